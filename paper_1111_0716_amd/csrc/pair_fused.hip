// Whole-pair kernels for cubic grids that fit one compute unit (L^3 with
// L in {16, 24, 32} in FP32, L = 16 in FP64).
//
// One workgroup of L*L threads owns one output band and walks its partner
// list (paper, "Our Implementation": the band-pair loops on the GPU, with
// every operation inside them on the device).  For each partner the pair
// grid never leaves the chip: each thread holds one line of L values in
// registers, transforms it there, and the three axis switches go through LDS
// transposes (in two rounds when the grid is larger than LDS):
//
//   layout A  thread (j1, j3) holds the line along axis 2   (coalesced loads)
//   layout B  thread (c2, j3) holds the line along axis 1
//   layout C  thread (c2, c1) holds the line along axis 3   (kernel multiply)
//
// forward: load rho in A -> FFT_2 -> B -> FFT_1 -> C -> FFT_3 -> x v_q/N
// inverse: IFFT_3 -> B -> IFFT_1 -> A -> IFFT_2 -> acc += coef u_m W
// The kernel table is stored for this path in C order, (c3*L + c2)*L + c1, so
// the multiply reads it coalesced.  V_x u is accumulated in registers when
// the accumulator fits beside the line, else read-modify-written per partner.
#include <algorithm>

#include "fft_lds.hpp"
#include "fock_internal.hpp"
#include "reg_fft.hpp"

namespace fock {

// Compiler-only barrier: memory operations are not moved across it (keeps the
// number of outstanding loads, and so the live registers, bounded).
__device__ __forceinline__ void mem_fence_compiler() { asm volatile("" ::: "memory"); }

// A copy of a uniform element offset the compiler cannot see through: loads
// made with it are issued where written, not hoisted out of the partner loop
// or reused from earlier loads (both would pin whole lines in registers).
__device__ __forceinline__ size_t opaque_idx(size_t v) {
  // the value is uniform over the workgroup; make that explicit for the SGPR constraint
  uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return (static_cast<size_t>(hi) << 32) | lo;
}

// Per-thread 32-bit element offset, re-materialised where used (not hoisted).
__device__ __forceinline__ uint32_t opaque_off(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <typename T, int L>
struct FusedShape {
  using C = typename cx<T>::t;
  // lines per thread: two when one line per thread would leave too few registers
  static constexpr int LPT = (L == 32) ? 2 : 1;
  static constexpr int NT = L * L / LPT;  // threads
  static constexpr int RPT = L / LPT;     // rows covered by one line index
  // rounds needed so one round of a transpose fits in LDS (160 KiB less a margin)
  static constexpr int NR = (static_cast<size_t>(L) * L * (L + 1) * sizeof(C) <= 150 * 1024) ? 1 : 2;
  static constexpr int CH = L / NR;
  static constexpr int LP = L + 1;
  static constexpr int XA = L * L * CH;   // [c2][j1][j3 - r*CH]
  static constexpr int XB = CH * L * LP;  // [c2 - r*CH][c1][j3] (padded rows)
  static constexpr int LDS = XA > XB ? XA : XB;
  // accumulate V_x u in registers when it fits beside the lines
  static constexpr bool ACC_REG = (L <= 16) || (L <= 24 && sizeof(T) == 4);
  // 128-byte lines of one orbital and of one table, and their share per thread
  static constexpr int ORB_LINES = (L * L * L * static_cast<int>(sizeof(C))) / 128;
  static constexpr int TAB_LINES = (L * L * L * static_cast<int>(sizeof(T))) / 128;
  static constexpr int PF_ORB = (ORB_LINES + NT - 1) / NT;
  static constexpr int PF_TAB = (TAB_LINES + NT - 1) / NT;
};

// Pull the next orbital and kernel table into L2 while the FFTs run: one
// dword of every 128-byte line is loaded with the LDS-DMA form of the load,
// which needs no destination register.  All waves land their dwords in the
// same dead 256-byte LDS area (`junk`); nothing ever reads it.
typedef __attribute__((address_space(1))) const void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;

// What to pull into L2 during the forward transform (null orb: nothing).
template <typename T>
struct Prefetch {
  const typename cx<T>::t* orb;
  const T* tab;
  float* junk;
};

template <typename T, int L>
__device__ __forceinline__ void prefetch_lines(const typename cx<T>::t* orb, const T* tab, int t, float* junk) {
  using Sh = FusedShape<T, L>;
  const float* o = reinterpret_cast<const float*>(orb);
  const float* b = reinterpret_cast<const float*>(tab);
#pragma unroll
  for (int k = 0; k < Sh::PF_ORB; ++k) {
    const int line = t + k * Sh::NT;
    if (line < Sh::ORB_LINES) __builtin_amdgcn_global_load_lds((gptr_t)(o + line * 32), (lptr_t)junk, 4, 0, 0);
  }
#pragma unroll
  for (int k = 0; k < Sh::PF_TAB; ++k) {
    const int line = t + k * Sh::NT;
    if (line < Sh::TAB_LINES) __builtin_amdgcn_global_load_lds((gptr_t)(b + line * 32), (lptr_t)junk, 4, 0, 0);
  }
}

// LDS element at a byte address (base VGPR + immediate offset when the
// offset is a compile-time constant below 64 KiB).
template <typename C>
__device__ __forceinline__ C& lds_at(unsigned char* s, uint32_t byte_off) {
  return *reinterpret_cast<C*>(s + byte_off);
}

// Accessor for the large-stride side of a transpose: element i of a run with
// a stride of STRIDE bytes from `base`.  Two opaque bases (for the first and
// second half of the run) keep every offset an immediate.
template <typename C, int L, int STRIDE>
struct StridedRun {
  static constexpr int H = (65535 / STRIDE) + 1 < L ? (65535 / STRIDE) + 1 : L;  // elements per base
  uint32_t b0, b1;
  __device__ __forceinline__ explicit StridedRun(uint32_t base)
      : b0(opaque_off(base)), b1(opaque_off(base + H * STRIDE)) {}
  __device__ __forceinline__ C& at(unsigned char* s, int i) const {
    return i < H ? lds_at<C>(s, b0 + i * STRIDE) : lds_at<C>(s, b1 + (i - H) * STRIDE);
  }
};

// Thread t owns lines (row0 + l*RPT, col) for l < LPT, with row0 = t / L.
//
// A (row = j1, col = j3, x over c2) <-> B (row = c2, col = j3, x over j1).
// The column index j3 is the same in both layouts; rounds split it.
// LDS layout [c2][j1][j3 - r*CH]: index (c2*L + j1)*CH + cc.
template <typename T, int L, bool A_TO_B>
__device__ __forceinline__ void xchg_ab(typename cx<T>::t (*x)[L], typename cx<T>::t* sp, int row0, int col) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  constexpr int SZ = sizeof(C);
  constexpr int BIG = L * Sh::CH * SZ;  // stride of c2
  unsigned char* s = reinterpret_cast<unsigned char*>(sp);
#pragma unroll
  for (int r = 0; r < Sh::NR; ++r) {
    const bool mine = (col / Sh::CH) == r;
    const int cc = col - r * Sh::CH;
    // write side: A writes x[c2 = i] at (i, row) (stride BIG); B writes x[j1 = i] at (row, i) (stride CH)
    if (mine) {
#pragma unroll
      for (int l = 0; l < Sh::LPT; ++l) {
        const int row = row0 + l * Sh::RPT;
        if (A_TO_B) {
          const StridedRun<C, L, BIG> run(static_cast<uint32_t>((row * Sh::CH + cc) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) run.at(s, i) = x[l][i];
        } else {
          const uint32_t b = opaque_off(static_cast<uint32_t>(((row * L) * Sh::CH + cc) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) lds_at<C>(s, b + i * Sh::CH * SZ) = x[l][i];
        }
      }
    }
    __syncthreads();
    if (mine) {
#pragma unroll
      for (int l = 0; l < Sh::LPT; ++l) {
        const int row = row0 + l * Sh::RPT;
        if (A_TO_B) {
          const uint32_t b = opaque_off(static_cast<uint32_t>(((row * L) * Sh::CH + cc) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) x[l][i] = lds_at<C>(s, b + i * Sh::CH * SZ);
        } else {
          const StridedRun<C, L, BIG> run(static_cast<uint32_t>((row * Sh::CH + cc) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) x[l][i] = run.at(s, i);
        }
      }
    }
    __syncthreads();
  }
}

// B (row = c2, col = j3, x over c1) <-> C (row = c2, col = c1, x over j3).
// The row index c2 is the same in both layouts; rounds split it.  When each
// thread has one line per round (LPT == NR), line l is exchanged in round l.
// LDS layout [c2 - r*CH][c1][j3] with padded rows: ((rr*L + c1)*LP + j3).
template <typename T, int L, bool B_TO_C>
__device__ __forceinline__ void xchg_bc(typename cx<T>::t (*x)[L], typename cx<T>::t* sp, int row0, int col,
                                        Prefetch<T> pf = Prefetch<T>{nullptr, nullptr, nullptr}) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  constexpr int SZ = sizeof(C);
  unsigned char* s = reinterpret_cast<unsigned char*>(sp);
#pragma unroll
  for (int r = 0; r < Sh::NR; ++r) {
#pragma unroll
    for (int l = 0; l < Sh::LPT; ++l) {
      const int row = row0 + l * Sh::RPT;
      const bool mine = (Sh::LPT == Sh::NR) ? (l == r) : ((row / Sh::CH) == r);
      if (mine) {
        const int rr = row - r * Sh::CH;
        if (B_TO_C) {  // B writes x[c1 = i] at (c1 = i, j3 = col)
          const uint32_t b = opaque_off(static_cast<uint32_t>(((rr * L) * Sh::LP + col) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) lds_at<C>(s, b + i * Sh::LP * SZ) = x[l][i];
        } else {  // C writes x[j3 = i] at (c1 = col, j3 = i)
          const uint32_t b = opaque_off(static_cast<uint32_t>(((rr * L + col) * Sh::LP) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) lds_at<C>(s, b + i * SZ) = x[l][i];
        }
      }
    }
    __syncthreads();
    // the line just written is dead until read back: the cheapest moment to
    // issue the L2 prefetch of the next partner
    if (r == 0 && pf.orb) prefetch_lines<T, L>(pf.orb, pf.tab, static_cast<int>(threadIdx.x), pf.junk);
#pragma unroll
    for (int l = 0; l < Sh::LPT; ++l) {
      const int row = row0 + l * Sh::RPT;
      const bool mine = (Sh::LPT == Sh::NR) ? (l == r) : ((row / Sh::CH) == r);
      if (mine) {
        const int rr = row - r * Sh::CH;
        if (B_TO_C) {  // C reads x[j3 = i] at (c1 = col, j3 = i)
          const uint32_t b = opaque_off(static_cast<uint32_t>(((rr * L + col) * Sh::LP) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) x[l][i] = lds_at<C>(s, b + i * SZ);
        } else {  // B reads x[c1 = i] at (c1 = i, j3 = col)
          const uint32_t b = opaque_off(static_cast<uint32_t>(((rr * L) * Sh::LP + col) * SZ));
#pragma unroll
          for (int i = 0; i < L; ++i) x[l][i] = lds_at<C>(s, b + i * Sh::LP * SZ);
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int L, int S>
__device__ __forceinline__ void reg_fft_lines(typename cx<T>::t (*x)[L]) {
  using Sh = FusedShape<T, L>;
#pragma unroll
  for (int l = 0; l < Sh::LPT; ++l) {
    __builtin_amdgcn_sched_barrier(0);  // one line at a time
    reg_fft<typename cx<T>::t, L, S>(x[l]);
  }
  __builtin_amdgcn_sched_barrier(0);
}

// rho in layout A -> P (c1, c2, c3) in layout C
template <typename T, int L>
__device__ __forceinline__ void fused_forward(typename cx<T>::t (*x)[L], typename cx<T>::t* s, int row0, int col,
                                              Prefetch<T> pf = Prefetch<T>{nullptr, nullptr, nullptr}) {
  reg_fft_lines<T, L, -1>(x);
  xchg_ab<T, L, true>(x, s, row0, col);
  reg_fft_lines<T, L, -1>(x);
  xchg_bc<T, L, true>(x, s, row0, col, pf);
  reg_fft_lines<T, L, -1>(x);
}

template <typename T, int L>
__device__ __forceinline__ void fused_inverse(typename cx<T>::t (*x)[L], typename cx<T>::t* s, int row0, int col) {
  reg_fft_lines<T, L, +1>(x);
  xchg_bc<T, L, false>(x, s, row0, col);
  reg_fft_lines<T, L, +1>(x);
  xchg_ab<T, L, false>(x, s, row0, col);
  reg_fft_lines<T, L, +1>(x);
}

// Element e of the thread's lines in layout A: line e / L, index e % L.
// Loads below are issued in batches of kB elements with the next batch in
// flight while the current one is consumed (two batches of registers), so a
// phase costs about one memory latency instead of one per batch.
constexpr int kB = 8;

// rho = conj(u_m) u_n, both orbitals double-buffered.
template <typename T, int L>
__device__ __forceinline__ void load_codensity(typename cx<T>::t (*x)[L], const typename cx<T>::t* __restrict__ bm,
                                               const typename cx<T>::t* __restrict__ bn, uint32_t toff) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  constexpr int E = Sh::LPT * L;
  constexpr int NB = E / kB;
  static_assert(E % kB == 0, "batch size must divide the thread's elements");
  C mb[2][kB], nb[2][kB];
#pragma unroll
  for (int j = 0; j < kB; ++j) {
    const uint32_t a = toff + (j / L) * (Sh::RPT * L * L) + (j % L) * L;
    mb[0][j] = bm[a];
    nb[0][j] = bn[a];
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b + 1 < NB) {
#pragma unroll
      for (int j = 0; j < kB; ++j) {
        const int e = (b + 1) * kB + j;
        const uint32_t a = toff + (e / L) * (Sh::RPT * L * L) + (e % L) * L;
        mb[(b + 1) & 1][j] = bm[a];
        nb[(b + 1) & 1][j] = bn[a];
      }
    }
    mem_fence_compiler();
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int e = b * kB + j;
      x[e / L][e % L] = cmulconj(mb[b & 1][j], nb[b & 1][j]);
    }
  }
}

// x *= v for the thread's lines in layout C (table in C order), double-buffered.
// EN: also es += v |x|^2 in FP64 (the pair's energy share of this thread).
template <typename T, int L, bool EN = false>
__device__ __forceinline__ void mul_kernel(typename cx<T>::t (*x)[L], const T* __restrict__ v, uint32_t tv,
                                           double& es) {
  using Sh = FusedShape<T, L>;
  constexpr int E = Sh::LPT * L;
  constexpr int NB = E / kB;
  T vb[2][kB];
#pragma unroll
  for (int j = 0; j < kB; ++j) vb[0][j] = v[tv + (j / L) * (Sh::RPT * L) + (j % L) * (L * L)];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b + 1 < NB) {
#pragma unroll
      for (int j = 0; j < kB; ++j) {
        const int e = (b + 1) * kB + j;
        vb[(b + 1) & 1][j] = v[tv + (e / L) * (Sh::RPT * L) + (e % L) * (L * L)];
      }
    }
    mem_fence_compiler();
#pragma unroll
    for (int j = 0; j < kB; ++j) {
      const int e = b * kB + j;
      if constexpr (EN) {
        const double px = static_cast<double>(x[e / L][e % L].x), py = static_cast<double>(x[e / L][e % L].y);
        es += static_cast<double>(vb[b & 1][j]) * (px * px + py * py);
      }
      x[e / L][e % L] = cscale(x[e / L][e % L], vb[b & 1][j]);
    }
  }
}

// ---------------------------------------------------------------------------
// apply / backward: one workgroup per output band, all partners of its list
// ---------------------------------------------------------------------------
// ENERGY (apply only): the forward transforms of the apply also give the
// pair energies; each block writes w_k f_n sum_p w'_p f'_p sum_c v/N |P|^2
// over its partners to eblk[block] (FP64), so that E_x needs no transforms
// of its own.
template <typename T, int L, bool ENERGY = false>
__global__ __launch_bounds__((FusedShape<T, L>::NT)) void k_pair_fused(
    int nbands, long long bs, int o0, int nout, const typename cx<T>::t* __restrict__ psi,
    const int2* __restrict__ parts, int npart, int nsplit, int nk, const int* __restrict__ qmap,
    const T* __restrict__ vtab, const double* __restrict__ occ, const double* __restrict__ kw,
    typename cx<T>::t* __restrict__ out, typename cx<T>::t* __restrict__ partial, const double* __restrict__ gscale,
    double hscale, int backward, double* __restrict__ eblk) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  constexpr int LL = L * L;
  constexpr int LPT = Sh::LPT;
  extern __shared__ unsigned char smem_raw[];
  __shared__ float junk[64];  // landing area of the L2 prefetch (never read)
  C* s = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x, row0 = t / L, col = t - (t / L) * L;
  // block = (output, partner slice); slice 0 writes the output, slice s > 0 a partial
  const int oi = blockIdx.x % nout, slice = blockIdx.x / nout;
  const int okn = o0 + oi;
  const int ok = okn / nbands;
  const int p0 = static_cast<int>((static_cast<long long>(npart) * slice) / nsplit);
  const int p1 = static_cast<int>((static_cast<long long>(npart) * (slice + 1)) / nsplit);
  double f = hscale;
  if (gscale) f *= gscale[0];
  if (backward) f *= kw[ok] * occ[okn];
  const size_t npts = static_cast<size_t>(LL) * L;
  const size_t on = static_cast<size_t>(okn) * bs;
  // destination of this block's sum: the output band, or its partial slot
  C* const dst = slice == 0 ? out : partial;
  const size_t od = slice == 0 ? on : (static_cast<size_t>(slice - 1) * nout + oi) * npts;
  const uint32_t toff0 = static_cast<uint32_t>(row0 * LL + col);  // layout A element (j1 = row0, 0, j3 = col)
  C acc[Sh::ACC_REG ? LPT : 1][Sh::ACC_REG ? L : 1];
  if constexpr (Sh::ACC_REG) {
#pragma unroll
    for (int l = 0; l < LPT; ++l)
#pragma unroll
      for (int i = 0; i < L; ++i) acc[l][i] = C{T(0), T(0)};
  }
  // ENERGY: per thread, sum over partners of w' f' e (its share), kept in LDS
  // so that no register is carried through the partner loop
  __shared__ double eslot[ENERGY ? Sh::NT : 1];
  if constexpr (ENERGY) eslot[t] = 0.0;
  const double wn = ENERGY ? kw[ok] * occ[okn] : 0.0;  // w_k f_n of the output
  for (int p = p0; p < p1; ++p) {
    const int2 r = parts[p];
    const int pkm = r.x * nbands + r.y;
    const size_t om = static_cast<size_t>(pkm) * bs;
    C x[LPT][L];
    load_codensity<T, L>(x, psi + opaque_idx(om), psi + opaque_idx(on), opaque_off(toff0));
    // warm L2 with the next partner's orbital and kernel table while the FFTs run
    Prefetch<T> pf{nullptr, nullptr, junk};
    if (p + 1 < p1) {
      const int2 rn = parts[p + 1];
      pf.orb = psi + static_cast<size_t>(rn.x * nbands + rn.y) * bs;
      pf.tab = vtab + static_cast<size_t>(qmap[ok * nk + rn.x]) * npts;
    }
    fused_forward<T, L>(x, s, row0, col, pf);
    double esum = 0.0;
    mul_kernel<T, L, ENERGY>(x, vtab + static_cast<size_t>(qmap[ok * nk + r.x]) * npts,
                             opaque_off(static_cast<uint32_t>(t)), esum);
    if constexpr (ENERGY) eslot[t] += wn * kw[r.x] * occ[pkm] * esum;  // only this thread touches eslot[t]
    fused_inverse<T, L>(x, s, row0, col);
    const T coef = static_cast<T>(-kw[r.x] * occ[pkm] * f);
    const C* bm = psi + opaque_idx(om);
    C* bo = dst + opaque_idx(od);
    const uint32_t toff = opaque_off(toff0);
    // accumulate: u_m (and the running output) in double-buffered batches
    constexpr int E = LPT * L;
    // smaller batches here: x, u_m and the output are live together (with the
    // energy epilogue two, which keeps its spill below the plain kernel's)
    constexpr int kA = ENERGY ? 2 : 4;
    constexpr int NB = E / kA;
    C mb[2][kA], ob[2][kA];
    const bool rmw = !Sh::ACC_REG && p > p0;
#pragma unroll
    for (int j = 0; j < kA; ++j) {
      const uint32_t a = toff + (j / L) * (Sh::RPT * LL) + (j % L) * L;
      mb[0][j] = bm[a];
      if (rmw) ob[0][j] = bo[a];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b + 1 < NB) {
#pragma unroll
        for (int j = 0; j < kA; ++j) {
          const int e = (b + 1) * kA + j;
          const uint32_t a = toff + (e / L) * (Sh::RPT * LL) + (e % L) * L;
          mb[(b + 1) & 1][j] = bm[a];
          if (rmw) ob[(b + 1) & 1][j] = bo[a];
        }
      }
      mem_fence_compiler();
#pragma unroll
      for (int j = 0; j < kA; ++j) {
        const int e = b * kA + j;
        const C w = cscale(cmul(mb[b & 1][j], x[e / L][e % L]), coef);
        if constexpr (Sh::ACC_REG) {
          acc[e / L][e % L] = cadd(acc[e / L][e % L], w);
        } else {
          const uint32_t a = toff + (e / L) * (Sh::RPT * LL) + (e % L) * L;
          bo[a] = rmw ? cadd(ob[b & 1][j], w) : w;
        }
      }
    }
  }
  if constexpr (Sh::ACC_REG) {
    C* bo = dst + od;
#pragma unroll
    for (int l = 0; l < LPT; ++l) {
      const uint32_t off = toff0 + static_cast<uint32_t>(l * Sh::RPT * LL);
#pragma unroll
      for (int i = 0; i < L; ++i) bo[off + i * L] = acc[l][i];
    }
  }
  if constexpr (ENERGY) {
    // fixed-order block sum by the first wave: lane l takes l, l + 64, ...
    __syncthreads();
    if (t < 64) {
      double e = 0.0;
      for (int i = t; i < Sh::NT; i += 64) e += eslot[i];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
      if (t == 0) eblk[blockIdx.x] = e;
    }
  }
}

// ---------------------------------------------------------------------------
// apply / backward by unordered pairs: one workgroup per pair of a round
// ---------------------------------------------------------------------------
// bo[j] += coef * bm[j] * x[j] (CONJ: * conj(x[j])) over the thread's lines in
// layout A, in double-buffered batches of kA (u and the output are read
// together, the sum written back).
template <typename T, int L, bool CONJ, int kA>
__device__ __forceinline__ void rmw_accumulate(typename cx<T>::t (*x)[L], const typename cx<T>::t* __restrict__ bm,
                                               typename cx<T>::t* __restrict__ bo, uint32_t toff, T coef) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  constexpr int LL = L * L;
  constexpr int E = Sh::LPT * L;
  constexpr int NB = E / kA;
  static_assert(E % kA == 0, "batch size must divide the thread's elements");
  C mb[2][kA], ob[2][kA];
#pragma unroll
  for (int j = 0; j < kA; ++j) {
    const uint32_t a = toff + (j / L) * (Sh::RPT * LL) + (j % L) * L;
    mb[0][j] = bm[a];
    ob[0][j] = bo[a];
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (b + 1 < NB) {
#pragma unroll
      for (int j = 0; j < kA; ++j) {
        const int e = (b + 1) * kA + j;
        const uint32_t a = toff + (e / L) * (Sh::RPT * LL) + (e % L) * L;
        mb[(b + 1) & 1][j] = bm[a];
        ob[(b + 1) & 1][j] = bo[a];
      }
    }
    mem_fence_compiler();
#pragma unroll
    for (int j = 0; j < kA; ++j) {
      const int e = b * kA + j;
      const C u = mb[b & 1][j];
      const C w = CONJ ? cmulconj(x[e / L][e % L], u) : cmul(u, x[e / L][e % L]);
      const uint32_t a = toff + (e / L) * (Sh::RPT * LL) + (e % L) * L;
      bo[a] = cadd(ob[b & 1][j], cscale(w, coef));
    }
  }
}

// One unordered pair (a, b), a <= b (global band indices k nbands + n), per
// workgroup: W_ab = IDFT(v_q DFT(conj(u_b) u_a)) once, then
//   out_a += -w_kb f_b F_a u_b W_ab,   out_b += -w_ka f_a F_b u_a conj(W_ab)
// (W_ba = conj(W_ab): the Nyquist-averaged kernel is even under (c, q) ->
// (-c, -q)); a == b adds the first only.  F_x is the output factor (hscale,
// gscale and, for the backward, w_kx f_x).  The pairs of one launch are
// pairwise disjoint, so no output is written by two workgroups; the outputs
// were zeroed before the first round.  ENERGY: eblk[pair] = w_a f_a w_b f_b
// sum_c v/N |P|^2, times 2 when a != b (the pair stands for both orders).
template <typename T, int L, bool ENERGY = false>
__global__ __launch_bounds__((FusedShape<T, L>::NT)) void k_pair_fused_sym(
    int nbands, long long bs, const typename cx<T>::t* __restrict__ psi, const int2* __restrict__ pairs, int nk,
    const int* __restrict__ qmap, const T* __restrict__ vtab, const double* __restrict__ occ,
    const double* __restrict__ kw, typename cx<T>::t* __restrict__ out, const double* __restrict__ gscale,
    double hscale, int backward, double* __restrict__ eblk) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  static_assert(!Sh::ACC_REG, "pair rounds serve the grids whose output is read-modify-written per pair");
  constexpr int LL = L * L;
  constexpr int LPT = Sh::LPT;
  extern __shared__ unsigned char smem_raw[];
  __shared__ float junk[64];  // landing area of the L2 prefetch (never read)
  __shared__ double eslot[ENERGY ? Sh::NT : 1];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x, row0 = t / L, col = t - (t / L) * L;
  const int2 pr = pairs[blockIdx.x];
  const int a = pr.x, b = pr.y;
  const int ka = a / nbands, kb = b / nbands;
  double g = hscale;
  if (gscale) g *= gscale[0];
  const double fa = backward ? g * kw[ka] * occ[a] : g;
  const double fb = backward ? g * kw[kb] * occ[b] : g;
  const size_t npts = static_cast<size_t>(LL) * L;
  const size_t oa = static_cast<size_t>(a) * bs, ob = static_cast<size_t>(b) * bs;
  const uint32_t toff0 = static_cast<uint32_t>(row0 * LL + col);  // layout A element (j1 = row0, 0, j3 = col)
  const T* tab = vtab + static_cast<size_t>(qmap[ka * nk + kb]) * npts;
  C x[LPT][L];
  load_codensity<T, L>(x, psi + opaque_idx(ob), psi + opaque_idx(oa), opaque_off(toff0));
  // warm L2 with the first output (read back after the transforms) and the table
  fused_forward<T, L>(x, s, row0, col, Prefetch<T>{out + oa, tab, junk});
  double esum = 0.0;
  mul_kernel<T, L, ENERGY>(x, tab, opaque_off(static_cast<uint32_t>(t)), esum);
  if constexpr (ENERGY) eslot[t] = esum;
  fused_inverse<T, L>(x, s, row0, col);
  constexpr int kA = ENERGY ? 2 : 4;
  rmw_accumulate<T, L, false, kA>(x, psi + opaque_idx(ob), out + opaque_idx(oa), opaque_off(toff0),
                                  static_cast<T>(-kw[kb] * occ[b] * fa));
  if (a != b)
    rmw_accumulate<T, L, true, kA>(x, psi + opaque_idx(oa), out + opaque_idx(ob), opaque_off(toff0),
                                   static_cast<T>(-kw[ka] * occ[a] * fb));
  if constexpr (ENERGY) {
    // fixed-order block sum by the first wave: lane l takes l, l + 64, ...
    __syncthreads();
    if (t < 64) {
      double e = 0.0;
      for (int i = t; i < Sh::NT; i += 64) e += eslot[i];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
      if (t == 0) eblk[blockIdx.x] = (a != b ? 2.0 : 1.0) * kw[ka] * occ[a] * kw[kb] * occ[b] * e;
    }
  }
}

// ---------------------------------------------------------------------------
// energy: per pair sum_c v_q(c)/N |P(c)|^2 in FP64, `per_wg` pairs per block
// ---------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__((FusedShape<T, L>::NT)) void k_pair_energy_fused(
    int nbands, long long bs, const typename cx<T>::t* __restrict__ psi, const PairRef* __restrict__ pairs,
    int npairs, int per_wg, const T* __restrict__ vtab, double* __restrict__ epart) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  constexpr int LL = L * L;
  constexpr int LPT = Sh::LPT;
  constexpr int NW = (Sh::NT + 63) / 64;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[NW];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x, row0 = t / L, col = t - (t / L) * L;
  const size_t npts = static_cast<size_t>(LL) * L;
  for (int i0 = 0; i0 < per_wg; ++i0) {
    const int pi = blockIdx.x * per_wg + i0;
    if (pi >= npairs) break;  // uniform over the block
    const PairRef pr = pairs[pi];
    C x[LPT][L];
    load_codensity<T, L>(x, psi + opaque_idx(static_cast<size_t>(pr.kp * nbands + pr.m) * bs),
                         psi + opaque_idx(static_cast<size_t>(pr.k * nbands + pr.n) * bs),
                         opaque_off(static_cast<uint32_t>(row0 * LL + col)));
    fused_forward<T, L>(x, s, row0, col);
    // |P|^2 in place (x[.].x), then weight by the table
#pragma unroll
    for (int l = 0; l < LPT; ++l)
#pragma unroll
      for (int i = 0; i < L; ++i) x[l][i] = C{x[l][i].x * x[l][i].x + x[l][i].y * x[l][i].y, T(0)};
    double e = 0.0;
    {
      const T* v = vtab + static_cast<size_t>(pr.q) * npts;
      const uint32_t tv = opaque_off(static_cast<uint32_t>(t));
      constexpr int E = LPT * L;
      constexpr int NB = E / kB;
      T vb[2][kB];
#pragma unroll
      for (int j = 0; j < kB; ++j) vb[0][j] = v[tv + (j / L) * (Sh::RPT * L) + (j % L) * LL];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB) {
#pragma unroll
          for (int j = 0; j < kB; ++j) {
            const int q = (b + 1) * kB + j;
            vb[(b + 1) & 1][j] = v[tv + (q / L) * (Sh::RPT * L) + (q % L) * LL];
          }
        }
        mem_fence_compiler();
#pragma unroll
        for (int j = 0; j < kB; ++j) {
          const int q = b * kB + j;
          e += static_cast<double>(vb[b & 1][j]) * static_cast<double>(x[q / L][q % L].x);
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if ((t & 63) == 0) red[t >> 6] = e;
    __syncthreads();
    if (t == 0) {
      double tot = 0.0;
      for (int w = 0; w < NW; ++w) tot += red[w];
      epart[pi] = tot;
    }
    __syncthreads();
  }
}

// out[o0 + o] += sum_s partial[s][o] (fixed order), one output per blockIdx.y
template <typename T>
__global__ __launch_bounds__(256) void k_add_partials(typename cx<T>::t* __restrict__ out, long long bs, int o0, int nout,
                                                       const typename cx<T>::t* __restrict__ partial, int nparts,
                                                       long long npts) {
  using C = typename cx<T>::t;
  const int o = blockIdx.y;
  C* dst = out + static_cast<size_t>(o0 + o) * bs;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < npts; e += static_cast<long long>(gridDim.x) * 256) {
    C v = dst[e];
    for (int sl = 0; sl < nparts; ++sl) v = cadd(v, partial[(static_cast<size_t>(sl) * nout + o) * npts + e]);
    dst[e] = v;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <typename T, int L, bool ENERGY>
void launch_pair_fused(const Plan& p, const FusedGroup& g, const void* psi, const double* occ, void* out,
                       const double* gscale, double hscale, bool backward, double* eblk) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  const Instance& in = p.inst[g.inst];
  const size_t lds = static_cast<size_t>(Sh::LDS) * sizeof(C);
  C* partial = reinterpret_cast<C*>(p.ws + p.partial_off);
  hipLaunchKernelGGL((k_pair_fused<T, L, ENERGY>), dim3(g.nout * g.nsplit), dim3(Sh::NT), lds, p.stream, in.nbands,
                     static_cast<long long>(in.band_stride), g.o0, g.nout, static_cast<const C*>(psi),
                     reinterpret_cast<const int2*>(p.ws + g.part_off), g.npart, g.nsplit, in.nk,
                     reinterpret_cast<const int*>(p.ws + in.qmap_off), reinterpret_cast<const T*>(p.ws + in.vtab_off),
                     occ, reinterpret_cast<const double*>(p.ws + in.kw_off), static_cast<C*>(out), partial, gscale,
                     hscale, backward ? 1 : 0, eblk);
}

// eblk: per-block energy partials of this group (null: no energy)
template <typename T, int L>
hipError_t fused_apply_L(const Plan& p, const FusedGroup& g, const void* psi, const double* occ, void* out,
                         const double* gscale, double hscale, bool backward, double* eblk) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[g.inst];
  C* partial = reinterpret_cast<C*>(p.ws + p.partial_off);
  p.prof.begin(FOCK_K_FUSED, p.stream);
  if (eblk)
    launch_pair_fused<T, L, true>(p, g, psi, occ, out, gscale, hscale, backward, eblk);
  else
    launch_pair_fused<T, L, false>(p, g, psi, occ, out, gscale, hscale, backward, nullptr);
  p.prof.end(FOCK_K_FUSED, p.stream);
  if (g.nsplit > 1) {
    const size_t npts = static_cast<size_t>(in.npts);
    const int gx = static_cast<int>(std::min<size_t>(4096, (npts + 255) / 256));
    p.prof.begin(FOCK_K_OTHER, p.stream);
    hipLaunchKernelGGL((k_add_partials<T>), dim3(gx, g.nout), dim3(256), 0, p.stream, static_cast<C*>(out),
                       static_cast<long long>(in.band_stride), g.o0, g.nout, static_cast<const C*>(partial),
                       g.nsplit - 1, static_cast<long long>(npts));
    p.prof.end(FOCK_K_OTHER, p.stream);
  }
  return hipGetLastError();
}

// The rounds of unordered pairs of one instance (outputs zeroed first).
template <typename T, int L>
hipError_t fused_rounds_L(const Plan& p, const FusedRounds& r, const void* psi, const double* occ, void* out,
                          const double* gscale, double hscale, bool backward, double* eblk) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  const Instance& in = p.inst[r.inst];
  const size_t lds = static_cast<size_t>(Sh::LDS) * sizeof(C);
  hipError_t e = launch_zero_all_bands(p, r.inst, out);
  if (e != hipSuccess) return e;
  const int2* pairs = reinterpret_cast<const int2*>(p.ws + r.pairs_off);
  const int* qmap = reinterpret_cast<const int*>(p.ws + in.qmap_off);
  const T* vtab = reinterpret_cast<const T*>(p.ws + in.vtab_off);
  const double* kw = reinterpret_cast<const double*>(p.ws + in.kw_off);
  for (size_t i = 0; i + 1 < r.round_start.size(); ++i) {
    const int p0 = r.round_start[i], n = r.round_start[i + 1] - p0;
    p.prof.begin(FOCK_K_FUSED, p.stream);
    if (eblk)
      hipLaunchKernelGGL((k_pair_fused_sym<T, L, true>), dim3(n), dim3(Sh::NT), lds, p.stream, in.nbands,
                         static_cast<long long>(in.band_stride), static_cast<const C*>(psi), pairs + p0, in.nk, qmap,
                         vtab, occ, kw, static_cast<C*>(out), gscale, hscale, backward ? 1 : 0, eblk + p0);
    else
      hipLaunchKernelGGL((k_pair_fused_sym<T, L, false>), dim3(n), dim3(Sh::NT), lds, p.stream, in.nbands,
                         static_cast<long long>(in.band_stride), static_cast<const C*>(psi), pairs + p0, in.nk, qmap,
                         vtab, occ, kw, static_cast<C*>(out), gscale, hscale, backward ? 1 : 0, nullptr);
    p.prof.end(FOCK_K_FUSED, p.stream);
  }
  return hipGetLastError();
}

template <typename T, int L>
hipError_t fused_energy_L(const Plan& p, const Batch& b, const void* psi) {
  using C = typename cx<T>::t;
  using Sh = FusedShape<T, L>;
  const Instance& in = p.inst[b.inst];
  const size_t lds = static_cast<size_t>(Sh::LDS) * sizeof(C);
  const int per_wg = b.per_wg;
  const int nwg = (b.npairs + per_wg - 1) / per_wg;
  p.prof.begin(FOCK_K_ENERGY_FUSED, p.stream);
  hipLaunchKernelGGL((k_pair_energy_fused<T, L>), dim3(nwg), dim3(Sh::NT), lds, p.stream, in.nbands,
                     static_cast<long long>(in.band_stride), static_cast<const C*>(psi),
                     reinterpret_cast<const PairRef*>(p.ws + b.pair_off), b.npairs, per_wg,
                     reinterpret_cast<const T*>(p.ws + in.vtab_off), reinterpret_cast<double*>(p.ws + p.epart_off));
  p.prof.end(FOCK_K_ENERGY_FUSED, p.stream);
  return hipGetLastError();
}

template <typename T>
hipError_t fused_apply_t(const Plan& p, const FusedGroup& g, const void* psi, const double* occ, void* out,
                         const double* gscale, double hscale, bool backward, double* eblk) {
  switch (p.inst[g.inst].grid[0]) {
    case 16: return fused_apply_L<T, 16>(p, g, psi, occ, out, gscale, hscale, backward, eblk);
    case 24:
      if constexpr (sizeof(T) == 4) return fused_apply_L<T, 24>(p, g, psi, occ, out, gscale, hscale, backward, eblk);
      break;
    case 32:
      if constexpr (sizeof(T) == 4) return fused_apply_L<T, 32>(p, g, psi, occ, out, gscale, hscale, backward, eblk);
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t fused_energy_t(const Plan& p, const Batch& b, const void* psi) {
  switch (p.inst[b.inst].grid[0]) {
    case 16: return fused_energy_L<T, 16>(p, b, psi);
    case 24:
      if constexpr (sizeof(T) == 4) return fused_energy_L<T, 24>(p, b, psi);
      break;
    case 32:
      if constexpr (sizeof(T) == 4) return fused_energy_L<T, 32>(p, b, psi);
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename T, int L>
void fused_lds_attr(int lim) {
  const void* fs[] = {reinterpret_cast<const void*>(&k_pair_fused<T, L, false>),
                      reinterpret_cast<const void*>(&k_pair_fused<T, L, true>),
                      reinterpret_cast<const void*>(&k_pair_energy_fused<T, L>)};
  for (const void* f : fs)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) (void)hipGetLastError();
  if constexpr (!FusedShape<T, L>::ACC_REG) {
    const void* fr[] = {reinterpret_cast<const void*>(&k_pair_fused_sym<T, L, false>),
                        reinterpret_cast<const void*>(&k_pair_fused_sym<T, L, true>)};
    for (const void* f : fr)
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
        (void)hipGetLastError();
  }
}

}  // namespace

bool fused_rounds_supported(fock_precision prec, const int grid[3]) {
  return prec == FOCK_C64 && grid[0] == 32 && grid[1] == 32 && grid[2] == 32 && !FusedShape<float, 32>::ACC_REG;
}

hipError_t launch_fused_rounds(const Plan& p, const FusedRounds& r, const void* psi, const double* occ, void* out,
                               const double* gscale, double hscale, bool backward, double* eblk) {
  if (p.prec != FOCK_C64 || p.inst[r.inst].grid[0] != 32) return hipErrorInvalidValue;
  return fused_rounds_L<float, 32>(p, r, psi, occ, out, gscale, hscale, backward, eblk);
}

bool fused_supported(fock_precision prec, const int grid[3]) {
  if (grid[0] != grid[1] || grid[0] != grid[2]) return false;
  const int L = grid[0];
  if (prec == FOCK_C64) return L == 16 || L == 24 || L == 32;
  return L == 16;  // FP64 24^3 would spill on this path; it takes the three-pass path
}

int fused_threads(fock_precision prec, int L) {
  if (prec == FOCK_C64) return L == 16 ? FusedShape<float, 16>::NT : L == 24 ? FusedShape<float, 24>::NT
                                                                            : FusedShape<float, 32>::NT;
  return FusedShape<double, 16>::NT;
}

size_t fused_lds_bytes(fock_precision prec, int L) {
  if (prec == FOCK_C64) {
    return L == 16 ? FusedShape<float, 16>::LDS * 8 : L == 24 ? FusedShape<float, 24>::LDS * 8
                                                              : FusedShape<float, 32>::LDS * 8;
  }
  return FusedShape<double, 16>::LDS * 16;
}

void prepare_fused_kernels(fock_precision prec, int lim) {
  if (prec == FOCK_C64) {
    fused_lds_attr<float, 16>(lim);
    fused_lds_attr<float, 24>(lim);
    fused_lds_attr<float, 32>(lim);
  } else {
    fused_lds_attr<double, 16>(lim);
  }
}

hipError_t launch_fused_apply(const Plan& p, const FusedGroup& g, const void* psi, const double* occ, void* out,
                              const double* gscale, double hscale, bool backward, double* eblk) {
  return p.prec == FOCK_C128 ? fused_apply_t<double>(p, g, psi, occ, out, gscale, hscale, backward, eblk)
                             : fused_apply_t<float>(p, g, psi, occ, out, gscale, hscale, backward, eblk);
}

hipError_t launch_fused_energy(const Plan& p, const Batch& b, const void* psi) {
  return p.prec == FOCK_C128 ? fused_energy_t<double>(p, b, psi) : fused_energy_t<float>(p, b, psi);
}

}  // namespace fock
