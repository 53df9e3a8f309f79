// Three-pass kernels with register-line FFTs for grids N1 x L x L that do not
// take the whole-pair kernels, N1 and L in {24, 32, 36, 40, 48, 50, 54, 60,
// 64, 72}: a line per lane (FP32 up to 60 in most passes, FP64 up to 32) or a
// line per lane pair (longer lines).  Same passes and batching as the LDS-Stockham kernels (paper,
// "Our Implementation": the band-pair loop on the GPU; NSIM-like blocks of
// outputs x partners), but every 1-D transform runs in one thread's registers
// on a whole line (reg_fft.hpp), a plane switches axes through one padded LDS
// transpose, and the pair buffer T is laid out [j1][c3][c2] (c2 fastest) so
// that every global access of every pass is coalesced across the lanes:
//
//   plane   thread (plane p, j3): column u along axis 2 -> FFT_2 -> LDS ->
//           thread (p, c2): row along axis 3 -> FFT_3 -> T[j1][c3][c2]
//   pencil  thread (c3, c2): line along axis 1 -> FFT_1 -> x v_q/N -> IFFT_1
//           (apply; the table is stored [c1][c3][c2]) or FP64 sum v |P|^2
//   acc     thread (p, c2): row of T -> IFFT_3 -> LDS -> thread (p, j3):
//           column -> IFFT_2 -> acc += -w' f' u_m W in registers, for every
//           partner of the batch; one write (or add) of the output per batch
//
// The plane and accumulate passes are compiled for the plane side L and take
// the plane count N1 at run time; the pencil pass is compiled for the line
// length N1 and takes the line count L^2 at run time.
#include <algorithm>

#include "fft_lds.hpp"
#include "fock_internal.hpp"
#include "reg_fft.hpp"
#include "split_fft.hpp"

namespace fock {

// Loads issued in batches with the next batch in flight while the current one
// is consumed: only two batches of operands are live beside the line, and a
// phase costs (elements / batch) - 1 memory latencies at most.
constexpr int kRegB = 8;

template <typename T, int L>
struct RegShape {
  using C = typename cx<T>::t;
  static constexpr int LP = L + 1;  // padded LDS row
  // axis switches go through LDS one component (real, then imaginary) at a time
  static constexpr int PLANE_LDS = L * LP * static_cast<int>(sizeof(T));
  // planes per workgroup: about 256 threads, two workgroups' LDS per compute unit
  static constexpr int PL0 = (256 / L) > 0 ? (256 / L) : 1;
  static constexpr int PL = (PL0 * PLANE_LDS <= 78 * 1024) ? PL0 : ((78 * 1024) / PLANE_LDS > 0 ? (78 * 1024) / PLANE_LDS : 1);
  static constexpr int NTP = PL * L;             // threads of the plane and accumulate passes
  static constexpr int LDS = PL * PLANE_LDS;
  // waves per SIMD each kernel is compiled for (register budget 512 / WPE):
  // two where the line (and the accumulator) leave room for the transform
  // without spilling, as measured on the compiled kernels
  static constexpr int LINE_REGS = L * static_cast<int>(sizeof(C)) / 4;
  static constexpr int WPE_PLANE = 2;
  static constexpr int WPE_PENCIL = L <= 48 ? 2 : 1;
  static constexpr int WPE_ACC = 2 * LINE_REGS <= 160 ? 2 : 1;
  // operand batches: larger where the kernel has a whole SIMD's registers
  static constexpr int PLANE_B = kRegB;
  static constexpr int ACC_B = (WPE_ACC == 1 && sizeof(T) == 4) ? 16 : kRegB;
  // 128-byte lines of a workgroup's planes of one pair, per thread
  static constexpr int PF_ACC = (PL * L * L * static_cast<int>(sizeof(C)) / 128 + NTP - 1) / NTP;
};


// Compiler-only barrier: loads are not hoisted across it.
__device__ __forceinline__ void reg_fence() { asm volatile("" ::: "memory"); }

// the largest batch size <= want that divides L
__host__ __device__ constexpr int batch_of(int L, int want) {
  int b = want < L ? want : L;
  while (L % b != 0) --b;
  return b;
}

// Output and partner slots (o, p) of pair slot pi of an apply batch: pi =
// o nP + p, or for a block paired with itself (tri) the unordered pairs
// o <= p, row-major over the upper triangle (row o starts at tri_slot(o, o)).
__host__ __device__ constexpr size_t tri_slot(int o, int p, int n) {
  return static_cast<size_t>(o) * n - static_cast<size_t>(o) * (o - 1) / 2 + static_cast<size_t>(p - o);
}

__device__ __forceinline__ void batch_pair(int pi, int nP, int tri, int* o, int* p) {
  if (!tri) {
    *o = pi / nP;
    *p = pi - *o * nP;
    return;
  }
  const double b = 2.0 * nP + 1.0;
  int r = static_cast<int>((b - sqrt(b * b - 8.0 * pi)) * 0.5);
  r = r < 0 ? 0 : (r > nP - 1 ? nP - 1 : r);
  while (r > 0 && tri_slot(r, r, nP) > static_cast<size_t>(pi)) --r;
  while (r + 1 < nP && tri_slot(r + 1, r + 1, nP) <= static_cast<size_t>(pi)) ++r;
  *o = r;
  *p = r + static_cast<int>(static_cast<size_t>(pi) - tri_slot(r, r, nP));
}

// complex value in another precision
template <typename C, typename CI>
__device__ __forceinline__ C cvt(CI v) {
  using T = decltype(C{}.x);
  return C{static_cast<T>(v.x), static_cast<T>(v.y)};
}

// x[j] = conj(b[j * stride]) a[j * stride], j < L: a straight into the line
// (all loads in flight at once), then b in batches of BW multiplied in place,
// so only one batch of operands is live beside the line.  The orbitals may
// be stored in a wider precision (CI) than the line (C): they are rounded on
// load.
template <typename C, int L, int BW = kRegB, typename CI = C>
__device__ __forceinline__ void load_codensity_line(C* x, const CI* __restrict__ a, const CI* __restrict__ b,
                                                    int stride) {
  constexpr int B = batch_of(L, BW);
  constexpr int NB = L / B;
#pragma unroll
  for (int j = 0; j < L; ++j) x[j] = cvt<C>(a[j * stride]);
  CI bb[2][B];
#pragma unroll
  for (int j = 0; j < B; ++j) bb[0][j] = b[j * stride];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    if (n + 1 < NB) {
#pragma unroll
      for (int j = 0; j < B; ++j) bb[(n + 1) & 1][j] = b[((n + 1) * B + j) * stride];
    }
    reg_fence();
#pragma unroll
    for (int j = 0; j < B; ++j) x[n * B + j] = cmulconj(cvt<C>(bb[n & 1][j]), x[n * B + j]);
  }
}

// x[j] *= v[j * stride], j < L
template <typename C, typename T, int L>
__device__ __forceinline__ void mul_table_line(C* x, const T* __restrict__ v, size_t stride) {
  constexpr int B = batch_of(L, kRegB);
  constexpr int NB = L / B;
  T vb[2][B];
#pragma unroll
  for (int j = 0; j < B; ++j) vb[0][j] = v[j * stride];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    if (n + 1 < NB) {
#pragma unroll
      for (int j = 0; j < B; ++j) vb[(n + 1) & 1][j] = v[((n + 1) * B + j) * stride];
    }
    reg_fence();
#pragma unroll
    for (int j = 0; j < B; ++j) x[n * B + j] = cscale(x[n * B + j], vb[n & 1][j]);
  }
}

// Pencil lines with the line count known only at run time: the address of
// element j is a wave-uniform base (scalar registers) plus the lane's 32-bit
// byte offset, so the loads of a line take no 64-bit address per element.
template <typename C>
__device__ __forceinline__ C* lane_at(C* u, unsigned o) {
  return reinterpret_cast<C*>(reinterpret_cast<uintptr_t>(u) + o);
}

// v, through an empty asm the compiler cannot see through: addresses built
// from the copy are formed where they are used instead of being kept live
// (two registers each) across the transform in between
__device__ __forceinline__ unsigned opaque(unsigned v) {
  asm volatile("" : "+v"(v));
  return v;
}

// x[j] *= u[j * stride] at the lane's byte offset o, j < L (u wave-uniform);
// EN: also *es += u |x|^2 in FP64, taken before the multiply
template <typename C, typename T, int L, bool EN = false>
__device__ __forceinline__ void mul_table_line_u(C* x, const T* __restrict__ u, unsigned o, size_t stride,
                                                 double* es = nullptr) {
  constexpr int B = batch_of(L, kRegB);
  constexpr int NB = L / B;
  T vb[2][B];
#pragma unroll
  for (int j = 0; j < B; ++j) vb[0][j] = *lane_at(u + j * stride, o);
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    if (n + 1 < NB) {
#pragma unroll
      for (int j = 0; j < B; ++j) vb[(n + 1) & 1][j] = *lane_at(u + ((n + 1) * B + j) * stride, o);
    }
    reg_fence();
#pragma unroll
    for (int j = 0; j < B; ++j) {
      if constexpr (EN) {
        const double px = static_cast<double>(x[n * B + j].x), py = static_cast<double>(x[n * B + j].y);
        *es += static_cast<double>(vb[n & 1][j]) * (px * px + py * py);
      }
      x[n * B + j] = cscale(x[n * B + j], vb[n & 1][j]);
    }
  }
}

// Block sum of the energy partials e of the 256 threads, times the pair
// weight w, into epart[pair * gridDim.x + block] (fixed order).
__device__ __forceinline__ void store_line_energy(double e, double w, double* __restrict__ epart) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0)
    epart[static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x] = w * (((red[0] + red[1]) + red[2]) + red[3]);
}

// Switch a plane's axis: thread `col` holds line x[i] = P[i][col]; afterwards
// it holds x[i] = P[col][i].  One component at a time through sp ([L][LP]
// of T, this plane's share of LDS); every thread of the block must call it.
template <typename C, typename T, int L>
__device__ __forceinline__ void transpose_plane(C* x, T* sp, int col) {
  constexpr int LP = L + 1;
  __syncthreads();  // earlier readers of sp are done
#pragma unroll
  for (int i = 0; i < L; ++i) sp[i * LP + col] = x[i].x;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < L; ++i) x[i].x = sp[col * LP + i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < L; ++i) sp[i * LP + col] = x[i].y;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < L; ++i) x[i].y = sp[col * LP + i];
}

// The line through LDS and back in place: each thread its own slots, after
// one barrier for earlier readers of sp.  The values do not change; after the
// last transform of the FP32 72-point plane pass it lets the compiler
// allocate that kernel without scratch (205 registers, where it otherwise
// keeps about 40 values of the second transform in 156 bytes of scratch per
// lane at the 256 registers of two waves per SIMD).
template <typename C, typename T, int L>
__device__ __forceinline__ void lds_round_trip(C* x, T* sp, int col) {
  constexpr int LP = L + 1;
  __syncthreads();  // earlier readers of sp are done
#pragma unroll
  for (int i = 0; i < L; ++i) sp[i * LP + col] = x[i].x;
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < L; ++i) x[i].x = sp[i * LP + col];
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < L; ++i) sp[i * LP + col] = x[i].y;
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < L; ++i) x[i].y = sp[i * LP + col];
}

// ---------------------------------------------------------------------------
// plane pass: rho = conj(u_m) u_n, FFT along axes 2 and 3, T[j1][c3][c2]
// ---------------------------------------------------------------------------
// (orbitals wider than the transform, FOCK_MIXED: one wave per SIMD, so the
// wide operands fit beside the line without spilling)
// SLAB: the pair buffer leaves as [j1][c2][c3] (one more transpose) for the
// slab pencil; otherwise as [j1][c3][c2]
template <typename T, int L, bool EXPLICIT, typename TI = T, bool SLAB = false>
__global__ __launch_bounds__((RegShape<T, L>::NTP), (sizeof(TI) == sizeof(T) ? RegShape<T, L>::WPE_PLANE : 1)) void k_plane_reg(
    int n1, int nbands, long long bs, const typename cx<TI>::t* __restrict__ psi, int o0, int nP, int tri,
    const int2* __restrict__ parts, const PairRef* __restrict__ pairs, typename cx<T>::t* __restrict__ tbuf, int pf) {
  using C = typename cx<T>::t;
  using Sh = RegShape<T, L>;
  constexpr int LL = L * L;
  extern __shared__ unsigned char smem_raw[];
  const int t = threadIdx.x, pl = t / L, col = t - (t / L) * L;
  // pf: pairs fastest in the grid (blockIdx.x the pair slot)
  const int j1 = static_cast<int>(pf ? blockIdx.y : blockIdx.x) * Sh::PL + pl;
  const bool valid = j1 < n1;
  const int pi = static_cast<int>(pf ? blockIdx.x : blockIdx.y);
  int okn, pkm;
  if (EXPLICIT) {
    const PairRef pr = pairs[pi];
    okn = pr.k * nbands + pr.n;
    pkm = pr.kp * nbands + pr.m;
  } else {
    int o, p;
    batch_pair(pi, nP, tri, &o, &p);
    okn = o0 + o;
    const int2 r = parts[p];
    pkm = r.x * nbands + r.y;
  }
  C x[L];
  if (valid) {
    load_codensity_line<C, L, Sh::PLANE_B, typename cx<TI>::t>(
        x, psi + static_cast<size_t>(okn) * bs + static_cast<size_t>(j1) * LL + col,
        psi + static_cast<size_t>(pkm) * bs + static_cast<size_t>(j1) * LL + col, L);
  } else {
#pragma unroll
    for (int j2 = 0; j2 < L; ++j2) x[j2] = C{T(0), T(0)};
  }
  reg_fft<C, L, -1>(x);  // axis 2: x[c2] at (j1, c2, j3 = col)
  transpose_plane<C, T, L>(x, reinterpret_cast<T*>(smem_raw) + pl * L * Sh::LP, col);  // now c2 = col
  reg_fft<C, L, -1>(x);  // axis 3: x[c3]
  if constexpr (SLAB)
    transpose_plane<C, T, L>(x, reinterpret_cast<T*>(smem_raw) + pl * L * Sh::LP, col);  // x[c2], c3 = col
  else if constexpr (sizeof(TI) == sizeof(T) && sizeof(T) == 4 && L == 72)
    lds_round_trip<C, T, L>(x, reinterpret_cast<T*>(smem_raw) + pl * L * Sh::LP, col);
  if (valid) {
    if constexpr (sizeof(TI) != sizeof(T)) {
      // wide orbitals: addresses formed at the stores (the form with the
      // fewest registers for these variants, by the compiled kernels)
      C* dst = tbuf + static_cast<size_t>(pi) * n1 * LL;
      const unsigned so = opaque((static_cast<unsigned>(j1) * LL + col) * sizeof(C));
#pragma unroll
      for (int c3 = 0; c3 < L; ++c3) *lane_at(dst + c3 * L, so) = x[c3];
    } else {
      C* dst = tbuf + (static_cast<size_t>(pi) * n1 + j1) * LL + col;
#pragma unroll
      for (int c3 = 0; c3 < L; ++c3) dst[c3 * L] = x[c3];
    }
  }
}

// ---------------------------------------------------------------------------
// pencil pass, apply: FFT_1, x v_q/N, IFFT_1 on lines (c3, c2) of T
// ---------------------------------------------------------------------------
// EN: the apply also yields the pair energies (the spectrum is at hand after
// FFT_1): w_o f_o w'_p f'_p sum v/N |P|^2 per line block into epart.
template <typename T, int L, bool EN>
__device__ __forceinline__ void pencil_apply_line(int l, int LL, int pi, int q, typename cx<T>::t* __restrict__ tbuf,
                                                  const T* __restrict__ vtab, double* es) {
  using C = typename cx<T>::t;
  C* base = tbuf + static_cast<size_t>(pi) * LL * L;
  const unsigned lo = static_cast<unsigned>(l) * sizeof(C);
  C x[L];
#pragma unroll
  for (int j1 = 0; j1 < L; ++j1) x[j1] = *lane_at(base + static_cast<size_t>(j1) * LL, lo);
  reg_fft<C, L, -1>(x);
  mul_table_line_u<C, T, L, EN>(x, vtab + static_cast<size_t>(q) * LL * L,
                                opaque(static_cast<unsigned>(l) * sizeof(T)), LL, es);
  reg_fft<C, L, +1>(x);
  const unsigned so = opaque(lo);
#pragma unroll
  for (int j1 = 0; j1 < L; ++j1) *lane_at(base + static_cast<size_t>(j1) * LL, so) = x[j1];
}

template <typename T, int L, bool EN = false>
__global__ __launch_bounds__(256, (RegShape<T, L>::WPE_PENCIL)) void k_pencil_apply_reg(int ll, int nbands, int nk, int o0, int nP,
                                                          int tri, const int2* __restrict__ parts, const int* __restrict__ qmap,
                                                          typename cx<T>::t* __restrict__ tbuf,
                                                          const T* __restrict__ vtab, const double* __restrict__ occ,
                                                          const double* __restrict__ kw, double* __restrict__ epart) {
  const int LL = ll;  // lines per pair (N2 N3); L is the line length N1
  const int l = blockIdx.x * 256 + threadIdx.x;  // line (c3, c2) = l
  const int pi = blockIdx.y;
  int o, p;
  batch_pair(pi, nP, tri, &o, &p);
  const int ok = (o0 + o) / nbands;
  const int2 r = parts[p];
  const int q = qmap[ok * nk + r.x];
  if constexpr (!EN) {
    if (l >= LL) return;  // no barrier in this variant
    pencil_apply_line<T, L, false>(l, LL, pi, q, tbuf, vtab, nullptr);
  } else {
    double e = 0.0;
    if (l < LL) pencil_apply_line<T, L, true>(l, LL, pi, q, tbuf, vtab, &e);
    // an unordered pair of a block with itself stands for both orders
    store_line_energy(e, (tri && o != p ? 2.0 : 1.0) * kw[ok] * occ[o0 + o] * kw[r.x] * occ[r.x * nbands + r.y],
                      epart);
  }
}

// ---------------------------------------------------------------------------
// pencil pass, energy: FFT_1 and sum v_q/N |P|^2 in FP64 per line block
// ---------------------------------------------------------------------------
template <typename T, int L, typename TV = T>
__global__ __launch_bounds__(256, (RegShape<T, L>::WPE_PENCIL)) void k_pencil_energy_reg(int ll, const PairRef* __restrict__ pairs,
                                                           const typename cx<T>::t* __restrict__ tbuf,
                                                           const TV* __restrict__ vtab, double* __restrict__ epart) {
  using C = typename cx<T>::t;
  const int LL = ll;
  __shared__ double red[4];
  const int l = blockIdx.x * 256 + threadIdx.x;
  const int pi = blockIdx.y;
  double e = 0.0;
  if (l < LL) {
    const int q = pairs[pi].q;
    const C* base = tbuf + static_cast<size_t>(pi) * LL * L;
    C x[L];
#pragma unroll
    for (int j1 = 0; j1 < L; ++j1) x[j1] = *lane_at(base + static_cast<size_t>(j1) * LL, static_cast<unsigned>(l) * sizeof(C));
    reg_fft<C, L, -1>(x);
    const TV* v = vtab + static_cast<size_t>(q) * LL * L;
    const unsigned lv = opaque(static_cast<unsigned>(l) * sizeof(TV));
#pragma unroll
    for (int c1 = 0; c1 < L; ++c1) {
      const double px = static_cast<double>(x[c1].x), py = static_cast<double>(x[c1].y);
      e += static_cast<double>(*lane_at(v + static_cast<size_t>(c1) * LL, lv)) * (px * px + py * py);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) epart[static_cast<size_t>(pi) * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ---------------------------------------------------------------------------
// accumulate pass: per (output, plane group), every partner of the batch
// ---------------------------------------------------------------------------
// Batch pairs are pi = o nP + p (output o0 + o, partner parts[p]).  One
// launch serves the batch's outputs (blockIdx.y = o < nO) and, for a batch of
// unordered pairs of two blocks (mirror), also its partners (blockIdx.y =
// nO + p): the outputs are disjoint, so the two halves never write the same
// band.
//   output o:    W of pair (o, p) for every p, times u_p.
//   partner p:   the partner is the output; for every o the pair's W_{o p}
//                gives W_{p o} = conj(W_{o p}), times u_{o0+o}.
//   tri (a block paired with itself, unordered pairs o <= p at tri_slot):
//                 output o takes W_{o p} from slot (o, p) for p >= o and
//                 conj(W_{p o}) from slot (p, o) for p < o.
// The global band index of the orbital that multiplies W, the pair slot, and
// whether the slot holds the conjugate of the W wanted.
__device__ __forceinline__ void acc_source(bool mirror, int j, int blk, int o0, int nP, int tri, int nbands,
                                           const int2* __restrict__ parts, int* band, size_t* pair, bool* cj) {
  if (mirror) {
    *band = o0 + j;
    *pair = static_cast<size_t>(j) * nP + blk;
    *cj = true;
  } else {
    const int2 r = parts[j];
    *band = r.x * nbands + r.y;
    if (tri) {
      *pair = j >= blk ? tri_slot(blk, j, nP) : tri_slot(j, blk, nP);
      *cj = j < blk;
    } else {
      *pair = static_cast<size_t>(blk) * nP + j;
      *cj = false;
    }
  }
}

// Pull a byte range into L2 ahead of its use: one dword of every 128-byte
// line is loaded into v[k].  Past the range the range's first line is
// loaded again, so that every lane issues every load (no branch, so the
// compiler counts the loads in flight exactly).  The caller consumes v with
// prefetch_done where it may wait for them.
template <int NT, int PER>
__device__ __forceinline__ void prefetch_l2(const void* base, unsigned bytes, int t, unsigned (&v)[PER]) {
  const unsigned* b = static_cast<const unsigned*>(base);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const unsigned off = static_cast<unsigned>(t + k * NT) * 128u;
    v[k] = b[(off < bytes ? off : 0u) / 4u];
  }
  reg_fence();  // issued here, not moved to their use
}

template <int PER>
__device__ __forceinline__ void prefetch_done(const unsigned (&v)[PER]) {
#pragma unroll
  for (int k = 0; k < PER; ++k) asm volatile("" ::"v"(v[k]));
}

// PF: while a partner is transformed, the next partner's pair-buffer rows of
// the workgroup's planes are pulled into L2 (prefetch_l2), so that their
// loads wait on L2 rather than on HBM
template <typename T, int L, typename TI = T, bool PF = false>
__global__ __launch_bounds__((RegShape<T, L>::NTP), (RegShape<T, L>::WPE_ACC)) void k_acc_reg(
    int n1, int nbands, long long bs, int o0, int nO, int nP, int tri, const int2* __restrict__ parts,
    const typename cx<T>::t* __restrict__ tbuf, const typename cx<TI>::t* __restrict__ psi,
    const double* __restrict__ occ, const double* __restrict__ kw, typename cx<TI>::t* __restrict__ out, int first,
    int first_mirror,
    const double* __restrict__ gscale, double hscale, int backward) {
  using C = typename cx<T>::t;
  using CI = typename cx<TI>::t;  // orbitals and outputs (wider than the transform for FOCK_MIXED_INV)
  using Sh = RegShape<T, L>;
  constexpr int LL = L * L;
  constexpr int B = batch_of(L, Sh::ACC_B);
  constexpr int NB = L / B;
  extern __shared__ unsigned char smem_raw[];
  T* sp = reinterpret_cast<T*>(smem_raw);
  const int t = threadIdx.x, pl = t / L, col = t - (t / L) * L;
  // rows fastest in the grid: the workgroups of one plane block for all rows,
  // which read the same slices of the partners' orbitals, run together
  const int xb = static_cast<int>(blockIdx.y);
  const int row = static_cast<int>(blockIdx.x);
  const int j1 = xb * Sh::PL + pl;
  const bool valid = j1 < n1;
  const bool mirror = row >= nO;
  const int o = mirror ? row - nO : row;
  const int nsrc = mirror ? nO : nP;
  sp += pl * L * Sh::LP;
  C acc[L];
#pragma unroll
  for (int j2 = 0; j2 < L; ++j2) acc[j2] = C{T(0), T(0)};
  for (int p = 0; p < nsrc; ++p) {
    int sb;
    size_t pair;
    bool cj;
    acc_source(mirror, p, o, o0, nP, tri, nbands, parts, &sb, &pair, &cj);
    C x[L];
    if (valid) {
      const C* src = tbuf + pair * LL * n1 + static_cast<size_t>(j1) * LL + col;
#pragma unroll
      for (int c3 = 0; c3 < L; ++c3) x[c3] = src[c3 * L];  // row (j1, c2 = col)
    } else {
#pragma unroll
      for (int c3 = 0; c3 < L; ++c3) x[c3] = C{T(0), T(0)};
    }
    unsigned pfv[Sh::PF_ACC];
    if constexpr (PF) {
      // the next partner's rows (the last partner: its own again), behind
      // this partner's: the transforms wait only for the latter
      int sb1;
      size_t pair1;
      bool cj1;
      acc_source(mirror, p + 1 < nsrc ? p + 1 : p, o, o0, nP, tri, nbands, parts, &sb1, &pair1, &cj1);
      const int j10 = xb * Sh::PL;
      const int planes = min(Sh::PL, n1 - j10);
      prefetch_l2<Sh::NTP, Sh::PF_ACC>(tbuf + (pair1 * n1 + j10) * LL, static_cast<unsigned>(planes * LL * sizeof(C)), t,
                                       pfv);
    }
    reg_fft<C, L, +1>(x);                   // inverse axis 3: x[j3] at (j1, c2 = col)
    transpose_plane<C, T, L>(x, sp, col);   // column (j1, j3 = col)
    reg_fft<C, L, +1>(x);                   // inverse axis 2: x[j2]
    if (cj) {
#pragma unroll
      for (int j2 = 0; j2 < L; ++j2) x[j2].y = -x[j2].y;
    }
    if (valid) {
      const T coef = static_cast<T>(-kw[sb / nbands] * occ[sb]);
      const CI* um = psi + static_cast<size_t>(sb) * bs + static_cast<size_t>(j1) * LL + col;
      C mb[2][B];
#pragma unroll
      for (int j = 0; j < B; ++j) mb[0][j] = cvt<C>(um[j * L]);
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        if (n + 1 < NB) {
#pragma unroll
          for (int j = 0; j < B; ++j) mb[(n + 1) & 1][j] = cvt<C>(um[((n + 1) * B + j) * L]);
        }
        reg_fence();
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const C w = cmul(mb[n & 1][j], x[n * B + j]);
          acc[n * B + j].x += coef * w.x;
          acc[n * B + j].y += coef * w.y;
        }
      }
    }
    if constexpr (PF) prefetch_done(pfv);
  }
  if (!valid) return;  // no barrier after this point
  const int okn = mirror ? parts[o].x * nbands + parts[o].y : o0 + o;
  double f = hscale;
  if (gscale) f *= gscale[0];
  if (backward) f *= kw[okn / nbands] * occ[okn];
  CI* dst = out + static_cast<size_t>(okn) * bs + static_cast<size_t>(j1) * LL + col;
  const bool add = !(mirror ? first_mirror : first);
  if constexpr (sizeof(TI) != sizeof(T)) {
    // wide outputs: scaled in FP64 and read-modify-written in batches
    constexpr int OB = batch_of(L, 8);
#pragma unroll
    for (int n = 0; n < L / OB; ++n) {
      CI old[OB];
#pragma unroll
      for (int j = 0; j < OB; ++j) old[j] = add ? dst[(n * OB + j) * L] : CI{TI(0), TI(0)};
#pragma unroll
      for (int j = 0; j < OB; ++j)
        dst[(n * OB + j) * L] = CI{old[j].x + f * static_cast<TI>(acc[n * OB + j].x),
                                   old[j].y + f * static_cast<TI>(acc[n * OB + j].y)};
    }
  } else {
    const T ft = static_cast<T>(f);
    if (add) {
      // every earlier value is loaded before the first store, so the loads
      // overlap instead of waiting one by one behind the stores
      C old[L];
#pragma unroll
      for (int j2 = 0; j2 < L; ++j2) old[j2] = dst[j2 * L];
#pragma unroll
      for (int j2 = 0; j2 < L; ++j2) dst[j2 * L] = cadd(old[j2], cscale(acc[j2], ft));
    } else {
#pragma unroll
      for (int j2 = 0; j2 < L; ++j2) dst[j2 * L] = cscale(acc[j2], ft);
    }
  }
}

// ---------------------------------------------------------------------------
// plain batched 3-D DFT in the natural layout (fock_dft3 on cubic grids)
// ---------------------------------------------------------------------------
// plane pass: axes 2 and 3 of plane j1, read and written as columns (one
// line per lane, coalesced); two transposes bring the rows in and back out
template <typename T, int L, int S>
__global__ __launch_bounds__((RegShape<T, L>::NTP), (RegShape<T, L>::WPE_PLANE)) void k_dft_plane_reg(
    int n1, typename cx<T>::t* __restrict__ data, long long stride) {
  using C = typename cx<T>::t;
  using Sh = RegShape<T, L>;
  constexpr int LL = L * L;
  extern __shared__ unsigned char smem_raw[];
  const int t = threadIdx.x, pl = t / L, col = t - (t / L) * L;
  const int j1 = blockIdx.x * Sh::PL + pl;
  const bool valid = j1 < n1;
  T* sp = reinterpret_cast<T*>(smem_raw) + pl * L * Sh::LP;
  C* g = data + static_cast<size_t>(blockIdx.y) * stride + static_cast<size_t>(j1) * LL + col;
  C x[L];
#pragma unroll
  for (int j2 = 0; j2 < L; ++j2) x[j2] = valid ? g[j2 * L] : C{T(0), T(0)};
  reg_fft<C, L, S>(x);                  // axis 2: x[c2] at j3 = col
  transpose_plane<C, T, L>(x, sp, col);  // row c2 = col
  reg_fft<C, L, S>(x);                  // axis 3: x[c3]
  transpose_plane<C, T, L>(x, sp, col);  // column c3 = col: x[c2]
  if (valid) {
#pragma unroll
    for (int c2 = 0; c2 < L; ++c2) g[c2 * L] = x[c2];
  }
}

// pencil pass: axis 1 of line (c2, c3) = l, coalesced across lanes
template <typename T, int L, int S>
__global__ __launch_bounds__(256, (RegShape<T, L>::WPE_PENCIL)) void k_dft_pencil_reg(
    int ll, typename cx<T>::t* __restrict__ data, long long stride) {
  using C = typename cx<T>::t;
  const int LL = ll;
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= LL) return;  // no barrier in this kernel
  C* g = data + static_cast<size_t>(blockIdx.y) * stride;
  const unsigned lo = static_cast<unsigned>(l) * sizeof(C);
  C x[L];
#pragma unroll
  for (int j1 = 0; j1 < L; ++j1) x[j1] = *lane_at(g + static_cast<size_t>(j1) * LL, lo);
  reg_fft<C, L, S>(x);
  const unsigned so = opaque(lo);
#pragma unroll
  for (int c1 = 0; c1 < L; ++c1) *lane_at(g + static_cast<size_t>(c1) * LL, so) = x[c1];
}

// ---------------------------------------------------------------------------
// two-lane lines (L >= 64 FP32, L >= 36 FP64): each line lives in a lane pair
// ---------------------------------------------------------------------------
// The lanes 2i and 2i+1 share a line; lane h holds the samples 2m + h, or
// after a forward transform the half h of the spectrum (split_fft_fwd /
// split_fft_inv in reg_fft.hpp).  Registers per lane halve, so these kernels
// keep two or more waves per SIMD where a whole line per lane could not.
template <typename T, int L>
struct SplitShape {
  using C = typename cx<T>::t;
  static constexpr int LH = L / 2;
  static constexpr int LP = L + 1;
  static constexpr int PLANE_LDS = L * LP * static_cast<int>(sizeof(T));
  static constexpr int TPP = 2 * L;  // threads per plane
  static constexpr int HALF_REGS = LH * static_cast<int>(sizeof(C)) / 4;
  // planes per workgroup: up to 320 threads, but at most four waves (a whole
  // SIMD's registers per wave) when the accumulator and the half line need
  // more than 160 registers
  static constexpr int TMAX = 2 * HALF_REGS > 160 ? 256 : 320;
  static constexpr int PL = (TMAX / TPP) > 0 ? (TMAX / TPP) : 1;
  static constexpr int NTP = PL * TPP;
  static constexpr int LDS = PL * PLANE_LDS;
  static constexpr int LPB = 128;  // lines per pencil block
  static constexpr int WPE_LINE = HALF_REGS <= 64 ? 3 : (HALF_REGS <= 72 ? 2 : 1);
  static constexpr int WPE_ACC = 2 * HALF_REGS <= 144 ? 2 : 1;
};

// Switch a plane's axis for split lines.  EO_IN: the lane holds the samples
// i = 2m + h of line `col` and receives the half i = h L/2 + k of line `col`
// of the other axis; otherwise the reverse.  Component-wise through sp.
template <typename C, typename T, int L, bool EO_IN>
__device__ __forceinline__ void transpose_split(C* y, T* sp, int col, int h) {
  constexpr int LH = L / 2, LP = L + 1;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < LH; ++k) sp[(EO_IN ? 2 * k + h : h * LH + k) * LP + col] = y[k].x;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < LH; ++k) y[k].x = sp[col * LP + (EO_IN ? h * LH + k : 2 * k + h)];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < LH; ++k) sp[(EO_IN ? 2 * k + h : h * LH + k) * LP + col] = y[k].y;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < LH; ++k) y[k].y = sp[col * LP + (EO_IN ? h * LH + k : 2 * k + h)];
}

template <typename T, int L, bool EXPLICIT>
__global__ __launch_bounds__((SplitShape<T, L>::NTP), (SplitShape<T, L>::WPE_LINE)) void k_plane_split(
    int n1, int nbands, long long bs, const typename cx<T>::t* __restrict__ psi, int o0, int nP, int tri,
    const int2* __restrict__ parts, const PairRef* __restrict__ pairs, typename cx<T>::t* __restrict__ tbuf) {
  using C = typename cx<T>::t;
  using Sh = SplitShape<T, L>;
  constexpr int LL = L * L, LH = Sh::LH;
  extern __shared__ unsigned char smem_raw[];
  const int t = threadIdx.x, pl = t / Sh::TPP, rem = t - pl * Sh::TPP, col = rem >> 1, h = rem & 1;
  const int j1 = blockIdx.x * Sh::PL + pl;
  const bool valid = j1 < n1;
  const int pi = blockIdx.y;
  int okn, pkm;
  if (EXPLICIT) {
    const PairRef pr = pairs[pi];
    okn = pr.k * nbands + pr.n;
    pkm = pr.kp * nbands + pr.m;
  } else {
    int o, p;
    batch_pair(pi, nP, tri, &o, &p);
    okn = o0 + o;
    const int2 r = parts[p];
    pkm = r.x * nbands + r.y;
  }
  C y[LH];
  if (valid) {
    const size_t off = static_cast<size_t>(j1) * LL + static_cast<size_t>(h) * L + col;  // j2 = 2m + h
    load_codensity_line<C, LH>(y, psi + static_cast<size_t>(okn) * bs + off, psi + static_cast<size_t>(pkm) * bs + off,
                               2 * L);
  } else {
#pragma unroll
    for (int m = 0; m < LH; ++m) y[m] = C{T(0), T(0)};
  }
  split_fft_fwd<C, L>(y, h);  // axis 2: y[k] at c2 = h L/2 + k, j3 = col
  transpose_split<C, T, L, false>(y, reinterpret_cast<T*>(smem_raw) + pl * L * Sh::LP, col, h);  // c2 = col
  split_fft_fwd<C, L>(y, h);  // axis 3: y[k] at c3 = h L/2 + k
  if (valid) {
    C* dst = tbuf + (static_cast<size_t>(pi) * n1 + j1) * LL + static_cast<size_t>(h) * LH * L + col;
#pragma unroll
    for (int k = 0; k < LH; ++k) dst[k * L] = y[k];
  }
}

template <typename T, int L, bool EN>
__device__ __forceinline__ void pencil_apply_split_line(int l, int h, int LL, int pi, int q,
                                                        typename cx<T>::t* __restrict__ tbuf,
                                                        const T* __restrict__ vtab, double* es) {
  using C = typename cx<T>::t;
  constexpr int LH = L / 2;
  C* base = tbuf + static_cast<size_t>(pi) * LL * L;
  const unsigned lo = (static_cast<unsigned>(h) * LL + l) * sizeof(C);
  C y[LH];
#pragma unroll
  for (int m = 0; m < LH; ++m) y[m] = *lane_at(base + static_cast<size_t>(2 * m) * LL, lo);  // j1 = 2m + h
  split_fft_fwd<C, L>(y, h);  // y[k] at c1 = h L/2 + k
  mul_table_line_u<C, T, LH, EN>(y, vtab + static_cast<size_t>(q) * LL * L,
                                 opaque((static_cast<unsigned>(h) * LH * LL + l) * sizeof(T)), LL, es);
  split_fft_inv<C, L>(y, h);
  const unsigned so = opaque(lo);
#pragma unroll
  for (int m = 0; m < LH; ++m) *lane_at(base + static_cast<size_t>(2 * m) * LL, so) = y[m];
}

template <typename T, int L, bool EN = false>
__global__ __launch_bounds__(256, (SplitShape<T, L>::WPE_LINE)) void k_pencil_apply_split(
    int ll, int nbands, int nk, int o0, int nP, int tri, const int2* __restrict__ parts, const int* __restrict__ qmap,
    typename cx<T>::t* __restrict__ tbuf, const T* __restrict__ vtab, const double* __restrict__ occ,
    const double* __restrict__ kw, double* __restrict__ epart) {
  using Sh = SplitShape<T, L>;
  const int LL = ll;
  const int h = threadIdx.x & 1;
  const int l = blockIdx.x * Sh::LPB + (threadIdx.x >> 1);  // line (c3, c2), shared by the lane pair
  const int pi = blockIdx.y;
  int o, p;
  batch_pair(pi, nP, tri, &o, &p);
  const int ok = (o0 + o) / nbands;
  const int2 r = parts[p];
  const int q = qmap[ok * nk + r.x];
  if constexpr (!EN) {
    if (l >= LL) return;  // uniform over the pair; no barrier in this variant
    pencil_apply_split_line<T, L, false>(l, h, LL, pi, q, tbuf, vtab, nullptr);
  } else {
    double e = 0.0;  // each lane: its half of the spectrum
    if (l < LL) pencil_apply_split_line<T, L, true>(l, h, LL, pi, q, tbuf, vtab, &e);
    store_line_energy(e, (tri && o != p ? 2.0 : 1.0) * kw[ok] * occ[o0 + o] * kw[r.x] * occ[r.x * nbands + r.y],
                      epart);
  }
}

// ---------------------------------------------------------------------------
// slab pencil (cubic L^3, pair buffer [j1][c2][c3] from the SLAB plane pass):
// one slab of fixed c2 per L threads, thread col = c3 holding the line
// (c2, c3) along axis 1: FFT_1, x v_q/N (pair energies with EN), IFFT_1; a
// transpose to lines along axis 3 for fixed j1 = col, IFFT_3; a transpose
// back (the same LDS round as the plane pass), so that the pair buffer
// leaves as [j1][c2][j3], read by the line accumulate along axis 2.  The
// table is in grid order [c1][c2][c3].
// ---------------------------------------------------------------------------
template <typename T, int L, bool EN>
__global__ __launch_bounds__((RegShape<T, L>::NTP), (RegShape<T, L>::WPE_PLANE)) void k_pencil_slab(
    int nbands, int nk, int o0, int nP, int tri, const int2* __restrict__ parts, const int* __restrict__ qmap,
    typename cx<T>::t* __restrict__ tbuf, const T* __restrict__ vtab, const double* __restrict__ occ,
    const double* __restrict__ kw, double* __restrict__ epart) {
  using C = typename cx<T>::t;
  using Sh = RegShape<T, L>;
  constexpr int LL = L * L;
  extern __shared__ unsigned char smem_raw[];
  const int t = threadIdx.x, pl = t / L, col = t - (t / L) * L;
  const int c2 = blockIdx.x * Sh::PL + pl;
  const bool valid = c2 < L;
  const int pi = blockIdx.y;
  int o, p;
  batch_pair(pi, nP, tri, &o, &p);
  const int ok = (o0 + o) / nbands;
  const int2 r = parts[p];
  const int q = qmap[ok * nk + r.x];
  T* sp = reinterpret_cast<T*>(smem_raw) + pl * L * Sh::LP;
  C* base = tbuf + static_cast<size_t>(pi) * LL * L;
  C x[L];
  double e = 0.0;
  if (valid) {
    const unsigned lo = (static_cast<unsigned>(c2) * L + col) * sizeof(C);
#pragma unroll
    for (int j1 = 0; j1 < L; ++j1) x[j1] = *lane_at(base + static_cast<size_t>(j1) * LL, lo);
    reg_fft<C, L, -1>(x);  // axis 1: x[c1] at (c2, c3 = col)
    mul_table_line_u<C, T, L, EN>(x, vtab + static_cast<size_t>(q) * LL * L,
                                  opaque((static_cast<unsigned>(c2) * L + col) * sizeof(T)), LL, &e);
    reg_fft<C, L, +1>(x);  // x[j1]
  } else {
#pragma unroll
    for (int j1 = 0; j1 < L; ++j1) x[j1] = C{T(0), T(0)};
  }
  transpose_plane<C, T, L>(x, sp, col);  // line j1 = col: x[c3]
  reg_fft<C, L, +1>(x);                  // x[j3]
  transpose_plane<C, T, L>(x, sp, col);  // line j3 = col: x[j1]
  if (valid) {
    const unsigned so = opaque((static_cast<unsigned>(c2) * L + col) * sizeof(C));
#pragma unroll
    for (int j1 = 0; j1 < L; ++j1) *lane_at(base + static_cast<size_t>(j1) * LL, so) = x[j1];
  }
  if constexpr (EN) {
    // block sum in a fixed order (the block's last wave may be partly empty):
    // the first wave adds the threads' partials with stride 64, then across
    // its lanes
    __shared__ double red[Sh::NTP];
    red[t] = e;
    __syncthreads();
    if (t < 64) {
      double sum = 0.0;
      for (int i = t; i < Sh::NTP; i += 64) sum += red[i];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
      if (t == 0)
        epart[static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x] =
            (tri && o != p ? 2.0 : 1.0) * kw[ok] * occ[o0 + o] * kw[r.x] * occ[r.x * nbands + r.y] * sum;
    }
  }
}

template <typename T, int L, typename TV = T>
__global__ __launch_bounds__(256, (SplitShape<T, L>::WPE_LINE)) void k_pencil_energy_split(
    int ll, const PairRef* __restrict__ pairs, const typename cx<T>::t* __restrict__ tbuf, const TV* __restrict__ vtab,
    double* __restrict__ epart) {
  using C = typename cx<T>::t;
  using Sh = SplitShape<T, L>;
  const int LL = ll;
  constexpr int LH = Sh::LH;
  __shared__ double red[4];
  const int h = threadIdx.x & 1;
  const int l = blockIdx.x * Sh::LPB + (threadIdx.x >> 1);
  const int pi = blockIdx.y;
  double e = 0.0;
  if (l < LL) {
    const int q = pairs[pi].q;
    const C* base = tbuf + static_cast<size_t>(pi) * LL * L;
    const unsigned lo = (static_cast<unsigned>(h) * LL + l) * sizeof(C);
    C y[LH];
#pragma unroll
    for (int m = 0; m < LH; ++m) y[m] = *lane_at(base + static_cast<size_t>(2 * m) * LL, lo);
    split_fft_fwd<C, L>(y, h);
    const TV* v = vtab + static_cast<size_t>(q) * LL * L;
    const unsigned lv = opaque((static_cast<unsigned>(h) * LH * LL + l) * sizeof(TV));
#pragma unroll
    for (int k = 0; k < LH; ++k) {
      const double px = static_cast<double>(y[k].x), py = static_cast<double>(y[k].y);
      e += static_cast<double>(*lane_at(v + static_cast<size_t>(k) * LL, lv)) * (px * px + py * py);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) epart[static_cast<size_t>(pi) * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename T, int L, typename TI = T>
__global__ __launch_bounds__((SplitShape<T, L>::NTP), (SplitShape<T, L>::WPE_ACC)) void k_acc_split(
    int n1, int nbands, long long bs, int o0, int nO, int nP, int tri, const int2* __restrict__ parts,
    const typename cx<T>::t* __restrict__ tbuf, const typename cx<TI>::t* __restrict__ psi,
    const double* __restrict__ occ, const double* __restrict__ kw, typename cx<TI>::t* __restrict__ out, int first,
    int first_mirror,
    const double* __restrict__ gscale, double hscale, int backward) {
  using C = typename cx<T>::t;
  using CI = typename cx<TI>::t;  // orbitals and outputs (wider than the transform for FOCK_MIXED_INV)
  using Sh = SplitShape<T, L>;
  constexpr int LL = L * L, LH = Sh::LH;
  constexpr int B = batch_of(LH, Sh::WPE_ACC == 1 ? 16 : kRegB);
  constexpr int NB = LH / B;
  extern __shared__ unsigned char smem_raw[];
  const int t = threadIdx.x, pl = t / Sh::TPP, rem = t - pl * Sh::TPP, col = rem >> 1, h = rem & 1;
  // rows fastest in the grid: the workgroups of one plane block for all rows,
  // which read the same slices of the partners' orbitals, run together
  const int xb = static_cast<int>(blockIdx.y);
  const int row = static_cast<int>(blockIdx.x);
  const int j1 = xb * Sh::PL + pl;
  const bool valid = j1 < n1;
  const bool mirror = row >= nO;
  const int o = mirror ? row - nO : row;
  T* sp = reinterpret_cast<T*>(smem_raw) + pl * L * Sh::LP;
  // element (j1, 2m + h, col) of a grid: the lane's samples along axis 2
  const size_t eo = static_cast<size_t>(j1) * LL + static_cast<size_t>(h) * L + col;
  const int nsrc = mirror ? nO : nP;
  C acc[LH];
#pragma unroll
  for (int m = 0; m < LH; ++m) acc[m] = C{T(0), T(0)};
  for (int p = 0; p < nsrc; ++p) {
    int sb;
    size_t pair;
    bool cj;
    acc_source(mirror, p, o, o0, nP, tri, nbands, parts, &sb, &pair, &cj);
    C y[LH];
    if (valid) {
      const C* src = tbuf + pair * LL * n1 + static_cast<size_t>(j1) * LL + static_cast<size_t>(h) * LH * L + col;
#pragma unroll
      for (int k = 0; k < LH; ++k) y[k] = src[k * L];  // row (j1, c2 = col), c3 = h L/2 + k
    } else {
#pragma unroll
      for (int k = 0; k < LH; ++k) y[k] = C{T(0), T(0)};
    }
    split_fft_inv<C, L>(y, h);                      // inverse axis 3: y[m] at j3 = 2m + h
    transpose_split<C, T, L, true>(y, sp, col, h);  // column j3 = col, c2 = h L/2 + k
    split_fft_inv<C, L>(y, h);                      // inverse axis 2: y[m] at j2 = 2m + h
    if (cj) {
#pragma unroll
      for (int m = 0; m < LH; ++m) y[m].y = -y[m].y;
    }
    if (valid) {
      const T coef = static_cast<T>(-kw[sb / nbands] * occ[sb]);
      const CI* um = psi + static_cast<size_t>(sb) * bs + eo;
      C mb[2][B];
#pragma unroll
      for (int j = 0; j < B; ++j) mb[0][j] = cvt<C>(um[j * 2 * L]);
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        if (n + 1 < NB) {
#pragma unroll
          for (int j = 0; j < B; ++j) mb[(n + 1) & 1][j] = cvt<C>(um[((n + 1) * B + j) * 2 * L]);
        }
        reg_fence();
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const C w = cmul(mb[n & 1][j], y[n * B + j]);
          acc[n * B + j].x += coef * w.x;
          acc[n * B + j].y += coef * w.y;
        }
      }
    }
  }
  if (!valid) return;  // no barrier after this point
  const int okn = mirror ? parts[o].x * nbands + parts[o].y : o0 + o;
  double f = hscale;
  if (gscale) f *= gscale[0];
  if (backward) f *= kw[okn / nbands] * occ[okn];
  CI* dst = out + static_cast<size_t>(okn) * bs + eo;
  const bool add = !(mirror ? first_mirror : first);
  if constexpr (sizeof(TI) != sizeof(T)) {
    // wide outputs: scaled in FP64 and read-modify-written in batches
    constexpr int OB = batch_of(LH, 8);
#pragma unroll
    for (int n = 0; n < LH / OB; ++n) {
      CI old[OB];
#pragma unroll
      for (int j = 0; j < OB; ++j) old[j] = add ? dst[(n * OB + j) * 2 * L] : CI{TI(0), TI(0)};
#pragma unroll
      for (int j = 0; j < OB; ++j)
        dst[(n * OB + j) * 2 * L] = CI{old[j].x + f * static_cast<TI>(acc[n * OB + j].x),
                                       old[j].y + f * static_cast<TI>(acc[n * OB + j].y)};
    }
  } else {
    const T ft = static_cast<T>(f);
    if (add) {
      C old[LH];  // loaded before the first store (see k_acc_reg)
#pragma unroll
      for (int m = 0; m < LH; ++m) old[m] = dst[m * 2 * L];
#pragma unroll
      for (int m = 0; m < LH; ++m) dst[m * 2 * L] = cadd(old[m], cscale(acc[m], ft));
    } else {
#pragma unroll
      for (int m = 0; m < LH; ++m) dst[m * 2 * L] = cscale(acc[m], ft);
    }
  }
}

// ---------------------------------------------------------------------------
// line accumulate (pair buffer [j1][c2][j3] from the slab pencil): each thread
// one line (j1, j3) along axis 2, for every partner IFFT_2 and the partner's
// orbital along j2 at (j1, j3).  No transpose, so no LDS and no barrier, and
// the lines need not fill whole planes: every lane of a workgroup works.
// Rows and partners as in k_acc_reg.
// ---------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(256, (RegShape<T, L>::WPE_ACC)) void k_acc_line(
    int nbands, long long bs, int o0, int nO, int nP, int tri, const int2* __restrict__ parts,
    const typename cx<T>::t* __restrict__ tbuf, const typename cx<T>::t* __restrict__ psi,
    const double* __restrict__ occ, const double* __restrict__ kw, typename cx<T>::t* __restrict__ out, int first,
    int first_mirror, const double* __restrict__ gscale, double hscale, int backward) {
  using C = typename cx<T>::t;
  constexpr int LL = L * L;
  constexpr int B = batch_of(L, 16);
  constexpr int NB = L / B;
  // rows run fastest in the grid, so that the workgroups of one line block
  // for all rows, which read the same slices of the partners' orbitals, are
  // in flight together (beta boron 6.59 against 7.20 s per step with line
  // blocks fastest: the orbitals then come from L2 rather than from further)
  const int l = static_cast<int>(blockIdx.y) * 256 + static_cast<int>(threadIdx.x);  // line (j1, j3)
  if (l >= LL) return;  // no barrier in this kernel
  const int row = static_cast<int>(blockIdx.x);
  const bool mirror = row >= nO;
  const int o = mirror ? row - nO : row;
  const int nsrc = mirror ? nO : nP;
  const int j1 = l / L, j3 = l - (l / L) * L;
  const size_t eoff = static_cast<size_t>(j1) * LL + j3;  // element (j1, 0, j3); axis 2 has stride L
  C acc[L];
#pragma unroll
  for (int j2 = 0; j2 < L; ++j2) acc[j2] = C{T(0), T(0)};
  for (int p = 0; p < nsrc; ++p) {
    int sb;
    size_t pair;
    bool cj;
    acc_source(mirror, p, o, o0, nP, tri, nbands, parts, &sb, &pair, &cj);
    const C* src = tbuf + pair * LL * L + eoff;
    C x[L];
#pragma unroll
    for (int c2 = 0; c2 < L; ++c2) x[c2] = src[c2 * L];
    reg_fft<C, L, +1>(x);  // inverse axis 2: x[j2] at (j1, j3)
    if (cj) {
#pragma unroll
      for (int j2 = 0; j2 < L; ++j2) x[j2].y = -x[j2].y;
    }
    const T coef = static_cast<T>(-kw[sb / nbands] * occ[sb]);
    const C* um = psi + static_cast<size_t>(sb) * bs + eoff;
    C mb[2][B];
#pragma unroll
    for (int j = 0; j < B; ++j) mb[0][j] = um[j * L];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      if (n + 1 < NB) {
#pragma unroll
        for (int j = 0; j < B; ++j) mb[(n + 1) & 1][j] = um[((n + 1) * B + j) * L];
      }
      reg_fence();
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const C w = cmul(mb[n & 1][j], x[n * B + j]);
        acc[n * B + j].x += coef * w.x;
        acc[n * B + j].y += coef * w.y;
      }
    }
  }
  const int okn = mirror ? parts[o].x * nbands + parts[o].y : o0 + o;
  double f = hscale;
  if (gscale) f *= gscale[0];
  if (backward) f *= kw[okn / nbands] * occ[okn];
  const T ft = static_cast<T>(f);
  C* dst = out + static_cast<size_t>(okn) * bs + eoff;
  if (!(mirror ? first_mirror : first)) {
    C old[L];  // loaded before the first store (see k_acc_reg)
#pragma unroll
    for (int j2 = 0; j2 < L; ++j2) old[j2] = dst[j2 * L];
#pragma unroll
    for (int j2 = 0; j2 < L; ++j2) dst[j2 * L] = cadd(old[j2], cscale(acc[j2], ft));
  } else {
#pragma unroll
    for (int j2 = 0; j2 < L; ++j2) dst[j2 * L] = cscale(acc[j2], ft);
  }
}

// the line accumulate over lane pairs, where one lane per line would need a
// whole SIMD's registers: lane h of a pair loads c2 = h L/2 + k of the line
// (j1, j3) and holds j2 = 2m + h after the transform (see split_fft.hpp)
template <typename T, int L>
__global__ __launch_bounds__(256, (SplitShape<T, L>::WPE_ACC)) void k_acc_line_split(
    int nbands, long long bs, int o0, int nO, int nP, int tri, const int2* __restrict__ parts,
    const typename cx<T>::t* __restrict__ tbuf, const typename cx<T>::t* __restrict__ psi,
    const double* __restrict__ occ, const double* __restrict__ kw, typename cx<T>::t* __restrict__ out, int first,
    int first_mirror, const double* __restrict__ gscale, double hscale, int backward) {
  using C = typename cx<T>::t;
  using Sh = SplitShape<T, L>;
  constexpr int LL = L * L, LH = Sh::LH;
  constexpr int B = batch_of(LH, Sh::WPE_ACC == 1 ? 16 : kRegB);
  constexpr int NB = LH / B;
  const int h = threadIdx.x & 1;
  // rows fastest in the grid (see k_acc_line)
  const int l = static_cast<int>(blockIdx.y) * 128 + static_cast<int>(threadIdx.x >> 1);  // line (j1, j3)
  if (l >= LL) return;  // both lanes of a pair together; no barrier in this kernel
  const int row = static_cast<int>(blockIdx.x);
  const bool mirror = row >= nO;
  const int o = mirror ? row - nO : row;
  const int nsrc = mirror ? nO : nP;
  const int j1 = l / L, j3 = l - (l / L) * L;
  const size_t eoff = static_cast<size_t>(j1) * LL + j3;  // element (j1, 0, j3); axis 2 has stride L
  C acc[LH];
#pragma unroll
  for (int m = 0; m < LH; ++m) acc[m] = C{T(0), T(0)};
  for (int p = 0; p < nsrc; ++p) {
    int sb;
    size_t pair;
    bool cj;
    acc_source(mirror, p, o, o0, nP, tri, nbands, parts, &sb, &pair, &cj);
    const C* src = tbuf + pair * LL * L + eoff + static_cast<size_t>(h) * LH * L;
    C y[LH];
#pragma unroll
    for (int k = 0; k < LH; ++k) y[k] = src[k * L];  // c2 = h L/2 + k
    split_fft_inv<C, L>(y, h);                       // y[m] at j2 = 2m + h
    if (cj) {
#pragma unroll
      for (int m = 0; m < LH; ++m) y[m].y = -y[m].y;
    }
    const T coef = static_cast<T>(-kw[sb / nbands] * occ[sb]);
    const C* um = psi + static_cast<size_t>(sb) * bs + eoff + static_cast<size_t>(h) * L;
    C mb[2][B];
#pragma unroll
    for (int j = 0; j < B; ++j) mb[0][j] = um[j * 2 * L];
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      if (n + 1 < NB) {
#pragma unroll
        for (int j = 0; j < B; ++j) mb[(n + 1) & 1][j] = um[((n + 1) * B + j) * 2 * L];
      }
      reg_fence();
#pragma unroll
      for (int j = 0; j < B; ++j) {
        const C w = cmul(mb[n & 1][j], y[n * B + j]);
        acc[n * B + j].x += coef * w.x;
        acc[n * B + j].y += coef * w.y;
      }
    }
  }
  const int okn = mirror ? parts[o].x * nbands + parts[o].y : o0 + o;
  double f = hscale;
  if (gscale) f *= gscale[0];
  if (backward) f *= kw[okn / nbands] * occ[okn];
  const T ft = static_cast<T>(f);
  C* dst = out + static_cast<size_t>(okn) * bs + eoff + static_cast<size_t>(h) * L;
  if (!(mirror ? first_mirror : first)) {
    C old[LH];  // loaded before the first store (see k_acc_reg)
#pragma unroll
    for (int m = 0; m < LH; ++m) old[m] = dst[m * 2 * L];
#pragma unroll
    for (int m = 0; m < LH; ++m) dst[m * 2 * L] = cadd(old[m], cscale(acc[m], ft));
  } else {
#pragma unroll
    for (int m = 0; m < LH; ++m) dst[m * 2 * L] = cscale(acc[m], ft);
  }
}

// ---------------------------------------------------------------------------
// mixed precision (FOCK_MIXED): pencil pass from the FP32 pair buffer to the
// FP64 one: forward axis 1 in FP32, kernel multiply and inverse in FP64
// ---------------------------------------------------------------------------
template <int L, bool EN>
__device__ __forceinline__ void pencil_apply_mixed_line(int l, int h, int LL, int pi, int q,
                                                        const float2* __restrict__ t32, double2* __restrict__ t64,
                                                        const double* __restrict__ vtab, double* es) {
  constexpr int LH = L / 2;
  const size_t base = static_cast<size_t>(pi) * LL * L;
  const unsigned le = static_cast<unsigned>(h) * LL + l;  // lane's element offset
  double2 y[LH];
  {
    float2 f[LH];
#pragma unroll
    for (int m = 0; m < LH; ++m) f[m] = *lane_at(t32 + base + static_cast<size_t>(2 * m) * LL, le * 8u);  // j1 = 2m + h
    split_fft_fwd<float2, L>(f, h);  // f[k] at c1 = h L/2 + k
#pragma unroll
    for (int k = 0; k < LH; ++k) y[k] = cvt<double2>(f[k]);
  }
  mul_table_line_u<double2, double, LH, EN>(y, vtab + static_cast<size_t>(q) * LL * L,
                                            opaque((static_cast<unsigned>(h) * LH * LL + l) * 8u), LL, es);
  split_fft_inv<double2, L>(y, h);
  const unsigned so = opaque(le * 16u);
#pragma unroll
  for (int m = 0; m < LH; ++m) *lane_at(t64 + base + static_cast<size_t>(2 * m) * LL, so) = y[m];
}

// EN: the energy variant (see k_pencil_apply_reg), from the FP32 forward
// spectrum widened to FP64
template <int L, bool EN = false>
__global__ __launch_bounds__(256, 1) void k_pencil_apply_mixed(int ll, int nbands, int nk, int o0, int nP, int tri,
                                                               const int2* __restrict__ parts,
                                                               const int* __restrict__ qmap,
                                                               const float2* __restrict__ t32,
                                                               double2* __restrict__ t64,
                                                               const double* __restrict__ vtab,
                                                               const double* __restrict__ occ,
                                                               const double* __restrict__ kw,
                                                               double* __restrict__ epart) {
  const int LL = ll;
  constexpr int LPB = 128;
  const int h = threadIdx.x & 1;
  const int l = blockIdx.x * LPB + (threadIdx.x >> 1);  // line (c3, c2), shared by the lane pair
  const int pi = blockIdx.y;
  int o, p;
  batch_pair(pi, nP, tri, &o, &p);
  const int ok = (o0 + o) / nbands;
  const int2 r = parts[p];
  const int q = qmap[ok * nk + r.x];
  if constexpr (!EN) {
    if (l >= LL) return;  // uniform over the pair; no barrier in this variant
    pencil_apply_mixed_line<L, false>(l, h, LL, pi, q, t32, t64, vtab, nullptr);
  } else {
    double e = 0.0;
    if (l < LL) pencil_apply_mixed_line<L, true>(l, h, LL, pi, q, t32, t64, vtab, &e);
    store_line_energy(e, (tri && o != p ? 2.0 : 1.0) * kw[ok] * occ[o0 + o] * kw[r.x] * occ[r.x * nbands + r.y],
                      epart);
  }
}

// ---------------------------------------------------------------------------
// the other mixed precision (FOCK_MIXED_INV): pencil pass from the FP64 pair
// buffer to the FP32 one: forward axis 1, kernel multiply (and the pair
// energies) in FP64, inverse axis 1 in FP32
// ---------------------------------------------------------------------------
template <int L, bool EN>
__device__ __forceinline__ void pencil_apply_mixinv_line(int l, int h, int LL, int pi, int q,
                                                         const double2* __restrict__ t64, float2* __restrict__ t32,
                                                         const double* __restrict__ vtab, double* es) {
  constexpr int LH = L / 2;
  const size_t base = static_cast<size_t>(pi) * LL * L;
  const unsigned le = static_cast<unsigned>(h) * LL + l;  // lane's element offset
  float2 f[LH];
  {
    double2 y[LH];
#pragma unroll
    for (int m = 0; m < LH; ++m) y[m] = *lane_at(t64 + base + static_cast<size_t>(2 * m) * LL, le * 16u);  // j1 = 2m + h
    split_fft_fwd<double2, L>(y, h);  // y[k] at c1 = h L/2 + k
    mul_table_line_u<double2, double, LH, EN>(y, vtab + static_cast<size_t>(q) * LL * L,
                                              opaque((static_cast<unsigned>(h) * LH * LL + l) * 8u), LL, es);
#pragma unroll
    for (int k = 0; k < LH; ++k) f[k] = cvt<float2>(y[k]);
  }
  split_fft_inv<float2, L>(f, h);
  const unsigned so = opaque(le * 8u);
#pragma unroll
  for (int m = 0; m < LH; ++m) *lane_at(t32 + base + static_cast<size_t>(2 * m) * LL, so) = f[m];
}

// EN: the energy variant (see k_pencil_apply_reg), from the FP64 spectrum
template <int L, bool EN = false>
__global__ __launch_bounds__(256, 1) void k_pencil_apply_mixinv(int ll, int nbands, int nk, int o0, int nP, int tri,
                                                                const int2* __restrict__ parts,
                                                                const int* __restrict__ qmap,
                                                                const double2* __restrict__ t64,
                                                                float2* __restrict__ t32,
                                                                const double* __restrict__ vtab,
                                                                const double* __restrict__ occ,
                                                                const double* __restrict__ kw,
                                                                double* __restrict__ epart) {
  const int LL = ll;
  constexpr int LPB = 128;
  const int h = threadIdx.x & 1;
  const int l = blockIdx.x * LPB + (threadIdx.x >> 1);  // line (c3, c2), shared by the lane pair
  const int pi = blockIdx.y;
  int o, p;
  batch_pair(pi, nP, tri, &o, &p);
  const int ok = (o0 + o) / nbands;
  const int2 r = parts[p];
  const int q = qmap[ok * nk + r.x];
  if constexpr (!EN) {
    if (l >= LL) return;  // uniform over the pair; no barrier in this variant
    pencil_apply_mixinv_line<L, false>(l, h, LL, pi, q, t64, t32, vtab, nullptr);
  } else {
    double e = 0.0;
    if (l < LL) pencil_apply_mixinv_line<L, true>(l, h, LL, pi, q, t64, t32, vtab, &e);
    store_line_energy(e, (tri && o != p ? 2.0 : 1.0) * kw[ok] * occ[o0 + o] * kw[r.x] * occ[r.x * nbands + r.y],
                      epart);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Every variant reads and writes the pair buffer in the same layout, so each
// pass picks its own: a line per lane where that fits the registers without
// spilling, a line per lane pair otherwise, and by measurement where both fit
// (FP32 54-64: two-lane accumulate; FP32 64 and 72: two-lane pencil).
template <typename T, int L>
struct RegPolicy {
  static constexpr bool FP32 = sizeof(T) == 4;
  static constexpr bool SPLIT_PLANE = !FP32 && L >= 36;
  static constexpr bool SPLIT_PENCIL = FP32 ? L >= 64 : L >= 36;
  // FP64 32 points over lane pairs too: alpha boron FP64 accumulate 462
  // against 518 ms per step for one lane (one-wave workgroups with the L2
  // prefetch, 586 ms as four-wave ones without)
  static constexpr bool SPLIT_ACC = FP32 ? (L >= 54 && L <= 64) : L >= 32;
  // L2 prefetch of the next partner in the one-lane accumulate, where that
  // kernel runs one wave per SIMD: FP32 72 points (beta boron 8.71 against
  // 8.89 s per step); at FP32 32 points, two waves per SIMD, it costs (428
  // against 382 ms per step at alpha boron)
  static constexpr bool ACC_PREFETCH = FP32 && L == 72;
  static constexpr int PLANE_LDS = SPLIT_PLANE ? SplitShape<T, L>::LDS : RegShape<T, L>::LDS;
  static constexpr int ACC_LDS = SPLIT_ACC ? SplitShape<T, L>::LDS : RegShape<T, L>::LDS;
  static constexpr int LDS = PLANE_LDS > ACC_LDS ? PLANE_LDS : ACC_LDS;
};

namespace {

// Grids N1 x L x L: the plane and accumulate passes are compiled for the
// plane side L and take the plane count N1 at run time; the pencil pass is
// compiled for the line length N1 and takes the line count L^2 at run time.
// Each pass is dispatched on its own length.

// lengths compiled with the slab pencil and the line accumulate
template <typename T, int L>
constexpr bool slab_len() {
  return sizeof(T) == 4 ? true : L <= 32;  // FP64: the one-lane plane lengths
}

// the line accumulate over lane pairs: FP64 where line and accumulator take
// over 160 registers, FP32 at 60 and 64 points.  Measured on the slab path
// (cubic cells, 2x2x2 k, apply + energy + gradient per step), one lane per
// line against lane pairs: 48^3 70.7 against 71.1 ms, 50^3 84.5 against
// 89.9, 54^3 111.9 against 119.0, 60^3 105.0 against 93.7, 64^3 54.9 against
// 42.8; at 72^3 one lane wins (beta boron)
template <typename T, int L>
constexpr bool line_split() {
  return sizeof(T) == 4 ? (L == 60 || L == 64) : 2 * RegShape<T, L>::LINE_REGS > 160;
}

template <typename T, int L, bool EXPLICIT, typename TI = T>
void launch_plane(const Plan& p, const Batch& b, const Instance& in, const void* psi, const int2* parts,
                  const PairRef* pairs, typename cx<T>::t* tbuf) {
  using C = typename cx<T>::t;
  using CI = typename cx<TI>::t;
  using Po = RegPolicy<T, L>;
  const int n1 = in.grid[0];
  const long long bs = static_cast<long long>(in.band_stride);
  const int o0 = EXPLICIT ? 0 : b.o0, nP = EXPLICIT ? 1 : b.nP, tri = EXPLICIT ? 0 : b.tri;
  if constexpr (sizeof(TI) != sizeof(T)) {  // FOCK_MIXED: one-lane FP32 lines from FP64 orbitals
    using Sh = RegShape<T, L>;
    hipLaunchKernelGGL((k_plane_reg<T, L, EXPLICIT, TI>), dim3((n1 + Sh::PL - 1) / Sh::PL, b.npairs), dim3(Sh::NTP),
                       Sh::LDS, p.stream, n1, in.nbands, bs, static_cast<const CI*>(psi), o0, nP, tri, parts, pairs, tbuf,
                       0);
  } else if constexpr (Po::SPLIT_PLANE) {
    using Sh = SplitShape<T, L>;
    hipLaunchKernelGGL((k_plane_split<T, L, EXPLICIT>), dim3((n1 + Sh::PL - 1) / Sh::PL, b.npairs), dim3(Sh::NTP),
                       Sh::LDS, p.stream, n1, in.nbands, bs, static_cast<const C*>(psi), o0, nP, tri, parts, pairs, tbuf);
  } else {
    using Sh = RegShape<T, L>;
    if constexpr (slab_len<T, L>()) {
      if (in.slab) {  // pair buffer [j1][c2][c3] for the slab pencil
        constexpr int pf = sizeof(T) == 8 ? 1 : 0;  // as below
        const int nxb = (n1 + Sh::PL - 1) / Sh::PL;
        hipLaunchKernelGGL((k_plane_reg<T, L, EXPLICIT, T, true>), pf ? dim3(b.npairs, nxb) : dim3(nxb, b.npairs),
                           dim3(Sh::NTP), Sh::LDS, p.stream, n1, in.nbands, bs, static_cast<const C*>(psi), o0, nP,
                           tri, parts, pairs, tbuf, pf);
        return;
      }
    }
    // FP64: pairs fastest in the grid (alpha boron FP64 plane pass 180 against
    // 207 ms per step; FP32 on the slab path loses with it)
    constexpr int pf = sizeof(T) == 8 ? 1 : 0;
    const int nxb = (n1 + Sh::PL - 1) / Sh::PL;
    hipLaunchKernelGGL((k_plane_reg<T, L, EXPLICIT>), pf ? dim3(b.npairs, nxb) : dim3(nxb, b.npairs), dim3(Sh::NTP),
                       Sh::LDS, p.stream, n1, in.nbands, bs, static_cast<const C*>(psi), o0, nP, tri, parts, pairs, tbuf,
                       pf);
  }
}

// the slab pencil of an apply batch (cubic grids); epart not null: the
// energy variant; returns the slabs' workgroups per pair (0: not compiled)
template <typename T, int L>
int launch_pencil_slab(const Plan& p, const Batch& b, const Instance& in, const int2* parts, const int* qmap,
                       typename cx<T>::t* tbuf, const T* vtab, const double* occ, const double* kw, double* epart) {
  if constexpr (slab_len<T, L>()) {
    using Sh = RegShape<T, L>;
    const int nlb = (L + Sh::PL - 1) / Sh::PL;
    if (epart)
      hipLaunchKernelGGL((k_pencil_slab<T, L, true>), dim3(nlb, b.npairs), dim3(Sh::NTP), Sh::LDS, p.stream,
                         in.nbands, in.nk, b.o0, b.nP, b.tri, parts, qmap, tbuf, vtab, occ, kw, epart);
    else
      hipLaunchKernelGGL((k_pencil_slab<T, L, false>), dim3(nlb, b.npairs), dim3(Sh::NTP), Sh::LDS, p.stream,
                         in.nbands, in.nk, b.o0, b.nP, b.tri, parts, qmap, tbuf, vtab, occ, kw, epart);
    return nlb;
  } else {
    return 0;
  }
}

// the line accumulate of an apply batch: its outputs and, for a batch of two
// blocks, its partners in the same launch (false: not compiled)
template <typename T, int L>
bool launch_acc_line(const Plan& p, const Batch& b, const Instance& in, const int2* parts,
                     const typename cx<T>::t* tbuf, const void* psi, const double* occ, const double* kw, void* out,
                     const double* gscale, double hscale, bool backward) {
  if constexpr (slab_len<T, L>()) {
    using C = typename cx<T>::t;
    const int rows = b.nO + (b.mirror ? b.nP : 0);
    if constexpr (line_split<T, L>())
      hipLaunchKernelGGL((k_acc_line_split<T, L>), dim3(rows, (L * L + 127) / 128), dim3(256), 0, p.stream,
                         in.nbands, static_cast<long long>(in.band_stride), b.o0, b.nO, b.nP, b.tri, parts, tbuf,
                         static_cast<const C*>(psi), occ, kw, static_cast<C*>(out), b.first, b.first_mirror, gscale,
                         hscale, backward ? 1 : 0);
    else
      hipLaunchKernelGGL((k_acc_line<T, L>), dim3(rows, (L * L + 255) / 256), dim3(256), 0, p.stream, in.nbands,
                         static_cast<long long>(in.band_stride), b.o0, b.nO, b.nP, b.tri, parts, tbuf,
                         static_cast<const C*>(psi), occ, kw, static_cast<C*>(out), b.first, b.first_mirror, gscale,
                         hscale, backward ? 1 : 0);
    return true;
  } else {
    return false;
  }
}

// epart not null: the energy variant, weighted partials per (pair, line
// block) into epart; returns the line blocks per pair
template <typename T, int L>
int launch_pencil_apply(const Plan& p, const Batch& b, const Instance& in, const int2* parts, const int* qmap,
                        typename cx<T>::t* tbuf, const T* vtab, const double* occ, const double* kw, double* epart) {
  const int ll = in.grid[1] * in.grid[2];
  if constexpr (RegPolicy<T, L>::SPLIT_PENCIL) {
    const int nlb = (ll + SplitShape<T, L>::LPB - 1) / SplitShape<T, L>::LPB;
    if (epart)
      hipLaunchKernelGGL((k_pencil_apply_split<T, L, true>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll,
                         in.nbands, in.nk, b.o0, b.nP, b.tri, parts, qmap, tbuf, vtab, occ, kw, epart);
    else
      hipLaunchKernelGGL((k_pencil_apply_split<T, L, false>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll,
                         in.nbands, in.nk, b.o0, b.nP, b.tri, parts, qmap, tbuf, vtab, occ, kw, epart);
    return nlb;
  } else {
    const int nlb = (ll + 255) / 256;
    if (epart)
      hipLaunchKernelGGL((k_pencil_apply_reg<T, L, true>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll,
                         in.nbands, in.nk, b.o0, b.nP, b.tri, parts, qmap, tbuf, vtab, occ, kw, epart);
    else
      hipLaunchKernelGGL((k_pencil_apply_reg<T, L, false>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll,
                         in.nbands, in.nk, b.o0, b.nP, b.tri, parts, qmap, tbuf, vtab, occ, kw, epart);
    return nlb;
  }
}

// returns the number of line blocks per pair (partial sums in epart)
template <typename T, int L, typename TV = T>
int launch_pencil_energy(const Plan& p, const Batch& b, const Instance& in, const PairRef* pairs,
                         const typename cx<T>::t* tbuf, const TV* vtab, double* epart) {
  const int ll = in.grid[1] * in.grid[2];
  if constexpr (RegPolicy<T, L>::SPLIT_PENCIL) {
    const int nlb = (ll + SplitShape<T, L>::LPB - 1) / SplitShape<T, L>::LPB;
    hipLaunchKernelGGL((k_pencil_energy_split<T, L, TV>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll, pairs,
                       tbuf, vtab, epart);
    return nlb;
  } else {
    const int nlb = (ll + 255) / 256;
    hipLaunchKernelGGL((k_pencil_energy_reg<T, L, TV>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll, pairs, tbuf,
                       vtab, epart);
    return nlb;
  }
}

// the lane-pair accumulate where the one-lane kernel would need too many
// registers: RegPolicy's choice, and for FP32 sums over FP64 orbitals and
// outputs (FOCK_MIXED_INV, whose wide operands add registers) from 40 up
template <typename T, int L, typename TI>
constexpr bool split_acc() {
  return sizeof(TI) != sizeof(T) ? L >= 40 : RegPolicy<T, L>::SPLIT_ACC;
}

template <typename T, int L, typename TI, bool SPLIT>
void launch_acc_kernel(const Plan& p, const Batch& b, const Instance& in, const int2* parts,
                       const typename cx<T>::t* tbuf, const void* psi, const double* occ, const double* kw, void* out,
                       const double* gscale, double hscale, bool backward) {
  using C = typename cx<TI>::t;
  const int n1 = in.grid[0];
  const long long bs = static_cast<long long>(in.band_stride);
  const int rows = b.nO + (b.mirror ? b.nP : 0);
  if constexpr (SPLIT) {
    using Sh = SplitShape<T, L>;
    hipLaunchKernelGGL((k_acc_split<T, L, TI>), dim3(rows, (n1 + Sh::PL - 1) / Sh::PL), dim3(Sh::NTP), Sh::LDS,
                       p.stream, n1, in.nbands, bs, b.o0, b.nO, b.nP, b.tri, parts, tbuf, static_cast<const C*>(psi),
                       occ, kw, static_cast<C*>(out), b.first, b.first_mirror, gscale, hscale, backward ? 1 : 0);
  } else {
    using Sh = RegShape<T, L>;
    constexpr bool PF = sizeof(TI) == sizeof(T) && RegPolicy<T, L>::ACC_PREFETCH;
    hipLaunchKernelGGL((k_acc_reg<T, L, TI, PF>), dim3(rows, (n1 + Sh::PL - 1) / Sh::PL), dim3(Sh::NTP), Sh::LDS,
                       p.stream, n1, in.nbands, bs, b.o0, b.nO, b.nP, b.tri, parts, tbuf, static_cast<const C*>(psi),
                       occ, kw, static_cast<C*>(out), b.first, b.first_mirror, gscale, hscale, backward ? 1 : 0);
  }
}

// the accumulate pass of a batch: its outputs, and for a batch of unordered
// pairs of two blocks also its partners (see k_acc_reg)
template <typename T, int L, typename TI = T>
void launch_acc_all(const Plan& p, const Batch& b, const Instance& in, const int2* parts, const typename cx<T>::t* tbuf,
                    const void* psi, const double* occ, const double* kw, void* out, const double* gscale,
                    double hscale, bool backward) {
  launch_acc_kernel<T, L, TI, split_acc<T, L, TI>()>(p, b, in, parts, tbuf, psi, occ, kw, out, gscale, hscale,
                                                     backward);
}

template <typename T, int L>
void reg_lds_attr(int lim) {
  using Po = RegPolicy<T, L>;
  const void* fs[4];
  if constexpr (Po::SPLIT_PLANE) {
    fs[0] = reinterpret_cast<const void*>(&k_plane_split<T, L, false>);
    fs[1] = reinterpret_cast<const void*>(&k_plane_split<T, L, true>);
  } else {
    fs[0] = reinterpret_cast<const void*>(&k_plane_reg<T, L, false>);
    fs[1] = reinterpret_cast<const void*>(&k_plane_reg<T, L, true>);
  }
  if constexpr (Po::SPLIT_ACC)
    fs[2] = reinterpret_cast<const void*>(&k_acc_split<T, L>);
  else
    fs[2] = reinterpret_cast<const void*>(&k_acc_reg<T, L, T, Po::ACC_PREFETCH>);
  fs[3] = fs[2];
  for (const void* f : fs)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) (void)hipGetLastError();
  if constexpr (slab_len<T, L>()) {
    const void* gs[4] = {reinterpret_cast<const void*>(&k_plane_reg<T, L, false, T, true>),
                         reinterpret_cast<const void*>(&k_plane_reg<T, L, true, T, true>),
                         reinterpret_cast<const void*>(&k_pencil_slab<T, L, false>),
                         reinterpret_cast<const void*>(&k_pencil_slab<T, L, true>)};
    for (const void* f : gs)
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) (void)hipGetLastError();
  }
}

// FOCK_MIXED: FP32 plane pass (FP64 orbitals rounded on load), mixed pencil
// pass, FP64 accumulate pass (the FP64 variant of the length)
template <int L>
struct MixedPolicy {
  using Acc = RegPolicy<double, L>;
  static constexpr int PLANE_LDS = RegShape<float, L>::LDS;
  static constexpr int LDS = PLANE_LDS > Acc::ACC_LDS ? PLANE_LDS : Acc::ACC_LDS;
};

template <int L>
int launch_pencil_mixed(const Plan& p, const Batch& b, const Instance& in, const int2* parts, const int* qmap,
                        const float2* t32, double2* t64, const double* vtab, const double* occ, const double* kw,
                        double* epart) {
  const int ll = in.grid[1] * in.grid[2];
  const int nlb = (ll + 127) / 128;
  if (epart)
    hipLaunchKernelGGL((k_pencil_apply_mixed<L, true>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll, in.nbands,
                       in.nk, b.o0, b.nP, b.tri, parts, qmap, t32, t64, vtab, occ, kw, epart);
  else
    hipLaunchKernelGGL((k_pencil_apply_mixed<L, false>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll, in.nbands,
                       in.nk, b.o0, b.nP, b.tri, parts, qmap, t32, t64, vtab, occ, kw, epart);
  return nlb;
}

template <int L>
void mixed_lds_attr(int lim) {
  using Acc = RegPolicy<double, L>;
  const void* fs[4] = {reinterpret_cast<const void*>(&k_plane_reg<float, L, false, double>),
                       reinterpret_cast<const void*>(&k_plane_reg<float, L, true, double>), nullptr, nullptr};
  if constexpr (Acc::SPLIT_ACC)
    fs[2] = reinterpret_cast<const void*>(&k_acc_split<double, L>);
  else
    fs[2] = reinterpret_cast<const void*>(&k_acc_reg<double, L, double, Acc::ACC_PREFETCH>);
  fs[3] = fs[2];
  for (const void* f : fs)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) (void)hipGetLastError();
}

// FOCK_MIXED_INV: FP64 plane pass, mixed pencil pass, FP32 accumulate pass
// reading FP64 orbitals and writing FP64 outputs
template <int L>
struct MixInvPolicy {
  static constexpr int ACC_LDS = L >= 40 ? SplitShape<float, L>::LDS : RegShape<float, L>::LDS;
  static constexpr int LDS = RegPolicy<double, L>::PLANE_LDS > ACC_LDS ? RegPolicy<double, L>::PLANE_LDS : ACC_LDS;
};

template <int L>
int launch_pencil_mixinv(const Plan& p, const Batch& b, const Instance& in, const int2* parts, const int* qmap,
                         const double2* t64, float2* t32, const double* vtab, const double* occ, const double* kw,
                         double* epart) {
  const int ll = in.grid[1] * in.grid[2];
  const int nlb = (ll + 127) / 128;
  if (epart)
    hipLaunchKernelGGL((k_pencil_apply_mixinv<L, true>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll, in.nbands,
                       in.nk, b.o0, b.nP, b.tri, parts, qmap, t64, t32, vtab, occ, kw, epart);
  else
    hipLaunchKernelGGL((k_pencil_apply_mixinv<L, false>), dim3(nlb, b.npairs), dim3(256), 0, p.stream, ll, in.nbands,
                       in.nk, b.o0, b.nP, b.tri, parts, qmap, t64, t32, vtab, occ, kw, epart);
  return nlb;
}

template <int L>
void mixinv_lds_attr(int lim) {
  const void* fs[4] = {nullptr, nullptr, nullptr, nullptr};
  if constexpr (RegPolicy<double, L>::SPLIT_PLANE) {
    fs[0] = reinterpret_cast<const void*>(&k_plane_split<double, L, false>);
    fs[1] = reinterpret_cast<const void*>(&k_plane_split<double, L, true>);
  } else {
    fs[0] = reinterpret_cast<const void*>(&k_plane_reg<double, L, false>);
    fs[1] = reinterpret_cast<const void*>(&k_plane_reg<double, L, true>);
  }
  if constexpr (split_acc<float, L, double>())
    fs[2] = reinterpret_cast<const void*>(&k_acc_split<float, L, double>);
  else
    fs[2] = reinterpret_cast<const void*>(&k_acc_reg<float, L, double>);
  fs[3] = fs[2];
  for (const void* f : fs)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) (void)hipGetLastError();
}

// the axis lengths with register-line kernels
#define FOCK_REG_L(X) X(24) X(32) X(36) X(40) X(48) X(50) X(54) X(60) X(64) X(72)

// `call` of the pass compiled for length n; false if there is none
#define FOCK_REG_DISPATCH(n, call)                 \
  [&]() -> bool {                                  \
    switch (n) {                                   \
      case 24: { constexpr int N = 24; call; return true; } \
      case 32: { constexpr int N = 32; call; return true; } \
      case 36: { constexpr int N = 36; call; return true; } \
      case 40: { constexpr int N = 40; call; return true; } \
      case 48: { constexpr int N = 48; call; return true; } \
      case 50: { constexpr int N = 50; call; return true; } \
      case 54: { constexpr int N = 54; call; return true; } \
      case 60: { constexpr int N = 60; call; return true; } \
      case 64: { constexpr int N = 64; call; return true; } \
      case 72: { constexpr int N = 72; call; return true; } \
      default: return false;                       \
    }                                              \
  }()

template <typename T>
hipError_t reg_apply_t(const Plan& p, const Batch& b, const void* psi, const double* occ, void* out,
                       const double* gscale, double hscale, bool backward, bool energy) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[b.inst];
  const int2* parts = reinterpret_cast<const int2*>(p.ws + b.part_off);
  const int* qmap = reinterpret_cast<const int*>(p.ws + in.qmap_off);
  const T* vtab = reinterpret_cast<const T*>(p.ws + in.vtab_off);
  const double* kw = reinterpret_cast<const double*>(p.ws + in.kw_off);
  C* tbuf = reinterpret_cast<C*>(p.ws + p.tbuf_off);
  double* epart = energy ? reinterpret_cast<double*>(p.ws + p.epart_off) : nullptr;
  int nlb = 0;
  bool ok;
  p.prof.begin(FOCK_K_PLANE, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[1], (launch_plane<T, N, false>(p, b, in, psi, parts, nullptr, tbuf)));
  p.prof.end(FOCK_K_PLANE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  p.prof.begin(FOCK_K_PENCIL, p.stream);
  if (in.slab)
    ok = FOCK_REG_DISPATCH(in.grid[0], (nlb = launch_pencil_slab<T, N>(p, b, in, parts, qmap, tbuf, vtab, occ, kw,
                                                                        epart))) &&
         nlb > 0;
  else
    ok = FOCK_REG_DISPATCH(in.grid[0], (nlb = launch_pencil_apply<T, N>(p, b, in, parts, qmap, tbuf, vtab, occ, kw,
                                                                         epart)));
  p.prof.end(FOCK_K_PENCIL, p.stream);
  if (!ok) return hipErrorInvalidValue;
  if (energy) {
    const hipError_t e = launch_sum_slot(p, static_cast<long long>(b.npairs) * nlb, b.eslot, b.mirror ? 2.0 : 1.0);
    if (e != hipSuccess) return e;
  }
  p.prof.begin(FOCK_K_ACCUMULATE, p.stream);
  if (in.slab) {
    bool launched = false;
    ok = FOCK_REG_DISPATCH(in.grid[1], (launched = launch_acc_line<T, N>(p, b, in, parts, tbuf, psi, occ, kw, out,
                                                                         gscale, hscale, backward))) &&
         launched;
  } else {
    ok = FOCK_REG_DISPATCH(in.grid[1], (launch_acc_all<T, N>(p, b, in, parts, tbuf, psi, occ, kw, out, gscale,
                                                              hscale, backward)));
  }
  p.prof.end(FOCK_K_ACCUMULATE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

// tbuf_off: the pair buffer (0: the plan's at tbuf_off)
template <typename T>
hipError_t reg_energy_t(const Plan& p, const Batch& b, const void* psi, const double* occ, size_t tbuf_off = 0) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[b.inst];
  const PairRef* pairs = reinterpret_cast<const PairRef*>(p.ws + b.pair_off);
  const T* vtab = reinterpret_cast<const T*>(p.ws + in.vtab_off);
  C* tbuf = reinterpret_cast<C*>(p.ws + (tbuf_off ? tbuf_off : p.tbuf_off));
  double* epart = reinterpret_cast<double*>(p.ws + p.epart_off);
  bool ok;
  int nlb = 0;
  p.prof.begin(FOCK_K_ENERGY_PLANE, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[1], (launch_plane<T, N, true>(p, b, in, psi, nullptr, pairs, tbuf)));
  p.prof.end(FOCK_K_ENERGY_PLANE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  p.prof.begin(FOCK_K_ENERGY_PENCIL, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[0], (nlb = launch_pencil_energy<T, N>(p, b, in, pairs, tbuf, vtab, epart)));
  p.prof.end(FOCK_K_ENERGY_PENCIL, p.stream);
  if (!ok) return hipErrorInvalidValue;
  return launch_energy_reduce(p, b, occ, nlb);
}

hipError_t mixed_apply_t(const Plan& p, const Batch& b, const void* psi, const double* occ, void* out,
                         const double* gscale, double hscale, bool backward, bool energy) {
  const Instance& in = p.inst[b.inst];
  const int2* parts = reinterpret_cast<const int2*>(p.ws + b.part_off);
  const int* qmap = reinterpret_cast<const int*>(p.ws + in.qmap_off);
  const double* vtab = reinterpret_cast<const double*>(p.ws + in.vtab_off);
  const double* kw = reinterpret_cast<const double*>(p.ws + in.kw_off);
  float2* t32 = reinterpret_cast<float2*>(p.ws + p.tbuf_off);
  double2* t64 = reinterpret_cast<double2*>(p.ws + p.tbuf64_off);
  double* epart = energy ? reinterpret_cast<double*>(p.ws + p.epart_off) : nullptr;
  int nlb = 0;
  bool ok;
  p.prof.begin(FOCK_K_PLANE, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[1], (launch_plane<float, N, false, double>(p, b, in, psi, parts, nullptr, t32)));
  p.prof.end(FOCK_K_PLANE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  p.prof.begin(FOCK_K_PENCIL, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[0], (nlb = launch_pencil_mixed<N>(p, b, in, parts, qmap, t32, t64, vtab, occ, kw,
                                                                      epart)));
  p.prof.end(FOCK_K_PENCIL, p.stream);
  if (!ok) return hipErrorInvalidValue;
  if (energy) {
    const hipError_t e = launch_sum_slot(p, static_cast<long long>(b.npairs) * nlb, b.eslot, b.mirror ? 2.0 : 1.0);
    if (e != hipSuccess) return e;
  }
  p.prof.begin(FOCK_K_ACCUMULATE, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[1], (launch_acc_all<double, N>(p, b, in, parts, t64, psi, occ, kw, out, gscale,
                                                                 hscale, backward)));
  p.prof.end(FOCK_K_ACCUMULATE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t mixinv_apply_t(const Plan& p, const Batch& b, const void* psi, const double* occ, void* out,
                          const double* gscale, double hscale, bool backward, bool energy) {
  const Instance& in = p.inst[b.inst];
  const int2* parts = reinterpret_cast<const int2*>(p.ws + b.part_off);
  const int* qmap = reinterpret_cast<const int*>(p.ws + in.qmap_off);
  const double* vtab = reinterpret_cast<const double*>(p.ws + in.vtab_off);
  const double* kw = reinterpret_cast<const double*>(p.ws + in.kw_off);
  float2* t32 = reinterpret_cast<float2*>(p.ws + p.tbuf_off);
  double2* t64 = reinterpret_cast<double2*>(p.ws + p.tbuf64_off);
  double* epart = energy ? reinterpret_cast<double*>(p.ws + p.epart_off) : nullptr;
  int nlb = 0;
  bool ok;
  p.prof.begin(FOCK_K_PLANE, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[1], (launch_plane<double, N, false>(p, b, in, psi, parts, nullptr, t64)));
  p.prof.end(FOCK_K_PLANE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  p.prof.begin(FOCK_K_PENCIL, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[0], (nlb = launch_pencil_mixinv<N>(p, b, in, parts, qmap, t64, t32, vtab, occ, kw,
                                                                       epart)));
  p.prof.end(FOCK_K_PENCIL, p.stream);
  if (!ok) return hipErrorInvalidValue;
  if (energy) {
    const hipError_t e = launch_sum_slot(p, static_cast<long long>(b.npairs) * nlb, b.eslot, b.mirror ? 2.0 : 1.0);
    if (e != hipSuccess) return e;
  }
  p.prof.begin(FOCK_K_ACCUMULATE, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[1], (launch_acc_all<float, N, double>(p, b, in, parts, t32, psi, occ, kw, out, gscale,
                                                                        hscale, backward)));
  p.prof.end(FOCK_K_ACCUMULATE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t mixed_energy_t(const Plan& p, const Batch& b, const void* psi, const double* occ) {
  const Instance& in = p.inst[b.inst];
  const PairRef* pairs = reinterpret_cast<const PairRef*>(p.ws + b.pair_off);
  const double* vtab = reinterpret_cast<const double*>(p.ws + in.vtab_off);
  float2* t32 = reinterpret_cast<float2*>(p.ws + p.tbuf_off);
  double* epart = reinterpret_cast<double*>(p.ws + p.epart_off);
  bool ok;
  int nlb = 0;
  p.prof.begin(FOCK_K_ENERGY_PLANE, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[1], (launch_plane<float, N, true, double>(p, b, in, psi, nullptr, pairs, t32)));
  p.prof.end(FOCK_K_ENERGY_PLANE, p.stream);
  if (!ok) return hipErrorInvalidValue;
  p.prof.begin(FOCK_K_ENERGY_PENCIL, p.stream);
  ok = FOCK_REG_DISPATCH(in.grid[0], (nlb = launch_pencil_energy<float, N, double>(p, b, in, pairs, t32, vtab,
                                                                                      epart)));
  p.prof.end(FOCK_K_ENERGY_PENCIL, p.stream);
  if (!ok) return hipErrorInvalidValue;
  return launch_energy_reduce(p, b, occ, nlb);
}

template <typename T, int L, int S>
void dft_plane_L(const Plan& p, int n1, int count, typename cx<T>::t* d, long long stride) {
  using Sh = RegShape<T, L>;
  hipLaunchKernelGGL((k_dft_plane_reg<T, L, S>), dim3((n1 + Sh::PL - 1) / Sh::PL, count), dim3(Sh::NTP), Sh::LDS,
                     p.stream, n1, d, stride);
}

template <typename T, int L, int S>
void dft_pencil_L(const Plan& p, int ll, int count, typename cx<T>::t* d, long long stride) {
  hipLaunchKernelGGL((k_dft_pencil_reg<T, L, S>), dim3((ll + 255) / 256, count), dim3(256), 0, p.stream, ll, d,
                     stride);
}

template <typename T, int L>
void dft_reg_lds_attr(int lim) {
  const void* fs[] = {reinterpret_cast<const void*>(&k_dft_plane_reg<T, L, -1>),
                      reinterpret_cast<const void*>(&k_dft_plane_reg<T, L, +1>)};
  for (const void* f : fs)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) (void)hipGetLastError();
}

// the lengths with one-lane DFT kernels, per precision (longer FP64 lines would spill)
#define FOCK_DFT_F32(X) X(16) X(24) X(32) X(36) X(40) X(48) X(50) X(54) X(60) X(64) X(72)
#define FOCK_DFT_F64(X) X(16) X(24) X(32)

bool reg_len(int n) {
  switch (n) {
    case 24: case 32: case 36: case 40: case 48: case 50: case 54: case 60: case 64: case 72: return true;
    default: return false;
  }
}

bool dft_len(fock_precision prec, int n) {
  switch (n) {
    case 16: case 24: case 32: return true;
    case 36: case 40: case 48: case 50: case 54: case 60: case 64: case 72: return prec == FOCK_C64;
    default: return false;
  }
}

template <typename T, int S>
hipError_t reg_dft3_t(const Plan& p, int inst, int count, void* data, long long stride) {
  using C = typename cx<T>::t;
  const int* g = p.inst[inst].grid;
  C* d = static_cast<C*>(data);
  bool ok = false;
#define CASE(N) \
  case N: dft_plane_L<T, N, S>(p, g[0], count, d, stride); ok = true; break;
  if constexpr (sizeof(T) == 4) {
    switch (g[1]) { FOCK_DFT_F32(CASE) default: break; }
  } else {
    switch (g[1]) { FOCK_DFT_F64(CASE) default: break; }
  }
#undef CASE
  if (!ok) return hipErrorInvalidValue;
  ok = false;
#define CASE(N) \
  case N: dft_pencil_L<T, N, S>(p, g[1] * g[2], count, d, stride); ok = true; break;
  if constexpr (sizeof(T) == 4) {
    switch (g[0]) { FOCK_DFT_F32(CASE) default: break; }
  } else {
    switch (g[0]) { FOCK_DFT_F64(CASE) default: break; }
  }
#undef CASE
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

bool reg_slab_supported(fock_precision prec, const int grid[3]) {
  const int n = grid[0];
  if (grid[1] != n || grid[2] != n || !reg_supported(prec, grid)) return false;
  if (prec == FOCK_C64) return true;
  return prec == FOCK_C128 && n <= 32;
}

// measured per step: alpha boron 32^3 FP32 370 against 385 ms, FP64 758
// against 886 ms; beta boron 72^3 7.20 against 8.04 s; the 64^3 preset FP32
// 42.8 against 46.5 ms (with the lane-pair line accumulate; one lane per
// line, a whole SIMD's registers, took 54.9 ms).  Cubic cells with 2x2x2 k
// (apply + energy + gradient): FP32 36^3 69.9 against 72.5 ms, 40^3 92.9
// against 100.9, 48^3 70.7 against 72.9, 50^3 84.5 against 100.5, 54^3 111.9
// against 116.5; FP64 24^3 34.7 against 43.9.  Kept plane-wise: FP32 60^3
// (93.7 against 87.6 ms); FP32 24^3 stays on the whole-pair kernel (17.1 ms
// against 19.8 on the slab path).
bool reg_slab_default(fock_precision prec, const int grid[3]) {
  const int n = grid[0];
  if (!reg_slab_supported(prec, grid)) return false;
  if (prec == FOCK_C128) return true;  // 24^3 and 32^3
  return n != 24 && n != 60;
}

bool reg_supported(fock_precision prec, const int grid[3]) {
  (void)prec;
  return grid[1] == grid[2] && reg_len(grid[0]) && reg_len(grid[1]);
}

size_t reg_lds_bytes(fock_precision prec, int L) {
  size_t r = 0;
#define CASE(N)                                                                                \
  case N:                                                                                      \
    r = prec == FOCK_C64     ? RegPolicy<float, N>::LDS                                        \
        : prec == FOCK_MIXED ? MixedPolicy<N>::LDS                                             \
        : prec == FOCK_MIXED_INV ? MixInvPolicy<N>::LDS                                        \
                                 : RegPolicy<double, N>::LDS;                                  \
    break;
  switch (L) { FOCK_REG_L(CASE) default: break; }
#undef CASE
  return r;
}

void prepare_reg_kernels(fock_precision prec, int lim) {
#define CASE(N)                                     \
  if (prec == FOCK_C64) reg_lds_attr<float, N>(lim); \
  else if (prec == FOCK_MIXED) mixed_lds_attr<N>(lim); \
  else if (prec == FOCK_MIXED_INV) { mixinv_lds_attr<N>(lim); reg_lds_attr<double, N>(lim); } \
  else reg_lds_attr<double, N>(lim);
  FOCK_REG_L(CASE)
#undef CASE
}

bool reg_dft_supported(fock_precision prec, const int grid[3]) {
  return grid[1] == grid[2] && dft_len(prec, grid[0]) && dft_len(prec, grid[1]);
}

hipError_t launch_reg_dft3(const Plan& p, int inst, int sign, int count, void* data, long long stride) {
  if (p.prec == FOCK_C64)
    return sign < 0 ? reg_dft3_t<float, -1>(p, inst, count, data, stride)
                    : reg_dft3_t<float, +1>(p, inst, count, data, stride);
  return sign < 0 ? reg_dft3_t<double, -1>(p, inst, count, data, stride)
                  : reg_dft3_t<double, +1>(p, inst, count, data, stride);
}

void prepare_reg_dft_kernels(fock_precision prec, int lim) {
#define CASE(N) dft_reg_lds_attr<float, N>(lim);
  if (prec == FOCK_C64) { FOCK_DFT_F32(CASE) }
#undef CASE
#define CASE(N) dft_reg_lds_attr<double, N>(lim);
  if (prec != FOCK_C64) { FOCK_DFT_F64(CASE) }
#undef CASE
}

hipError_t launch_reg_apply_batch(const Plan& p, const Batch& b, const void* psi, const double* occ, void* out,
                                  const double* gscale, double hscale, bool backward, bool energy) {
  if (p.prec == FOCK_MIXED) return mixed_apply_t(p, b, psi, occ, out, gscale, hscale, backward, energy);
  if (p.prec == FOCK_MIXED_INV) return mixinv_apply_t(p, b, psi, occ, out, gscale, hscale, backward, energy);
  return p.prec == FOCK_C128 ? reg_apply_t<double>(p, b, psi, occ, out, gscale, hscale, backward, energy)
                             : reg_apply_t<float>(p, b, psi, occ, out, gscale, hscale, backward, energy);
}


hipError_t launch_reg_energy_batch(const Plan& p, const Batch& b, const void* psi, const double* occ) {
  if (p.prec == FOCK_MIXED) return mixed_energy_t(p, b, psi, occ);
  // FOCK_MIXED_INV: the energy takes the FP64 forward transforms (its FP64 pair buffer)
  if (p.prec == FOCK_MIXED_INV) return reg_energy_t<double>(p, b, psi, occ, p.tbuf64_off);
  return p.prec == FOCK_C128 ? reg_energy_t<double>(p, b, psi, occ) : reg_energy_t<float>(p, b, psi, occ);
}

}  // namespace fock
