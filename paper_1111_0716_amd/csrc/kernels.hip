// HIP kernels of the exchange hot path for gfx950 and their launchers.
//
// One band pair (output n at k, partner m at k') is carried through three
// passes over the FFT grid (paper, "Our Implementation": the band-pair loop
// that runs on the GPU; "CPU Performance Analysis": FFTs, data manipulation
// and the accumulate that make up FOCK_ACC):
//
//   plane pass   per j1-plane: rho = conj(u_m) u_n (coalesced reads of both
//                orbitals), forward FFT along axis 3 then axis 2 in LDS,
//                plane stored to the pair buffer T.
//   pencil pass  per c2-slab [j1][c3]: forward FFT along axis 1, multiply by
//                v_q(c)/N (apply) or accumulate sum v_q |P|^2 in FP64
//                (energy), inverse FFT along axis 1 (apply).
//   acc pass     per (output n, j1-plane): for every partner of the batch,
//                inverse FFT along axis 2 then axis 3 and
//                acc += -w_k' f_k'm u_m * W in registers; one write of the
//                output plane per batch (no atomics, fixed order).
//
// Energies: per (pair, c2) partial sums in FP64, then a fixed-order tree per
// batch and a compensated (Neumaier) sum over batches.
#include <algorithm>

#include "fft_lds.hpp"
#include "fock_internal.hpp"

namespace fock {

struct Geo {
  int n1, n2, n3;
  int nk, nbands;
  long long bs;  // band stride in elements
};

// ---------------------------------------------------------------------------
// deterministic block reduction of a double (kBlock threads, wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
  }
  __syncthreads();
  return t;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// plane pass
// ---------------------------------------------------------------------------
template <typename T, bool EXPLICIT>
__global__ __launch_bounds__(kBlock) void k_fwd_plane(Geo g, const typename cx<T>::t* __restrict__ psi, int o0,
                                                      int nP, const int2* __restrict__ parts,
                                                      const PairRef* __restrict__ pairs,
                                                      typename cx<T>::t* __restrict__ tbuf,
                                                      const typename cx<T>::t* __restrict__ tw) {
  using C = typename cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int j1 = blockIdx.x, pi = blockIdx.y;
  int okn, pkm;  // global band indices k*nbands + n
  if (EXPLICIT) {
    const PairRef pr = pairs[pi];
    okn = pr.k * g.nbands + pr.n;
    pkm = pr.kp * g.nbands + pr.m;
  } else {
    const int o = pi / nP, p = pi - o * nP;
    okn = o0 + o;
    const int2 r = parts[p];
    pkm = r.x * g.nbands + r.y;
  }
  const int plane = g.n2 * g.n3;
  const C* a = psi + static_cast<size_t>(okn) * g.bs + static_cast<size_t>(j1) * plane;
  const C* b = psi + static_cast<size_t>(pkm) * g.bs + static_cast<size_t>(j1) * plane;
  for (int e = threadIdx.x; e < plane; e += kBlock) s[e] = cmulconj(b[e], a[e]);
  __syncthreads();
  fft_lines<C, -1, true>(s, g.n3, g.n2, g.n3, 1, tw);   // axis 3 (rows)
  fft_lines<C, -1, false>(s, g.n2, g.n3, 1, g.n3, tw);  // axis 2 (columns)
  C* t = tbuf + (static_cast<size_t>(pi) * g.n1 + j1) * plane;
  for (int e = threadIdx.x; e < plane; e += kBlock) t[e] = s[e];
}

// ---------------------------------------------------------------------------
// pencil pass, apply: FFT_1, x v_q / N, IFFT_1
// ---------------------------------------------------------------------------
// EN (fock_apply_energy): also w_o f_o w'_p f'_p sum v/N |P|^2 of the slab,
// in FP64, into epart[pair * n2 + c2]
template <typename T, bool EN = false>
__global__ __launch_bounds__(kBlock) void k_pencil_apply(Geo g, int o0, int nP, const int2* __restrict__ parts,
                                                         const int* __restrict__ qmap,
                                                         typename cx<T>::t* __restrict__ tbuf,
                                                         const T* __restrict__ vtab,
                                                         const typename cx<T>::t* __restrict__ tw,
                                                         const double* __restrict__ occ,
                                                         const double* __restrict__ kw,
                                                         double* __restrict__ epart) {
  using C = typename cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int c2 = blockIdx.x, pi = blockIdx.y;
  const int o = pi / nP, p = pi - o * nP;
  const int ok = (o0 + o) / g.nbands;
  const int q = qmap[ok * g.nk + parts[p].x];
  const int plane = g.n2 * g.n3, tile = g.n1 * g.n3;
  const size_t npts = static_cast<size_t>(g.n1) * plane;
  C* base = tbuf + static_cast<size_t>(pi) * npts + static_cast<size_t>(c2) * g.n3;
  const float rcp3 = 1.0f / static_cast<float>(g.n3);
  for (int e = threadIdx.x; e < tile; e += kBlock) {
    const int j1 = fdiv(e, rcp3), c3 = e - j1 * g.n3;
    s[e] = base[static_cast<size_t>(j1) * plane + c3];
  }
  __syncthreads();
  fft_lines<C, -1, false>(s, g.n1, g.n3, 1, g.n3, tw);  // axis 1
  const T* v = vtab + static_cast<size_t>(q) * npts + static_cast<size_t>(c2) * g.n3;
  double en = 0.0;
  for (int e = threadIdx.x; e < tile; e += kBlock) {
    const int c1 = fdiv(e, rcp3), c3 = e - c1 * g.n3;
    const T vv = v[static_cast<size_t>(c1) * plane + c3];
    if constexpr (EN) {
      const double px = static_cast<double>(s[e].x), py = static_cast<double>(s[e].y);
      en += static_cast<double>(vv) * (px * px + py * py);
    }
    s[e] = cscale(s[e], vv);
  }
  if constexpr (EN) {
    __shared__ double red[kBlock / 64];
    const double tot = block_sum(en, red);  // ends with a barrier
    if (threadIdx.x == 0) {
      const int2 r = parts[p];
      epart[static_cast<size_t>(pi) * g.n2 + c2] =
          kw[ok] * occ[o0 + o] * kw[r.x] * occ[r.x * g.nbands + r.y] * tot;
    }
  } else {
    __syncthreads();
  }
  fft_lines<C, +1, false>(s, g.n1, g.n3, 1, g.n3, tw);  // inverse axis 1
  for (int e = threadIdx.x; e < tile; e += kBlock) {
    const int j1 = fdiv(e, rcp3), c3 = e - j1 * g.n3;
    base[static_cast<size_t>(j1) * plane + c3] = s[e];
  }
}

// ---------------------------------------------------------------------------
// pencil pass, energy: FFT_1 and sum_c v_q(c)/N |P(c)|^2 in FP64
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pencil_energy(Geo g, const PairRef* __restrict__ pairs,
                                                          const typename cx<T>::t* __restrict__ tbuf,
                                                          const T* __restrict__ vtab,
                                                          const typename cx<T>::t* __restrict__ tw,
                                                          double* __restrict__ epart) {
  using C = typename cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[kBlock / 64];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int c2 = blockIdx.x, pi = blockIdx.y;
  const int q = pairs[pi].q;
  const int plane = g.n2 * g.n3, tile = g.n1 * g.n3;
  const size_t npts = static_cast<size_t>(g.n1) * plane;
  const C* base = tbuf + static_cast<size_t>(pi) * npts + static_cast<size_t>(c2) * g.n3;
  const float rcp3 = 1.0f / static_cast<float>(g.n3);
  for (int e = threadIdx.x; e < tile; e += kBlock) {
    const int j1 = fdiv(e, rcp3), c3 = e - j1 * g.n3;
    s[e] = base[static_cast<size_t>(j1) * plane + c3];
  }
  __syncthreads();
  fft_lines<C, -1, false>(s, g.n1, g.n3, 1, g.n3, tw);
  const T* v = vtab + static_cast<size_t>(q) * npts + static_cast<size_t>(c2) * g.n3;
  double acc = 0.0;
  for (int e = threadIdx.x; e < tile; e += kBlock) {
    const int c1 = fdiv(e, rcp3), c3 = e - c1 * g.n3;
    const double px = static_cast<double>(s[e].x), py = static_cast<double>(s[e].y);
    acc += static_cast<double>(v[static_cast<size_t>(c1) * plane + c3]) * (px * px + py * py);
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) epart[static_cast<size_t>(pi) * g.n2 + c2] = tot;
}

// ---------------------------------------------------------------------------
// accumulate pass: inverse FFT of axes 2 and 3 per partner, acc in registers
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_inv_plane_acc(Geo g, int o0, int nP, const int2* __restrict__ parts,
                                                          const typename cx<T>::t* __restrict__ tbuf,
                                                          const typename cx<T>::t* __restrict__ psi,
                                                          const double* __restrict__ occ,
                                                          const double* __restrict__ kw,
                                                          typename cx<T>::t* __restrict__ out, int first,
                                                          const double* __restrict__ gscale, double hscale,
                                                          int backward, const typename cx<T>::t* __restrict__ tw) {
  using C = typename cx<T>::t;
  constexpr int E = (kNMax * kNMax + kBlock - 1) / kBlock;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int j1 = blockIdx.x, o = blockIdx.y;
  const int plane = g.n2 * g.n3;
  const size_t npts = static_cast<size_t>(g.n1) * plane;
  C acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = C{T(0), T(0)};
  for (int p = 0; p < nP; ++p) {
    const int2 r = parts[p];
    const C* src = tbuf + (static_cast<size_t>(o) * nP + p) * npts + static_cast<size_t>(j1) * plane;
    for (int e = threadIdx.x; e < plane; e += kBlock) s[e] = src[e];
    __syncthreads();
    fft_lines_call<C, +1, false>(s, g.n2, g.n3, 1, g.n3, tw);  // inverse axis 2
    fft_lines_call<C, +1, true>(s, g.n3, g.n2, g.n3, 1, tw);   // inverse axis 3
    const T coef = static_cast<T>(-kw[r.x] * occ[r.x * g.nbands + r.y]);
    const C* um = psi + static_cast<size_t>(r.x * g.nbands + r.y) * g.bs + static_cast<size_t>(j1) * plane;
    // elements past the plane load element 0 (in bounds) and are not used:
    // the loads stay unconditional and overlap
    C u[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = threadIdx.x + i * kBlock;
      u[i] = um[e < plane ? e : 0];
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = threadIdx.x + i * kBlock;
      if (e < plane) {
        const C w = cmul(u[i], s[e]);
        acc[i].x += coef * w.x;
        acc[i].y += coef * w.y;
      }
    }
    __syncthreads();
  }
  const int okn = o0 + o;
  double f = hscale;
  if (gscale) f *= gscale[0];
  if (backward) {
    const int ok = okn / g.nbands;
    f *= kw[ok] * occ[okn];
  }
  const T ft = static_cast<T>(f);
  C* dst = out + static_cast<size_t>(okn) * g.bs + static_cast<size_t>(j1) * plane;
  C old[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = threadIdx.x + i * kBlock;
    old[i] = first ? C{T(0), T(0)} : dst[e < plane ? e : 0];  // all loads before the first store
  }
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = threadIdx.x + i * kBlock;
    if (e < plane) dst[e] = cadd(old[i], cscale(acc[i], ft));
  }
}

// ---------------------------------------------------------------------------
// energy reductions
// ---------------------------------------------------------------------------
// one workgroup per energy batch: sum_c2 per pair, weight, fixed-order tree
__global__ __launch_bounds__(kBlock) void k_energy_batch(const PairRef* __restrict__ pairs, int npairs, int n2,
                                                         const double* __restrict__ epart,
                                                         const double* __restrict__ occ,
                                                         const double* __restrict__ kw, int nbands,
                                                         double* __restrict__ ebsum, int slot) {
  __shared__ double red[kBlock / 64];
  double sum = 0.0, comp = 0.0;
  for (int pi = threadIdx.x; pi < npairs; pi += kBlock) {
    const PairRef pr = pairs[pi];
    double e = 0.0;
    for (int c = 0; c < n2; ++c) e += epart[static_cast<size_t>(pi) * n2 + c];
    const double w = pr.mult * kw[pr.k] * occ[pr.k * nbands + pr.n] * kw[pr.kp] * occ[pr.kp * nbands + pr.m];
    const double x = w * e;
    const double t = sum + x;  // Neumaier
    comp += (fabs(sum) >= fabs(x)) ? (sum - t) + x : (x - t) + sum;
    sum = t;
  }
  const double tot = block_sum(sum + comp, red);
  if (threadIdx.x == 0) ebsum[slot] = tot;
}

// slots[slot] = mult * (sum of part[0..n)) in a fixed order: Neumaier per
// thread over a strided share, then the waves in order (1024 threads: the
// partials of a batch run to tens of thousands, read once).  mult is 2 for a
// batch of unordered pairs (each stands for both orders), else 1.
constexpr int kSumBlock = 1024;
__global__ __launch_bounds__(kSumBlock) void k_sum_slot(const double* __restrict__ part, long long n,
                                                        double* __restrict__ slots, int slot, double mult) {
  __shared__ double red[kSumBlock / 64];
  double sum = 0.0, comp = 0.0;
  for (long long i = threadIdx.x; i < n; i += kSumBlock) {
    const double x = part[i];
    const double t = sum + x;
    comp += (fabs(sum) >= fabs(x)) ? (sum - t) + x : (x - t) + sum;
    sum = t;
  }
  double v = sum + comp;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kSumBlock / 64; ++w) t += red[w];
    slots[slot] = mult * t;
  }
}

__global__ void k_energy_finish(const double* __restrict__ ebsum, int first, int count, double factor,
                                double* __restrict__ ex) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sum = 0.0, comp = 0.0;
  for (int i = 0; i < count; ++i) {
    const double x = ebsum[first + i];
    const double t = sum + x;
    comp += (fabs(sum) >= fabs(x)) ? (sum - t) + x : (x - t) + sum;
    sum = t;
  }
  ex[0] = factor * (sum + comp);
}

// ---------------------------------------------------------------------------
// zero the outputs of k-points that have no partner in the k-pair list
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_bands(typename cx<T>::t* __restrict__ out, int b0, long long bs,
                                                       long long npts) {
  using C = typename cx<T>::t;
  C* dst = out + static_cast<size_t>(b0 + blockIdx.y) * bs;
  for (long long e = blockIdx.x * static_cast<long long>(kBlock) + threadIdx.x; e < npts;
       e += static_cast<long long>(gridDim.x) * kBlock)
    dst[e] = C{T(0), T(0)};
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

inline Geo geo_of(const Instance& in) {
  return Geo{in.grid[0], in.grid[1], in.grid[2], in.nk, in.nbands, static_cast<long long>(in.band_stride)};
}

template <typename T>
hipError_t apply_batch_t(const Plan& p, const Batch& b, const void* psi, const double* occ, void* out, bool energy,
                         const double* gscale, double hscale, bool backward) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[b.inst];
  energy = energy && batch_apply_energy(p, b.inst);
  if (in.reg) return launch_reg_apply_batch(p, b, psi, occ, out, gscale, hscale, backward, energy);
  const Geo g = geo_of(in);
  const C* tw = reinterpret_cast<const C*>(p.ws + p.tw_off);
  const int2* parts = reinterpret_cast<const int2*>(p.ws + b.part_off);
  const int* qmap = reinterpret_cast<const int*>(p.ws + in.qmap_off);
  const T* vtab = reinterpret_cast<const T*>(p.ws + in.vtab_off);
  const double* kw = reinterpret_cast<const double*>(p.ws + in.kw_off);
  C* tbuf = reinterpret_cast<C*>(p.ws + p.tbuf_off);
  const size_t lds_plane = static_cast<size_t>(g.n2) * g.n3 * sizeof(C);
  const size_t lds_tile = static_cast<size_t>(g.n1) * g.n3 * sizeof(C);
  p.prof.begin(FOCK_K_PLANE, p.stream);
  hipLaunchKernelGGL((k_fwd_plane<T, false>), dim3(g.n1, b.npairs), dim3(kBlock), lds_plane, p.stream, g,
                     static_cast<const C*>(psi), b.o0, b.nP, parts, static_cast<const PairRef*>(nullptr), tbuf, tw);
  p.prof.end(FOCK_K_PLANE, p.stream);
  p.prof.begin(FOCK_K_PENCIL, p.stream);
  if (energy)
    hipLaunchKernelGGL((k_pencil_apply<T, true>), dim3(g.n2, b.npairs), dim3(kBlock), lds_tile, p.stream, g, b.o0,
                       b.nP, parts, qmap, tbuf, vtab, tw, occ, kw, reinterpret_cast<double*>(p.ws + p.epart_off));
  else
    hipLaunchKernelGGL((k_pencil_apply<T, false>), dim3(g.n2, b.npairs), dim3(kBlock), lds_tile, p.stream, g, b.o0,
                       b.nP, parts, qmap, tbuf, vtab, tw, occ, kw, static_cast<double*>(nullptr));
  p.prof.end(FOCK_K_PENCIL, p.stream);
  if (energy) {
    const hipError_t e = launch_sum_slot(p, static_cast<long long>(b.npairs) * g.n2, b.eslot, 1.0);
    if (e != hipSuccess) return e;
  }
  p.prof.begin(FOCK_K_ACCUMULATE, p.stream);
  hipLaunchKernelGGL((k_inv_plane_acc<T>), dim3(g.n1, b.nO), dim3(kBlock), lds_plane, p.stream, g, b.o0, b.nP,
                     parts, static_cast<const C*>(tbuf), static_cast<const C*>(psi), occ, kw, static_cast<C*>(out),
                     b.first, gscale, hscale, backward ? 1 : 0, tw);
  p.prof.end(FOCK_K_ACCUMULATE, p.stream);
  return hipGetLastError();
}

template <typename T>
hipError_t energy_batch_t(const Plan& p, const Batch& b, const void* psi, const double* occ) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[b.inst];
  if (in.reg) return launch_reg_energy_batch(p, b, psi, occ);
  const Geo g = geo_of(in);
  const C* tw = reinterpret_cast<const C*>(p.ws + p.tw_off);
  const PairRef* pairs = reinterpret_cast<const PairRef*>(p.ws + b.pair_off);
  const T* vtab = reinterpret_cast<const T*>(p.ws + in.vtab_off);
  C* tbuf = reinterpret_cast<C*>(p.ws + p.tbuf_off);
  double* epart = reinterpret_cast<double*>(p.ws + p.epart_off);
  const size_t lds_plane = static_cast<size_t>(g.n2) * g.n3 * sizeof(C);
  const size_t lds_tile = static_cast<size_t>(g.n1) * g.n3 * sizeof(C);
  p.prof.begin(FOCK_K_ENERGY_PLANE, p.stream);
  hipLaunchKernelGGL((k_fwd_plane<T, true>), dim3(g.n1, b.npairs), dim3(kBlock), lds_plane, p.stream, g,
                     static_cast<const C*>(psi), 0, 1, static_cast<const int2*>(nullptr), pairs, tbuf, tw);
  p.prof.end(FOCK_K_ENERGY_PLANE, p.stream);
  p.prof.begin(FOCK_K_ENERGY_PENCIL, p.stream);
  hipLaunchKernelGGL((k_pencil_energy<T>), dim3(g.n2, b.npairs), dim3(kBlock), lds_tile, p.stream, g, pairs,
                     static_cast<const C*>(tbuf), vtab, tw, epart);
  p.prof.end(FOCK_K_ENERGY_PENCIL, p.stream);
  return launch_energy_reduce(p, b, occ, g.n2);
}


// Dynamic LDS above 64 KiB: ask for the device's per-block limit.  The call
// is advisory on ROCm (launches beyond 64 KiB succeed up to the hardware
// limit); a refusal is cleared so it does not surface at an unrelated call.
template <typename T>
void allow_large_lds(int lim) {
  const void* fs[] = {reinterpret_cast<const void*>(&k_fwd_plane<T, false>),
                      reinterpret_cast<const void*>(&k_fwd_plane<T, true>),
                      reinterpret_cast<const void*>(&k_pencil_apply<T, false>),
                      reinterpret_cast<const void*>(&k_pencil_apply<T, true>),
                      reinterpret_cast<const void*>(&k_pencil_energy<T>),
                      reinterpret_cast<const void*>(&k_inv_plane_acc<T>)};
  for (const void* f : fs) {
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
      (void)hipGetLastError();
  }
}

template <typename T>
hipError_t zero_outputs_t(const Plan& p, int inst, void* out) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[inst];
  for (int k = 0; k < in.nk; ++k) {
    if (!in.kpartners[k].empty()) continue;
    const int gx = static_cast<int>(std::min<long long>(1024, (in.npts + kBlock - 1) / kBlock));
    p.prof.begin(FOCK_K_OTHER, p.stream);
    hipLaunchKernelGGL((k_zero_bands<T>), dim3(gx, in.nbands), dim3(kBlock), 0, p.stream, static_cast<C*>(out),
                       k * in.nbands, static_cast<long long>(in.band_stride), static_cast<long long>(in.npts));
    p.prof.end(FOCK_K_OTHER, p.stream);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_all_bands(const Plan& p, int inst, void* out) {
  const Instance& in = p.inst[inst];
  const int gx = static_cast<int>(std::min<long long>(1024, (in.npts + kBlock - 1) / kBlock));
  const int nbt = in.nk * in.nbands;
  for (int b0 = 0; b0 < nbt; b0 += 65535) {
    const int nb = std::min(65535, nbt - b0);
    p.prof.begin(FOCK_K_OTHER, p.stream);
    if (p.io64()) {
      hipLaunchKernelGGL((k_zero_bands<double>), dim3(gx, nb), dim3(kBlock), 0, p.stream, static_cast<double2*>(out),
                         b0, static_cast<long long>(in.band_stride), static_cast<long long>(in.npts));
    } else {
      hipLaunchKernelGGL((k_zero_bands<float>), dim3(gx, nb), dim3(kBlock), 0, p.stream, static_cast<float2*>(out),
                         b0, static_cast<long long>(in.band_stride), static_cast<long long>(in.npts));
    }
    p.prof.end(FOCK_K_OTHER, p.stream);
  }
  return hipGetLastError();
}

hipError_t launch_zero_outputs(const Plan& p, int inst, void* out) {
  return p.io64() ? zero_outputs_t<double>(p, inst, out) : zero_outputs_t<float>(p, inst, out);
}

hipError_t prepare_kernels(fock_precision prec, size_t* max_lds) {
  int dev = 0, lim = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  *max_lds = static_cast<size_t>(lim);
  prepare_fused_kernels(prec, lim - 256);
  prepare_reg_kernels(prec, lim - 64);
  prepare_dft_kernels(prec, lim - 64);
  if (lim > 65536) {
    if (prec != FOCK_C64)
      allow_large_lds<double>(lim - 64);
    else
      allow_large_lds<float>(lim - 64);
  }
  return hipSuccess;
}

hipError_t launch_apply_batch(const Plan& p, const Batch& b, const void* psi, const double* occ, void* out,
                              bool energy, const double* gscale, double hscale, bool backward) {
  return p.io64() ? apply_batch_t<double>(p, b, psi, occ, out, energy, gscale, hscale, backward)
                  : apply_batch_t<float>(p, b, psi, occ, out, energy, gscale, hscale, backward);
}

hipError_t launch_energy_batch(const Plan& p, const Batch& b, const void* psi, const double* occ) {
  return p.io64() ? energy_batch_t<double>(p, b, psi, occ) : energy_batch_t<float>(p, b, psi, occ);
}

hipError_t launch_energy_reduce(const Plan& p, const Batch& b, const double* occ, int n2) {
  const Instance& in = p.inst[b.inst];
  p.prof.begin(FOCK_K_ENERGY_REDUCE, p.stream);
  hipLaunchKernelGGL(k_energy_batch, dim3(1), dim3(kBlock), 0, p.stream,
                     reinterpret_cast<const PairRef*>(p.ws + b.pair_off), b.npairs, n2,
                     reinterpret_cast<const double*>(p.ws + p.epart_off), occ,
                     reinterpret_cast<const double*>(p.ws + in.kw_off), in.nbands,
                     reinterpret_cast<double*>(p.ws + p.ebsum_off), b.slot);
  p.prof.end(FOCK_K_ENERGY_REDUCE, p.stream);
  return hipGetLastError();
}

bool batch_apply_energy(const Plan& p, int inst) { return !p.inst[inst].fused; }

hipError_t launch_sum_slot(const Plan& p, long long n, int slot, double mult) {
  p.prof.begin(FOCK_K_ENERGY_REDUCE, p.stream);
  hipLaunchKernelGGL(k_sum_slot, dim3(1), dim3(kSumBlock), 0, p.stream, reinterpret_cast<const double*>(p.ws + p.epart_off),
                     n, reinterpret_cast<double*>(p.ws + p.ebsum_off), slot, mult);
  p.prof.end(FOCK_K_ENERGY_REDUCE, p.stream);
  return hipGetLastError();
}

hipError_t launch_aslot_finish(const Plan& p, int inst, double* ex) {
  const Instance& in = p.inst[inst];
  const double factor = -0.5 * in.omega / static_cast<double>(in.npts);  // as in launch_energy_finish
  p.prof.begin(FOCK_K_ENERGY_REDUCE, p.stream);
  hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(64), 0, p.stream,
                     reinterpret_cast<const double*>(p.ws + p.ebsum_off), in.first_aslot, in.n_aslot, factor, ex);
  p.prof.end(FOCK_K_ENERGY_REDUCE, p.stream);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const Plan& p, const double* part, long long n, int slot) {
  p.prof.begin(FOCK_K_ENERGY_REDUCE, p.stream);
  hipLaunchKernelGGL(k_sum_slot, dim3(1), dim3(kSumBlock), 0, p.stream, part, n,
                     reinterpret_cast<double*>(p.ws + p.ebsum_off), slot, 1.0);
  p.prof.end(FOCK_K_ENERGY_REDUCE, p.stream);
  return hipGetLastError();
}

hipError_t launch_eblk_finish(const Plan& p, int inst, double* ex) {
  const Instance& in = p.inst[inst];
  const double factor = -0.5 * in.omega / static_cast<double>(in.npts);  // as in launch_energy_finish
  if (in.rounds >= 0) {
    // one partial per unordered pair: summed in a fixed order into the
    // instance's slot, then scaled
    const FusedRounds& r = p.fused_rounds[in.rounds];
    hipError_t e = launch_sum_partials(p, reinterpret_cast<const double*>(p.ws + p.eblk_off) + r.eblk0, r.npairs,
                                       r.eslot);
    if (e != hipSuccess) return e;
    p.prof.begin(FOCK_K_ENERGY_REDUCE, p.stream);
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(64), 0, p.stream,
                       reinterpret_cast<const double*>(p.ws + p.ebsum_off), r.eslot, 1, factor, ex);
    p.prof.end(FOCK_K_ENERGY_REDUCE, p.stream);
    return hipGetLastError();
  }
  p.prof.begin(FOCK_K_ENERGY_REDUCE, p.stream);
  hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(64), 0, p.stream,
                     reinterpret_cast<const double*>(p.ws + p.eblk_off), in.first_eblk, in.n_eblk, factor, ex);
  p.prof.end(FOCK_K_ENERGY_REDUCE, p.stream);
  return hipGetLastError();
}

hipError_t launch_energy_finish(const Plan& p, int inst, double* ex) {
  const Instance& in = p.inst[inst];
  // the tables hold v/N, so e = N * sum; E_x = -1/2 (Omega/N^2) * N * sum
  const double factor = -0.5 * in.omega / static_cast<double>(in.npts);
  p.prof.begin(FOCK_K_ENERGY_REDUCE, p.stream);
  hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(64), 0, p.stream,
                     reinterpret_cast<const double*>(p.ws + p.ebsum_off), in.first_ebatch, in.n_ebatches, factor,
                     ex);
  p.prof.end(FOCK_K_ENERGY_REDUCE, p.stream);
  return hipGetLastError();
}


}  // namespace fock
