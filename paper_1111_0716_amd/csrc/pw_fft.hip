// Batched 3-D DFT on a plan's grid, and the plane-wave boundary of the
// exchange path: coefficients on the cutoff sphere to orbitals on the FFT
// grid and back (paper, "CPU Performance Analysis": the scatter/gather
// between sphere and grid around the FFTs of FOCK_ACC).
//
// The conversions run once per band (N_k N_b transforms against N_k^2 N_b^2
// pair transforms of the apply), so they are separate batched passes rather
// than part of the pair kernels:
//
//   to the grid    zero the bands, scatter c(G) / sqrt(Omega) to the grid
//                  class of G, inverse DFT (unnormalised, exp(+))
//   to the sphere  forward DFT in place, gather sqrt(Omega)/N F(class of G)
//
// DFT passes: on grids N1 x L x L with register-line kernels (pass_reg.hip) a
// plane pass (axes 2 and 3, one line per lane) and a pencil pass (axis 1);
// elsewhere per (grid, j1-plane) the axes 3 and 2 in LDS and per (grid,
// c2-slab) the axis 1 in LDS (the LDS Stockham transforms of fft_lds.hpp),
// so every {2,3,5}-smooth axis up to 72 works.
#include <algorithm>

#include "fft_lds.hpp"
#include "fock_internal.hpp"

namespace fock {

template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_dft_planes(int n2, int n3, typename cx<T>::t* __restrict__ data,
                                                       long long stride, long long plane0,
                                                       const typename cx<T>::t* __restrict__ tw) {
  using C = typename cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int plane = n2 * n3;
  C* g = data + static_cast<size_t>(blockIdx.y) * stride + (plane0 + blockIdx.x) * static_cast<size_t>(plane);
  for (int e = threadIdx.x; e < plane; e += kBlock) s[e] = g[e];
  __syncthreads();
  fft_lines<C, S, true>(s, n3, n2, n3, 1, tw);   // axis 3 (rows)
  fft_lines<C, S, false>(s, n2, n3, 1, n3, tw);  // axis 2 (columns)
  for (int e = threadIdx.x; e < plane; e += kBlock) g[e] = s[e];
}

template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_dft_pencils(int n1, int n2, int n3, typename cx<T>::t* __restrict__ data,
                                                        long long stride, const typename cx<T>::t* __restrict__ tw) {
  using C = typename cx<T>::t;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int c2 = blockIdx.x, plane = n2 * n3, tile = n1 * n3;
  C* base = data + static_cast<size_t>(blockIdx.y) * stride + static_cast<size_t>(c2) * n3;
  const float rcp3 = 1.0f / static_cast<float>(n3);
  for (int e = threadIdx.x; e < tile; e += kBlock) {
    const int j1 = fdiv(e, rcp3), c3 = e - j1 * n3;
    s[e] = base[static_cast<size_t>(j1) * plane + c3];
  }
  __syncthreads();
  fft_lines<C, S, false>(s, n1, n3, 1, n3, tw);  // axis 1
  for (int e = threadIdx.x; e < tile; e += kBlock) {
    const int j1 = fdiv(e, rcp3), c3 = e - j1 * n3;
    base[static_cast<size_t>(j1) * plane + c3] = s[e];
  }
}

// out[b][gidx[k][p]] = scale * coef[b][p] for p < min(npw[k], npw_max), b = k nbands + n;
// slots whose class lies outside the grid are skipped
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pw_scatter(const typename cx<T>::t* __restrict__ coef,
                                                       const int* __restrict__ gidx, const int* __restrict__ npw,
                                                       int npw_max, int nbands, int b0, long long bs, long long npts,
                                                       typename cx<T>::t* __restrict__ out, T scale) {
  const int b = b0 + blockIdx.y, k = b / nbands;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  const int np = min(npw[k], npw_max);
  if (p >= np) return;
  const int c = gidx[static_cast<size_t>(k) * npw_max + p];
  if (c < 0 || c >= npts) return;
  out[static_cast<size_t>(b) * bs + c] = cscale(coef[static_cast<size_t>(b) * npw_max + p], scale);
}

// coef[b][p] = scale * f[b][gidx[k][p]] for p < min(npw[k], npw_max), else 0
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pw_gather(const typename cx<T>::t* __restrict__ f,
                                                      const int* __restrict__ gidx, const int* __restrict__ npw,
                                                      int npw_max, int nbands, int b0, long long bs, long long npts,
                                                      typename cx<T>::t* __restrict__ coef, T scale) {
  using C = typename cx<T>::t;
  const int b = b0 + blockIdx.y, k = b / nbands;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= npw_max) return;
  C v{T(0), T(0)};
  if (p < npw[k]) {
    const int c = gidx[static_cast<size_t>(k) * npw_max + p];
    if (c >= 0 && c < npts) v = cscale(f[static_cast<size_t>(b) * bs + c], scale);
  }
  coef[static_cast<size_t>(b) * npw_max + p] = v;
}

namespace {

template <typename T>
hipError_t dft3_t(const Plan& p, int inst, int sign, long long count, void* data, long long stride) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[inst];
  const int n1 = in.grid[0], n2 = in.grid[1], n3 = in.grid[2];
  const C* tw = reinterpret_cast<const C*>(p.ws + p.tw_off);
  const size_t lds_plane = static_cast<size_t>(n2) * n3 * sizeof(C);
  const size_t lds_tile = static_cast<size_t>(n1) * n3 * sizeof(C);
  C* d = static_cast<C*>(data);
  for (long long b0 = 0; b0 < count; b0 += 65535) {
    const int nb = static_cast<int>(std::min<long long>(65535, count - b0));
    C* db = d + static_cast<size_t>(b0) * stride;
    p.prof.begin(FOCK_K_DFT, p.stream);
    if (reg_dft_supported(p.prec, in.grid)) {
      const hipError_t e = launch_reg_dft3(p, inst, sign, nb, db, stride);
      p.prof.end(FOCK_K_DFT, p.stream);
      if (e != hipSuccess) return e;
      continue;
    }
    if (sign < 0) {
      hipLaunchKernelGGL((k_dft_planes<T, -1>), dim3(n1, nb), dim3(kBlock), lds_plane, p.stream, n2, n3, db, stride,
                         0LL, tw);
      hipLaunchKernelGGL((k_dft_pencils<T, -1>), dim3(n2, nb), dim3(kBlock), lds_tile, p.stream, n1, n2, n3, db,
                         stride, tw);
    } else {
      hipLaunchKernelGGL((k_dft_planes<T, +1>), dim3(n1, nb), dim3(kBlock), lds_plane, p.stream, n2, n3, db, stride,
                         0LL, tw);
      hipLaunchKernelGGL((k_dft_pencils<T, +1>), dim3(n2, nb), dim3(kBlock), lds_tile, p.stream, n1, n2, n3, db,
                         stride, tw);
    }
    p.prof.end(FOCK_K_DFT, p.stream);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t pw_to_grid_t(const Plan& p, int inst, const void* coef, const int* gidx, const int* npw, int npw_max,
                        void* psi) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[inst];
  const int nbt = in.nk * in.nbands;
  hipError_t e = launch_zero_all_bands(p, inst, psi);
  if (e != hipSuccess) return e;
  const T scale = static_cast<T>(1.0 / std::sqrt(in.omega));
  const int gx = (npw_max + kBlock - 1) / kBlock;
  for (int b0 = 0; b0 < nbt; b0 += 65535) {
    const int nb = std::min(65535, nbt - b0);
    p.prof.begin(FOCK_K_PW, p.stream);
    hipLaunchKernelGGL((k_pw_scatter<T>), dim3(gx, nb), dim3(kBlock), 0, p.stream, static_cast<const C*>(coef), gidx,
                       npw, npw_max, in.nbands, b0, static_cast<long long>(in.band_stride),
                       static_cast<long long>(in.npts), static_cast<C*>(psi), scale);
    p.prof.end(FOCK_K_PW, p.stream);
  }
  return dft3_t<T>(p, inst, +1, nbt, psi, static_cast<long long>(in.band_stride));
}

template <typename T>
hipError_t grid_to_pw_t(const Plan& p, int inst, void* f, const int* gidx, const int* npw, int npw_max, void* coef) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[inst];
  const int nbt = in.nk * in.nbands;
  hipError_t e = dft3_t<T>(p, inst, -1, nbt, f, static_cast<long long>(in.band_stride));
  if (e != hipSuccess) return e;
  const T scale = static_cast<T>(std::sqrt(in.omega) / static_cast<double>(in.npts));
  const int gx = (npw_max + kBlock - 1) / kBlock;
  for (int b0 = 0; b0 < nbt; b0 += 65535) {
    const int nb = std::min(65535, nbt - b0);
    p.prof.begin(FOCK_K_PW, p.stream);
    hipLaunchKernelGGL((k_pw_gather<T>), dim3(gx, nb), dim3(kBlock), 0, p.stream, static_cast<const C*>(f), gidx, npw,
                       npw_max, in.nbands, b0, static_cast<long long>(in.band_stride),
                       static_cast<long long>(in.npts), static_cast<C*>(coef), scale);
    p.prof.end(FOCK_K_PW, p.stream);
  }
  return hipGetLastError();
}

template <typename T>
void dft_lds_attr(int lim) {
  const void* fs[] = {reinterpret_cast<const void*>(&k_dft_planes<T, -1>),
                      reinterpret_cast<const void*>(&k_dft_planes<T, +1>),
                      reinterpret_cast<const void*>(&k_dft_pencils<T, -1>),
                      reinterpret_cast<const void*>(&k_dft_pencils<T, +1>)};
  for (const void* f : fs)
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess) (void)hipGetLastError();
}

}  // namespace

void prepare_dft_kernels(fock_precision prec, int lim) {
  prepare_reg_dft_kernels(prec, lim);
  if (prec != FOCK_C64)
    dft_lds_attr<double>(lim);
  else
    dft_lds_attr<float>(lim);
}

hipError_t launch_dft3(const Plan& p, int inst, int sign, long long count, void* data, long long stride) {
  return p.io64() ? dft3_t<double>(p, inst, sign, count, data, stride)
                             : dft3_t<float>(p, inst, sign, count, data, stride);
}

hipError_t launch_pw_to_grid(const Plan& p, int inst, const void* coef, const int* gidx, const int* npw, int npw_max,
                             void* psi) {
  return p.io64() ? pw_to_grid_t<double>(p, inst, coef, gidx, npw, npw_max, psi)
                             : pw_to_grid_t<float>(p, inst, coef, gidx, npw, npw_max, psi);
}

hipError_t launch_grid_to_pw(const Plan& p, int inst, void* f, const int* gidx, const int* npw, int npw_max,
                             void* coef) {
  return p.io64() ? grid_to_pw_t<double>(p, inst, f, gidx, npw, npw_max, coef)
                             : grid_to_pw_t<float>(p, inst, f, gidx, npw, npw_max, coef);
}

}  // namespace fock
