// Band overlap M[k][i][j] = dV sum_e conj(u_{k,i}[e]) (V_x u)_{k,j}[e] on the
// matrix cores (the dense contraction on the path; paper, "CPU Performance
// Analysis": the BLAS share of FOCK).
//
// A complex N_b x N_b product over K = N grid points, split over K: each
// wave multiplies a 16 x 16 output tile over its share of a K chunk with
// 16x16x4 MFMA instructions (four real products per complex step:
// Re += ar br + ai bi, Im += ar bi - ai br), the four waves of a workgroup
// are summed in LDS in a fixed order, and the chunk partials (FP64) are summed
// over chunks in a fixed order by a second kernel, which also applies dV.
//
// Operand layout of the 16x16x4 instruction (both precisions): lane l gives
// A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16]; it receives
// D[i][j = l % 16] for v = 0..3 with i = 4 (l / 16) + v (FP32) or
// i = l / 16 + 4 v (FP64), as measured on gfx950.  Lane (i, kk) reads four
// consecutive grid points e0 + 4 kk .. e0 + 4 kk + 3 of band i (32 or 64
// contiguous bytes), one MFMA step per point.
#include "fock_internal.hpp"
#include "fft_lds.hpp"

namespace fock {

namespace {

constexpr int kOvWaves = 4;
constexpr int kOvChunk = 2048;  // grid points per workgroup (split-K chunk)

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = f32x4;
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  using acc_t = f64x4;
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// grid: (tile_i * ntj + tile_j, chunk, k); 256 threads
template <typename T>
__global__ __launch_bounds__(64 * kOvWaves) void k_overlap_mfma(const typename cx<T>::t* __restrict__ psi,
                                                                 const typename cx<T>::t* __restrict__ vx, int nbands,
                                                                 long long bs, long long npts, int ntj,
                                                                 double* __restrict__ part) {
  using C = typename cx<T>::t;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  __shared__ double red[kOvWaves][2][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ti = blockIdx.x / ntj, tj = blockIdx.x - ti * ntj;
  const int chunk = blockIdx.y, k = blockIdx.z;
  const int i = ti * 16 + (lane & 15), j = tj * 16 + (lane & 15), kk = lane >> 4;
  const bool ai = i < nbands, bj = j < nbands;
  const C* a = psi + (static_cast<size_t>(k) * nbands + (ai ? i : 0)) * bs;
  const C* b = vx + (static_cast<size_t>(k) * nbands + (bj ? j : 0)) * bs;
  acc_t re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  const long long c0 = static_cast<long long>(chunk) * kOvChunk;
  const long long c1 = c0 + kOvChunk < npts ? c0 + kOvChunk : npts;
  constexpr int WSPAN = kOvChunk / kOvWaves;  // points per wave
  const long long w0 = c0 + static_cast<long long>(wave) * WSPAN;
  const long long w1 = w0 + WSPAN < c1 ? w0 + WSPAN : c1;
  for (long long e0 = w0; e0 < w1; e0 += 16) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const long long e = e0 + 4 * kk + s;
      C av = C{T(0), T(0)}, bv = C{T(0), T(0)};
      if (e < w1) {
        if (ai) av = a[e];
        if (bj) bv = b[e];
      }
      re = M::step(av.x, bv.x, re);
      re = M::step(av.y, bv.y, re);
      im = M::step(av.x, bv.y, im);
      im = M::step(-av.y, bv.x, im);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wave][0][v][lane] = static_cast<double>(re[v]);
    red[wave][1][v][lane] = static_cast<double>(im[v]);
  }
  __syncthreads();
  if (wave == 0) {
    const int ntiles = gridDim.x;
    double* dst = part + ((static_cast<size_t>(chunk) * gridDim.z + k) * ntiles + blockIdx.x) * 512;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double sr = 0.0, si = 0.0;
      for (int w = 0; w < kOvWaves; ++w) {
        sr += red[w][0][v][lane];
        si += red[w][1][v][lane];
      }
      const int row = M::row(lane, v), col = lane & 15;
      dst[(row * 16 + col) * 2] = sr;
      dst[(row * 16 + col) * 2 + 1] = si;
    }
  }
}

// vmat[k][i][j] = dV sum_chunks part[chunk][k][tile][row][col]
template <typename T>
__global__ __launch_bounds__(256) void k_overlap_reduce(const double* __restrict__ part, int nchunks, int nk,
                                                        int nbands, int ntj, double dv,
                                                        typename cx<T>::t* __restrict__ vmat) {
  using C = typename cx<T>::t;
  const long long total = static_cast<long long>(nk) * nbands * nbands;
  for (long long id = blockIdx.x * 256LL + threadIdx.x; id < total; id += static_cast<long long>(gridDim.x) * 256) {
    const int k = static_cast<int>(id / (static_cast<long long>(nbands) * nbands));
    const int ij = static_cast<int>(id - static_cast<long long>(k) * nbands * nbands);
    const int i = ij / nbands, j = ij - i * nbands;
    const int tile = (i / 16) * ntj + (j / 16), row = i % 16, col = j % 16;
    const int ntiles = ((nbands + 15) / 16) * ntj;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nchunks; ++c) {
      const double* src = part + ((static_cast<size_t>(c) * nk + k) * ntiles + tile) * 512 + (row * 16 + col) * 2;
      sr += src[0];
      si += src[1];
    }
    vmat[id] = C{static_cast<T>(sr * dv), static_cast<T>(si * dv)};
  }
}

template <typename T>
hipError_t overlap_t(const Plan& p, int inst, const void* psi, const void* vx, void* vmat) {
  using C = typename cx<T>::t;
  const Instance& in = p.inst[inst];
  const int nt = (in.nbands + 15) / 16;
  const int nchunks = static_cast<int>((in.npts + kOvChunk - 1) / kOvChunk);
  double* part = reinterpret_cast<double*>(p.ws + p.ovl_off);
  p.prof.begin(FOCK_K_OVERLAP, p.stream);
  hipLaunchKernelGGL((k_overlap_mfma<T>), dim3(nt * nt, nchunks, in.nk), dim3(64 * kOvWaves), 0, p.stream,
                     static_cast<const C*>(psi), static_cast<const C*>(vx), in.nbands,
                     static_cast<long long>(in.band_stride), static_cast<long long>(in.npts), nt, part);
  const long long total = static_cast<long long>(in.nk) * in.nbands * in.nbands;
  const int gx = static_cast<int>(std::min<long long>(1024, (total + 255) / 256));
  hipLaunchKernelGGL((k_overlap_reduce<T>), dim3(gx), dim3(256), 0, p.stream, static_cast<const double*>(part),
                     nchunks, in.nk, in.nbands, nt, in.omega / static_cast<double>(in.npts), static_cast<C*>(vmat));
  p.prof.end(FOCK_K_OVERLAP, p.stream);
  return hipGetLastError();
}

}  // namespace

size_t overlap_scratch_bytes(const Instance& in) {
  const size_t nt = (in.nbands + 15) / 16;
  const size_t nchunks = (in.npts + kOvChunk - 1) / kOvChunk;
  return nchunks * in.nk * nt * nt * 512 * sizeof(double);
}

hipError_t launch_overlap(const Plan& p, int inst, const void* psi, const void* vx, void* vmat) {
  return p.io64() ? overlap_t<double>(p, inst, psi, vx, vmat) : overlap_t<float>(p, inst, psi, vx, vmat);
}

}  // namespace fock
