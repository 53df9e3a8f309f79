// Band overlap M[k][i][j] = dV sum_e conj(u_{k,i}[e]) (V_x u)_{k,j}[e] on the
// matrix cores (the dense contraction on the path; paper, "CPU Performance
// Analysis": the BLAS share of FOCK).
//
// A complex N_b x N_b product over K = N grid points, split over K chunks.
// One workgroup of four waves owns a 32 x 32 block of M (four 16 x 16
// tiles, one per wave) over one chunk: the 32 bands of u and the 32 bands of
// V_x u of the block are staged through LDS a slab of kSlab grid points at a
// time (16-byte loads, two slabs in flight), so each operand element read
// from memory serves two tiles.  Each wave multiplies its tile with 16x16x4
// MFMA instructions, four real products per complex step
// (Re += ar br + ai bi, Im += ar bi - ai br), and writes its chunk partial in
// FP64; a second kernel sums the chunk partials in a fixed order and applies
// dV.
//
// Operand layout of the 16x16x4 instruction (both precisions): lane l gives
// A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16]; it receives
// D[i][j = l % 16] for v = 0..3 with i = 4 (l / 16) + v (FP32) or
// i = l / 16 + 4 v (FP64), as measured on gfx950.
#include <type_traits>

#include "fock_internal.hpp"
#include "fft_lds.hpp"

namespace fock {

namespace {

constexpr int kOvWaves = 4;
constexpr int kOvChunk = 4096;  // grid points per workgroup (split-K chunk)
constexpr int kOvSub = 1024;    // points accumulated in the MFMA precision before an FP64 fold
constexpr int kBlk = 32;        // bands per block side (2 x 2 tiles of 16)

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

// One slab: the 32 bands of each operand times kSlab grid points, stored
// [band][point] (rows padded by one element); each thread moves kVec
// consecutive complex elements (16 bytes) of each operand kLoads times.
template <typename T>
struct OvStage {
  using C = typename cx<T>::t;
  using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;  // 16 bytes
  static constexpr int kSlab = sizeof(T) == 4 ? 32 : 16;  // two slabs of both operands within 64 KiB of LDS
  static constexpr int kVec = 16 / static_cast<int>(sizeof(C));
  static constexpr int kPerBand = kSlab / kVec;
  static constexpr int kLoads = kBlk * kPerBand / (64 * kOvWaves);
  static_assert(kLoads >= 1 && kBlk * kPerBand % (64 * kOvWaves) == 0, "slab does not divide over the threads");
  static_assert(kOvChunk % kOvSub == 0 && kOvSub % kSlab == 0, "chunk of whole sub-chunks of whole slabs");
};

// grid: (block_i * nbj + block_j, chunk, k); 256 threads
template <typename T>
__global__ __launch_bounds__(64 * kOvWaves) void k_overlap_mfma(const typename cx<T>::t* __restrict__ psi,
                                                                 const typename cx<T>::t* __restrict__ vx, int nbands,
                                                                 long long bs, long long npts, int nt,
                                                                 double* __restrict__ part) {
  using C = typename cx<T>::t;
  using M = Mfma<T>;
  using S = OvStage<T>;
  using V = typename S::V;
  using acc_t = typename M::acc_t;
  constexpr int kSlab = S::kSlab;
  __shared__ C sa[2][kBlk][kSlab + 1];
  __shared__ C sb[2][kBlk][kSlab + 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int nbj = (nt + 1) / 2;
  const int bi = blockIdx.x / nbj, bj = blockIdx.x - bi * nbj;
  const int chunk = blockIdx.y, k = blockIdx.z;
  const long long c0 = static_cast<long long>(chunk) * kOvChunk;
  const long long c1 = c0 + kOvChunk < npts ? c0 + kOvChunk : npts;
  const size_t kb = static_cast<size_t>(k) * nbands;
  // this wave's tile (ti, tj) of the block, and whether it lies inside M
  const int ti = 2 * bi + (wave >> 1), tj = 2 * bj + (wave & 1);
  const bool live = ti < nt && tj < nt;
  // thread t moves, per operand and load q, band row r and points p0 .. p0 + kVec - 1 of the slab
  V ra[S::kLoads], rb[S::kLoads];
  auto load = [&](long long e0) {
#pragma unroll
    for (int q = 0; q < S::kLoads; ++q) {
      const int id = t + q * 64 * kOvWaves;
      const int r = id / S::kPerBand, p0 = (id - r * S::kPerBand) * S::kVec;
      const long long e = e0 + p0;
      const int ia = bi * kBlk + r, jb = bj * kBlk + r;
      const C* pa = psi + (kb + (ia < nbands ? ia : 0)) * bs + e;
      const C* pb = vx + (kb + (jb < nbands ? jb : 0)) * bs + e;
      V va = {}, vb = {};
      const bool whole = e + S::kVec <= c1;
      if (whole && ia < nbands && (reinterpret_cast<uintptr_t>(pa) & 15) == 0) {
        va = *reinterpret_cast<const V*>(pa);
      } else if (ia < nbands) {  // grid end or an odd band stride: element by element
        C* x = reinterpret_cast<C*>(&va);
#pragma unroll
        for (int u = 0; u < S::kVec; ++u) x[u] = e + u < c1 ? pa[u] : C{T(0), T(0)};
      }
      if (whole && jb < nbands && (reinterpret_cast<uintptr_t>(pb) & 15) == 0) {
        vb = *reinterpret_cast<const V*>(pb);
      } else if (jb < nbands) {
        C* x = reinterpret_cast<C*>(&vb);
#pragma unroll
        for (int u = 0; u < S::kVec; ++u) x[u] = e + u < c1 ? pb[u] : C{T(0), T(0)};
      }
      ra[q] = va;
      rb[q] = vb;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < S::kLoads; ++q) {
      const int id = t + q * 64 * kOvWaves;
      const int r = id / S::kPerBand, p0 = (id - r * S::kPerBand) * S::kVec;
      const C* ea = reinterpret_cast<const C*>(&ra[q]);
      const C* eb = reinterpret_cast<const C*>(&rb[q]);
#pragma unroll
      for (int u = 0; u < S::kVec; ++u) {
        sa[buf][r][p0 + u] = ea[u];
        sb[buf][r][p0 + u] = eb[u];
      }
    }
  };
  acc_t re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
  double dre[4] = {0.0, 0.0, 0.0, 0.0}, dim[4] = {0.0, 0.0, 0.0, 0.0};  // FP64 sums of the sub-chunks
  const int ia = (wave >> 1) * 16 + (lane & 15), jb = (wave & 1) * 16 + (lane & 15), kk = lane >> 4;
  int buf = 0;
  load(c0);
  store(0);
  __syncthreads();
  for (long long e0 = c0; e0 < c1; e0 += kSlab) {
    const bool more = e0 + kSlab < c1;
    if (more) load(e0 + kSlab);  // the next slab's loads are in flight while this one is multiplied
    if (live) {
#pragma unroll
      for (int s4 = 0; s4 < kSlab; s4 += 4) {
        const C av = sa[buf][ia][s4 + kk];
        const C bv = sb[buf][jb][s4 + kk];
        re = M::step(av.x, bv.x, re);
        re = M::step(av.y, bv.y, re);
        im = M::step(av.x, bv.y, im);
        im = M::step(-av.y, bv.x, im);
      }
      if (!more || (e0 + kSlab - c0) % kOvSub == 0) {  // end of a sub-chunk: fold into FP64
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          dre[v] += static_cast<double>(re[v]);
          dim[v] += static_cast<double>(im[v]);
        }
        re = acc_t{0, 0, 0, 0};
        im = acc_t{0, 0, 0, 0};
      }
    }
    if (more) store(buf ^ 1);  // that buffer was last read before the previous barrier
    __syncthreads();
    buf ^= 1;
  }
  if (!live) return;
  double* dst = part + ((static_cast<size_t>(chunk) * gridDim.z + k) * (static_cast<size_t>(nt) * nt) +
                        static_cast<size_t>(ti) * nt + tj) * 512;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = M::row(lane, v), col = lane & 15;
    dst[(row * 16 + col) * 2] = dre[v];
    dst[(row * 16 + col) * 2 + 1] = dim[v];
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
  const int nbj = (nt + 1) / 2;
  const int nchunks = static_cast<int>((in.npts + kOvChunk - 1) / kOvChunk);
  double* part = reinterpret_cast<double*>(p.ws + p.ovl_off);
  p.prof.begin(FOCK_K_OVERLAP, p.stream);
  hipLaunchKernelGGL((k_overlap_mfma<T>), dim3(nbj * nbj, nchunks, in.nk), dim3(64 * kOvWaves), 0, p.stream,
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
