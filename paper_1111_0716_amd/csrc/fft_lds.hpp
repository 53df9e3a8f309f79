// LDS-staged mixed-radix FFT building blocks for gfx950.
//
// A workgroup transforms many lines (rows or columns of a 2-D tile held in
// LDS) of one compile-time length L at once.  Each radix pass is a Stockham
// step: every thread loads R elements of its butterflies into registers,
// applies the inter-pass twiddles, runs an in-register radix-R DFT, and after
// a barrier writes the R results to their autosorted positions in the same
// LDS tile (in place; the barrier separates all reads from all writes).
//
// Lengths: every {2,3,5}-smooth L in [2, 72].  Radices 8, 4, 2, 3, 5 are
// taken greedily from the remaining factor, so L = 72 runs as 8*3*3.
// Twiddles come from a per-L table W_L^t = exp(-2 pi i t / L) built in FP64
// on the host and rounded once to the working precision.
#pragma once

#include <hip/hip_runtime.h>

namespace fock {

constexpr int kNMax = 72;   // largest supported grid axis
constexpr int kBlock = 256; // threads per workgroup of the plane/pencil kernels

// ---------------------------------------------------------------------------
// complex helpers on HIP vector types (x = real, y = imaginary)
// ---------------------------------------------------------------------------
template <typename T> struct cx;
template <> struct cx<float> { using t = float2; };
template <> struct cx<double> { using t = double2; };

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cmulconj(C a, C b) {  // conj(a) * b
  return C{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { return C{a.x * s, a.y * s}; }
// multiply by s*i with s = +1 or -1
template <int S, typename C> __device__ __forceinline__ C cmul_si(C a) {
  return S > 0 ? C{-a.y, a.x} : C{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// in-register DFTs, X[k] = sum_n x[n] exp(S * 2 pi i n k / R), S = -1 forward
// ---------------------------------------------------------------------------
template <int R, int S, typename C> struct Dft;

template <int S, typename C> struct Dft<2, S, C> {
  static __device__ __forceinline__ void run(C* x) {
    C a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int S, typename C> struct Dft<3, S, C> {
  static __device__ __forceinline__ void run(C* x) {
    using T = decltype(x[0].x);
    const T h = T(0.8660254037844386467637231707529362);  // sin(2 pi / 3)
    C t1 = cadd(x[1], x[2]);
    C t2 = csub(x[1], x[2]);
    C m = C{x[0].x - T(0.5) * t1.x, x[0].y - T(0.5) * t1.y};
    C r = cmul_si<S>(cscale(t2, h));
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <int S, typename C> struct Dft<4, S, C> {
  static __device__ __forceinline__ void run(C* x) {
    C a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    C c = cadd(x[1], x[3]), d = cmul_si<S>(csub(x[1], x[3]));
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, d);
    x[3] = csub(b, d);
  }
};

template <int S, typename C> struct Dft<5, S, C> {
  static __device__ __forceinline__ void run(C* x) {
    using T = decltype(x[0].x);
    const T c1 = T(0.3090169943749474241022934171828191);   // cos(2 pi / 5)
    const T c2 = T(-0.8090169943749474241022934171828191);  // cos(4 pi / 5)
    const T s1 = T(0.9510565162951535721164393333793821);   // sin(2 pi / 5)
    const T s2 = T(0.5877852522924731291687059546390728);   // sin(4 pi / 5)
    C a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    C a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    C x0 = x[0];
    C m1 = C{x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
    C m2 = C{x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
    C n1 = cmul_si<S>(C{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    C n2 = cmul_si<S>(C{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    x[0] = cadd(x0, cadd(a1, a2));
    x[1] = cadd(m1, n1);
    x[4] = csub(m1, n1);
    x[2] = cadd(m2, n2);
    x[3] = csub(m2, n2);
  }
};

template <int S, typename C> struct Dft<8, S, C> {
  // two length-4 DFTs over even and odd inputs, combined with w8^k
  static __device__ __forceinline__ void run(C* x) {
    using T = decltype(x[0].x);
    const T r2 = T(0.7071067811865475244008443621048490);  // 1/sqrt(2)
    C e[4] = {x[0], x[2], x[4], x[6]};
    C o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4, S, C>::run(e);
    Dft<4, S, C>::run(o);
    // w8^1 = (1 + S i)/sqrt2, w8^2 = S i, w8^3 = (-1 + S i)/sqrt2
    C o1 = cscale(cadd(o[1], cmul_si<S>(o[1])), r2);
    C o2 = cmul_si<S>(o[2]);
    C o3 = cscale(csub(cmul_si<S>(o[3]), o[3]), r2);
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], o1);
    x[5] = csub(e[1], o1);
    x[2] = cadd(e[2], o2);
    x[6] = csub(e[2], o2);
    x[3] = cadd(e[3], o3);
    x[7] = csub(e[3], o3);
  }
};

// ---------------------------------------------------------------------------
// compile-time factorisation
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pick_radix(int rem) {
  return rem % 8 == 0 ? 8 : rem % 4 == 0 ? 4 : rem % 2 == 0 ? 2 : rem % 3 == 0 ? 3 : 5;
}

__host__ __device__ constexpr bool smooth235(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}

// Twiddle tables of every supported length, concatenated in increasing L.
__host__ __device__ constexpr int twiddle_offset(int L) {
  int off = 0;
  for (int n = 2; n < L; ++n)
    if (smooth235(n)) off += n;
  return off;
}
constexpr int kTwiddleTotal = twiddle_offset(kNMax + 1);

// fast quotient for idx < 2^20 and 1 <= n <= kNMax: the fractional part of
// (idx + 0.5)/n stays >= 0.5/n away from an integer, far above FP32 error.
__device__ __forceinline__ int fdiv(int idx, float rcp) {
  return static_cast<int>((static_cast<float>(idx) + 0.5f) * rcp);
}

// ---------------------------------------------------------------------------
// one Stockham pass of radix R over `nlines` lines of length L in LDS.
// ROWS: elements of a line are contiguous (estride 1) and consecutive lanes
// take consecutive butterflies of one line; otherwise lines are contiguous
// (lstride 1) and consecutive lanes take consecutive lines.
// ---------------------------------------------------------------------------
template <typename C, int L, int R, int NS, int S, bool ROWS>
__device__ __forceinline__ void stockham_pass(C* s, int nlines, float rcp_lines, int lstride, int estride,
                                              const C* __restrict__ tw) {
  constexpr int M = L / R;
  constexpr int MAXB = (kNMax * M + kBlock - 1) / kBlock;
  const int nbf = nlines * M;
  C v[MAXB][R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int idx = static_cast<int>(threadIdx.x) + b * kBlock;
    if (idx < nbf) {
      int line, j;
      if (ROWS) {
        line = idx / M;
        j = idx - line * M;
      } else {
        j = fdiv(idx, rcp_lines);
        line = idx - j * nlines;
      }
      const C* src = s + line * lstride;
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C x = src[(j + r * M) * estride];
        if (NS > 1 && r > 0) {
          C w = tw[r * k * (L / (NS * R))];
          if (S > 0) w.y = -w.y;
          x = cmul(x, w);
        }
        v[b][r] = x;
      }
      Dft<R, S, C>::run(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int idx = static_cast<int>(threadIdx.x) + b * kBlock;
    if (idx < nbf) {
      int line, j;
      if (ROWS) {
        line = idx / M;
        j = idx - line * M;
      } else {
        j = fdiv(idx, rcp_lines);
        line = idx - j * nlines;
      }
      C* dst = s + line * lstride;
      const int k = j % NS;
      const int d = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[(d + r * NS) * estride] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename C, int L, int NS, int S, bool ROWS>
__device__ __forceinline__ void stockham_passes(C* s, int nlines, float rcp_lines, int lstride, int estride,
                                                const C* __restrict__ tw) {
  if constexpr (NS < L) {
    constexpr int R = pick_radix(L / NS);
    stockham_pass<C, L, R, NS, S, ROWS>(s, nlines, rcp_lines, lstride, estride, tw);
    stockham_passes<C, L, NS * R, S, ROWS>(s, nlines, rcp_lines, lstride, estride, tw);
  }
}

// Transform `nlines` lines of runtime length L (a supported size) in LDS.
// `twall` is the concatenated twiddle table.  Must be called by all threads.
template <typename C, int S, bool ROWS>
__device__ __forceinline__ void fft_lines(C* s, int L, int nlines, int lstride, int estride,
                                       const C* __restrict__ twall) {
  const float rcp = 1.0f / static_cast<float>(nlines);
#define FOCK_FFT_CASE(LL)                                                                  \
  case LL:                                                                                 \
    stockham_passes<C, LL, 1, S, ROWS>(s, nlines, rcp, lstride, estride, twall + twiddle_offset(LL)); \
    break;
  switch (L) {
    FOCK_FFT_CASE(2) FOCK_FFT_CASE(3) FOCK_FFT_CASE(4) FOCK_FFT_CASE(5) FOCK_FFT_CASE(6)
    FOCK_FFT_CASE(8) FOCK_FFT_CASE(9) FOCK_FFT_CASE(10) FOCK_FFT_CASE(12) FOCK_FFT_CASE(15)
    FOCK_FFT_CASE(16) FOCK_FFT_CASE(18) FOCK_FFT_CASE(20) FOCK_FFT_CASE(24) FOCK_FFT_CASE(25)
    FOCK_FFT_CASE(27) FOCK_FFT_CASE(30) FOCK_FFT_CASE(32) FOCK_FFT_CASE(36) FOCK_FFT_CASE(40)
    FOCK_FFT_CASE(45) FOCK_FFT_CASE(48) FOCK_FFT_CASE(50) FOCK_FFT_CASE(54) FOCK_FFT_CASE(60)
    FOCK_FFT_CASE(64) FOCK_FFT_CASE(72)
    default:
      break;  // unreachable: the planner admits supported lengths only
  }
#undef FOCK_FFT_CASE
}

// Out-of-line copy for kernels that keep large register state live across
// several transforms (the accumulate pass): keeps the allocator from spilling.
template <typename C, int S, bool ROWS>
__device__ __noinline__ void fft_lines_call(C* s, int L, int nlines, int lstride, int estride,
                                            const C* __restrict__ twall) {
  fft_lines<C, S, ROWS>(s, L, nlines, lstride, estride, twall);
}

}  // namespace fock
