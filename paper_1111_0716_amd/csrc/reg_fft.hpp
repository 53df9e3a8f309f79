// In-register Stockham FFT of a compile-time length L on x[L] (one line per
// thread).  Radix-8/4/5/3/2 stages; the twiddles are compile-time constants
// (twiddle_ce.hpp), so an unrolled stage multiplies by instruction literals.
#pragma once

#include "fft_lds.hpp"
#include "twiddle_ce.hpp"

namespace fock {

// ---------------------------------------------------------------------------
// in-register Stockham FFT of a compile-time length L on x[L]
// ---------------------------------------------------------------------------
template <typename C, int L, int NS, int S>
__device__ __forceinline__ void reg_fft_stages(C* x) {
  if constexpr (NS < L) {
    constexpr int R = pick_radix(L / NS);
    constexpr int M = L / R;
    C y[L];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      C v[R];
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C a = x[j + r * M];
        if (NS > 1 && r > 0 && k > 0) {
          using T = decltype(a.x);
          const int e = r * k * (L / (NS * R));
          const C w = C{static_cast<T>(kTwiddle<L>.re[e]), static_cast<T>(S > 0 ? -kTwiddle<L>.im[e] : kTwiddle<L>.im[e])};
          a = cmul(a, w);
        }
        v[r] = a;
      }
      Dft<R, S, C>::run(v);
      const int d = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) y[d + r * NS] = v[r];
    }
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = y[i];
    __builtin_amdgcn_sched_barrier(0);  // keep stages apart: bounds the live values to ~2 lines
    reg_fft_stages<C, L, NS * R, S>(x);
  }
}

template <typename C, int L, int S>
__device__ __forceinline__ void reg_fft(C* x) {
  reg_fft_stages<C, L, 1, S>(x);
}

}  // namespace fock
