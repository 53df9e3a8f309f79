// Register FFT of a line shared by a lane pair (see split_fft_fwd).
#pragma once

#include "reg_fft.hpp"

namespace fock {

// ---------------------------------------------------------------------------
// a line of even length L shared by two adjacent lanes (lane ^ 1)
// ---------------------------------------------------------------------------
// Input of the forward transform: the lane with h = lane & 1 holds x[2m + h]
// in y[m], m < L/2.  Output: it holds X[h L/2 + k] in y[k], k < L/2.  The
// inverse takes that split of the spectrum back to the even/odd split of the
// line.  Each lane runs an L/2-point register FFT; the radix-2 step across
// the pair exchanges the halves with one DPP move per 32-bit word.

// value of the partner lane (lane ^ 1): DPP quad_perm [1, 0, 3, 2]
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// e^{S 2 pi i k / L} as a compile-time constant
template <typename C, int L, int S>
__device__ __forceinline__ C twiddle_ce(int k) {
  using T = decltype(C{}.x);
  return C{static_cast<T>(kTwiddle<L>.re[k]), static_cast<T>(S > 0 ? -kTwiddle<L>.im[k] : kTwiddle<L>.im[k])};
}

// forward (S = -1): decimation in time over the lane pair
template <typename C, int L>
__device__ __forceinline__ void split_fft_fwd(C* y, int h) {
  constexpr int LH = L / 2;
  static_assert(L % 2 == 0, "split lines need an even length");
  reg_fft<C, LH, -1>(y);  // E (h = 0) or O (h = 1)
#pragma unroll
  for (int k = 0; k < LH; ++k) {
    const C o = C{pair_swap(y[k].x), pair_swap(y[k].y)};
    const C e = h ? o : y[k];
    const C t = cmul(h ? y[k] : o, twiddle_ce<C, L, -1>(k));
    y[k] = h ? csub(e, t) : cadd(e, t);
  }
}

// inverse (S = +1): decimation in frequency over the lane pair
template <typename C, int L>
__device__ __forceinline__ void split_fft_inv(C* y, int h) {
  constexpr int LH = L / 2;
  static_assert(L % 2 == 0, "split lines need an even length");
#pragma unroll
  for (int k = 0; k < LH; ++k) {
    const C o = C{pair_swap(y[k].x), pair_swap(y[k].y)};
    const C a = h ? o : y[k];  // X[k]
    const C b = h ? y[k] : o;  // X[k + L/2]
    y[k] = h ? cmul(csub(a, b), twiddle_ce<C, L, +1>(k)) : cadd(a, b);
  }
  reg_fft<C, LH, +1>(y);  // x[2m] (h = 0) or x[2m + 1] (h = 1)
}

}  // namespace fock
