// Compile-time twiddle factors W_L^t = exp(-2 pi i t / L).
//
// sin and cos of 2 pi t / L are evaluated in FP64 at compile time: the angle
// is reduced exactly with integer arithmetic to an octant and a residual
// phi in [0, pi/4], where the Taylor series of sin and cos converge to
// rounding within 12 terms; the octant symmetries of sin/cos rebuild the
// value.  Kernels that index these tables with unrolled constant indices get
// the values as instruction literals (no registers, no loads).
#pragma once

namespace fock {

namespace ce {

constexpr double kQuarterPi = 0.78539816339744830961566084581987572;

constexpr double sin_poly(double x) {  // |x| <= pi/4
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 12; ++n) {
    term *= -x2 / static_cast<double>((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}

constexpr double cos_poly(double x) {  // |x| <= pi/4
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 12; ++n) {
    term *= -x2 / static_cast<double>((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}

// cos and sin of 2 pi t / L for integers t, L > 0
struct SinCos {
  double c, s;
};

constexpr SinCos sincos_frac(long t, long L) {
  t %= L;
  if (t < 0) t += L;
  const long u = 8 * t;          // angle in units of (pi/4) / L
  const long oct = u / L;        // octant 0..7
  const long r = u - oct * L;    // residual phi = (pi/4) r / L in [0, pi/4)
  const double phi = kQuarterPi * static_cast<double>(r) / static_cast<double>(L);
  const double psi = kQuarterPi * static_cast<double>(L - r) / static_cast<double>(L);  // pi/4 - phi
  const double sp = sin_poly(phi), cp = cos_poly(phi), sq = sin_poly(psi), cq = cos_poly(psi);
  switch (oct) {
    case 0: return {cp, sp};
    case 1: return {sq, cq};
    case 2: return {-sp, cp};
    case 3: return {-cq, sq};
    case 4: return {-cp, -sp};
    case 5: return {-sq, -cq};
    case 6: return {sp, -cp};
    default: return {cq, -sq};
  }
}

}  // namespace ce

// exp(-2 pi i t / L) for t = 0..L-1
template <int L>
struct TwTable {
  double re[L], im[L];
  constexpr TwTable() : re(), im() {
    for (int t = 0; t < L; ++t) {
      const ce::SinCos v = ce::sincos_frac(t, L);
      re[t] = v.c;
      im[t] = -v.s;
    }
  }
};

template <int L>
inline constexpr TwTable<L> kTwiddle{};

}  // namespace fock
