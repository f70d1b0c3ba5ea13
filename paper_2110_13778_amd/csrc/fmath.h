// FP64 device helpers for the kernel evaluations (internal).
//
// inv_sqrt: single-precision reciprocal square root as the seed, then two
//   Newton steps y <- y (3 - x y^2) / 2 in FP64 (each step squares the
//   relative error: ~1e-7 -> ~1e-14 -> rounding level).
// exp_expm1: e^x and e^x - 1 together by Cody-Waite argument reduction
//   x = k ln2 + f, |f| <= ln2/2 (ln2 split into a 32-bit head, so k ln2_hi is
//   exact, and a tail), the Taylor series of (e^f - 1)/f to degree 12
//   (truncation below 2e-17), and e^x - 1 = 2^k q + (2^k - 1) with q = e^f - 1,
//   which has no cancellation when k = 0.
#pragma once
#include <hip/hip_runtime.h>

namespace fagbi {

__device__ inline double inv_sqrt(double x) {
  double y = (double)__frsqrt_rn((float)x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

__device__ inline void exp_expm1(double x, double& e, double& em1) {
  constexpr double LOG2E = 1.4426950408889634074;
  constexpr double LN2_HI = 6.93147180369123816490e-01;   // 0x3fe62e42fee00000
  constexpr double LN2_LO = 1.90821492927058770002e-10;   // 0x3dea39ef35793c76
  const double k = rint(x * LOG2E);
  double f = fma(-k, LN2_HI, x);
  f = fma(-k, LN2_LO, f);
  // sum_{n=0}^{12} f^n / (n+1)!
  double p = 1.6059043836821614599e-10;                  // 1/13!
  p = fma(p, f, 2.0876756987868098979e-09);               // 1/12!
  p = fma(p, f, 2.5052108385441718775e-08);               // 1/11!
  p = fma(p, f, 2.7557319223985890653e-07);               // 1/10!
  p = fma(p, f, 2.7557319223985890653e-06);               // 1/9!
  p = fma(p, f, 2.4801587301587301587e-05);               // 1/8!
  p = fma(p, f, 1.9841269841269841270e-04);               // 1/7!
  p = fma(p, f, 1.3888888888888888889e-03);               // 1/6!
  p = fma(p, f, 8.3333333333333333333e-03);               // 1/5!
  p = fma(p, f, 4.1666666666666666667e-02);               // 1/4!
  p = fma(p, f, 1.6666666666666666667e-01);               // 1/3!
  p = fma(p, f, 0.5);                                     // 1/2!
  p = fma(p, f, 1.0);                                     // 1/1!
  const double q = f * p;
  const int ki = (int)fmax(k, -1100.0);
  const double s = ldexp(1.0, ki);
  em1 = fma(s, q, s - 1.0);
  e = fma(s, q, s);
}

}  // namespace fagbi
