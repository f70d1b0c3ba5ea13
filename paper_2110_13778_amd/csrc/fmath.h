// FP64 device helpers for the kernel evaluations (internal).
//
// inv_sqrt: single-precision reciprocal square root as the seed, then one
//   Newton step y <- y (3 - x y^2) / 2 in FP64 (the step squares the seed's
//   relative error: below 2e-14, always from below).
// exp_expm1: e^x and e^x - 1 together by table-driven Cody-Waite reduction
//   x = (32 m + j) ln2/32 + f, |f| <= ln2/64 (ln2/32 split into a 32-bit head,
//   so k ln2_hi/32 is exact, and a tail), the Taylor series of (e^f - 1)/f to
//   degree 6 (truncation below 1e-18), s = 2^m 2^(j/32), and
//   e^x - 1 = s q + (s - 1) with q = e^f - 1, which is q itself when the
//   reduced index is 0 (no cancellation for small |x|); relative error below
//   5e-15 for both on x <= 0.
#pragma once
#include <hip/hip_runtime.h>

namespace fagbi {

// 2^(j/32), j = 0..31, correctly rounded
__device__ constexpr double kExp2Frac[32] = {
    1.0, 1.0218971486541166, 1.0442737824274138, 1.0671404006768237, 1.0905077326652577, 1.1143867425958924,
    1.1387886347566916, 1.1637248587775775, 1.189207115002721, 1.215247359980469, 1.241857812073484,
    1.2690509571917332, 1.2968395546510096, 1.3252366431597413, 1.3542555469368927, 1.383909881963832,
    1.4142135623730951, 1.4451808069770467, 1.4768261459394993, 1.5091644275934228, 1.5422108254079407,
    1.5759808451078865, 1.6104903319492543, 1.6457554781539649, 1.681792830507429, 1.7186192981224779,
    1.7562521603732995, 1.7947090750031072, 1.8340080864093424, 1.8741676341103, 1.9152065613971474,
    1.9571441241754002};

__device__ inline double inv_sqrt(double x) {
  const double y = (double)__frsqrt_rn((float)x);
  return y * fma(-0.5 * x * y, y, 1.5);
}

__device__ inline void exp_expm1(double x, double& e, double& em1) {
  constexpr double INV = 46.166241308446828;              // 32 / ln2
  constexpr double LN2_32_HI = 0.021660834550857544;      // 0x1.62e42p-6 (32 trailing zero bits)
  constexpr double LN2_32_LO = 1.4841640746973977e-08;    // ln2/32 - LN2_32_HI
  const double k = rint(fmax(x, -745.0) * INV);
  double f = fma(-k, LN2_32_HI, x);
  f = fma(-k, LN2_32_LO, f);
  // sum_{n=0}^{6} f^n / (n+1)!
  double p = 1.9841269841269841270e-04;                   // 1/7!
  p = fma(p, f, 1.3888888888888888889e-03);               // 1/6!
  p = fma(p, f, 8.3333333333333333333e-03);               // 1/5!
  p = fma(p, f, 4.1666666666666666667e-02);               // 1/4!
  p = fma(p, f, 1.6666666666666666667e-01);               // 1/3!
  p = fma(p, f, 0.5);                                     // 1/2!
  p = fma(p, f, 1.0);                                     // 1/1!
  const double q = f * p;
  const int ki = (int)k;
  const double s = ldexp(kExp2Frac[ki & 31], ki >> 5);
  em1 = fma(s, q, s - 1.0);
  e = fma(s, q, s);
}

}  // namespace fagbi
