// Natural logarithm of a positive finite double for the per-cell reductions
// (H-functional sum F ln F, entropy production sum Q ln F).  Host and device,
// so the CPU tests check the code the kernels run.
//
// x = m 2^e with m in [1/sqrt 2, sqrt 2) (frexp, then one doubling when
// m < 1/sqrt 2); s = (m - 1) / (m + 1), |s| <= (sqrt 2 - 1)/(sqrt 2 + 1) <
// 0.1716; ln m = 2 atanh s = 2 s sum_{k >= 0} s^{2k} / (2k + 1), summed to
// k = 10 (the remainder is below s^22 / 23 < 7e-19 of the sum).  Then
// ln x = e ln 2 + ln m with ln 2 split into the double nearest to it and the
// remainder, so e ln 2 carries no rounding beyond the final additions.
// Every product that feeds an addition is an explicit fma, so host and device
// evaluate the same operations (the division is correctly rounded on both).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define EFM_LOG_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define EFM_LOG_HD inline
#endif

namespace efm {

#if !defined(__HIPCC__)
using std::fma;
using std::frexp;
#endif

EFM_LOG_HD double log_pos(double x) {
  int e;
  double m = frexp(x, &e);                  // [0.5, 1)
  if (m < 0.7071067811865476) {             // the double nearest 1/sqrt 2
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);   // m - 1 is exact (m in [1/2, 2])
  const double s2 = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, s2, 1.0 / 19.0);
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  const double t = 2.0 * s;
  const double lnm = fma(t * s2, p, t);     // 2 s (1 + s^2 p)
  const double de = (double)e;
  constexpr double LN2 = 0x1.62e42fefa39efp-1, LN2_LO = 0x1.abc9e3b39803fp-56;
  return fma(de, LN2, fma(de, LN2_LO, lnm));
}

}  // namespace efm
