// Float64 reciprocal, quotient and natural logarithm for the objective terms
// (d_beta of the KL and IS divergences), written for throughput: a float32
// reciprocal seed refined by Newton steps in float64 instead of the float64
// division sequence, and the logarithm from the atanh series on a reduced
// argument.  Both are accurate to a few units in the last place for the
// positive, finite, normal arguments they receive (data and Lambda are float32
// values, so every quotient of two of them is a normal float64).
//
// log method (textbook argument reduction + series):
//   x = 2^e m,  m in [sqrt(1/2), sqrt(2)),  s = (m - 1) / (m + 1),
//   log m = 2 atanh s = 2 s (1 + s^2/3 + s^4/5 + ...),   |s| <= 0.1716,
// and e log 2 is added as e * ln2_hi + e * ln2_lo with ln2_hi holding 42
// significant bits (e * ln2_hi is exact for |e| < 2^11).
//
// The functions compile for the host as well (the seed is then an exact
// float32 division), which is how they are checked against the C library.
#pragma once

#if defined(__HIPCC__)
#define NMF_HD __host__ __device__
#else
#define NMF_HD
#endif

#include <math.h>

namespace nmf {

NMF_HD inline float rcp_seed(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

NMF_HD inline float rsq_seed(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}

// 1 / sqrt(x) for x a positive normal float64 within the float32 range:
// float32 seed, two Newton steps y <- y (3 - x y^2) / 2.
NMF_HD inline double rsqrt64(double x) {
  double y = (double)rsq_seed((float)x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// sqrt(x) = x / sqrt(x) with one residual correction; `r` is rsqrt64(x).
NMF_HD inline double sqrt64(double x, double r) {
  const double s = x * r;
  return fma(fma(-s, s, x), 0.5 * r, s);
}

// 1 / x for x a positive normal float64 within the float32 range.
NMF_HD inline double rcp64(double x) {
  double y = (double)rcp_seed((float)x);   // about 2^-23 relative
  y = fma(y, fma(-x, y, 1.0), y);          // about 2^-46
  y = fma(y, fma(-x, y, 1.0), y);          // float64 rounding
  return y;
}

// a / b: quotient from the reciprocal plus one residual correction.
NMF_HD inline double div64(double a, double b) {
  const double r = rcp64(b);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

// Natural logarithm of a positive finite normal float64.
NMF_HD inline double log64(double x) {
  int e;
  double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;  // exact (Sterbenz)
  const double s = div64(f, m + 1.0);
  const double z = s * s;
  // 1/3 + z/5 + z^2/7 + ... + z^10/23 (the next term is below 2^-55 relative)
  double p = 1.0 / 23.0;
  p = fma(p, z, 1.0 / 21.0);
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double t = 2.0 * s;
  const double lm = fma(t * z, p, t);  // log m
  const double de = (double)e;
  constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;   // ln 2 to 42 bits
  constexpr double kLn2Lo = 0x1.ef35793c76730p-45;  // ln 2 - kLn2Hi
  return fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
}

}  // namespace nmf
