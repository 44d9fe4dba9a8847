// mpt_math.h -- FP64 elementary functions on the restricted ranges that the
// particle step needs, written from their Taylor series: no tables, no
// large-argument reduction, no special-value handling beyond what the
// ranges require.  Each stays within a few ulp of the exact value on its
// range.  Host and device compile the same code, so their accuracy can be
// checked on the host.
#pragma once
#include <hip/hip_runtime.h>

namespace mpt {
namespace m64 {

constexpr double kPiD = 3.14159265358979323846;
// ln 2 = kLn2Hi + kLn2Lo; the head has 32 significant bits, so e * kLn2Hi is
// exact for |e| < 2^21.
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;

// Seeds of 1/x and 1/sqrt(x): the hardware approximations on the device
// (about 26 good bits); on the host the FP32 operations (24 bits) stand in
// for them, so the refinements below are exercised from seeds of the same
// quality.
__host__ __device__ __forceinline__ double rcp_seed(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(x);
#else
  return (double)(1.0f / (float)x);
#endif
}
__host__ __device__ __forceinline__ double rsq_seed(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsq(x);
#else
  return (double)(1.0f / sqrtf((float)x));
#endif
}

// a / b for b in [1, 4] (no special values): one Newton step on the
// reciprocal seed, the quotient, one correction by its residual; within
// 1 ulp (the library division also handles every exponent and special
// value, at twice the instructions).
__host__ __device__ __forceinline__ double div_1to4(double a, double b) {
  double r = rcp_seed(b);
  r = fma(r, fma(-b, r, 1.0), r);
  const double q = a * r;
  return fma(fma(-q, b, a), r, q);
}

// sqrt(x) for a positive normal x in [2^-900, 2^900] (no scaling, no special
// values): Goldschmidt iteration from the reciprocal square-root seed,
// g -> sqrt(x) and h -> 1/(2 sqrt(x)), then two corrections of g by its
// residual x - g^2; within 1 ulp.
__host__ __device__ __forceinline__ double sqrt_pos(double x) {
  const double y = rsq_seed(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// ln x for a positive normal x.  x = m 2^e with m in [1/sqrt 2, sqrt 2);
// ln m = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716 (m - 1 is exact);
// atanh s = s (1 + z/3 + z^2/5 + ... + z^10/21), z = s^2 <= 0.0295, whose
// remainder is below 1e-18 relative.
__host__ __device__ __forceinline__ double ln_pos(double x) {
  int e;
  double m = frexp(x, &e);                            // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m = m + m;
    e = e - 1;
  }
  const double s = div_1to4(m - 1.0, m + 1.0);
  const double z = s * s;
  double q = 1.0 / 21.0;
  q = fma(q, z, 1.0 / 19.0);
  q = fma(q, z, 1.0 / 17.0);
  q = fma(q, z, 1.0 / 15.0);
  q = fma(q, z, 1.0 / 13.0);
  q = fma(q, z, 1.0 / 11.0);
  q = fma(q, z, 1.0 / 9.0);
  q = fma(q, z, 1.0 / 7.0);
  q = fma(q, z, 1.0 / 5.0);
  q = fma(q, z, 1.0 / 3.0);
  const double t = s + s;
  const double lnm = fma(t * z, q, t);
  const double fe = (double)e;
  return fma(fe, kLn2Hi, fma(fe, kLn2Lo, lnm));
}

// sin x for |x| <= pi/2 (and a little beyond): odd Taylor series to x^21;
// the first omitted term is below 1.2e-18 at pi/2.
__host__ __device__ __forceinline__ double sin_half(double x) {
  const double z = x * x;
  double q = 1.0 / 51090942171709440000.0;            // 1/21!
  q = fma(q, z, -1.0 / 121645100408832000.0);         // 1/19!
  q = fma(q, z, 1.0 / 355687428096000.0);             // 1/17!
  q = fma(q, z, -1.0 / 1307674368000.0);              // 1/15!
  q = fma(q, z, 1.0 / 6227020800.0);                  // 1/13!
  q = fma(q, z, -1.0 / 39916800.0);                   // 1/11!
  q = fma(q, z, 1.0 / 362880.0);                      // 1/9!
  q = fma(q, z, -1.0 / 5040.0);                       // 1/7!
  q = fma(q, z, 1.0 / 120.0);                         // 1/5!
  q = fma(q, z, -1.0 / 6.0);                          // 1/3!
  return fma(x * z, q, x);
}

// cos of a latitude in degrees, |lat| <= 90 plus a small overshoot, as the
// sine of the co-latitude: keeps its relative accuracy near the poles, and
// is negative past them.
__host__ __device__ __forceinline__ double cos_lat_deg(double lat) {
  return sin_half((90.0 - fabs(lat)) * (kPiD / 180.0));
}

// sin(pi t) and cos(pi t) for t in [0, 2].  n = rint(2 t) quarter periods,
// r = t - n/2 in [-1/4, 1/4] (exact), x = pi r: sine to x^17 and cosine to
// x^16 by Taylor (first omitted terms below 1e-19 and 3e-18), then the
// rotation by n quarter turns.
__host__ __device__ __forceinline__ void sincospi_02(double t, double *s, double *c) {
  const double n = rint(t + t);
  const double r = fma(-0.5, n, t);
  const double x = r * kPiD;
  const double z = x * x;
  double ps = 1.0 / 355687428096000.0;                // 1/17!
  ps = fma(ps, z, -1.0 / 1307674368000.0);
  ps = fma(ps, z, 1.0 / 6227020800.0);
  ps = fma(ps, z, -1.0 / 39916800.0);
  ps = fma(ps, z, 1.0 / 362880.0);
  ps = fma(ps, z, -1.0 / 5040.0);
  ps = fma(ps, z, 1.0 / 120.0);
  ps = fma(ps, z, -1.0 / 6.0);
  ps = fma(x * z, ps, x);
  double pc = 1.0 / 20922789888000.0;                 // 1/16!
  pc = fma(pc, z, -1.0 / 87178291200.0);              // 1/14!
  pc = fma(pc, z, 1.0 / 479001600.0);                 // 1/12!
  pc = fma(pc, z, -1.0 / 3628800.0);                  // 1/10!
  pc = fma(pc, z, 1.0 / 40320.0);                     // 1/8!
  pc = fma(pc, z, -1.0 / 720.0);                      // 1/6!
  pc = fma(pc, z, 1.0 / 24.0);                        // 1/4!
  pc = fma(pc, z, -0.5);
  pc = fma(pc, z, 1.0);
  const int q = (int)n & 3;
  double ss = (q & 1) ? pc : ps;
  double cc = (q & 1) ? ps : pc;
  if (q == 1 || q == 2) cc = -cc;
  if (q >= 2) ss = -ss;
  *s = ss;
  *c = cc;
}

}  // namespace m64
}  // namespace mpt
