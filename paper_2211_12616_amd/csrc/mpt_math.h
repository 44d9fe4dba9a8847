// mpt_math.h -- FP64 elementary functions on the restricted ranges that the
// particle step needs: argument reductions written out, then minimax
// polynomials for the smooth remainders of the series (coefficients from
// gen_minimax.py, a Remez exchange in 50-digit arithmetic, rounded to
// double).  No tables, no large-argument reduction, no special-value
// handling beyond what the ranges require.  Each stays within a few ulp of
// the exact value on its range.  Host and device compile the same code, so
// their accuracy can be checked on the host.
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
// values): one Goldschmidt step from the reciprocal square-root seed,
// g -> sqrt(x) and h -> 1/(2 sqrt(x)) (relative errors near the square of
// the seed's, below 2^-46), then one correction of g by its residual
// x - g^2 (an FMA, exact), which squares the error again; within 1 ulp
// (correctly rounded on the tested ranges).
__host__ __device__ __forceinline__ double sqrt_pos(double x) {
  const double y = rsq_seed(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

// ln x for a positive normal x.  x = m 2^e with m in [1/sqrt 2, sqrt 2);
// ln m = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716 (m - 1 is exact);
// atanh s = s (1 + z q(z)), z = s^2 <= 0.0295, with q the degree-6 minimax
// polynomial of (atanh(s)/s - 1)/z (1/3 + z/5 + ...), whose error adds
// below 2e-18 relative.
__host__ __device__ __forceinline__ double ln_pos(double x) {
  int e;
  double m = frexp(x, &e);                            // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m = m + m;
    e = e - 1;
  }
  const double s = div_1to4(m - 1.0, m + 1.0);
  const double z = s * s;
  double q = 0x1.2f0008a2b99ecp-4;
  q = fma(q, z, 0x1.39a2503857f5bp-4);
  q = fma(q, z, 0x1.74663874e7961p-4);
  q = fma(q, z, 0x1.c71c522d05652p-4);                 // ~1/9
  q = fma(q, z, 0x1.24924941be083p-3);                 // ~1/7
  q = fma(q, z, 0x1.999999998021bp-3);                 // ~1/5
  q = fma(q, z, 0x1.5555555555591p-2);                 // ~1/3
  const double t = s + s;
  const double lnm = fma(t * z, q, t);
  const double fe = (double)e;
  return fma(fe, kLn2Hi, fma(fe, kLn2Lo, lnm));
}

// sin x for |x| <= pi/2 + 0.02: sin x = x + x z h(z), z = x^2, with h the
// degree-7 minimax polynomial of (sin(x)/x - 1)/z (-1/6 + z/120 - ...),
// whose error adds below 4e-18 relative.
__host__ __device__ __forceinline__ double sin_half(double x) {
  const double z = x * x;
  double q = 0x1.88019a32e3114p-49;
  q = fma(q, z, -0x1.ae41c365249b1p-41);
  q = fma(q, z, 0x1.6123c688a4d1cp-33);
  q = fma(q, z, -0x1.ae6454bb7bb20p-26);
  q = fma(q, z, 0x1.71de3a526b757p-19);
  q = fma(q, z, -0x1.a01a01a0145aap-13);               // ~-1/7!
  q = fma(q, z, 0x1.11111111110bfp-7);                 // ~1/5!
  q = fma(q, z, -0x1.5555555555555p-3);                // ~-1/3!
  return fma(x * z, q, x);
}

// cos of a latitude in degrees, |lat| <= 90 plus a small overshoot, as the
// sine of the co-latitude: keeps its relative accuracy near the poles, and
// is negative past them.
__host__ __device__ __forceinline__ double cos_lat_deg(double lat) {
  return sin_half((90.0 - fabs(lat)) * (kPiD / 180.0));
}

// sin(pi t) and cos(pi t) for t in [0, 2].  n = rint(2 t) quarter periods,
// r = t - n/2 in [-1/4, 1/4] (exact), x = pi r, z = x^2: sin x = x + x z h(z)
// and cos x = 1 - z/2 + z^2 g(z) with degree-5 minimax polynomials h and g
// (errors adding below 4e-18 and 1e-18), then the rotation by n quarter
// turns.
__host__ __device__ __forceinline__ void sincospi_02(double t, double *s, double *c) {
  const double n = rint(t + t);
  const double r = fma(-0.5, n, t);
  const double x = r * kPiD;
  const double z = x * x;
  double ps = 0x1.5d93a7ca6a89dp-33;
  ps = fma(ps, z, -0x1.ae5e68bcab28fp-26);
  ps = fma(ps, z, 0x1.71de357b5cdfap-19);
  ps = fma(ps, z, -0x1.a01a019c16899p-13);             // ~-1/7!
  ps = fma(ps, z, 0x1.111111110f8abp-7);               // ~1/5!
  ps = fma(ps, z, -0x1.5555555555549p-3);              // ~-1/3!
  ps = fma(x * z, ps, x);
  double pc = -0x1.8fae9e9c70fa5p-37;
  pc = fma(pc, z, 0x1.1ee9ebedb59f5p-29);
  pc = fma(pc, z, -0x1.27e4f809f803ap-22);
  pc = fma(pc, z, 0x1.a01a019cb1c94p-16);               // ~1/8!
  pc = fma(pc, z, -0x1.6c16c16c1517ep-10);              // ~-1/6!
  pc = fma(pc, z, 0x1.555555555554cp-5);                // ~1/4!
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

// cos(pi t) for t in (0, 2) a multiple of 2^-24 (twice a uniform): with
// h = 1/2 - t (exact), n = rint(h) in {-1, 0} and y = h - n in [-1/2, 1/2]
// (exact), cos(pi t) = sin(pi h) = (-1)^n sin(pi y); one polynomial
// (sin_half) where the quarter-period form evaluates two.
__host__ __device__ __forceinline__ double cospi_02(double t) {
  const double h = 0.5 - t;
  const double n = rint(h);
  const double s = sin_half((h - n) * kPiD);
  return n != 0.0 ? -s : s;
}

}  // namespace m64
}  // namespace mpt
