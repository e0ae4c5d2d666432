// fastmath.hpp -- FP64 elementary functions for the push, accurate to a few
// ulp on the argument ranges that occur there and much shorter than the
// general-purpose library versions (which handle every IEEE corner case).
#pragma once
#include <hip/hip_runtime.h>

namespace grpic {

// 1/x for finite, normal x: the hardware estimate y (relative error below
// 2^-24 on this device) refined by one third-order step,
// 1/x = y / (1 - e) = y (1 + e + e^2 + ...) with e = 1 - x y; the omitted
// terms are below 2^-72 relative.
__device__ __forceinline__ double frcp(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, fma(e, e, e), y);
}

// sqrt(x) for finite x > 0 away from the denormal range: the hardware
// estimate of 1/sqrt(x) (relative error below 2^-24) refined by one step of
// Goldschmidt's coupled iteration for sqrt(x) and 1/(2 sqrt(x)) (error ~2^-48)
// and a final residual correction (Newton step on s^2 = x), which rounds
// correctly in practice.
__device__ __forceinline__ double fsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  r = fma(-s, s, x);
  return fma(h, r, s);
}

// 1/sqrt(x) for finite x > 0 away from the denormal range: the hardware
// estimate y (relative error below 2^-24) refined by one third-order step,
// 1/sqrt(x) = y (1 - e)^(-1/2) = y (1 + e/2 + 3 e^2/8 + ...) with
// e = 1 - x y^2; the omitted terms are below 2^-70 relative.
__device__ __forceinline__ double frsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x, y * y, 1.0);
  return fma(y, e * fma(e, 0.375, 0.5), y);
}

// sin and cos of x for |x| < 100 (polar angles here lie near [0, pi]):
// Cody-Waite reduction x = k pi/2 + t with pi/2 split in two parts, t in
// [-pi/4, pi/4]; Taylor polynomials of degree 17 (sin) and 16 (cos), whose
// truncation error is below 1e-18 on that interval; quadrant from k mod 4.
__device__ __forceinline__ void fsincos(double x, double* sn, double* cs) {
  const double two_over_pi = 0.63661977236758134308;
  const double pio2_hi = 1.5707963267948966;     // pi/2 rounded to double
  const double pio2_lo = 6.123233995736766e-17;  // pi/2 - pio2_hi
  double k = rint(x * two_over_pi);
  double t = fma(-k, pio2_hi, x);
  t = fma(-k, pio2_lo, t);
  double t2 = t * t;
  double ps = -1.0 / 1307674368000.0 + t2 * (1.0 / 355687428096000.0);
  ps = 1.0 / 6227020800.0 + t2 * ps;
  ps = -1.0 / 39916800.0 + t2 * ps;
  ps = 1.0 / 362880.0 + t2 * ps;
  ps = -1.0 / 5040.0 + t2 * ps;
  ps = 1.0 / 120.0 + t2 * ps;
  ps = -1.0 / 6.0 + t2 * ps;
  ps = fma(t * t2, ps, t);
  double pc = -1.0 / 87178291200.0 + t2 * (1.0 / 20922789888000.0);
  pc = 1.0 / 479001600.0 + t2 * pc;
  pc = -1.0 / 3628800.0 + t2 * pc;
  pc = 1.0 / 40320.0 + t2 * pc;
  pc = -1.0 / 720.0 + t2 * pc;
  pc = 1.0 / 24.0 + t2 * pc;
  pc = -0.5 + t2 * pc;
  pc = fma(t2, pc, 1.0);
  int q = ((int)k) & 3;
  double s = (q & 1) ? pc : ps;
  double c = (q & 1) ? ps : pc;
  *sn = (q & 2) ? -s : s;
  *cs = ((q + 1) & 2) ? -c : c;
}

// sin and cos of t from those of a nearby angle t0 (s0, c0): with d = t - t0
// (exact for nearby arguments), Taylor series of sin d and cos d - 1 to d^7
// and d^8 (the next terms are below 3e-22 relative for |d| <= 0.01, far
// under one ulp) and the angle-addition formulas arranged as corrections to
// s0, c0.  Farther angles (a stage or midpoint moves theta by much less
// than 0.01 at the time steps used here) use fsincos.
__device__ __forceinline__ void sincos_near(double t, double t0, double s0,
                                            double c0, double* sn, double* cs) {
  const double d = t - t0;
  if (fabs(d) > 0.01) {
    fsincos(t, sn, cs);
    return;
  }
  const double d2 = d * d;
  double ps = -1.0 / 5040.0;
  ps = 1.0 / 120.0 + d2 * ps;
  ps = -1.0 / 6.0 + d2 * ps;
  const double sd = fma(d * d2, ps, d);  // sin d
  double pc = 1.0 / 40320.0;
  pc = -1.0 / 720.0 + d2 * pc;
  pc = 1.0 / 24.0 + d2 * pc;
  pc = -0.5 + d2 * pc;
  const double cm1 = d2 * pc;            // cos d - 1
  *sn = fma(s0, cm1, fma(c0, sd, s0));
  *cs = fma(c0, cm1, fma(-s0, sd, c0));
}

}  // namespace grpic
