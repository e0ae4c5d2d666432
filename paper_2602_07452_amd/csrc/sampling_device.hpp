// sampling_device.hpp -- seeded particle draws shared by the initial data
// and the pair injection: counter-based SplitMix64 (Steele, Lea & Flood
// 2014; draw k of stream s uses counter s * 256 + k), positions uniform in
// proper volume over a shell [r0, r1] x [t0, t1] by rejection against
// r^2 sin(theta) proposals (at most 64 tries), Maxwell-Juettner speeds by
// inverting a tabulated cumulative distribution, and FIDO-frame momenta
// mapped to covariant u_i with the Cholesky factor of gamma_ij (order r,
// theta, phi).
#pragma once
#include "kerr_device.hpp"

namespace grpic {

__device__ __forceinline__ double splitmix_u01(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ double draw(uint64_t seed, long stream, int k) {
  return splitmix_u01(seed, (uint64_t)stream * 256ull + (uint64_t)k);
}

// z[0..2] = (r, theta, phi) uniform in proper volume over the shell
__device__ __forceinline__ void sample_position(double a, uint64_t seed, long stream,
                                                double r0, double r1, double t0, double t1,
                                                double* z) {
  double C = (1.0 + a * a / (r0 * r0)) * sqrt(1.0 + 2.0 / r0);
  double c0 = cos(t0), c1 = cos(t1);
  double r = r0, th = t0;
  double r03 = r0 * r0 * r0, r13 = r1 * r1 * r1;
  for (int t = 0; t < 64; ++t) {
    double u1 = draw(seed, stream, 3 * t), u2 = draw(seed, stream, 3 * t + 1),
           u3 = draw(seed, stream, 3 * t + 2);
    r = cbrt(r03 + u1 * (r13 - r03));
    th = acos(c0 - u2 * (c0 - c1));
    double c = cos(th);
    double rho2 = r * r + a * a * c * c;
    double ratio = rho2 / (r * r) * sqrt(1.0 + 2.0 * r / rho2);
    if (u3 * C < ratio) break;
  }
  z[0] = r;
  z[1] = th;
  z[2] = 2.0 * kPi * draw(seed, stream, 192);
}

// speed from the cumulative table mj[0..K] (spacing h) at the quantile x
__device__ __forceinline__ double mj_speed(const double* mj, int K, double h, double x) {
  int lo = 0, hi = K;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (mj[mid] <= x) lo = mid;
    else hi = mid;
  }
  double dc = mj[lo + 1] - mj[lo];
  double f = dc > 0.0 ? (x - mj[lo]) / dc : 0.0;
  return (lo + f) * h;
}

// covariant u_i of FIDO momentum magnitude mag in the direction drawn from
// stream draws 201 (cos of the polar angle to e_r) and 202 (azimuth)
__device__ __forceinline__ void fido_momentum(double a, uint64_t seed, long stream, double mag,
                                              double r, double th, double* u) {
  double mu = 2.0 * draw(seed, stream, 201) - 1.0;
  double az = 2.0 * kPi * draw(seed, stream, 202);
  double sn = sqrt(1.0 - mu * mu);
  double fr = mag * mu, ft = mag * sn * cos(az), fp = mag * sn * sin(az);
  Met m;
  metric(a, r, th, m);
  double Lrr = sqrt(m.grr), Ltt = sqrt(m.gtt), Lpr = m.grp / Lrr;
  double Lpp = sqrt(m.gpp - Lpr * Lpr);
  u[0] = Lrr * fr;
  u[1] = Ltt * ft;
  u[2] = Lpr * fr + Lpp * fp;
}

}  // namespace grpic
