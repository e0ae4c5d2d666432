/*
 * om_init.c -- reference oracle (TEST INFRASTRUCTURE ONLY): seeded particle
 * initial data for the synthetic workloads.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea & Flood 2014, "Fast splittable pseudorandom number
 * generators") applied to the state seed + (counter + 1) * golden gamma,
 * top 53 bits -> [0, 1).  Counter of draw k of stream s: s * 256 + k.
 */
#include <math.h>
#include <stdlib.h>

#include "om_internal.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

double om_uniform(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53;
}

static double U(uint64_t seed, long stream, int k) {
  return om_uniform(seed, (uint64_t)stream * 256ULL + (uint64_t)k);
}

/* Positions uniform in proper volume sqrt(gamma) dr dtheta dphi over the
 * shell [r0,r1] x [t0,t1] (reading of "uniform in volume"): proposals with
 * density r^2 sin(theta) are accepted with probability
 * (rho^2 / r^2) sqrt(xi) / C, C >= that ratio on the shell.  At most 64
 * proposals; the last one is kept if all are rejected.                    */
static void sample_position(double a, uint64_t seed, long stream, double r0,
                            double r1, double t0, double t1, double *r,
                            double *th, double *ph) {
  double C = (1.0 + a * a / (r0 * r0)) * sqrt(1.0 + 2.0 / r0);
  double c0 = cos(t0), c1 = cos(t1);
  for (int t = 0; t < 64; ++t) {
    double u1 = U(seed, stream, 3 * t), u2 = U(seed, stream, 3 * t + 1),
           u3 = U(seed, stream, 3 * t + 2);
    *r = cbrt(r0 * r0 * r0 + u1 * (r1 * r1 * r1 - r0 * r0 * r0));
    *th = acos(c0 - u2 * (c0 - c1));
    double c = cos(*th);
    double rho2 = (*r) * (*r) + a * a * c * c;
    double xi = 1.0 + 2.0 * (*r) / rho2;
    double ratio = rho2 / ((*r) * (*r)) * sqrt(xi);
    if (u3 * C < ratio) break;
  }
  *ph = 2.0 * M_PI * U(seed, stream, 192);
}

/* Maxwell-Juettner speed distribution f(u) ~ u^2 exp(-(gamma-1)/Theta),
 * inverted through its cumulative table (trapezoidal rule on 4096 equal
 * intervals of [0, u_max], gamma_max - 1 = 50 Theta) and linear
 * interpolation inside an interval.                                       */
#define MJ_K 4096
typedef struct {
  double h;
  double C[MJ_K + 1];
} mj_table;

static void mj_build(double theta, mj_table *T) {
  double gm = 1.0 + 50.0 * theta;
  double umax = sqrt(gm * gm - 1.0);
  T->h = umax / MJ_K;
  double fprev = 0.0;
  T->C[0] = 0.0;
  for (int k = 1; k <= MJ_K; ++k) {
    double u = k * T->h;
    double f = u * u * exp(-(sqrt(1.0 + u * u) - 1.0) / theta);
    T->C[k] = T->C[k - 1] + 0.5 * (fprev + f) * T->h;
    fprev = f;
  }
  double tot = T->C[MJ_K];
  for (int k = 0; k <= MJ_K; ++k) T->C[k] /= tot;
}

static double mj_sample(const mj_table *T, double x) {
  int lo = 0, hi = MJ_K;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (T->C[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  double dc = T->C[lo + 1] - T->C[lo];
  double f = dc > 0.0 ? (x - T->C[lo]) / dc : 0.0;
  return (lo + f) * T->h;
}

/* FIDO orthonormal components (r, theta, phi order) -> covariant u_i via
 * the Cholesky factor of gamma_ij taken in the order r, theta, phi.       */
static void fido_to_covariant(double a, double r, double th, const double *f,
                              double *u) {
  double m[13];
  om_metric(a, r, th, m);
  double Lrr = sqrt(m[2]);
  double Ltt = sqrt(m[3]);
  double Lpr = m[5] / Lrr;
  double Lpp = sqrt(m[4] - Lpr * Lpr);
  u[0] = Lrr * f[0];
  u[1] = Ltt * f[1];
  u[2] = Lpr * f[0] + Lpp * f[2];
}

void om_init_particles(int kind, double a, uint64_t seed, long n, double r0,
                       double r1, double t0, double t1, double p0, double w,
                       om_particles *p) {
  mj_table *T = NULL;
  if (kind == 2) {
    T = (mj_table *)malloc(sizeof(mj_table));
    mj_build(p0, T);
  }
#pragma omp parallel for schedule(static)
  for (long id = 0; id < n; ++id) {
    double z[6];
    double qm;
    if (kind == 0) {
      /* Schwarzschild (a = 0) test orbits: circular orbit constants at r
       * (textbook closed forms), inclined by starting at theta with
       * u_theta = 0 and u_phi = L sin(theta); Kerr-Schild u_r = 2E/(r-2).
       * Odd ids get an extra u_r offset uniform in [-p0, p0].            */
      double r = r0 + (r1 - r0) * U(seed, id, 0);
      double th = t0 + (t1 - t0) * U(seed, id, 1);
      double E = (1.0 - 2.0 / r) / sqrt(1.0 - 3.0 / r);
      double L = sqrt(r) / sqrt(1.0 - 3.0 / r);
      z[0] = r, z[1] = th, z[2] = 0.0;
      z[3] = 2.0 * E / (r - 2.0);
      if (id & 1) z[3] += -p0 + 2.0 * p0 * U(seed, id, 2);
      z[4] = 0.0;
      z[5] = L * sin(th);
      qm = 0.0;
    } else {
      long pid = (kind == 2) ? id / 2 : id;
      sample_position(a, seed, pid, r0, r1, t0, t1, &z[0], &z[1], &z[2]);
      double mag = (kind == 2) ? mj_sample(T, U(seed, id, 200))
                               : p0 * U(seed, id, 200);
      double mu = 2.0 * U(seed, id, 201) - 1.0;
      double az = 2.0 * M_PI * U(seed, id, 202);
      double sn = sqrt(1.0 - mu * mu);
      double f[3] = {mag * mu, mag * sn * cos(az), mag * sn * sin(az)};
      fido_to_covariant(a, z[0], z[1], f, &z[3]);
      qm = (id & 1) ? -1.0 : 1.0;
    }
    p->r[id] = z[0];
    p->th[id] = z[1];
    p->ph[id] = z[2];
    p->ur[id] = z[3];
    p->uth[id] = z[4];
    p->uph[id] = z[5];
    p->qm[id] = qm;
    p->w[id] = w;
    p->H0[id] = om_energy(a, z);
    p->herr[id] = 0.0;
    p->flags[id] = OM_ALIVE;
    p->iters[id] = 0;
    p->crit[id] = NAN;
  }
  free(T);
}

/* ------------------------------------------------------------------------
 * Pair injection (Sec. 3.3).  Every node cell (p, q) whose centre
 * (r_{p+1/2}, theta_{q+1/2}) lies in [r0, r1] receives one e+/e- pair at one
 * position when its plasma density n = sum of the weights of the charged
 * particles in the cell / V_cell is below mult * n_GJ.  Readings:
 *   n_GJ = Omega_H |Omega . B| / (4 pi) per unit Omega_H, with the rotation
 *          axis direction taken as the gradient of z = r cos(theta):
 *          Omega . B = Omega_H (cos(theta) B^r - r sin(theta) B^theta),
 *          Omega_H = a / (2 r_+), B at the cell centre as the mean of the
 *          densitized values on the two faces over sqrt(g) at the centre;
 *   V_cell = 2 pi sqrt(g)(centre) (r_{p+1} - r_p) dtheta;
 *   each particle of the pair weighs density * n_GJ * V_cell / 2, so the
 *          pair adds density * n_GJ;
 *   cells are visited in index order q n_r + p while there is room for a
 *          pair; the pair's position is uniform in proper volume over the
 *          cell (stream c = q n_r + p), the momenta Maxwell-Juettner at
 *          temperature theta in the FIDO frame (streams 2c and 2c + 1), all
 *          from the seed seed + event * golden gamma.
 * B: plain B^r (at (r_i, theta_{j+1/2})) and B^theta (at (r_{i+1/2},
 * theta_j)).  Writes 8 values per new particle (r, theta, phi, u_r, u_theta,
 * u_phi, q/m, w) and returns the number written.
 * ------------------------------------------------------------------------ */
long om_inject(const om_grid *g, const om_inject_params *I, uint64_t event,
               const double *Br, const double *Bt, long n, const double *r,
               const double *th, const double *qm, const double *w,
               const int *flags, long room, double *out) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  double a = g->a, rp = 1.0 + sqrt(1.0 - a * a), OmH = a / (2.0 * rp);
  double *wsum = (double *)calloc((size_t)nr * nth, sizeof(double));
  for (long k = 0; k < n; ++k) {
    if (!(flags[k] & OM_ALIVE) || qm[k] == 0.0) continue;
    int p = om_locate(g->rn, nr + 1, r[k]), q = om_locate(g->tn, nth + 1, th[k]);
    wsum[(long)q * nr + p] += w[k];
  }
  mj_table *T = (mj_table *)malloc(sizeof(mj_table));
  mj_build(I->theta, T);
  uint64_t seed = I->seed + event * 0x9E3779B97F4A7C15ULL;
  long made = 0;
  for (int q = 0; q < nth; ++q)
    for (int p = 0; p < nr; ++p) {
      double rc = g->rh[p], tc = g->th[q];
      if (rc < I->r0 || rc > I->r1) continue;
      if (room - made < 2) continue;
      double sc = om_sqrtg(a, rc, tc);
      double br = 0.5 * (om_sqrtg(a, g->rn[p], tc) * Br[(long)q * nrn + p] +
                         om_sqrtg(a, g->rn[p + 1], tc) * Br[(long)q * nrn + p + 1]) / sc;
      double bt = 0.5 * (om_sqrtg(a, rc, g->tn[q]) * Bt[(long)q * nr + p] +
                         om_sqrtg(a, rc, g->tn[q + 1]) * Bt[(long)(q + 1) * nr + p]) / sc;
      double ngj = OmH * fabs(cos(tc) * br - rc * sin(tc) * bt) / (4.0 * M_PI);
      double V = 2.0 * M_PI * sc * (g->rn[p + 1] - g->rn[p]) * g->dth;
      long c = (long)q * nr + p;
      if (!(wsum[c] / V < I->mult * ngj)) continue;
      double z[3];
      sample_position(a, seed, c, g->rn[p], g->rn[p + 1], g->tn[q], g->tn[q + 1],
                      &z[0], &z[1], &z[2]);
      for (int s = 0; s < 2; ++s) {
        long id = 2 * c + s;
        double mag = mj_sample(T, U(seed, id, 200));
        double mu = 2.0 * U(seed, id, 201) - 1.0;
        double az = 2.0 * M_PI * U(seed, id, 202);
        double sn = sqrt(1.0 - mu * mu);
        double f[3] = {mag * mu, mag * sn * cos(az), mag * sn * sin(az)};
        double *o = out + 8 * (made + s);
        o[0] = z[0], o[1] = z[1], o[2] = z[2];
        fido_to_covariant(a, z[0], z[1], f, &o[3]);
        o[6] = s == 0 ? 1.0 : -1.0;
        o[7] = 0.5 * I->density * ngj * V;
      }
      made += 2;
    }
  free(T);
  free(wsum);
  return made;
}
