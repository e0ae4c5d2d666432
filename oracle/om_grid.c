/*
 * om_grid.c -- reference oracle (TEST INFRASTRUCTURE ONLY): spherical Yee
 * grid, field gather, volume-weighted charge-conserving deposit, the
 * two-chain leapfrog Maxwell solver and grid diagnostics of
 * arXiv:2602.07452, in plain FP64 C.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "om_internal.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* component arrays: r fastest, index j nR + i                               */
#define IDX(nR, i, j) ((long)(j) * (nR) + (i))

/* ------------------------------------------------------------------------
 * Grid: r log-spaced between r_in and r_out, theta uniform on
 * [theta0, pi - theta0] (half-theta domain, Sec. 2.5); half radii are the
 * geometric means of neighbouring nodes (reading for a log-spaced grid).
 * ------------------------------------------------------------------------ */
om_grid *om_grid_new(double a, int nr, int nth, double r_in, double r_out,
                     double th0) {
  om_grid *g = (om_grid *)calloc(1, sizeof(om_grid));
  g->a = a;
  g->nr = nr;
  g->nth = nth;
  g->r_in = r_in;
  g->r_out = r_out;
  g->th0 = th0;
  g->dlnr = log(r_out / r_in) / nr;
  g->dth = (M_PI - 2.0 * th0) / nth;
  g->rn = (double *)malloc(sizeof(double) * (nr + 1));
  g->rh = (double *)malloc(sizeof(double) * nr);
  g->tn = (double *)malloc(sizeof(double) * (nth + 1));
  g->th = (double *)malloc(sizeof(double) * nth);
  for (int i = 0; i <= nr; ++i) g->rn[i] = r_in * exp(i * g->dlnr);
  for (int i = 0; i < nr; ++i) g->rh[i] = sqrt(g->rn[i] * g->rn[i + 1]);
  for (int j = 0; j <= nth; ++j) g->tn[j] = th0 + j * g->dth;
  for (int j = 0; j < nth; ++j) g->th[j] = th0 + (j + 0.5) * g->dth;
  return g;
}

void om_grid_free(om_grid *g) {
  if (!g) return;
  free(g->rn);
  free(g->rh);
  free(g->tn);
  free(g->th);
  free(g);
}

void om_grid_coords(const om_grid *g, double *rn, double *rh, double *tn,
                    double *th) {
  memcpy(rn, g->rn, sizeof(double) * (g->nr + 1));
  memcpy(rh, g->rh, sizeof(double) * g->nr);
  memcpy(tn, g->tn, sizeof(double) * (g->nth + 1));
  memcpy(th, g->th, sizeof(double) * g->nth);
}

void om_comp_shape(const om_grid *g, int c, int *nR, int *nT) {
  if (c >= 6) {
    *nR = g->nr + 1;
    *nT = g->nth + 1;
    return;
  }
  *nR = om_comp_rhalf(c) ? g->nr : g->nr + 1;
  *nT = om_comp_thalf(c) ? g->nth : g->nth + 1;
}

static double comp_r(const om_grid *g, int c, int i) {
  return (c < 6 && om_comp_rhalf(c)) ? g->rh[i] : g->rn[i];
}
static double comp_t(const om_grid *g, int c, int j) {
  return (c < 6 && om_comp_thalf(c)) ? g->th[j] : g->tn[j];
}

void om_densitize(const om_grid *g, int c, int dir, const double *in,
                  double *out) {
  int nR, nT;
  om_comp_shape(g, c, &nR, &nT);
  for (int j = 0; j < nT; ++j)
    for (int i = 0; i < nR; ++i) {
      double s = om_sqrtg(g->a, comp_r(g, c, i), comp_t(g, c, j));
      out[j * nR + i] = dir > 0 ? in[j * nR + i] * s : in[j * nR + i] / s;
    }
}

/* largest p in [0, n-2] with x[p] <= v (clamped at both ends)             */
static int locate(const double *x, int n, double v) {
  if (v <= x[0]) return 0;
  if (v >= x[n - 1]) return n - 2;
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (x[mid] <= v)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

int om_locate(const double *x, int n, double v) { return locate(x, n, v); }

static double clamp01(double f) { return f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f); }

/* ------------------------------------------------------------------------
 * Gather (reading: the paper names no scheme).  Each component is
 * interpolated on its own staggered sub-grid with the metric-weighted
 * linear rule of Sec. 2.1 extended to two dimensions:
 *   F(x) = sum_c w_c (sqrt(g) F)_c / sqrt(g)(x),
 * w_c the bilinear weights in (r, theta); outside the sub-grid the nearest
 * cell's edge value is used (fractions clamped to [0,1]).
 * ------------------------------------------------------------------------ */
void om_gather(const om_grid *g, const double *const *G, double r, double th,
               double *D, double *B) {
  double out[6];
  for (int c = 0; c < 6; ++c) {
    int rhf = om_comp_rhalf(c), thf = om_comp_thalf(c);
    const double *R = rhf ? g->rh : g->rn;
    const double *T = thf ? g->th : g->tn;
    int nR = rhf ? g->nr : g->nr + 1;
    int nT = thf ? g->nth : g->nth + 1;
    int p = locate(R, nR, r), q = locate(T, nT, th);
    double fr = clamp01((r - R[p]) / (R[p + 1] - R[p]));
    double ft = clamp01((th - T[q]) / (T[q + 1] - T[q]));
    const double *A = G[c];
    double v = (1.0 - fr) * (1.0 - ft) * A[q * nR + p] +
               fr * (1.0 - ft) * A[q * nR + p + 1] +
               (1.0 - fr) * ft * A[(q + 1) * nR + p] +
               fr * ft * A[(q + 1) * nR + p + 1];
    out[c] = v;
  }
  double s = om_sqrtg(g->a, r, th);
  for (int c = 0; c < 3; ++c) D[c] = out[c] / s;
  for (int c = 0; c < 3; ++c) B[c] = out[3 + c] / s;
}

/* ------------------------------------------------------------------------
 * Deposit weights (Sec. 2.3, eqs. v1-v5): the charge given to a node is the
 * sub-volume opposite to it over the cell volume.  Sub-volumes are
 * integrals of sqrt(gamma) dr dtheta evaluated with the 2-D trapezoidal
 * rule on 4 x 4 points per sub-rectangle; the cell volume is the sum of the
 * four sub-volumes (reading), so the weights sum to one.
 * ------------------------------------------------------------------------ */
static double subvol(double a, int flat, double r0, double r1, double t0,
                     double t1) {
  static const double cw[4] = {0.5, 1.0, 1.0, 0.5};
  double hr = (r1 - r0) / 3.0, ht = (t1 - t0) / 3.0, sum = 0.0;
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) {
      double f = flat ? 1.0 : om_sqrtg(a, r0 + i * hr, t0 + j * ht);
      sum += cw[i] * cw[j] * f;
    }
  return hr * ht * sum;
}

/* weights of the corners (ra,ta), (rb,ta), (ra,tb), (rb,tb) of any cell  */
static void box_weights(double a, int flat, double r, double th, double ra,
                        double rb, double ta, double tb, double *W) {
  double V00 = subvol(a, flat, ra, r, ta, th);
  double V10 = subvol(a, flat, r, rb, ta, th);
  double V01 = subvol(a, flat, ra, r, th, tb);
  double V11 = subvol(a, flat, r, rb, th, tb);
  double V = V00 + V10 + V01 + V11;
  W[0] = V11 / V;
  W[1] = V01 / V;
  W[2] = V10 / V;
  W[3] = V00 / V;
}

void om_dep_weights(const om_grid *g, double r, double th, int p, int q,
                    int flat, double *W) {
  double ra = g->rn[p], rb = g->rn[p + 1], ta = g->tn[q], tb = g->tn[q + 1];
  double V00 = subvol(g->a, flat, ra, r, ta, th);
  double V10 = subvol(g->a, flat, r, rb, ta, th);
  double V01 = subvol(g->a, flat, ra, r, th, tb);
  double V11 = subvol(g->a, flat, r, rb, th, tb);
  double V = V00 + V10 + V01 + V11;
  W[0] = V11 / V; /* node (p,   q  ) */
  W[1] = V01 / V; /* node (p+1, q  ) */
  W[2] = V10 / V; /* node (p,   q+1) */
  W[3] = V00 / V; /* node (p+1, q+1) */
}

static void node_cell(const om_grid *g, double r, double th, int *p, int *q) {
  *p = locate(g->rn, g->nr + 1, r);
  *q = locate(g->tn, g->nth + 1, th);
}

/* Dual lengths of node (i, j): half cells at the domain edges.             */
static double Lr(const om_grid *g, int i) {
  if (i == 0) return g->rh[0] - g->rn[0];
  if (i == g->nr) return g->rn[g->nr] - g->rh[g->nr - 1];
  return g->rh[i] - g->rh[i - 1];
}
static double Lt(const om_grid *g, int j) {
  return (j == 0 || j == g->nth) ? 0.5 * g->dth : g->dth;
}

/* ------------------------------------------------------------------------
 * Charge-conserving current (reading; the paper's own current is not
 * conserving and is corrected by cleaning).  The straight move in (r,
 * theta) is split where it crosses node-cell boundaries; inside a cell the
 * weight change is turned into four face fluxes with
 *   S_r = W10 + W11, S_t = W01 + W11,
 *   Fr1 = dS_r (S_t + S_t') / 2, Fr0 = dS_r - Fr1,
 *   Ft1 = dW11 - Fr1,            Ft0 = dS_t - Ft1,
 * which reproduces every node's weight change exactly.  Because the
 * volume weights of two cells disagree on their common edge, the jump at a
 * crossing is carried by a flux along that edge.  Fluxes F (charge per
 * time) become densitized currents sqrt(g) J = F / (2 pi L), charges
 * sqrt(g) rho = Q / (2 pi Lr Lt); J^phi = q w (W + W')/2 dphi/dt on the
 * nodes of both the old and the new cell.
 * ------------------------------------------------------------------------ */
typedef struct {
  const om_grid *g;
  double *Fr, *Ft; /* raw face fluxes, hn and nh layouts                  */
} flux_acc;

static void add_fr(flux_acc *A, int i, int j, double v) {
  A->Fr[j * A->g->nr + i] += v;
}
static void add_ft(flux_acc *A, int i, int j, double v) {
  A->Ft[j * (A->g->nr + 1) + i] += v;
}

static void cell_flux(flux_acc *A, int p, int q, const double *W0,
                      const double *W1, double s) {
  double Sr0 = W0[1] + W0[3], Sr1 = W1[1] + W1[3];
  double St0 = W0[2] + W0[3], St1 = W1[2] + W1[3];
  double dSr = Sr1 - Sr0, dSt = St1 - St0, dW11 = W1[3] - W0[3];
  double Fr1 = 0.5 * dSr * (St0 + St1);
  double Fr0 = dSr - Fr1;
  double Ft1 = dW11 - Fr1;
  double Ft0 = dSt - Ft1;
  add_fr(A, p, q, s * Fr0);
  add_fr(A, p, q + 1, s * Fr1);
  add_ft(A, p, q, s * Ft0);
  add_ft(A, p + 1, q, s * Ft1);
}

static void deposit_one(const om_grid *g, flux_acc *A, double dt, double r0,
                        double t0, double ph0, double r1, double t1,
                        double ph1, double qw, double *Q, double *Jp) {
  int nrn = g->nr + 1;
  int p0, q0, p1, q1;
  node_cell(g, r0, t0, &p0, &q0);
  node_cell(g, r1, t1, &p1, &q1);
  double Wo[4], Wn[4];
  om_dep_weights(g, r0, t0, p0, q0, 0, Wo);
  om_dep_weights(g, r1, t1, p1, q1, 0, Wn);
  static const int off[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
  double dphi = (ph1 - ph0) / dt;
  for (int c = 0; c < 4; ++c) {
    int io = p0 + off[c][0], jo = q0 + off[c][1];
    int in = p1 + off[c][0], jn = q1 + off[c][1];
    Q[jn * nrn + in] += qw * Wn[c];
    Jp[jo * nrn + io] += 0.5 * qw * Wo[c] * dphi;
    Jp[jn * nrn + in] += 0.5 * qw * Wn[c] * dphi;
  }
  double s = qw / dt;
  if (p0 == p1 && q0 == q1) {
    cell_flux(A, p0, q0, Wo, Wn, s);
    return;
  }
  /* crossings of node-cell boundaries along the straight move: parameter
   * t in (0,1), kind 0 = radius r_b, kind 1 = angle theta_b              */
  double ts[16];
  int kind[16], bnd[16], nt = 0;
  int lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
  for (int b = lo + 1; b <= hi && nt < 16; ++b) {
    ts[nt] = (g->rn[b] - r0) / (r1 - r0);
    kind[nt] = 0, bnd[nt] = b, ++nt;
  }
  lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
  for (int b = lo + 1; b <= hi && nt < 16; ++b) {
    ts[nt] = (g->tn[b] - t0) / (t1 - t0);
    kind[nt] = 1, bnd[nt] = b, ++nt;
  }
  for (int i = 1; i < nt; ++i) /* insertion sort by t */
    for (int k = i; k > 0 && ts[k] < ts[k - 1]; --k) {
      double tt = ts[k];
      int tk = kind[k], tb = bnd[k];
      ts[k] = ts[k - 1], kind[k] = kind[k - 1], bnd[k] = bnd[k - 1];
      ts[k - 1] = tt, kind[k - 1] = tk, bnd[k - 1] = tb;
    }
  /* the crossing point itself, with the crossed coordinate set exactly on
   * the boundary                                                          */
  double xr[16], xt[16];
  for (int k = 0; k < nt; ++k) {
    xr[k] = kind[k] == 0 ? g->rn[bnd[k]] : r0 + ts[k] * (r1 - r0);
    xt[k] = kind[k] == 1 ? g->tn[bnd[k]] : t0 + ts[k] * (t1 - t0);
  }
  double prevW[4];
  int pp = p0, pq = q0;
  for (int k = 0; k <= nt; ++k) {
    int cp, cq;
    double Wa[4], Wb[4];
    if (k == 0) {
      cp = p0, cq = q0;
      memcpy(Wa, Wo, sizeof(Wa));
    } else {
      /* next cell: step across the boundary just crossed */
      cp = pp, cq = pq;
      if (kind[k - 1] == 0)
        cp = (bnd[k - 1] > pp) ? pp + 1 : pp - 1;
      else
        cq = (bnd[k - 1] > pq) ? pq + 1 : pq - 1;
      om_dep_weights(g, xr[k - 1], xt[k - 1], cp, cq, 0, Wa);
      /* the two cells' weights at the crossing point both live on the
       * shared edge; the difference moves along that edge as a flux      */
      double jump[4];
      for (int c = 0; c < 4; ++c) {
        int ni = cp + off[c][0], nj = cq + off[c][1];
        double prev = 0.0;
        for (int d = 0; d < 4; ++d)
          if (pp + off[d][0] == ni && pq + off[d][1] == nj) prev = prevW[d];
        jump[c] = Wa[c] - prev;
      }
      if (kind[k - 1] == 0) {
        int e = bnd[k - 1];
        int c_hi = (e == cp) ? 2 : 3; /* node (e, cq+1) of the new cell */
        add_ft(A, e, cq, s * jump[c_hi]);
      } else {
        int e = bnd[k - 1];
        int c_hi = (e == cq) ? 1 : 3; /* node (cp+1, e) of the new cell */
        add_fr(A, cp, e, s * jump[c_hi]);
      }
    }
    if (k == nt)
      memcpy(Wb, Wn, sizeof(Wb));
    else
      om_dep_weights(g, xr[k], xt[k], cp, cq, 0, Wb);
    cell_flux(A, cp, cq, Wa, Wb, s);
    memcpy(prevW, Wb, sizeof(prevW));
    pp = cp, pq = cq;
  }
}

void om_deposit(const om_grid *g, double dt, long n, const double *r0,
                const double *th0, const double *ph0, const double *r1,
                const double *th1, const double *ph1, const double *qw,
                const int *mode, double *rho, double *Jr, double *Jth,
                double *Jph) {
  int nrn = g->nr + 1, ntn = g->nth + 1;
  long nn = (long)nrn * ntn;
  long nhn = (long)g->nr * ntn, nnh = (long)nrn * g->nth;
  double *Q = (double *)calloc(nn, sizeof(double));
  double *P = (double *)calloc(nn, sizeof(double));
  flux_acc A = {g, (double *)calloc(nhn, sizeof(double)),
                (double *)calloc(nnh, sizeof(double))};
  /* sequential in particle order: the plain definition of a sum */
  for (long k = 0; k < n; ++k) {
    if (!mode[k]) continue;
    deposit_one(g, &A, dt, r0[k], th0[k], ph0[k], r1[k], th1[k], ph1[k],
                qw[k], Q, P);
  }
  double tp = 2.0 * M_PI;
  for (int j = 0; j < ntn; ++j)
    for (int i = 0; i < nrn; ++i) {
      double L = tp * Lr(g, i) * Lt(g, j);
      rho[j * nrn + i] += Q[j * nrn + i] / L;
      Jph[j * nrn + i] += P[j * nrn + i] / L;
    }
  for (int j = 0; j < ntn; ++j)
    for (int i = 0; i < g->nr; ++i)
      Jr[j * g->nr + i] += A.Fr[j * g->nr + i] / (tp * Lt(g, j));
  for (int j = 0; j < g->nth; ++j)
    for (int i = 0; i < nrn; ++i)
      Jth[j * nrn + i] += A.Ft[j * nrn + i] / (tp * Lr(g, i));
  free(Q);
  free(P);
  free(A.Fr);
  free(A.Ft);
}

/* ------------------------------------------------------------------------
 * The paper's own current (Sec. 2.3), a deposit mode of its own.  Every
 * particle alive after the push deposits at its new position x^{n+2} with
 * u^{n+2}: rho with the node weights, each current component on its own Yee
 * subgrid (J^r at (r_{i+1/2}, theta_j), J^theta at (r_i, theta_{j+1/2}),
 * J^phi at the nodes) with the volume weights of that subgrid's cell, each
 * carried by the coordinate velocity dx^i/dt = alpha v^i - beta^i of eq. p1.
 * The sums of the paper give the FIDO current j; q w (alpha v - beta) is the
 * grid current J = alpha j - rho beta that eq. m3 needs (reading).  A
 * position outside a half subgrid's range (below r_{1/2}, above
 * r_{N-1/2}, or within half a cell of a theta edge) is moved onto its edge
 * for that component.  Densitized values: sqrt(g) rho = Q / (2 pi Lr Lt),
 * sqrt(g) J^r = sum q w W dr/dt / (2 pi (r_{i+1} - r_i) Lt_j), sqrt(g)
 * J^theta = sum q w W dth/dt / (2 pi Lr_i dth), sqrt(g) J^phi = sum q w W
 * dphi/dt / (2 pi Lr Lt).  Not charge-conserving: Gauss's law is restored
 * by cleaning (om_div_clean).
 * ------------------------------------------------------------------------ */
static double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

void om_deposit_paper(const om_grid *g, long n, const double *r,
                      const double *th, const double *ur, const double *uth,
                      const double *uph, const double *qw, const int *mode,
                      double *rho, double *Jr, double *Jth, double *Jph) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1, ntn = nth + 1;
  double tp = 2.0 * M_PI;
  for (long k = 0; k < n; ++k) {
    if (!mode[k]) continue;
    double z[6] = {r[k], th[k], 0.0, ur[k], uth[k], uph[k]};
    double f[6], zero[3] = {0.0, 0.0, 0.0};
    om_rhs(g->a, 0.0, z, zero, zero, f); /* f[0..2] = dx^i/dt, eq. p1   */
    double W[4];
    int p, q;
    /* rho and J^phi at the nodes                                          */
    node_cell(g, z[0], z[1], &p, &q);
    om_dep_weights(g, z[0], z[1], p, q, 0, W);
    for (int c = 0; c < 4; ++c) {
      int i = p + (c & 1), j = q + (c >> 1);
      double L = tp * Lr(g, i) * Lt(g, j);
      rho[IDX(nrn, i, j)] += qw[k] * W[c] / L;
      Jph[IDX(nrn, i, j)] += qw[k] * W[c] * f[2] / L;
    }
    /* J^r on (r_{i+1/2}, theta_j)                                          */
    {
      double rc = clampd(z[0], g->rh[0], g->rh[nr - 1]);
      int pr = locate(g->rh, nr, rc);
      box_weights(g->a, 0, rc, z[1], g->rh[pr], g->rh[pr + 1], g->tn[q],
                  g->tn[q + 1], W);
      for (int c = 0; c < 4; ++c) {
        int i = pr + (c & 1), j = q + (c >> 1);
        double L = tp * (g->rn[i + 1] - g->rn[i]) * Lt(g, j);
        Jr[IDX(nr, i, j)] += qw[k] * W[c] * f[0] / L;
      }
    }
    /* J^theta on (r_i, theta_{j+1/2})                                      */
    {
      double tc = clampd(z[1], g->th[0], g->th[nth - 1]);
      int qt = locate(g->th, nth, tc);
      box_weights(g->a, 0, z[0], tc, g->rn[p], g->rn[p + 1], g->th[qt],
                  g->th[qt + 1], W);
      for (int c = 0; c < 4; ++c) {
        int i = p + (c & 1), j = qt + (c >> 1);
        double L = tp * Lr(g, i) * g->dth;
        Jth[IDX(nrn, i, j)] += qw[k] * W[c] * f[1] / L;
      }
    }
  }
  (void)ntn;
}

/* ------------------------------------------------------------------------
 * Divergence cleaning (Sec. 2.4, eq. phi) in densitized form on the nodes:
 *   d_r(sqrt(g) g^rr d_r phi) + d_th(sqrt(g) g^thth d_th phi) = G,
 * G the Gauss residual div_h(sqrt(g) D) - 4 pi sqrt(g) rho of
 * om_gauss_residual at the interior nodes (d_phi = 0, and g^rth = 0).
 * d_r phi lives at (r_{i+1/2}, theta_j), d_th phi at (r_i, theta_{j+1/2}),
 * where D^r and D^theta do, so the discrete operator is the discrete
 * divergence of the discrete gradient.  phi = 0 on the boundary nodes
 * (reading); phi starts at 0 and takes `iters` Jacobi sweeps; then
 * D^i -= g^ij d_j phi (D^phi with g^phir and the mean of the two radial
 * differences at interior nodes).
 * ------------------------------------------------------------------------ */
static double *dup0(long n) { return (double *)calloc(n, sizeof(double)); }

static double gupper(const om_grid *g, double r, double th, int which) {
  double m[13];
  om_metric(g->a, r, th, m);
  return m[which];
}

void om_div_clean(const om_grid *g, double *const *D, const double *rho_d,
                  int iters, double *phi_out) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1, ntn = nth + 1;
  long nn = (long)nrn * ntn;
  double *G = dup0(nn), *phi = dup0(nn), *nxt = dup0(nn);
  om_gauss_residual(g, (const double *const *)D, rho_d, G);
  double dth = g->dth;
  for (int it = 0; it < iters; ++it) {
    for (int j = 1; j < nth; ++j)
      for (int i = 1; i < nr; ++i) {
        double Lri = g->rh[i] - g->rh[i - 1];
        double aE = om_sqrtg(g->a, g->rh[i], g->tn[j]) *
                    gupper(g, g->rh[i], g->tn[j], 6) /
                    (g->rn[i + 1] - g->rn[i]) / Lri;
        double aW = om_sqrtg(g->a, g->rh[i - 1], g->tn[j]) *
                    gupper(g, g->rh[i - 1], g->tn[j], 6) /
                    (g->rn[i] - g->rn[i - 1]) / Lri;
        double aN = om_sqrtg(g->a, g->rn[i], g->th[j]) *
                    gupper(g, g->rn[i], g->th[j], 7) / (dth * dth);
        double aS = om_sqrtg(g->a, g->rn[i], g->th[j - 1]) *
                    gupper(g, g->rn[i], g->th[j - 1], 7) / (dth * dth);
        double nb = aE * phi[IDX(nrn, i + 1, j)] + aW * phi[IDX(nrn, i - 1, j)] +
                    aN * phi[IDX(nrn, i, j + 1)] + aS * phi[IDX(nrn, i, j - 1)];
        nxt[IDX(nrn, i, j)] = (nb - G[IDX(nrn, i, j)]) / (aE + aW + aN + aS);
      }
    double *t = phi;
    phi = nxt;
    nxt = t;
  }
  for (int j = 0; j <= nth; ++j)
    for (int i = 0; i < nr; ++i)
      D[0][IDX(nr, i, j)] -= gupper(g, g->rh[i], g->tn[j], 6) *
                             (phi[IDX(nrn, i + 1, j)] - phi[IDX(nrn, i, j)]) /
                             (g->rn[i + 1] - g->rn[i]);
  for (int j = 0; j < nth; ++j)
    for (int i = 0; i <= nr; ++i)
      D[1][IDX(nrn, i, j)] -= gupper(g, g->rn[i], g->th[j], 7) *
                              (phi[IDX(nrn, i, j + 1)] - phi[IDX(nrn, i, j)]) /
                              dth;
  for (int j = 1; j < nth; ++j)
    for (int i = 1; i < nr; ++i) {
      double dr = 0.5 * ((phi[IDX(nrn, i + 1, j)] - phi[IDX(nrn, i, j)]) /
                             (g->rn[i + 1] - g->rn[i]) +
                         (phi[IDX(nrn, i, j)] - phi[IDX(nrn, i - 1, j)]) /
                             (g->rn[i] - g->rn[i - 1]));
      D[2][IDX(nrn, i, j)] -= gupper(g, g->rn[i], g->tn[j], 9) * dr;
    }
  if (phi_out) memcpy(phi_out, phi, sizeof(double) * nn);
  free(G);
  free(phi);
  free(nxt);
}

/* ------------------------------------------------------------------------
 * Maxwell solver (Sec. 2.1).  Grid fields
 *   E_i = alpha D_i + sqrt(g) eta_ijk beta^j B^k,
 *   H_i = alpha B_i - sqrt(g) eta_ijk beta^j D^k,
 * with components not native to a Yee point brought there by the
 * metric-weighted average of the two neighbours (sqrt(g) F averaged, then
 * divided by sqrt(g) at the target); at the radial ends of the grid the
 * single available neighbour is used.  E_phi vanishes on the theta edges
 * (axis condition, reading).
 * ------------------------------------------------------------------------ */

/* densitized average of a component at two positions (either may be -1) */
static double davg2(const om_grid *g, int c, const double *F, int nR, int i0,
                    int j0, int i1, int j1) {
  double s = 0.0;
  int k = 0;
  if (i0 >= 0) {
    s += om_sqrtg(g->a, comp_r(g, c, i0), comp_t(g, c, j0)) *
         F[IDX(nR, i0, j0)];
    ++k;
  }
  if (i1 >= 0) {
    s += om_sqrtg(g->a, comp_r(g, c, i1), comp_t(g, c, j1)) *
         F[IDX(nR, i1, j1)];
    ++k;
  }
  return s / k;
}

void om_compute_E(const om_grid *g, const double *const *D,
                  const double *const *B, double *const *E) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  double m[13];
  /* E_r at (i+1/2, j) */
  for (int j = 0; j <= nth; ++j)
    for (int i = 0; i < nr; ++i) {
      om_metric(g->a, g->rh[i], g->tn[j], m);
      double Dp = davg2(g, 2, D[2], nrn, i, j, i + 1, j) / m[10];
      E[0][IDX(nr, i, j)] = m[0] * (m[2] * D[0][IDX(nr, i, j)] + m[5] * Dp);
    }
  /* E_theta at (i, j+1/2) */
  for (int j = 0; j < nth; ++j)
    for (int i = 0; i <= nr; ++i) {
      om_metric(g->a, g->rn[i], g->th[j], m);
      double sBp = davg2(g, 5, B[2], nr, i > 0 ? i - 1 : -1, j,
                         i < nr ? i : -1, j);
      E[1][IDX(nrn, i, j)] = m[0] * m[3] * D[1][IDX(nrn, i, j)] - m[1] * sBp;
    }
  /* E_phi at (i, j) */
  for (int j = 0; j <= nth; ++j)
    for (int i = 0; i <= nr; ++i) {
      if (j == 0 || j == nth) {
        E[2][IDX(nrn, i, j)] = 0.0;
        continue;
      }
      om_metric(g->a, g->rn[i], g->tn[j], m);
      int i0 = i > 0 ? i - 1 : -1, i1 = i < nr ? i : -1;
      double Dr = davg2(g, 0, D[0], nr, i0, j, i1, j) / m[10];
      double sBt = davg2(g, 4, B[1], nr, i0, j, i1, j);
      E[2][IDX(nrn, i, j)] =
          m[0] * (m[5] * Dr + m[4] * D[2][IDX(nrn, i, j)]) + m[1] * sBt;
    }
}

void om_compute_H(const om_grid *g, const double *const *B,
                  const double *const *D, double *const *H) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  double m[13];
  /* H_r at (i, j+1/2) */
  for (int j = 0; j < nth; ++j)
    for (int i = 0; i <= nr; ++i) {
      om_metric(g->a, g->rn[i], g->th[j], m);
      double Bp = davg2(g, 5, B[2], nr, i > 0 ? i - 1 : -1, j,
                        i < nr ? i : -1, j) /
                  m[10];
      H[0][IDX(nrn, i, j)] = m[0] * (m[2] * B[0][IDX(nrn, i, j)] + m[5] * Bp);
    }
  /* H_theta at (i+1/2, j) */
  for (int j = 0; j <= nth; ++j)
    for (int i = 0; i < nr; ++i) {
      om_metric(g->a, g->rh[i], g->tn[j], m);
      double sDp = davg2(g, 2, D[2], nrn, i, j, i + 1, j);
      H[1][IDX(nr, i, j)] = m[0] * m[3] * B[1][IDX(nr, i, j)] + m[1] * sDp;
    }
  /* H_phi at (i+1/2, j+1/2) */
  for (int j = 0; j < nth; ++j)
    for (int i = 0; i < nr; ++i) {
      om_metric(g->a, g->rh[i], g->th[j], m);
      double Br = davg2(g, 3, B[0], nrn, i, j, i + 1, j) / m[10];
      double sDt = davg2(g, 1, D[1], nrn, i, j, i + 1, j);
      H[2][IDX(nr, i, j)] =
          m[0] * (m[5] * Br + m[4] * B[2][IDX(nr, i, j)]) - m[1] * sDt;
    }
}

/* absorbing layer (eqs. abs0-abs2), applied as the factor exp(-chi dt)    */
static double damp(const om_grid *g, const double *ab, double r, double dt) {
  if (!ab || ab[1] <= 0.0 || r <= ab[0]) return 1.0;
  double x = (r - ab[0]) / (g->r_out - ab[0]);
  return exp(-ab[1] * pow(x, ab[2]) * dt);
}

void om_faraday(const om_grid *g, double dt, const double *ab,
                const double *const *Bin, const double *const *E,
                double *const *Bout) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  double dth = g->dth;
  /* B^r at (i, j+1/2): dB/dt = -(1/sqrt g) d_theta E_phi */
  for (int j = 0; j < nth; ++j)
    for (int i = 0; i <= nr; ++i) {
      double s = om_sqrtg(g->a, g->rn[i], g->th[j]);
      double c = (E[2][IDX(nrn, i, j + 1)] - E[2][IDX(nrn, i, j)]) / dth;
      Bout[0][IDX(nrn, i, j)] =
          damp(g, ab, g->rn[i], dt) * (Bin[0][IDX(nrn, i, j)] - dt * c / s);
    }
  /* B^theta at (i+1/2, j): dB/dt = +(1/sqrt g) d_r E_phi */
  for (int j = 0; j <= nth; ++j)
    for (int i = 0; i < nr; ++i) {
      double s = om_sqrtg(g->a, g->rh[i], g->tn[j]);
      double c = -(E[2][IDX(nrn, i + 1, j)] - E[2][IDX(nrn, i, j)]) /
                 (g->rn[i + 1] - g->rn[i]);
      Bout[1][IDX(nr, i, j)] =
          damp(g, ab, g->rh[i], dt) * (Bin[1][IDX(nr, i, j)] - dt * c / s);
    }
  /* B^phi at (i+1/2, j+1/2): dB/dt = -(1/sqrt g)(d_r E_th - d_th E_r) */
  for (int j = 0; j < nth; ++j)
    for (int i = 0; i < nr; ++i) {
      double s = om_sqrtg(g->a, g->rh[i], g->th[j]);
      double c = (E[1][IDX(nrn, i + 1, j)] - E[1][IDX(nrn, i, j)]) /
                     (g->rn[i + 1] - g->rn[i]) -
                 (E[0][IDX(nr, i, j + 1)] - E[0][IDX(nr, i, j)]) / dth;
      Bout[2][IDX(nr, i, j)] =
          damp(g, ab, g->rh[i], dt) * (Bin[2][IDX(nr, i, j)] - dt * c / s);
    }
}

/* zero gradient at the radial ends of the grid (Sec. 2.5): copy F from
 * (is, js) to (id, jd)                                                     */
static void zcopy(double *F, int nR, int id, int jd, int is, int js) {
  F[IDX(nR, id, jd)] = F[IDX(nR, is, js)];
}

void om_ampere(const om_grid *g, double dt, const double *ab,
               const double *const *Din, const double *const *H,
               const double *const *Jd, double *const *Dout) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  double dth = g->dth, fp = 4.0 * M_PI;
  /* D^r at (i+1/2, j): dD/dt = (1/sqrt g) d_th H_phi - 4 pi J.  On the
   * theta edges the axis condition H_phi = 0 closes the derivative over the
   * half cell (dual length dth/2).                                         */
  for (int j = 0; j <= nth; ++j)
    for (int i = 0; i < nr; ++i) {
      double s = om_sqrtg(g->a, g->rh[i], g->tn[j]);
      double c;
      if (j == 0)
        c = H[2][IDX(nr, i, 0)] / (0.5 * dth);
      else if (j == nth)
        c = -H[2][IDX(nr, i, nth - 1)] / (0.5 * dth);
      else
        c = (H[2][IDX(nr, i, j)] - H[2][IDX(nr, i, j - 1)]) / dth;
      Dout[0][IDX(nr, i, j)] =
          damp(g, ab, g->rh[i], dt) *
          (Din[0][IDX(nr, i, j)] + dt * (c - fp * Jd[0][IDX(nr, i, j)]) / s);
    }
  /* D^theta at (i, j+1/2), interior i: dD/dt = -(1/sqrt g) d_r H_phi - .. */
  for (int j = 0; j < nth; ++j)
    for (int i = 1; i < nr; ++i) {
      double s = om_sqrtg(g->a, g->rn[i], g->th[j]);
      double c = -(H[2][IDX(nr, i, j)] - H[2][IDX(nr, i - 1, j)]) /
                 (g->rh[i] - g->rh[i - 1]);
      Dout[1][IDX(nrn, i, j)] =
          damp(g, ab, g->rn[i], dt) *
          (Din[1][IDX(nrn, i, j)] + dt * (c - fp * Jd[1][IDX(nrn, i, j)]) / s);
    }
  /* D^phi at (i, j), interior: dD/dt = (1/sqrt g)(d_r H_th - d_th H_r) - ..*/
  for (int j = 1; j < nth; ++j)
    for (int i = 1; i < nr; ++i) {
      double s = om_sqrtg(g->a, g->rn[i], g->tn[j]);
      double c = (H[1][IDX(nr, i, j)] - H[1][IDX(nr, i - 1, j)]) /
                     (g->rh[i] - g->rh[i - 1]) -
                 (H[0][IDX(nrn, i, j)] - H[0][IDX(nrn, i, j - 1)]) / dth;
      Dout[2][IDX(nrn, i, j)] =
          damp(g, ab, g->rn[i], dt) *
          (Din[2][IDX(nrn, i, j)] + dt * (c - fp * Jd[2][IDX(nrn, i, j)]) / s);
    }
  /* radial ends: zero radial gradient (inner end inside the horizon, outer
   * end inside the absorbing layer)                                        */
  for (int j = 0; j < nth; ++j) {
    zcopy(Dout[1], nrn, 0, j, 1, j);
    zcopy(Dout[1], nrn, nr, j, nr - 1, j);
  }
  for (int j = 1; j < nth; ++j) {
    zcopy(Dout[2], nrn, 0, j, 1, j);
    zcopy(Dout[2], nrn, nr, j, nr - 1, j);
  }
  /* theta edges: D^phi = 0 (axis condition)                                */
  for (int i = 0; i <= nr; ++i) {
    Dout[2][IDX(nrn, i, 0)] = 0.0;
    Dout[2][IDX(nrn, i, nth)] = 0.0;
  }
}

/* ------------------------------------------------------------------------
 * One PIC step, the ten sub-steps of Sec. 2.1 in order:
 *  1 E^{n+1}   = E(<D>^{n+1}, B^{n+1}),  <D>^{n+1} = (D^{n+1/2}+D^{n+3/2})/2
 *  2 B^{n+3/2} = <B>^{n+1/2} - dt curl E^{n+1}, <B>^{n+1/2} = (B^n+B^{n+1})/2
 *  3 E^{n+3/2} = E(D^{n+3/2}, B^{n+3/2})
 *  4 B^{n+2}   = B^{n+1} - dt curl E^{n+3/2}
 *  5 push x^{n+1} -> x^{n+2} in D^{n+3/2}, B^{n+3/2}
 *  6 deposit rho^{n+2}, J^{n+3/2} (conserving) or J^{n+2} (paper mode)
 *  7 H^{n+3/2} = H(B^{n+3/2}, D^{n+3/2})
 *  8 D^{n+2}   = D^{n+1} + dt (curl H^{n+3/2} - 4 pi <J>^{n+3/2}),
 *    <J>^{n+3/2} = J^{n+3/2}, or (J^{n+1} + J^{n+2}) / 2 in paper mode
 *  9 H^{n+2}   = H(B^{n+2}, D^{n+2})
 * 10 D^{n+5/2} = D^{n+3/2} + dt (curl H^{n+2} - 4 pi J^{n+2}),
 *    J^{n+2} = 1.5 J^{n+3/2} - 0.5 J^{n+1/2} (reading) or, in paper mode,
 *    the deposited J^{n+2}
 * ------------------------------------------------------------------------ */
static double *dup_zero(long n) { return (double *)calloc(n, sizeof(double)); }

void om_pic_step(const om_push_params *P, const om_grid *g, const double *ab,
                 om_fields *F, om_particles *p, const double *guess,
                 const int *force, int push_mode) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1, ntn = nth + 1;
  long sz[3] = {(long)nr * ntn, (long)nrn * nth, (long)nrn * ntn};
  long szB[3] = {(long)nrn * nth, (long)nr * ntn, (long)nr * nth};
  double dt = P->dt;
  double *T1[3], *T2[3], *E[3], *H[3], *Bnew[3], *Dnew[3], *Dh2[3], *J[3],
      *J2[3], *Bavg[3], *Davg[3];
  for (int c = 0; c < 3; ++c) {
    E[c] = dup_zero(sz[c]);
    H[c] = dup_zero(szB[c]);
    Bnew[c] = dup_zero(szB[c]);
    Dnew[c] = dup_zero(sz[c]);
    Dh2[c] = dup_zero(sz[c]);
    J[c] = dup_zero(sz[c]);
    J2[c] = dup_zero(sz[c]);
    Bavg[c] = dup_zero(szB[c]);
    Davg[c] = dup_zero(sz[c]);
    T1[c] = T2[c] = NULL;
  }
  (void)T1;
  (void)T2;
  double *rho_new = dup_zero(sz[2]);
  /* 1 */
  for (int c = 0; c < 3; ++c)
    for (long k = 0; k < sz[c]; ++k)
      Davg[c][k] = 0.5 * (F->Dh0[c][k] + F->Dh1[c][k]);
  om_compute_E(g, (const double *const *)Davg, (const double *const *)F->Bn,
               E);
  /* 2 */
  for (int c = 0; c < 3; ++c)
    for (long k = 0; k < szB[c]; ++k)
      Bavg[c][k] = 0.5 * (F->Bm[c][k] + F->Bn[c][k]);
  om_faraday(g, dt, ab, (const double *const *)Bavg, (const double *const *)E,
             F->Bh);
  /* 3 */
  om_compute_E(g, (const double *const *)F->Dh1, (const double *const *)F->Bh,
               E);
  /* 4 */
  om_faraday(g, dt, ab, (const double *const *)F->Bn, (const double *const *)E,
             Bnew);
  /* 5, 6 */
  if (push_mode == 0 && p && p->n > 0) {
    double *G[6];
    for (int c = 0; c < 3; ++c) {
      G[c] = dup_zero(sz[c]);
      om_densitize(g, c, +1, F->Dh1[c], G[c]);
      G[3 + c] = dup_zero(szB[c]);
      om_densitize(g, 3 + c, +1, F->Bh[c], G[3 + c]);
    }
    long n = p->n;
    double *o[3], *qw = dup_zero(n);
    int *mode = (int *)calloc(n, sizeof(int));
    for (int c = 0; c < 3; ++c) o[c] = dup_zero(n);
    memcpy(o[0], p->r, n * sizeof(double));
    memcpy(o[1], p->th, n * sizeof(double));
    memcpy(o[2], p->ph, n * sizeof(double));
    int *was_alive = (int *)calloc(n, sizeof(int));
    for (long k = 0; k < n; ++k) was_alive[k] = p->flags[k] & OM_ALIVE;
    om_push(P, g, (const double *const *)G, p, guess, force);
    for (long k = 0; k < n; ++k) {
      qw[k] = (p->qm[k] > 0 ? 1.0 : (p->qm[k] < 0 ? -1.0 : 0.0)) * p->w[k];
      mode[k] = was_alive[k] && (p->flags[k] & OM_ALIVE);
    }
    if (P->deposit_mode == OM_DEPOSIT_PAPER)
      om_deposit_paper(g, n, p->r, p->th, p->ur, p->uth, p->uph, qw, mode,
                       rho_new, J[0], J[1], J[2]);
    else
      om_deposit(g, dt, n, o[0], o[1], o[2], p->r, p->th, p->ph, qw, mode,
                 rho_new, J[0], J[1], J[2]);
    for (int c = 0; c < 6; ++c) free(G[c]);
    for (int c = 0; c < 3; ++c) free(o[c]);
    free(qw);
    free(mode);
    free(was_alive);
  }
  /* 7 */
  om_compute_H(g, (const double *const *)F->Bh, (const double *const *)F->Dh1,
               H);
  /* 8: the conserving current is J^{n+3/2} itself; the paper's current is
   * J^{n+2} at the new positions, averaged with J^{n+1}                   */
  const int paper = P->deposit_mode == OM_DEPOSIT_PAPER;
  for (int c = 0; c < 3; ++c)
    for (long k = 0; k < sz[c]; ++k)
      J2[c][k] = paper ? 0.5 * (J[c][k] + F->Jprev[c][k]) : J[c][k];
  om_ampere(g, dt, ab, (const double *const *)F->Dn, (const double *const *)H,
            (const double *const *)J2, Dnew);
  /* 9 */
  om_compute_H(g, (const double *const *)Bnew, (const double *const *)Dnew, H);
  /* 10 */
  for (int c = 0; c < 3; ++c)
    for (long k = 0; k < sz[c]; ++k)
      J2[c][k] = paper ? J[c][k] : 1.5 * J[c][k] - 0.5 * F->Jprev[c][k];
  om_ampere(g, dt, ab, (const double *const *)F->Dh1, (const double *const *)H,
            (const double *const *)J2, Dh2);
  /* rotate the time levels */
  for (int c = 0; c < 3; ++c) {
    memcpy(F->Bm[c], F->Bn[c], szB[c] * sizeof(double));
    memcpy(F->Bn[c], Bnew[c], szB[c] * sizeof(double));
    memcpy(F->Dn[c], Dnew[c], sz[c] * sizeof(double));
    memcpy(F->Dh0[c], F->Dh1[c], sz[c] * sizeof(double));
    memcpy(F->Dh1[c], Dh2[c], sz[c] * sizeof(double));
    memcpy(F->Jprev[c], J[c], sz[c] * sizeof(double));
  }
  memcpy(F->rho, rho_new, sz[2] * sizeof(double));
  for (int c = 0; c < 3; ++c) {
    free(E[c]);
    free(H[c]);
    free(Bnew[c]);
    free(Dnew[c]);
    free(Dh2[c]);
    free(J[c]);
    free(J2[c]);
    free(Bavg[c]);
    free(Davg[c]);
  }
  free(rho_new);
}

/* ------------------------------------------------------------------------
 * Diagnostics.
 * Gauss residual at interior nodes, eq. m1 in densitized form:
 *   div_h(sqrt(g) D) - 4 pi sqrt(g) rho  (0 on the boundary nodes).
 * div B at cell centres (eq. m2).  Poynting luminosity through the sphere
 * r_i (eq. Pbz): P = (1/2) sum_j (E_th H_ph - E_ph H_th) dth at theta_{j+1/2}.
 * ------------------------------------------------------------------------ */
void om_gauss_residual(const om_grid *g, const double *const *D,
                       const double *rho_d, double *out) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  for (int j = 0; j <= nth; ++j)
    for (int i = 0; i <= nr; ++i) {
      if (i == 0 || i == nr || j == 0 || j == nth) {
        out[IDX(nrn, i, j)] = 0.0;
        continue;
      }
      double a = g->a;
      double fr = om_sqrtg(a, g->rh[i], g->tn[j]) * D[0][IDX(nr, i, j)] -
                  om_sqrtg(a, g->rh[i - 1], g->tn[j]) * D[0][IDX(nr, i - 1, j)];
      double ft = om_sqrtg(a, g->rn[i], g->th[j]) * D[1][IDX(nrn, i, j)] -
                  om_sqrtg(a, g->rn[i], g->th[j - 1]) * D[1][IDX(nrn, i, j - 1)];
      out[IDX(nrn, i, j)] = fr / (g->rh[i] - g->rh[i - 1]) + ft / g->dth -
                            4.0 * M_PI * rho_d[IDX(nrn, i, j)];
    }
}

void om_div_B(const om_grid *g, const double *const *B, double *out) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  for (int j = 0; j < nth; ++j)
    for (int i = 0; i < nr; ++i) {
      double a = g->a;
      double fr = om_sqrtg(a, g->rn[i + 1], g->th[j]) * B[0][IDX(nrn, i + 1, j)] -
                  om_sqrtg(a, g->rn[i], g->th[j]) * B[0][IDX(nrn, i, j)];
      double ft = om_sqrtg(a, g->rh[i], g->tn[j + 1]) * B[1][IDX(nr, i, j + 1)] -
                  om_sqrtg(a, g->rh[i], g->tn[j]) * B[1][IDX(nr, i, j)];
      out[IDX(nr, i, j)] = fr / (g->rn[i + 1] - g->rn[i]) + ft / g->dth;
    }
}

void om_poynting(const om_grid *g, const double *const *D,
                 const double *const *B, double *out) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  double *E[3], *H[3];
  long sz[3] = {(long)nr * (nth + 1), (long)nrn * nth, (long)nrn * (nth + 1)};
  long szB[3] = {(long)nrn * nth, (long)nr * (nth + 1), (long)nr * nth};
  for (int c = 0; c < 3; ++c) {
    E[c] = dup_zero(sz[c]);
    H[c] = dup_zero(szB[c]);
  }
  om_compute_E(g, D, B, E);
  om_compute_H(g, B, D, H);
  for (int i = 0; i <= nr; ++i) {
    double sum = 0.0;
    int i0 = i > 0 ? i - 1 : -1, i1 = i < nr ? i : -1;
    for (int j = 0; j < nth; ++j) {
      double s = om_sqrtg(g->a, g->rn[i], g->th[j]);
      double Et = E[1][IDX(nrn, i, j)];
      /* H_phi from the half radii, E_phi from the nodes j, j+1, H_theta
       * from the four surrounding (i+-1/2, j or j+1) points; all by
       * densitized averages */
      double Hp = 0.0, Ht = 0.0;
      int k = 0;
      if (i0 >= 0) Hp += om_sqrtg(g->a, g->rh[i0], g->th[j]) * H[2][IDX(nr, i0, j)], ++k;
      if (i1 >= 0) Hp += om_sqrtg(g->a, g->rh[i1], g->th[j]) * H[2][IDX(nr, i1, j)], ++k;
      Hp /= (k * s);
      double Ep = 0.5 * (om_sqrtg(g->a, g->rn[i], g->tn[j]) * E[2][IDX(nrn, i, j)] +
                         om_sqrtg(g->a, g->rn[i], g->tn[j + 1]) * E[2][IDX(nrn, i, j + 1)]) /
                  s;
      k = 0;
      for (int jj = j; jj <= j + 1; ++jj) {
        if (i0 >= 0) Ht += om_sqrtg(g->a, g->rh[i0], g->tn[jj]) * H[1][IDX(nr, i0, jj)], ++k;
        if (i1 >= 0) Ht += om_sqrtg(g->a, g->rh[i1], g->tn[jj]) * H[1][IDX(nr, i1, jj)], ++k;
      }
      Ht /= (k * s);
      sum += (Et * Hp - Ep * Ht) * g->dth;
    }
    out[i] = 0.5 * sum;
  }
  for (int c = 0; c < 3; ++c) {
    free(E[c]);
    free(H[c]);
  }
}

/* ------------------------------------------------------------------------
 * Initial data.
 * Wald (App. B.1): every component sampled from the closed form at its own
 * Yee point.  Split monopole (App. B.2): flux function
 * Psi = 4 B0 zeta(theta) (1 - cos theta), zeta = (2/pi) atan(zeta0 (theta -
 * pi/2)); B^r = dPsi/dtheta / sqrt(g) taken as the difference of Psi over
 * the cell edge so that the discrete div B vanishes; B^theta = B^phi = 0,
 * and D = -beta x B / alpha = 0 for a radial B.
 * ------------------------------------------------------------------------ */
void om_wald_grid(const om_grid *g, double B0, double af, double *const *D,
                  double *const *B) {
  for (int c = 0; c < 6; ++c) {
    int nR, nT;
    om_comp_shape(g, c, &nR, &nT);
    double *A = c < 3 ? D[c] : B[c - 3];
    for (int j = 0; j < nT; ++j)
      for (int i = 0; i < nR; ++i) {
        double d[3], b[3];
        om_wald_fields_spin(g->a, af, B0, comp_r(g, c, i), comp_t(g, c, j), d,
                            b);
        A[IDX(nR, i, j)] = c < 3 ? d[c] : b[c - 3];
      }
  }
}

static double psi_sm(double B0, double zeta0, double th) {
  double zeta = 2.0 / M_PI * atan(zeta0 * (th - 0.5 * M_PI));
  return 4.0 * B0 * zeta * (1.0 - cos(th));
}

void om_split_monopole_grid(const om_grid *g, double B0, double zeta0,
                            double *const *D, double *const *B) {
  int nr = g->nr, nth = g->nth, nrn = nr + 1;
  for (int c = 0; c < 3; ++c) {
    int nR, nT;
    om_comp_shape(g, c, &nR, &nT);
    memset(D[c], 0, sizeof(double) * nR * nT);
    om_comp_shape(g, 3 + c, &nR, &nT);
    memset(B[c], 0, sizeof(double) * nR * nT);
  }
  for (int j = 0; j < nth; ++j) {
    double dpsi = psi_sm(B0, zeta0, g->tn[j + 1]) - psi_sm(B0, zeta0, g->tn[j]);
    for (int i = 0; i <= nr; ++i)
      B[0][IDX(nrn, i, j)] =
          dpsi / (g->dth * om_sqrtg(g->a, g->rn[i], g->th[j]));
  }
}
