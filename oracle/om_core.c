/*
 * om_core.c -- reference oracle (TEST INFRASTRUCTURE ONLY): Kerr-Schild
 * 3+1 metric, particle equations of motion, Wald field and the particle
 * pushers of arXiv:2602.07452, in plain FP64 C.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "om_internal.h"

/* ------------------------------------------------------------------------
 * Metric, App. A (eqs. gsf, gsf_2, det).  M = 1.
 * gamma_{r phi} is printed with a^2; only -a xi sin^2(theta) is the inverse
 * of the printed gamma^{ij} (reading adopted), beta^theta = beta^phi = 0.
 * sqrt(gamma) uses |sin(theta)| so that it is the positive root.
 * ------------------------------------------------------------------------ */
void om_metric(double a, double r, double th, double *o) {
  double s = sin(th), c = cos(th);
  double rho2 = r * r + a * a * c * c;
  double xi = 1.0 + 2.0 * r / rho2;
  o[0] = 1.0 / sqrt(xi);          /* alpha = xi^{-1/2}                    */
  o[1] = (xi - 1.0) / xi;         /* beta^r                               */
  o[2] = xi;                      /* gamma_rr                             */
  o[3] = rho2;                    /* gamma_thth                           */
  o[4] = s * s * (rho2 + a * a * xi * s * s); /* gamma_phph               */
  o[5] = -a * xi * s * s;         /* gamma_rph                            */
  o[6] = a * a * s * s / rho2 + 1.0 / xi; /* gamma^rr                     */
  o[7] = 1.0 / rho2;              /* gamma^thth                           */
  o[8] = 1.0 / (rho2 * s * s);    /* gamma^phph                           */
  o[9] = a / rho2;                /* gamma^rph                            */
  o[10] = rho2 * sqrt(xi) * fabs(s); /* sqrt(gamma) = rho^2 xi^1/2 sin    */
  o[11] = xi;
  o[12] = rho2;
}

double om_sqrtg(double a, double r, double th) {
  double s = sin(th), c = cos(th);
  double rho2 = r * r + a * a * c * c;
  double xi = 1.0 + 2.0 * r / rho2;
  return rho2 * sqrt(xi) * fabs(s);
}

/* Analytic r- and theta-derivatives of the metric functions that enter the
 * gravitational acceleration (eq. O1), "computed analytically at the
 * position of the particle" (Sec. 2.2).                                    */
void om_metric_deriv(double a, double r, double th, double *o) {
  double s = sin(th), c = cos(th);
  double rho2 = r * r + a * a * c * c;
  double rho4 = rho2 * rho2;
  double xi = 1.0 + 2.0 * r / rho2;
  double drho2[2] = {2.0 * r, -2.0 * a * a * s * c};
  double dxi[2];
  dxi[0] = 2.0 / rho2 - 2.0 * r * drho2[0] / rho4;
  dxi[1] = -2.0 * r * drho2[1] / rho4;
  for (int k = 0; k < 2; ++k) {
    /* alpha = xi^{-1/2} */
    o[0 + k] = -0.5 * dxi[k] / (xi * sqrt(xi));
    /* beta^r = 1 - 1/xi */
    o[2 + k] = dxi[k] / (xi * xi);
    /* gamma^rr = a^2 s^2 / rho^2 + 1/xi */
    double d_s2 = (k == 0) ? 0.0 : 2.0 * s * c;
    o[4 + k] = a * a * d_s2 / rho2 - a * a * s * s * drho2[k] / rho4 -
               dxi[k] / (xi * xi);
    /* gamma^thth = 1/rho^2 */
    o[6 + k] = -drho2[k] / rho4;
    /* gamma^phph = 1/(rho^2 s^2) */
    double den = rho2 * s * s;
    double dden = drho2[k] * s * s + rho2 * d_s2;
    o[8 + k] = -dden / (den * den);
    /* gamma^rph = a/rho^2 */
    o[10 + k] = -a * drho2[k] / rho4;
  }
}

/* e = alpha Gamma - beta^r u_r; Gamma = sqrt(1 + gamma^ij u_i u_j)       */
double om_energy(double a, const double *z) {
  double m[13];
  om_metric(a, z[0], z[1], m);
  double ur = z[3], ut = z[4], up = z[5];
  double q = m[6] * ur * ur + m[7] * ut * ut + m[8] * up * up +
             2.0 * m[9] * ur * up;
  return m[0] * sqrt(1.0 + q) - m[1] * ur;
}

/* Equations of motion, eqs. p1, p2, O1, O2: f = (dx^i/dt, du_i/dt).
 * eta_ijk is the Levi-Civita symbol with eta_{r theta phi} = +1.          */
void om_rhs(double a, double qm, const double *z, const double *D,
            const double *B, double *f) {
  double m[13], d[12];
  om_metric(a, z[0], z[1], m);
  om_metric_deriv(a, z[0], z[1], d);
  double alpha = m[0], betar = m[1];
  double ur = z[3], ut = z[4], up = z[5];
  /* u^i = gamma^ij u_j */
  double Ur = m[6] * ur + m[9] * up;
  double Ut = m[7] * ut;
  double Up = m[9] * ur + m[8] * up;
  double Gam = sqrt(1.0 + ur * Ur + ut * Ut + up * Up);
  f[0] = alpha * Ur / Gam - betar;
  f[1] = alpha * Ut / Gam;
  f[2] = alpha * Up / Gam;
  double Ag[2];
  for (int k = 0; k < 2; ++k) {
    double quad = ur * ur * d[4 + k] + ut * ut * d[6 + k] +
                  up * up * d[8 + k] + 2.0 * ur * up * d[10 + k];
    Ag[k] = -Gam * d[0 + k] + ur * d[2 + k] - alpha / (2.0 * Gam) * quad;
  }
  /* lowered D: D_i = gamma_ij D^j */
  double Dr = m[2] * D[0] + m[5] * D[2];
  double Dt = m[3] * D[1];
  double Dp = m[5] * D[0] + m[4] * D[2];
  /* eta_ijk u^j B^k */
  double cr = Ut * B[2] - Up * B[1];
  double ct = Up * B[0] - Ur * B[2];
  double cp = Ur * B[1] - Ut * B[0];
  double sg = m[10];
  f[3] = Ag[0] + qm * alpha * (Dr + sg * cr / Gam);
  f[4] = Ag[1] + qm * alpha * (Dt + sg * ct / Gam);
  f[5] = qm * alpha * (Dp + sg * cp / Gam);
}

/* (q/m) E_i dx^i/dt with E_i = alpha D_i + sqrt(g) eta_ijk beta^j B^k
 * (eq. Ei): the rate of change of e along the motion.                      */
static double om_power(double a, double qm, const double *z, const double *D,
                       const double *B, const double *f) {
  if (qm == 0.0) return 0.0;
  double m[13];
  om_metric(a, z[0], z[1], m);
  double alpha = m[0], betar = m[1], sg = m[10];
  double Dr = m[2] * D[0] + m[5] * D[2];
  double Dt = m[3] * D[1];
  double Dp = m[5] * D[0] + m[4] * D[2];
  double Er = alpha * Dr;
  double Et = alpha * Dt - sg * betar * B[2];
  double Ep = alpha * Dp + sg * betar * B[1];
  return qm * (Er * f[0] + Et * f[1] + Ep * f[2]);
}

/* ------------------------------------------------------------------------
 * Wald field, App. B.1 (eqs. wald1-wald6) with the readings: E_i = +d_i A_0
 * (so E_theta carries a single factor a), D_i from eq. Ei, D^j = gamma^ij
 * D_i.  A_0 in the form used for the conserved energy (Sec. 3.1.3), A_phi
 * with the factor B0, A_r from eq. Amu.
 *
 * The potential of eq. Amu may be taken with a spin af of its own while the
 * spacetime has spin a (Sec. 3.3 starts a Kerr hole with the af = 0 field):
 * the curl eta^ijk d_j A_k and E_i = d_i A_0 are those of the af solution,
 * and sqrt(gamma), alpha, beta, gamma^ij those of the spacetime.  af = a is
 * the Wald vacuum solution itself; af = 0 has A_0 = 0, so E_i = 0 and
 * D = -beta x B / alpha.
 * ------------------------------------------------------------------------ */
void om_wald_fields_spin(double a, double af, double B0, double r, double th,
                         double *D, double *B) {
  double m[13];
  om_metric(a, r, th, m);
  double s = sin(th), c = cos(th);
  double a2 = af * af, r2 = r * r;
  double rho2 = r2 + a2 * c * c, rho4 = rho2 * rho2, sg = m[10];
  /* eta^ijk d_j A_k of the af potential, divided by the spacetime's sqrt(g) */
  B[0] = B0 / sg * (r2 + a2 - 2.0 * r + 2.0 * r * (r2 * r2 - a2 * a2) / rho4) *
         s * c;
  B[1] = -B0 / sg * (r + a2 * (1.0 + c * c) * (2.0 * r2 - rho2) / rho4) * s *
         s;
  B[2] = -B0 / sg * (2.0 * af * r * (a2 - r2) / rho4 - af) * s * c;
  double Er = B0 * af * (1.0 + c * c) * (a2 * c * c - r2) / rho4;
  double Et = B0 * af * 2.0 * r * (a2 - r2) / rho4 * s * c;
  double Ep = 0.0;
  double alpha = m[0], betar = m[1];
  double Dr_l = Er / alpha;
  double Dt_l = (Et + sg * betar * B[2]) / alpha;
  double Dp_l = (Ep - sg * betar * B[1]) / alpha;
  D[0] = m[6] * Dr_l + m[9] * Dp_l;
  D[1] = m[7] * Dt_l;
  D[2] = m[9] * Dr_l + m[8] * Dp_l;
}

void om_wald_fields(double a, double B0, double r, double th, double *D,
                    double *B) {
  om_wald_fields_spin(a, a, B0, r, th, D, B);
}

void om_wald_potential(double a, double B0, double r, double th, double *A) {
  double s = sin(th), c = cos(th);
  double rho2 = r * r + a * a * c * c;
  double xi = 1.0 + 2.0 * r / rho2;
  A[0] = B0 * a * r * (1.0 + c * c) / rho2;
  A[1] = 0.5 * B0 * (-a * xi * s * s + 4.0 * a * r / rho2);
  A[2] = 0.0;
  A[3] = 0.5 * B0 * s * s * (r * r + a * a - 2.0 * a * a * r * (1.0 + c * c) / rho2);
}

/* ------------------------------------------------------------------------
 * Field source seen by the pusher.
 * ------------------------------------------------------------------------ */
static void fields_at(const om_push_params *P, const om_grid *g,
                      const double *const *G, double r, double th, double *D,
                      double *B) {
  if (P->field_kind == OM_FIELDS_GRID) {
    om_gather(g, G, r, th, D, B);
  } else if (P->field_kind == OM_FIELDS_WALD) {
    om_wald_fields(P->a, P->B0, r, th, D, B);
  } else {
    D[0] = D[1] = D[2] = B[0] = B[1] = B[2] = 0.0;
  }
}

/* f = F(z) with the fields re-gathered at z's position; *pw = power.       */
static void eval_rhs(const om_push_params *P, const om_grid *g,
                     const double *const *G, double qm, const double *z,
                     double *f, double *pw) {
  double D[3], B[3];
  fields_at(P, g, G, z[0], z[1], D, B);
  om_rhs(P->a, qm, z, D, B, f);
  if (pw) *pw = om_power(P->a, qm, z, D, B, f);
}

/* ------------------------------------------------------------------------
 * RK4 (Sec. 2.2.1): four stages, fields re-gathered at each stage position
 * (reading: fields frozen at the push time level).  Wq = the same stage
 * quadrature applied to the power (q/m) E_i dx^i/dt.
 * ------------------------------------------------------------------------ */
void om_step_rk4(const om_push_params *P, const om_grid *g,
                 const double *const *G, double qm, const double *z,
                 double *out, double *Wq) {
  double dt = P->dt;
  double k1[6], k2[6], k3[6], k4[6], y[6], p1, p2, p3, p4;
  eval_rhs(P, g, G, qm, z, k1, &p1);
  for (int i = 0; i < 6; ++i) y[i] = z[i] + 0.5 * dt * k1[i];
  eval_rhs(P, g, G, qm, y, k2, &p2);
  for (int i = 0; i < 6; ++i) y[i] = z[i] + 0.5 * dt * k2[i];
  eval_rhs(P, g, G, qm, y, k3, &p3);
  for (int i = 0; i < 6; ++i) y[i] = z[i] + dt * k3[i];
  eval_rhs(P, g, G, qm, y, k4, &p4);
  for (int i = 0; i < 6; ++i)
    out[i] = z[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  if (Wq) *Wq = dt / 6.0 * (p1 + 2.0 * p2 + 2.0 * p3 + p4);
}

/* Stopping rule shared by both implicit schemes: the largest change of any
 * component, relative to max(|z_j|, 1), is at most tol.                    */
static int converged(const double *znew, const double *zold, double tol) {
  double m = 0.0;
  for (int i = 0; i < 6; ++i) {
    double sc = fabs(znew[i]) > 1.0 ? fabs(znew[i]) : 1.0;
    double d = fabs(znew[i] - zold[i]) / sc;
    if (d > m) m = d;
  }
  return m <= tol;
}

/* ------------------------------------------------------------------------
 * Implicit midpoint rule (Sec. 2.2.2, eq. imr1) solved by fixed-point
 * (Picard) iteration  z[k] = z^n + dt F((z^n + z[k-1])/2)  from a guess.
 * Returns the iteration count (negative if the cap was reached).
 * ------------------------------------------------------------------------ */
/* Newton's method on the same equation, the solver the paper names (the
 * Picard iteration above is the default reading):
 *   G(y) = y - z - dt F((z + y)/2),  J = I - (dt/2) dF/dx at the midpoint,
 * dF/dx by forward differences with steps h_j = 2^-26 max(|m_j|, 1) (the
 * step actually taken, (m_j + h_j) - m_j, divides), y <- y - J^{-1} G(y)
 * by Gaussian elimination with partial pivoting.  Same stopping test and
 * cap as the Picard iteration; Wq from the last midpoint evaluation.      */
static int imr_newton(const om_push_params *P, const om_grid *g,
                      const double *const *G, double qm, const double *z,
                      double *zk, double *Wq) {
  double pw = 0.0;
  for (int k = 1; k <= P->kmax; ++k) {
    double m[6], f0[6], A[6][7];
    for (int i = 0; i < 6; ++i) m[i] = 0.5 * (z[i] + zk[i]);
    eval_rhs(P, g, G, qm, m, f0, &pw);
    for (int j = 0; j < 6; ++j) {
      double mj[6], fj[6], pj;
      memcpy(mj, m, sizeof(mj));
      double h = 0x1p-26 * (fabs(m[j]) > 1.0 ? fabs(m[j]) : 1.0);
      mj[j] = m[j] + h;
      h = mj[j] - m[j];
      eval_rhs(P, g, G, qm, mj, fj, &pj);
      for (int i = 0; i < 6; ++i)
        A[i][j] = (i == j ? 1.0 : 0.0) - 0.5 * P->dt * (fj[i] - f0[i]) / h;
    }
    for (int i = 0; i < 6; ++i) A[i][6] = -(zk[i] - z[i] - P->dt * f0[i]);
    for (int c = 0; c < 6; ++c) { /* elimination with partial pivoting */
      int piv = c;
      for (int i = c + 1; i < 6; ++i)
        if (fabs(A[i][c]) > fabs(A[piv][c])) piv = i;
      if (piv != c)
        for (int j = c; j < 7; ++j) {
          double t = A[c][j];
          A[c][j] = A[piv][j];
          A[piv][j] = t;
        }
      for (int i = c + 1; i < 6; ++i) {
        double l = A[i][c] / A[c][c];
        for (int j = c; j < 7; ++j) A[i][j] -= l * A[c][j];
      }
    }
    double dy[6], zn[6];
    for (int i = 5; i >= 0; --i) {
      double v = A[i][6];
      for (int j = i + 1; j < 6; ++j) v -= A[i][j] * dy[j];
      dy[i] = v / A[i][i];
    }
    for (int i = 0; i < 6; ++i) zn[i] = zk[i] + dy[i];
    int c = converged(zn, zk, P->tol);
    memcpy(zk, zn, sizeof(zn));
    if (c) {
      if (Wq) *Wq = P->dt * pw;
      return k;
    }
  }
  if (Wq) *Wq = P->dt * pw;
  return -P->kmax;
}

int om_step_imr(const om_push_params *P, const om_grid *g,
                const double *const *G, double qm, const double *z,
                const double *guess, double *out, double *Wq) {
  double zk[6], zm[6], f[6], zn[6], pw = 0.0;
  memcpy(zk, guess ? guess : z, sizeof(zk));
  if (P->solver == OM_SOLVER_NEWTON) {
    int it = imr_newton(P, g, G, qm, z, zk, Wq);
    memcpy(out, zk, sizeof(zk));
    return it;
  }
  for (int k = 1; k <= P->kmax; ++k) {
    for (int i = 0; i < 6; ++i) zm[i] = 0.5 * (z[i] + zk[i]);
    eval_rhs(P, g, G, qm, zm, f, &pw);
    for (int i = 0; i < 6; ++i) zn[i] = z[i] + P->dt * f[i];
    int c = converged(zn, zk, P->tol);
    memcpy(zk, zn, sizeof(zk));
    if (c) {
      memcpy(out, zk, sizeof(zk));
      if (Wq) *Wq = P->dt * pw;
      return k;
    }
  }
  memcpy(out, zk, sizeof(zk));
  if (Wq) *Wq = P->dt * pw;
  return -P->kmax;
}

/* ------------------------------------------------------------------------
 * Hamiltonian discrete-gradient scheme (Sec. 2.2.3, App. D) for geodesic
 * motion, H = alpha sqrt(1 + gamma^lm u_l u_m) - beta^r u_r.
 *   dx^i/dt = Dbar_{u_i} H,  du_i/dt = -Dbar_{x^i} H,
 * where Dbar is the mean over six variable orderings of the partial
 * difference quotients obtained by changing one variable at a time from
 * time level n to n+1 (reading of the garbled App. D: the three cyclic
 * orders r->theta->phi with x before u, and their time reverses).  Each
 * ordering telescopes, so H is conserved exactly up to round-off.
 * The u-quotients are rationalised exactly; the x-quotients use the exact
 * product split d(alpha Gamma) = <alpha> dGamma + <Gamma> dalpha with the
 * metric quotients df/dx evaluated as cancellation-free divided differences
 * (same value as the plain quotient in exact arithmetic); a quotient is
 * replaced by the analytic derivative at the midpoint when |dx| < eps
 * (App. D, last paragraph).
 * Variables: 0 r, 1 theta, 2 phi, 3 u_r, 4 u_theta, 5 u_phi.
 * ------------------------------------------------------------------------ */
static const int om_orders[6][6] = {
    {0, 3, 1, 4, 2, 5}, {1, 4, 2, 5, 0, 3}, {2, 5, 0, 3, 1, 4},
    {5, 2, 4, 1, 3, 0}, {3, 0, 5, 2, 4, 1}, {4, 1, 3, 0, 5, 2}};

static double gamma_of(const double *m, const double *y) {
  double ur = y[3], ut = y[4], up = y[5];
  return sqrt(1.0 + m[6] * ur * ur + m[7] * ut * ut + m[8] * up * up +
              2.0 * m[9] * ur * up);
}

/* Divided differences [f(x') - f(x)] / (x'^k - x^k) of the metric
 * functions alpha, beta^r, gamma^rr, gamma^thth, gamma^phph, gamma^rph between
 * two positions that differ only in coordinate k (0 = r, 1 = theta),
 * written without cancellation (identical to the plain quotient in exact
 * arithmetic, but accurate to rounding for any step):
 *   r:     d(rho^2) = r + r',        d(S) = r + r' + 2   (S = rho^2 + 2r)
 *   theta: d(cos^2) = -sin(t + t') sin(t' - t)/(t' - t) = -d(sin^2)
 * and d(1/g) = -d(g)/(g g'), d(g h) = g' d(h) + h d(g),
 * d(sqrt g) = d(g)/(sqrt g + sqrt g').                                      */
static double sinc(double x) {
  return fabs(x) < 1e-4 ? 1.0 - x * x / 6.0 : sin(x) / x;
}

void om_metric_divdiff(double a, int k, double r0, double t0, double r1,
                       double t1, double *q) {
  double A = a * a;
  double c0 = cos(t0), c1 = cos(t1), s0 = sin(t0), s1 = sin(t1);
  double C0 = c0 * c0, C1 = c1 * c1, Ss0 = s0 * s0, Ss1 = s1 * s1;
  double P0 = r0 * r0 + A * C0, P1 = r1 * r1 + A * C1; /* rho^2 */
  double S0 = P0 + 2.0 * r0, S1 = P1 + 2.0 * r1;
  double dP, dS, dSs, dC;
  if (k == 0) {
    dP = r0 + r1;
    dS = r0 + r1 + 2.0;
    dSs = 0.0;
    dC = 0.0;
  } else {
    dC = -sin(t0 + t1) * sinc(t1 - t0);
    dSs = -dC;
    dP = A * dC;
    dS = A * dC;
  }
  double d_irho2 = -dP / (P0 * P1);
  /* 1/xi = rho^2 / S */
  double d_ixi = (dP * S0 - P0 * dS) / (S0 * S1);
  double ixi0 = P0 / S0, ixi1 = P1 / S1;
  double al0 = sqrt(ixi0), al1 = sqrt(ixi1);
  q[0] = d_ixi / (al0 + al1);               /* alpha = sqrt(1/xi)        */
  q[1] = -d_ixi;                            /* beta^r = 1 - 1/xi         */
  q[2] = A * (Ss1 * d_irho2 + dSs / P0) + d_ixi; /* gamma^rr             */
  q[3] = d_irho2;                           /* gamma^thth                */
  double dPS = P1 * dSs + Ss0 * dP;         /* d(rho^2 sin^2)            */
  q[4] = -dPS / (P0 * Ss0 * P1 * Ss1);      /* gamma^phph                */
  q[5] = a * d_irho2;                       /* gamma^rph                 */
}

/* [H(y1) - H(y0)] / (y1[k] - y0[k]) for y0, y1 differing only in slot k   */
static double ham_quotient(double a, double eps, int k, const double *y0,
                           const double *y1) {
  if (k == 2) return 0.0; /* H does not depend on phi (axisymmetry)        */
  if (k >= 3) {
    double m[13];
    om_metric(a, y0[0], y0[1], m);
    double G0 = gamma_of(m, y0), G1 = gamma_of(m, y1);
    double num;
    if (k == 3)
      num = m[6] * (y1[3] + y0[3]) + 2.0 * m[9] * y0[5];
    else if (k == 4)
      num = m[7] * (y1[4] + y0[4]);
    else
      num = m[8] * (y1[5] + y0[5]) + 2.0 * m[9] * y0[3];
    double q = m[0] * num / (G0 + G1);
    if (k == 3) q -= m[1];
    return q;
  }
  double m0[13], m1[13];
  om_metric(a, y0[0], y0[1], m0);
  om_metric(a, y1[0], y1[1], m1);
  double G0 = gamma_of(m0, y0), G1 = gamma_of(m1, y1);
  double dx = y1[k] - y0[k];
  double qa, qb, qg[4];
  if (fabs(dx) >= eps) {
    double q[6];
    om_metric_divdiff(a, k, y0[0], y0[1], y1[0], y1[1], q);
    qa = q[0];
    qb = q[1];
    for (int i = 0; i < 4; ++i) qg[i] = q[2 + i];
  } else {
    double d[12];
    double rm = (k == 0) ? 0.5 * (y0[0] + y1[0]) : y0[0];
    double tm = (k == 1) ? 0.5 * (y0[1] + y1[1]) : y0[1];
    om_metric_deriv(a, rm, tm, d);
    qa = d[0 + k];
    qb = d[2 + k];
    for (int i = 0; i < 4; ++i) qg[i] = d[4 + 2 * i + k];
  }
  double ur = y0[3], ut = y0[4], up = y0[5];
  double quad = qg[0] * ur * ur + qg[1] * ut * ut + qg[2] * up * up +
                2.0 * qg[3] * ur * up;
  return 0.5 * (G0 + G1) * qa + 0.5 * (m0[0] + m1[0]) * quad / (G0 + G1) -
         ur * qb;
}

static void ham_gradient(double a, double eps, const double *zn,
                         const double *zp, double *grad) {
  for (int i = 0; i < 6; ++i) grad[i] = 0.0;
  for (int o = 0; o < 6; ++o) {
    double y[6], y1[6];
    memcpy(y, zn, sizeof(y));
    for (int s = 0; s < 6; ++s) {
      int k = om_orders[o][s];
      memcpy(y1, y, sizeof(y));
      y1[k] = zp[k];
      grad[k] += ham_quotient(a, eps, k, y, y1) / 6.0;
      memcpy(y, y1, sizeof(y));
    }
  }
}

int om_step_ham(const om_push_params *P, const double *z, const double *guess,
                double *out) {
  double zk[6], zn[6], grad[6];
  memcpy(zk, guess ? guess : z, sizeof(zk));
  for (int k = 1; k <= P->kmax; ++k) {
    ham_gradient(P->a, P->ham_eps, z, zk, grad);
    zn[0] = z[0] + P->dt * grad[3];
    zn[1] = z[1] + P->dt * grad[4];
    zn[2] = z[2] + P->dt * grad[5];
    zn[3] = z[3] - P->dt * grad[0];
    zn[4] = z[4] - P->dt * grad[1];
    zn[5] = z[5] - P->dt * grad[2];
    int c = converged(zn, zk, P->tol);
    memcpy(zk, zn, sizeof(zk));
    if (c) {
      memcpy(out, zk, sizeof(zk));
      return k;
    }
  }
  memcpy(out, zk, sizeof(zk));
  return -P->kmax;
}

/* ------------------------------------------------------------------------
 * Hybrid switch (Sec. 3.1.2) and the per-particle step.
 * Neutral particles: Ht = |H - H_0| / |H_0| (cumulative).  Charged
 * particles: per-step energy-budget residual |e' - e - W| / |e|, W the
 * scheme's own quadrature of (q/m) E_i dx^i/dt (reading: no exactly
 * conserved H in grid fields).  Hyb2 bounds the value, Hyb1 its relative
 * rate (value - previous) / (dt max(previous, 2^-52)).  A rejected RK4 step
 * is redone implicitly: Ham-DG for neutral, IMR for charged particles.
 * ------------------------------------------------------------------------ */
static double crit_value(const om_push_params *P, double qm, double H0,
                         const double *z, const double *zn, double Wq) {
  if (qm == 0.0) return fabs(om_energy(P->a, zn) - H0) / fabs(H0);
  double e0 = om_energy(P->a, z);
  return fabs(om_energy(P->a, zn) - e0 - Wq) / fabs(e0);
}

/* Steps of their own length (Sec. 3.1.2 with Table 2): the explicit trial
 * advances by dt, the implicit scheme by dt_impl; with particle clocks each
 * particle's time grows by the step it took, and with t_end both lengths
 * are clipped to the time left, so every particle ends exactly at t_end and
 * then stays (flags ALIVE, no iterations, state and criterion unchanged). */
static void push_one(const om_push_params *P0, const om_grid *g,
                     const double *const *G, om_particles *p, long k,
                     const double *guess, int force) {
  int fl = p->flags[k];
  if (!(fl & OM_ALIVE)) return;
  fl &= OM_ALIVE;
  p->crit[k] = NAN;
  om_push_params Pe = *P0, Pi = *P0; /* explicit, implicit step lengths */
  Pi.dt = P0->dt_impl > 0.0 ? P0->dt_impl : P0->dt;
  int end_e = 0, end_i = 0; /* the step reaches t_end                      */
  if (p->t && P0->t_end > 0.0) {
    double left = P0->t_end - p->t[k];
    if (!(left > 0.0)) {
      p->flags[k] = OM_ALIVE;
      p->iters[k] = 0;
      return;
    }
    if (left <= Pe.dt) Pe.dt = left, end_e = 1;
    if (left <= Pi.dt) Pi.dt = left, end_i = 1;
  }
  const om_push_params *P = &Pe;
  double z[6] = {p->r[k], p->th[k], p->ph[k], p->ur[k], p->uth[k], p->uph[k]};
  double qm = p->qm[k], out[6], trial[6], Wq = 0.0;
  int it = 0;
  double herr_new;
  int implicit = 0;
  if (P->pusher == OM_RK4) {
    om_step_rk4(P, g, G, qm, z, out, &Wq);
  } else if (P->pusher == OM_IMR || P->pusher == OM_HAM) {
    implicit = 1;
  } else {
    om_step_rk4(P, g, G, qm, z, trial, &Wq);
    double v = crit_value(P, qm, p->H0[k], z, trial, Wq);
    double c = v;
    if (P->pusher == OM_HYB1) {
      double prev = p->herr[k];
      double den = prev > 0x1p-52 ? prev : 0x1p-52;
      c = (v - prev) / (P->dt * den);
    }
    p->crit[k] = c;
    int accept = (force == 0) || (force != 1 && c < P->thr);
    if (accept) {
      memcpy(out, trial, sizeof(out));
    } else {
      implicit = 1;
    }
  }
  if (implicit) {
    const double *gs = z;
    if (P->guess == OM_GUESS_RK4 && P->pusher >= OM_HYB1) gs = trial;
    if (P->guess == OM_GUESS_EXTERNAL && guess) gs = guess + 6 * k;
    if (qm == 0.0 && P->pusher != OM_IMR)
      it = om_step_ham(&Pi, z, gs, out), Wq = 0.0;
    else
      it = om_step_imr(&Pi, g, G, qm, z, gs, out, &Wq);
    fl |= OM_IMPLICIT;
    if (it < 0) fl |= OM_NOCONV, it = -it;
  }
  herr_new = crit_value(P, qm, p->H0[k], z, out, Wq);
  /* a state that is no number takes the particle out of the run; then the
   * particle boundary conditions (Sec. 2.5) */
  int finite = 1;
  for (int i = 0; i < 6; ++i) finite = finite && isfinite(out[i]);
  if (!finite) {
    fl = OM_REMOVED | OM_NONFINITE;
  } else if (out[0] < P->r_min || out[0] > P->r_max) {
    fl = (fl & ~OM_ALIVE) | OM_REMOVED;
  } else if (P->th_lo >= 0.0) {
    if (out[1] < P->th_lo) {
      out[1] = 2.0 * P->th_lo - out[1];
      out[4] = -out[4];
      fl |= OM_REFLECTED;
    } else if (out[1] > P->th_hi) {
      out[1] = 2.0 * P->th_hi - out[1];
      out[4] = -out[4];
      fl |= OM_REFLECTED;
    }
  }
  p->r[k] = out[0];
  p->th[k] = out[1];
  p->ph[k] = out[2];
  p->ur[k] = out[3];
  p->uth[k] = out[4];
  p->uph[k] = out[5];
  p->herr[k] = herr_new;
  p->flags[k] = fl;
  p->iters[k] = it;
  if (p->t) {
    /* a step clipped to the time left lands on t_end exactly */
    if (implicit ? end_i : end_e)
      p->t[k] = P0->t_end;
    else
      p->t[k] += implicit ? Pi.dt : Pe.dt;
  }
}

void om_push(const om_push_params *P, const om_grid *g,
             const double *const *G, om_particles *p, const double *guess,
             const int *force) {
#pragma omp parallel for schedule(dynamic, 64)
  for (long k = 0; k < p->n; ++k)
    push_one(P, g, G, p, k, guess, force ? force[k] : -1);
}
