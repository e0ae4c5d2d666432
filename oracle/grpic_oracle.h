/*
 * grpic_oracle.h -- reference (test-only) CPU implementation of the GRPIC
 * particle hot path of Meringolo & Rezzolla, "FPIC: a new Particle-In-Cell
 * code for stationary and axisymmetric black-hole spacetimes"
 * (arXiv:2602.07452).
 *
 * THIS IS TEST INFRASTRUCTURE.  It is plain, slow, FP64 C written from the
 * paper so that the GPU library can be checked against it.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no source with the GPU library.
 *
 * Conventions (M = 1, G = c = 1):
 *   particle state z = (r, theta, phi, u_r, u_theta, u_phi): contravariant
 *   position, covariant four-velocity (paper Sec. 2.2).
 *   Grid: N_r x N_theta cells; node radii r_i = r_in exp(i dlnr), i=0..N_r,
 *   dlnr = ln(r_out/r_in)/N_r; half radii r_{i+1/2} = sqrt(r_i r_{i+1});
 *   theta_j = theta0 + j dth, dth = (pi - 2 theta0)/N_theta; theta_{j+1/2}
 *   the midpoints.
 *   Yee positions (Sec. 2.1, Fig. 1): D^r,J^r,E_r,B^theta,H_theta at
 *   (i+1/2, j) ["hn"]; D^theta,J^theta,E_theta,B^r,H_r at (i, j+1/2) ["nh"];
 *   D^phi,J^phi,E_phi,rho at (i, j) ["nn"]; B^phi,H_phi at (i+1/2, j+1/2)
 *   ["hh"].  Arrays are r-fastest: index = jT * nR + iR.
 *   Component order for 6-field arrays: D^r, D^theta, D^phi, B^r, B^theta,
 *   B^phi.
 *   "Densitized" arrays hold sqrt(gamma) * F at the component's position.
 */
#ifndef GRPIC_ORACLE_H
#define GRPIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- pointwise spacetime (App. A) ------------------------------------- */
/* out[13] = alpha, beta^r, g_rr, g_thth, g_phph, g_rph, gi_rr, gi_thth,
 *           gi_phph, gi_rph, sqrt(gamma), xi, rho^2                         */
void om_metric(double a, double r, double th, double *out);
/* out[12] = d_r,d_th of alpha, beta^r, gi_rr, gi_thth, gi_phph, gi_rph      */
void om_metric_deriv(double a, double r, double th, double *out);
/* q[6] = divided differences [f(x1) - f(x0)] / (x1^k - x0^k), f = alpha,
 * beta^r, gamma^rr, gamma^thth, gamma^phph, gamma^rph; x0, x1 differ only in
 * coordinate k (0 = r, 1 = theta); evaluated without cancellation           */
void om_metric_divdiff(double a, int k, double r0, double t0, double r1,
                       double t1, double *q);
/* e = alpha Gamma - beta^r u_r  (eq. Ham with A_0 dropped)                  */
double om_energy(double a, const double *z);
/* equations of motion (eqs. p1, p2, O1, O2) at fields D^i, B^i             */
void om_rhs(double a, double qm, const double *z, const double *D,
            const double *B, double *f);

/* ---- Wald field (Sec. 3.1.3, App. B.1) --------------------------------- */
void om_wald_fields(double a, double B0, double r, double th, double *D,
                    double *B);
/* the potential of eq. Amu taken with spin af in the spacetime of spin a
 * (af = 0: the Schwarzschild-Wald start of Sec. 3.3, E_i = 0)             */
void om_wald_fields_spin(double a, double af, double B0, double r, double th,
                         double *D, double *B);
/* A[4] = A_0 (form used for the conserved energy), A_r, A_theta, A_phi     */
void om_wald_potential(double a, double B0, double r, double th, double *A);

/* ---- grid ---------------------------------------------------------------*/
typedef struct om_grid om_grid;
om_grid *om_grid_new(double a, int nr, int nth, double r_in, double r_out,
                     double th0);
void om_grid_free(om_grid *g);
/* copies rn[nr+1], rh[nr], tn[nth+1], th[nth]                               */
void om_grid_coords(const om_grid *g, double *rn, double *rh, double *tn,
                    double *th);
/* component c (0..5 for D^r..B^phi, 6 = rho/J^phi nodes) sizes              */
void om_comp_shape(const om_grid *g, int c, int *nR, int *nT);
/* multiply (dir=+1) or divide (dir=-1) by sqrt(gamma) at component c's
 * positions                                                                 */
void om_densitize(const om_grid *g, int c, int dir, const double *in,
                  double *out);

/* ---- gather (R16: metric-weighted bilinear) ---------------------------- */
void om_gather(const om_grid *g, const double *const *G, double r, double th,
               double *D, double *B);

/* ---- particles ----------------------------------------------------------*/
enum { OM_RK4 = 0, OM_IMR = 1, OM_HAM = 2, OM_HYB1 = 3, OM_HYB2 = 4 };
enum { OM_GUESS_PLAIN = 0, OM_GUESS_RK4 = 1, OM_GUESS_EXTERNAL = 2 };
enum { OM_FIELDS_NONE = 0, OM_FIELDS_GRID = 1, OM_FIELDS_WALD = 2 };
enum { OM_DEPOSIT_CONSERVING = 0, OM_DEPOSIT_PAPER = 1 };
enum { OM_SOLVER_PICARD = 0, OM_SOLVER_NEWTON = 1 };
enum {
  OM_ALIVE = 1,
  OM_IMPLICIT = 2,
  OM_NOCONV = 4,
  OM_REMOVED = 8,
  OM_REFLECTED = 16,
  OM_NONFINITE = 32 /* non-finite state after the step (with OM_REMOVED) */
};

typedef struct {
  double a, dt;
  int pusher, guess;
  double thr;       /* hybrid threshold                                    */
  double tol;       /* implicit stopping tolerance                        */
  int kmax;         /* implicit iteration cap                              */
  int field_kind;   /* OM_FIELDS_*                                         */
  double B0;        /* analytic Wald strength (field_kind == WALD)         */
  double r_min, r_max; /* particles outside are removed                   */
  double th_lo, th_hi; /* reflecting edges; th_lo < 0 disables            */
  double ham_eps;   /* |dx| below which Ham-DG uses analytic derivatives   */
  double dt_impl;   /* step of the implicit scheme (0: dt); Table 2 pairs a
                       Delta t_RK4 with a larger Delta t_Ham               */
  double t_end;     /* with particle clocks: steps are clipped to end at
                       t_end and particles that reached it stay (0: none) */
  int deposit_mode; /* OM_DEPOSIT_CONSERVING or OM_DEPOSIT_PAPER (pic step) */
  int solver;       /* implicit midpoint: OM_SOLVER_PICARD or _NEWTON      */
} om_push_params;

typedef struct {
  long n;
  double *r, *th, *ph, *ur, *uth, *uph;
  double *qm;   /* charge-to-mass ratio (+1, -1 or 0)                      */
  double *w;    /* macro weight                                            */
  double *H0;   /* initial energy (neutral criterion)                      */
  double *herr; /* criterion value after the last step                     */
  int *flags;   /* OM_ALIVE | ...                                          */
  int *iters;   /* implicit iterations of the last step (0 = explicit)     */
  double *crit; /* RK4 trial criterion of the last step (NaN if none)      */
  double *t;    /* each particle's own time, advanced by the step it took
                   (NULL: no clocks, every step is dt)                     */
} om_particles;

/* one step of every alive particle.  G: 6 densitized field arrays (only for
 * OM_FIELDS_GRID).  guess: n*6 (OM_GUESS_EXTERNAL) or NULL.  force: NULL or
 * per particle -1 (none) / 0 (force explicit) / 1 (force implicit).       */
void om_push(const om_push_params *P, const om_grid *g,
             const double *const *G, om_particles *p, const double *guess,
             const int *force);

/* single-particle building blocks, exposed for the pins                    */
void om_step_rk4(const om_push_params *P, const om_grid *g,
                 const double *const *G, double qm, const double *z,
                 double *out, double *Wq);
int om_step_imr(const om_push_params *P, const om_grid *g,
                const double *const *G, double qm, const double *z,
                const double *guess, double *out, double *Wq);
int om_step_ham(const om_push_params *P, const double *z,
                const double *guess, double *out);

/* ---- deposit (Sec. 2.3) -------------------------------------------------*/
/* W[4] for nodes (p,q),(p+1,q),(p,q+1),(p+1,q+1) of node cell (p,q).
 * flat != 0 replaces sqrt(gamma) by 1 (test hook).                         */
void om_dep_weights(const om_grid *g, double r, double th, int p, int q,
                    int flat, double *W);
/* accumulate (+=) densitized sqrt(g) rho (at new positions), sqrt(g) J^r,
 * J^theta, J^phi over the move (r0,th0,ph0) -> (r1,th1,ph1).  mode[k]: 0
 * skip, 1 deposit.                                                          */
void om_deposit(const om_grid *g, double dt, long n, const double *r0,
                const double *th0, const double *ph0, const double *r1,
                const double *th1, const double *ph1, const double *qw,
                const int *mode, double *rho, double *Jr, double *Jth,
                double *Jph);
/* the paper's own current (Sec. 2.3) at the pushed state, every component
 * on its own Yee subgrid; densitized like om_deposit (adds to the arrays)  */
void om_deposit_paper(const om_grid *g, long n, const double *r,
                      const double *th, const double *ur, const double *uth,
                      const double *uph, const double *qw, const int *mode,
                      double *rho, double *Jr, double *Jth, double *Jph);
/* divergence cleaning (Sec. 2.4, eq. phi): `iters` Jacobi sweeps from phi = 0
 * on the Gauss residual of D (plain values, corrected in place) and the
 * densitized rho; phi_out (nodes, may be NULL) receives phi              */
void om_div_clean(const om_grid *g, double *const *D, const double *rho_d,
                  int iters, double *phi_out);

/* ---- Maxwell solver (Sec. 2.1) ------------------------------------------*/
/* non-densitized D^i, B^i; E_i, H_i are grid fields at their Yee points    */
void om_compute_E(const om_grid *g, const double *const *D,
                  const double *const *B, double *const *E);
void om_compute_H(const om_grid *g, const double *const *B,
                  const double *const *D, double *const *H);
/* Bout = damp * (Bin - dt curl E)                                          */
void om_faraday(const om_grid *g, double dt, const double *absorber,
                const double *const *Bin, const double *const *E,
                double *const *Bout);
/* Dout = damp * (Din + dt (curl H - 4 pi J)); Jd densitized               */
void om_ampere(const om_grid *g, double dt, const double *absorber,
               const double *const *Din, const double *const *H,
               const double *const *Jd, double *const *Dout);
/* absorber[3] = r_abs, chi0, lambda (chi0 = 0 disables)                    */

typedef struct {
  double *Dn[3];    /* D^{n+1}                                            */
  double *Dh0[3];   /* D^{n+1/2}                                          */
  double *Dh1[3];   /* D^{n+3/2}                                          */
  double *Bm[3];    /* B^{n}                                              */
  double *Bn[3];    /* B^{n+1}                                            */
  double *Bh[3];    /* B^{n+3/2} (rebuilt each step)                      */
  double *Jprev[3]; /* densitized J^{n+1/2}                               */
  double *rho;      /* densitized rho^{n+1}                               */
} om_fields;

/* one full PIC step, sub-steps 1-10 of Sec. 2.1.  push_mode: 0 = push and
 * deposit, 1 = fields only (no particles).                                 */
void om_pic_step(const om_push_params *P, const om_grid *g,
                 const double *absorber, om_fields *F, om_particles *p,
                 const double *guess, const int *force, int push_mode);

/* ---- diagnostics ---------------------------------------------------------*/
void om_gauss_residual(const om_grid *g, const double *const *D,
                       const double *rho_d, double *out);
void om_div_B(const om_grid *g, const double *const *B, double *out);
void om_poynting(const om_grid *g, const double *const *D,
                 const double *const *B, double *out);

/* ---- pair injection (Sec. 3.3) -------------------------------------------*/
typedef struct {
  double r0, r1;   /* cells whose centre radius lies in [r0, r1]            */
  double mult;     /* inject while n < mult * n_GJ                          */
  double density;  /* an injected pair adds density * n_GJ                  */
  double theta;    /* Maxwell-Juettner temperature of the injected momenta  */
  uint64_t seed;
} om_inject_params;
long om_inject(const om_grid *g, const om_inject_params *I, uint64_t event,
               const double *Br, const double *Bt, long n, const double *r,
               const double *th, const double *qm, const double *w,
               const int *flags, long room, double *out);

/* ---- initial data (App. B, Sec. 3.3) -------------------------------------*/
void om_wald_grid(const om_grid *g, double B0, double af, double *const *D,
                  double *const *B);
void om_split_monopole_grid(const om_grid *g, double B0, double zeta0,
                            double *const *D, double *const *B);
double om_uniform(uint64_t seed, uint64_t counter);
/* kind 0: Schwarzschild orbits; 1: shell, isotropic |u|~U[0,p0];
 * 2: shell, Maxwell-Juettner pairs at temperature p0.                      */
void om_init_particles(int kind, double a, uint64_t seed, long n, double r0,
                       double r1, double t0, double t1, double p0, double w,
                       om_particles *p);

/* ---- MLP guess network (project extension) -------------------------------*/
/* parameters packed: W1[64][14] b1[64] W2[64][64] b2[64] W3[6][64] b3[6]   */
#define OM_MLP_NPARAM 5510
void om_mlp_forward(const double *theta, long n, const double *X, double *Y);
double om_mlp_loss_grad(const double *theta, long n, const double *X,
                        const double *T, double *grad);

#ifdef __cplusplus
}
#endif
#endif
