/*
 * grpic.h -- C ABI of the MI355X GRPIC particle hot path.
 *
 * Method: C. Meringolo & L. Rezzolla, "FPIC: a new Particle-In-Cell code for
 * stationary and axisymmetric black-hole spacetimes", arXiv:2602.07452.
 * The library advances charged or neutral test particles and (optionally)
 * the electromagnetic field of a Kerr black hole (mass M = 1, spin a) in
 * spherical Kerr-Schild coordinates (r, theta) with axisymmetric fields:
 * field gather, particle push (RK4, implicit midpoint, Hamiltonian
 * discrete-gradient scheme, and the Hyb1/Hyb2 hybrid switch), charge and
 * current deposit, and the two-chain leapfrog Maxwell update (Sec. 2).
 *
 * Conventions
 *  - Every entry point returns 0 on success or a negative GRPIC_E_* code;
 *    grpic_last_error() gives a message.  No entry point aborts.
 *  - The context owns all device memory (allocated in grpic_create and
 *    grpic_*_particles); host buffers belong to the caller and are copied
 *    synchronously on the context's stream unless stated otherwise.
 *  - Particle state z = (r, theta, phi, u_r, u_theta, u_phi): contravariant
 *    position and covariant four-velocity per unit mass (Sec. 2.2), FP64.
 *    qm is the charge-to-mass ratio q/m in {+1, -1, 0}; w the macro weight.
 *  - Grid (Sec. 2.1, Fig. 1): N_r x N_theta cells, r_i = r_in exp(i dlnr),
 *    dlnr = ln(r_out / r_in) / N_r, half radii r_{i+1/2} = sqrt(r_i r_{i+1});
 *    theta_j = theta0 + j dth, dth = (pi - 2 theta0) / N_theta.
 *  - Field arrays exchanged through the ABI are FP32, "densitized"
 *    (sqrt(gamma) * F at the component's Yee point), r-fastest, with shapes
 *      D^r, J^r, B^theta : N_r     x (N_theta+1)   at (i+1/2, j)
 *      D^th, J^th, B^r   : (N_r+1) x N_theta       at (i, j+1/2)
 *      D^phi, J^phi, rho : (N_r+1) x (N_theta+1)   at (i, j)
 *      B^phi             : N_r     x N_theta       at (i+1/2, j+1/2)
 *    (row = theta index, column = r index).
 */
#ifndef GRPIC_H
#define GRPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------- */
#define GRPIC_OK 0
#define GRPIC_E_INVALID (-1)   /* bad argument or configuration          */
#define GRPIC_E_CFL (-2)       /* dt above the Courant limit of the grid */
#define GRPIC_E_OOM (-3)       /* device allocation failed               */
#define GRPIC_E_HIP (-4)       /* HIP runtime error                      */
#define GRPIC_E_STATE (-5)     /* call not valid in the current state    */
#define GRPIC_E_NODEVICE (-6)  /* no usable GPU                          */

/* ---- enumerations ------------------------------------------------------*/
enum grpic_pusher {
  GRPIC_PUSH_RK4 = 0,  /* explicit RK4, Sec. 2.2.1                         */
  GRPIC_PUSH_IMR = 1,  /* implicit midpoint rule, Sec. 2.2.2                */
  GRPIC_PUSH_HAM = 2,  /* discrete-gradient scheme (neutral), Sec. 2.2.3;
                          charged particles fall back to the IMR             */
  GRPIC_PUSH_HYB1 = 3, /* RK4, redone implicitly when the relative growth
                          rate of the energy violation exceeds the threshold
                          (Sec. 3.1.2, "Hyb1")                               */
  GRPIC_PUSH_HYB2 = 4  /* RK4, redone implicitly when the energy violation
                          itself exceeds the threshold ("Hyb2")              */
};
enum grpic_guess {
  GRPIC_GUESS_PLAIN = 0, /* implicit iteration starts from z^n             */
  GRPIC_GUESS_RK4 = 1,   /* hybrid: starts from the rejected RK4 result    */
  GRPIC_GUESS_MLP = 2    /* starts from the learned guess network          */
};
enum grpic_field_mode {
  GRPIC_FIELDS_NONE = 0,   /* geodesic motion, no grid                     */
  GRPIC_FIELDS_STATIC = 1, /* gather + push in fixed grid fields           */
  GRPIC_FIELDS_EVOLVE = 2  /* full PIC step: Maxwell + gather + push +
                              deposit                                      */
};
enum grpic_solver {
  GRPIC_SOLVER_PICARD = 0, /* fixed-point iteration of eq. imr1 (default)  */
  GRPIC_SOLVER_NEWTON = 1  /* Newton's method (Sec. 2.2.2): forward-
                              difference Jacobian of the midpoint map,
                              Gaussian elimination with partial pivoting   */
};
enum grpic_deposit_mode {
  GRPIC_DEPOSIT_CONSERVING = 0, /* charge-conserving face fluxes over the
                                   move (default); J^{n+3/2} in sub-step 8,
                                   1.5 J^{n+3/2} - 0.5 J^{n+1/2} in 10      */
  GRPIC_DEPOSIT_PAPER = 1       /* the paper's current (Sec. 2.3) at the
                                   pushed state: each component on its own
                                   Yee subgrid with that subgrid's volume
                                   weights, carried by dx^i/dt (the grid
                                   current alpha j - rho beta); sub-step 8
                                   uses (J^{n+1} + J^{n+2}) / 2, 10 J^{n+2};
                                   not charge-conserving: use cleaning     */
};
/* field time levels (Sec. 2.1 sub-steps; the push reads DH1 and BH) */
enum grpic_level {
  GRPIC_LEVEL_DN = 0,  /* D^{n+1}                                          */
  GRPIC_LEVEL_DH0 = 1, /* D^{n+1/2}                                        */
  GRPIC_LEVEL_DH1 = 2, /* D^{n+3/2}                                        */
  GRPIC_LEVEL_BM = 3,  /* B^{n}                                            */
  GRPIC_LEVEL_BN = 4,  /* B^{n+1}                                          */
  GRPIC_LEVEL_BH = 5,  /* B^{n+3/2} (rebuilt every step)                   */
  GRPIC_LEVEL_J = 6,   /* J^{n+3/2} comps 0..2, rho^{n+2} comp 3 (after a
                          step: the current step's deposit)                */
  GRPIC_LEVEL_JPREV = 7 /* J^{n+1/2}, rho^{n+1}                            */
};
/* particle flags */
#define GRPIC_FLAG_ALIVE 1
#define GRPIC_FLAG_IMPLICIT 2  /* last step taken by the implicit scheme   */
#define GRPIC_FLAG_NOCONV 4    /* implicit iteration hit kmax              */
#define GRPIC_FLAG_REMOVED 8   /* left the domain in the last step         */
#define GRPIC_FLAG_REFLECTED 16 /* reflected at a theta edge last step     */
#define GRPIC_FLAG_NONFINITE 32 /* the step gave a non-finite state: the
                                   particle was removed (with REMOVED)     */

/* ---- configuration ---------------------------------------------------- */
typedef struct grpic_config {
  double a;              /* spin a_* in [0, 1)                              */
  int nr, nth;           /* grid cells (ignored for GRPIC_FIELDS_NONE);     *
                          * at least 2 and at most 2^22 - 2 each, with     *
                          * (nr + 1)(nth + 1) <= 2^30 (else                *
                          * GRPIC_E_INVALID)                               */
  double r_in, r_out;    /* radial extent of the grid                       */
  double theta0;         /* theta edges at theta0, pi - theta0 (Sec. 2.5)   */
  double dt;             /* time step (0 with a grid: half the Courant
                            limit, see grpic_cfl_dt)                       */
  int field_mode;        /* enum grpic_field_mode                           */
  int pusher;            /* enum grpic_pusher                               */
  int guess;             /* enum grpic_guess                                */
  double hyb_threshold;  /* Hyb1: rate bound; Hyb2: value bound             */
  double tol;            /* implicit stopping tolerance (max relative change
                            per component, relative to max(|z|,1))          */
  int kmax;              /* implicit iteration cap (<= 255)                 */
  double ham_eps;        /* |dx| below which the DG scheme uses analytic
                            derivatives (App. D: 1e-10)                    */
  double r_abs, chi0, lambda_abs; /* absorbing layer, eqs. abs0-abs2;
                                     chi0 = 0 disables                      */
  double r_remove_in, r_remove_out; /* particles outside are removed        */
  int reflect;           /* reflect particles at the theta edges (1) or not */
  long max_particles;    /* capacity                                        */
  int sort_every;        /* re-sort particles by tile every N steps (0: only
                            when particles are loaded)                      */
  int tile_r, tile_th;   /* tile size in cells for sorting / deposit bins  */
  int block;             /* threads per block for particle kernels (0 = 256)*/
  int persistent_waves;  /* waves per CU of the implicit-queue kernel (0=8) */
  int push_waves_per_simd; /* register budget of the explicit push: 0 = the
                              compiler's choice, 4 = at most 128 VGPRs so that
                              4 waves fit per SIMD (set by grpic_autotune)  */
  /* Steps of their own length (Sec. 3.1.2, Table 2), field_mode NONE only:
   * every particle keeps its own time; the explicit RK4 trial advances it by
   * dt, the implicit scheme by dt_implicit; with t_end > 0 both are clipped
   * to the time left (a clipped step lands on t_end exactly) and particles
   * that reached t_end are no longer advanced (flags ALIVE, iters 0).     */
  double dt_implicit;    /* step of the implicit scheme (0: dt)            */
  double t_end;          /* end time of the particle clocks (0: none)      */
  /* field_mode EVOLVE only: */
  int deposit_mode;      /* enum grpic_deposit_mode                        */
  int clean_every;       /* divergence cleaning after every N-th step (0:
                            never; Sec. 2.4 uses 25)                       */
  int clean_iters;       /* Jacobi sweeps per cleaning (Sec. 2.4: 500)     */
  /* Pair injection (Sec. 3.3), field_mode EVOLVE only; see grpic_inject.  */
  int inj_every;         /* inject after every N-th step (0: never)        */
  double inj_r0, inj_r1; /* cells whose centre radius lies in [r0, r1]     */
  double inj_mult;       /* inject while n < inj_mult * n_GJ (Sec. 3.3: 3) */
  double inj_density;    /* an injected pair adds inj_density * n_GJ (5)   */
  double inj_theta;      /* Maxwell-Juettner temperature (0.5)             */
  uint64_t inj_seed;     /* seed of the injection draws                    */
  int solver;            /* implicit midpoint: enum grpic_solver           */
} grpic_config;

/* Fill *cfg with defaults (no grid, RK4, dt = 0.01, tol 1e-13, kmax 50).  */
int grpic_config_default(grpic_config *cfg);

typedef struct grpic_ctx grpic_ctx;

/* Validate cfg, allocate grid/field storage on the current HIP device and
 * tabulate the metric at every Yee point (Sec. 2.1, "computed only
 * initially").  Errors: GRPIC_E_INVALID (ranges), GRPIC_E_CFL (dt above the
 * grid's Courant limit for field_mode EVOLVE), GRPIC_E_OOM, GRPIC_E_HIP,
 * GRPIC_E_NODEVICE.  *out is NULL on failure.                             */
int grpic_create(const grpic_config *cfg, grpic_ctx **out);
/* The context's configuration as it is now: dt resolved, and the launch
 * settings grpic_autotune may have changed.                               */
int grpic_get_config(grpic_ctx *ctx, grpic_config *out);
void grpic_destroy(grpic_ctx *ctx);
/* Message of the last failing call on ctx (ctx may be NULL: last failure
 * of grpic_create).  Owned by the library.                                */
const char *grpic_last_error(const grpic_ctx *ctx);
/* Largest stable dt of the field solver on this grid (Courant limit).    */
int grpic_cfl_dt(const grpic_config *cfg, double *dt_out);

/* Run all following work on the given hipStream_t (NULL: the context's own
 * stream).  The caller keeps ownership of the stream.                     */
int grpic_set_stream(grpic_ctx *ctx, void *hip_stream);
int grpic_sync(grpic_ctx *ctx);

/* Host copies of the grid coordinates: rn[N_r+1], rh[N_r], tn[N_th+1],
 * th[N_th].  Any pointer may be NULL.                                     */
int grpic_grid_coords(grpic_ctx *ctx, double *rn, double *rh, double *tn,
                      double *th);

/* ---- fields ----------------------------------------------------------- */
/* Wald field of strength B0 on every D and B level (App. B.1, with
 * E_i = +d_i A_0 and D_i from eq. Ei); J and rho are cleared.  a_field is
 * the spin in the potential of eq. Amu, 0 <= a_field < 1: a_field = cfg.a
 * gives the Wald vacuum solution of the spacetime; a_field = 0 gives the
 * start of Sec. 3.3 (the Schwarzschild Wald field laid on the Kerr
 * spacetime: grid E_i = 0, D = -beta x B / alpha).  The densitized B is the
 * curl of that potential, alpha, beta, gamma those of cfg.a.
 * GRPIC_E_INVALID for a non-finite B0 or a_field out of range.            */
int grpic_set_fields_wald(grpic_ctx *ctx, double B0, double a_field);
/* Split monopole (App. B.2): flux function 4 B0 zeta(theta)(1 - cos theta),
 * zeta = (2/pi) atan(zeta0 (theta - pi/2)); D = 0.                        */
int grpic_set_fields_split_monopole(grpic_ctx *ctx, double B0, double zeta0);
/* Copy one densitized component (comp 0..2 = D^r,D^th,D^ph for D levels,
 * B^r,B^th,B^ph for B levels; J levels: 0..2 = J^r,J^th,J^ph, 3 = rho)
 * from / to a host FP32 array of the component's shape.                   */
int grpic_set_field(grpic_ctx *ctx, int level, int comp, const float *host);
int grpic_get_field(grpic_ctx *ctx, int level, int comp, float *host);

/* ---- particles -------------------------------------------------------- */
enum grpic_init_kind {
  GRPIC_INIT_ORBITS = 0,    /* Schwarzschild (a = 0) test orbits: r ~
                               U[r0,r1], theta ~ U[t0,t1], circular orbit
                               constants, even ids circular, odd ids with a
                               u_r offset ~ U[-p0, p0]; neutral             */
  GRPIC_INIT_SHELL_ISO = 1, /* uniform in proper volume over the shell,
                               isotropic FIDO momenta |u| ~ U[0, p0];
                               q/m = +1 (even ids), -1 (odd ids)            */
  GRPIC_INIT_SHELL_MJ = 2   /* e+/e- pairs sharing a position uniform in
                               proper volume, Maxwell-Juettner FIDO momenta
                               at temperature p0                            */
};
typedef struct grpic_init_spec {
  int kind;              /* enum grpic_init_kind                            */
  long n;                /* number of particles (<= max_particles)          */
  uint64_t seed;         /* SplitMix64 seed (counter-based, per particle)   */
  double r0, r1, t0, t1; /* sampling shell                                  */
  double p0;             /* momentum scale / temperature / u_r spread       */
  double w;              /* macro weight of every particle                  */
} grpic_init_spec;
/* Sample the initial particles on the device, compute H_0, sort them by
 * tile and deposit rho at the initial positions (for EVOLVE).            */
int grpic_init_particles(grpic_ctx *ctx, const grpic_init_spec *spec);
/* Load n particles from host arrays (ids 0..n-1 in array order).  H0 and
 * herr may be NULL (H0 = e(z^0) = alpha Gamma - beta^r u_r, herr = 0).    */
int grpic_load_particles(grpic_ctx *ctx, long n, const double *r,
                         const double *th, const double *ph, const double *ur,
                         const double *uth, const double *uph,
                         const double *qm, const double *w, const double *H0,
                         const double *herr);
/* Copy the particles back in id order.  Any pointer may be NULL.  flags
 * and iters describe the last step: iters is the implicit iteration count
 * (0 for an explicit step); after a restart from z^n (learned guess) it is
 * kmax plus the restart's count, capped at 255.                           */
int grpic_get_particles(grpic_ctx *ctx, long n, double *r, double *th,
                        double *ph, double *ur, double *uth, double *uph,
                        double *qm, double *w, double *H0, double *herr,
                        int32_t *flags, int32_t *iters);
int grpic_num_particles(grpic_ctx *ctx, long *n);
/* Copy the particles' own times (field_mode NONE) in id order into t[n];
 * they start at 0 when particles are loaded.  GRPIC_E_STATE with a grid. */
int grpic_get_times(grpic_ctx *ctx, long n, double *t);
/* Copy the particles with the given ids (m <= 2^24 distinct ids in
 * [0, n)): rec receives 10 doubles per id (r, theta, phi, u_r, u_theta,
 * u_phi, q/m, w, H0, herr), flags and iters (may be NULL) one int each.
 * For checks of large runs without copying every particle.  Allocates a
 * temporary id map of n ints on the device.  GRPIC_E_INVALID for ids out of
 * range or repeated.                                                       */
int grpic_sample_particles(grpic_ctx *ctx, long m, const long *ids,
                           double *rec, int32_t *flags, int32_t *iters);

/* ---- state snapshot (checkpoint / resume) ------------------------------ */
/* A snapshot is one host byte block: a grpic_state_header, then every
 * field level (D^{n+1}, D^{n+1/2}, D^{n+3/2}, B^n, B^{n+1}, B^{n+3/2}: 3
 * FP32 components each; J, J_prev: 4 each; in level and component order,
 * each of its own shape) when the context has a grid, then the particles in
 * storage order (r, theta, phi, u_r, u_theta, u_phi, H0, herr, w as FP64;
 * q/m as int8; flags, iters as uint8; id as uint32; with a grid the
 * deposit weights W1..W3 of the current position as uint32 fixed point
 * (round(W 2^31)) and the cell index as int32; without a grid the
 * particle times as FP64), then the
 * diagnostic counters.  Restoring it into a
 * context of the same grid, field mode and dt continues the run exactly as
 * the uninterrupted one (the deposit sums are order-independent).  The
 * learned-guess network is not part of it (grpic_mlp_get / grpic_mlp_set). */
typedef struct grpic_state_header {
  char magic[8];          /* "GRPICST" and a zero byte                      */
  int32_t version;        /* 2                                              */
  int32_t field_mode;     /* enum grpic_field_mode                          */
  int32_t nr, nth;        /* grid cells                                     */
  double a, r_in, r_out, theta0, dt;
  int64_t n;              /* particles                                      */
  int64_t steps;          /* steps taken since the particles were loaded    */
  double qw_max;          /* largest |q w| (the deposit's fixed-point unit) */
  int32_t has_neutral;    /* some particle has q/m = 0                      */
  int32_t reserved;
  uint64_t bytes;         /* size of the whole snapshot, header included    */
} grpic_state_header;
/* Size in bytes of a snapshot of the context as it is now.               */
int grpic_state_size(grpic_ctx *ctx, size_t *bytes);
/* Write the snapshot into host[0..bytes); GRPIC_E_INVALID if bytes is
 * smaller than grpic_state_size.  Synchronizes the context's stream.      */
int grpic_get_state(grpic_ctx *ctx, void *host, size_t bytes);
/* Replace the context's fields, particles, step count and counters by a
 * snapshot.  GRPIC_E_INVALID if the block is short, not a snapshot, or
 * taken on another grid (nr, nth, a, r_in, r_out, theta0), field mode or
 * dt, or holds more particles than max_particles.  Cached step graphs are
 * dropped.                                                                */
int grpic_set_state(grpic_ctx *ctx, const void *host, size_t bytes);

/* ---- stepping ---------------------------------------------------------- */
/* Advance nsteps steps, asynchronously on the context's stream.  One step
 * is the cycle of Sec. 2.1: with field_mode EVOLVE the Maxwell sub-steps
 * 1-4, the push of sub-step 5 (gather at every stage, RK4 of Sec. 2.2.1,
 * the hybrid switch of Sec. 3.1.2 and the implicit redo of Sec. 2.2.2 or
 * 2.2.3, particle boundaries of Sec. 2.5), the deposit of sub-step 6
 * (Sec. 2.3) and sub-steps 7-10; without a grid or with static fields the
 * push alone (no particles: the fields alone).  Errors: GRPIC_E_INVALID
 * for nsteps < 0, GRPIC_E_STATE with guess MLP and no network set (and no
 * sample collection running), GRPIC_E_HIP.                               */
int grpic_step(grpic_ctx *ctx, int nsteps);
/* Capture one step in a hipGraph and replay it for grpic_step (1) or go
 * back to eager launches (0).                                             */
int grpic_use_graph(grpic_ctx *ctx, int enable);

/* ---- diagnostics ------------------------------------------------------- */
#define GRPIC_HIST_BINS 64
typedef struct grpic_diag {
  long steps;            /* steps taken since load                          */
  long alive;            /* particles alive (counted from the particle
                            arrays when the diagnostics are read)          */
  long removed;          /* removed since load                              */
  long implicit_steps;   /* particle-steps taken implicitly (cumulative)    */
  long noconv;           /* implicit solves that hit kmax (cumulative)      */
  long reflected;        /* pole reflections (cumulative)                   */
  long iter_hist[GRPIC_HIST_BINS]; /* implicit iteration counts             */
  long herr_hist[GRPIC_HIST_BINS]; /* log10 energy-violation bins of the
                                      alive particles, the values their
                                      last step wrote (0 before the
                                      first): bin b holds values in
                                      [10^(b/2-30), 10^((b+1)/2-30)), bin
                                      0 also those below 1e-30            */
  long deposit_fallback; /* deposit blocks whose node box did not fit the
                            on-chip bins (cumulative)                      */
  long nonfinite;        /* particles removed for a non-finite state
                            (cumulative, also counted in removed)          */
  long deposit_outside;  /* particles deposited through global atomics
                            because they had left the node box planned for
                            their chunk at the last sort (cumulative)      */
} grpic_diag;
/* The counters above (synchronises the stream).  The energy violation is
 * the hybrid switch quantity of Sec. 3.1.2 (|H - H_0| / |H_0| for neutral
 * particles, the per-step energy-budget residual for charged ones).        */
int grpic_get_diagnostics(grpic_ctx *ctx, grpic_diag *out);
/* Grid diagnostics on the integer chain: max |Gauss residual| over interior
 * nodes (eq. m1, densitized), max |div B| (eq. m2) and the Poynting
 * luminosity P(r_i) of eq. Pbz at every node radius (pbz may be NULL).    */
int grpic_field_diagnostics(grpic_ctx *ctx, double *gauss_max,
                            double *divb_max, double *pbz);
/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc): the same results as grpic_field_diagnostics
 * without any device allocation or free.  Its scratch (the two maxima and
 * the N_r + 1 luminosities) is a static device array of fixed size that
 * every GPU running the library holds until the process ends; it is set up
 * by grpic_create on the context's device.  Limit: N_r <= 16384
 * (GRPIC_E_INVALID above).  Calls on one GPU share that array: the library
 * serialises its own calls (each clears the maxima, launches, copies the
 * results to the host outputs and synchronises the context's stream before
 * the next may start), so a call is not capturable in a graph, and work of
 * another process on the same GPU must not overlap it.  Errors as
 * grpic_field_diagnostics; GRPIC_E_STATE without a grid.                  */
int grpic_field_diagnostics_noalloc(grpic_ctx *ctx, double *gauss_max,
                                    double *divb_max, double *pbz);
/* Divergence cleaning now (Sec. 2.4, eq. phi), as clean_every does after a
 * step: on each D chain, iters Jacobi sweeps (FP64, from phi = 0, phi = 0 on
 * the boundary nodes) of div(sqrt(g) g^kk d_k phi) = G with G the
 * densitized Gauss residual at the interior nodes, then
 * sqrt(g) D^i -= sqrt(g) g^ij d_j phi (D^r, D^theta on their faces, D^phi
 * at interior nodes with the mean radial difference).  The integer chain
 * (GRPIC_LEVEL_DN) is cleaned against rho of the last deposit, the half
 * chain (GRPIC_LEVEL_DH1, half a step later) against 1.5 rho - 0.5 rho_prev.
 * Allocates the solver's buffers on first use (five FP64 node arrays).
 * GRPIC_E_STATE without field_mode EVOLVE; GRPIC_E_INVALID for iters < 1. */
int grpic_clean(grpic_ctx *ctx, int iters);

/* ---- pair injection (Sec. 3.3) ---------------------------------------- */
/* Inject now, as inj_every does after a step: every node cell whose centre
 * radius lies in [inj_r0, inj_r1] and whose plasma density n (the weights
 * of its charged particles over V_cell = 2 pi sqrt(g)(centre) dr dtheta)
 * is below inj_mult * n_GJ receives one co-located e+/e- pair, each
 * particle of weight inj_density * n_GJ * V_cell / 2, at a position
 * uniform in proper volume over the cell, with Maxwell-Juettner FIDO
 * momenta at inj_theta.  n_GJ = Omega_H |cos(theta) B^r - r sin(theta)
 * B^theta| / (4 pi) at the cell centre from the integer-chain B, Omega_H =
 * a / (2 r_+).  Cells are taken in index order (theta row, then radius)
 * while max_particles leaves room for a pair; the new particles take the
 * next ids.  Draws: SplitMix64 keyed by inj_seed + steps * 0x9E3779B97F4A7C15
 * (streams: cell index c for the position, 2c and 2c + 1 for the momenta).
 * *added (may be NULL) receives the number of particles added.
 * GRPIC_E_STATE without field_mode EVOLVE; GRPIC_E_INVALID for
 * non-positive inj_mult, inj_density or inj_theta.                        */
int grpic_inject(grpic_ctx *ctx, long *added);

/* ---- timing ----------------------------------------------------------- */
enum grpic_kernel_id {
  GRPIC_K_FIELDS = 0,   /* Maxwell sub-steps 1-4 and 7-10                  */
  GRPIC_K_PUSH = 1,     /* explicit pass: gather + RK4 + switch            */
  GRPIC_K_IMPLICIT = 2, /* implicit-queue pass                             */
  GRPIC_K_DEPOSIT = 3,  /* deposit + finalize                              */
  GRPIC_K_SORT = 4,     /* tile sort                                       */
  GRPIC_K_GUESS = 5,    /* learned guess                                   */
  GRPIC_K_CLEAN = 6,    /* divergence cleaning                             */
  GRPIC_K_COUNT = 7
};
/* Enable (1) or disable (0) HIP-event timing of each kernel group on the
 * context's stream; grpic_get_timings returns the summed milliseconds and
 * the number of timed launches per group since the last reset.            */
int grpic_enable_timing(grpic_ctx *ctx, int enable);
int grpic_get_timings(grpic_ctx *ctx, double *ms, long *count);
int grpic_reset_timings(grpic_ctx *ctx);

/* ---- autotuner (project extension, not in the paper) -------------------
 * Times the step under candidate launch settings and keeps the fastest, by
 * coordinate search: sort tile (tile_r x tile_th in {16x16, 32x16, 32x32,
 * 64x16, 64x32}; grid contexts), implicit-pass waves per CU {4, 8, 16, 32}
 * (implicit pushers), explicit-push waves per SIMD {0 = compiler choice, 4}.
 * Each candidate runs one untimed and trial_steps timed steps (no re-sort
 * inside a trial): the trials are real steps of the simulation, which
 * advances by them.  Results are identical for every setting (the deposit
 * is order-independent), only the speed changes.  Needs loaded particles
 * (GRPIC_E_STATE otherwise); trial_steps >= 1.                           */
typedef struct grpic_tune_result {
  int tile_r, tile_th;      /* chosen sort tile                          */
  int persistent_waves;     /* chosen implicit-pass waves per CU         */
  int push_waves_per_simd;  /* chosen explicit-push occupancy            */
  int trials;               /* settings timed                            */
  int steps;                /* simulation steps taken by the trials      */
  double ms_start;          /* ms per step of the starting setting       */
  double ms_best;           /* ms per step of the chosen setting         */
} grpic_tune_result;
int grpic_autotune(grpic_ctx *ctx, int trial_steps, grpic_tune_result *out);

/* ---- measured ceilings (measurement aid, not part of the method) --------
 * Times, on the context's device and stream, (i) a kernel of independent
 * FP64 fused multiply-adds on every compute unit, no memory traffic, giving
 * the achievable FP64 vector rate in TFLOP/s (an FMA counts 2 FLOP; the
 * best of 8 or 16 waves per SIMD and 8 or 16 chains per thread), and (ii) a
 * grid-stride copy of 16-byte elements between two 1 GiB buffers (read +
 * write counted), giving the streaming HBM rate in TB/s (the best of 4, 8
 * or 16 blocks per compute unit, cached or nontemporal accesses, and the
 * HIP runtime's device-to-device copy of the same buffers).  Each
 * setting is the mean of 10 launches after 2 warm-up launches.  Allocates and
 * frees 2 GiB of device memory (GRPIC_E_OOM if that fails); synchronises
 * the stream.  GRPIC_E_INVALID on a null pointer.                          */
int grpic_probe_peaks(grpic_ctx *ctx, double *fp64_fma_tflops, double *copy_tbs);

/* ---- learned implicit guess (project extension, not in the paper) -----
 * A 14 -> 64 -> 64 -> 6 GELU network gives the implicit pusher's first
 * iterate as  base + scale (.) net((x - mean) * inv_std),  where base is the
 * RK4 result for the hybrid pushers (which compute it anyway) and the Euler
 * step z^n + dt F(z^n) otherwise, and
 * x = (r, theta, phi, u_r, u_theta, u_phi, (q/m) D^r, (q/m) D^theta,
 * (q/m) D^phi, (q/m) B^r, (q/m) B^theta, (q/m) B^phi, alpha, beta^r) at
 * step n (fields gathered as in the push).
 * The iteration decides the result (Sec. 2.2.2), so the guess changes only
 * the number of iterations; a particle whose iteration from it does not
 * converge is restarted from z^n.  Selected with guess = GRPIC_GUESS_MLP.
 * Parameters are packed W1[64][14] b1[64] W2[64][64] b2[64] W3[6][64] b3[6]
 * (FP32 master values; weights are rounded to BF16, nearest even, for the
 * matrix-core products, which accumulate in FP32; biases stay FP32).      */
#define GRPIC_MLP_NPARAM 5510
#define GRPIC_MLP_NIN 14
#define GRPIC_MLP_NOUT 6

/* Load parameters (host arrays: theta[5510], mean[14], inv_std[14],
 * scale[6]); the context owns its device copy.  Returns GRPIC_E_INVALID on
 * a null pointer.                                                          */
int grpic_mlp_set(grpic_ctx *ctx, const float *theta, const float *mean,
                  const float *inv_std, const float *scale);
/* Copy the current parameters and normalisation to host arrays of the same
 * sizes.                                                                   */
int grpic_mlp_get(grpic_ctx *ctx, float *theta, float *mean, float *inv_std,
                  float *scale);

/* Training samples.  grpic_mlp_collect(ctx, max_rows > 0) allocates room
 * for max_rows samples and starts collecting: during each following step
 * every particle of the implicit queue adds one row, its raw features x
 * (14 FP32) and the target z^{n+1} - base of its converged iteration
 * (6 FP32), plus valid = 1 if the iteration converged; the iteration then
 * starts from the base.  Rows beyond max_rows are dropped.  max_rows = 0
 * stops collecting (samples are kept).                                    */
int grpic_mlp_collect(grpic_ctx *ctx, long max_rows);
int grpic_mlp_num_samples(grpic_ctx *ctx, long *n);
/* Copy the first n samples (X: n x 14, T: n x 6, valid: n; any may be
 * NULL); GRPIC_E_INVALID if fewer than n were collected.                  */
int grpic_mlp_get_samples(grpic_ctx *ctx, long n, float *X, float *T,
                          unsigned char *valid);

typedef struct grpic_mlp_train_config {
  long epochs;                /* passes over the samples                     */
  long batch;                 /* rows per gradient step (>= 64)              */
  double lr, lr_final;        /* Adam step size, cosine-decayed to lr_final  */
  double beta1, beta2, eps;   /* Adam moments                                */
  unsigned long long seed;    /* initialisation and batch order              */
} grpic_mlp_train_config;

/* Train on the collected samples, on the GPU: feature mean / inv_std and
 * the output scale (RMS of each target component) from the valid samples,
 * uniform initialisation in +-1/sqrt(fan_in), then Adam on the mean squared
 * error of the scaled target, one shuffled pass per epoch.  epoch_loss (may
 * be NULL) receives the mean batch loss of each epoch.  The trained network
 * is then the one the learned guess uses.  GRPIC_E_STATE with fewer than 64
 * samples, GRPIC_E_INVALID for a bad configuration.                       */
int grpic_mlp_train(grpic_ctx *ctx, const grpic_mlp_train_config *cfg,
                    double *epoch_loss);

/* The network alone, for checks: Y (n x 6) = net(X) for normalised inputs
 * X (n x 14), host arrays.  grpic_mlp_loss_grad: loss = mean over rows and
 * outputs of (net(X) - T)^2 and its gradient with respect to the packed
 * parameters (grad[5510]).  Both use the same matrix-core kernels as the
 * guess and the training; GRPIC_E_STATE when no network is loaded.       */
int grpic_mlp_forward(grpic_ctx *ctx, long n, const float *X, float *Y);
int grpic_mlp_loss_grad(grpic_ctx *ctx, long n, const float *X,
                        const float *T, float *grad, double *loss);

#ifdef __cplusplus
}
#endif
#endif
