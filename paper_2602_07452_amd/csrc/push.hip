// push.hip -- particle push of the GRPIC step (sub-step 5 of Sec. 2.1):
// field gather, RK4 (Sec. 2.2.1), the Hyb1/Hyb2 energy switch (Sec. 3.1.2),
// the implicit midpoint rule (Sec. 2.2.2) and the discrete-gradient
// Hamiltonian scheme (Sec. 2.2.3, App. D), particle boundary conditions
// (Sec. 2.5) and the deposit weights of the pushed positions (Sec. 2.3).
//
// Two passes per step:
//  * k_push_explicit: one thread per particle.  RK4 with fields re-gathered
//    at every stage; the switch either accepts the step or appends the
//    particle to the implicit queue (wave ballots, one atomic per block on
//    one of kQueueSegs segment counters).
//  * k_push_implicit: persistent kernel; its waves take groups of kGrab
//    entries of the concatenated segments in fixed round-robin shares until
//    the queue is drained.
#include "deposit_device.hpp"
#include "queue_device.hpp"

namespace grpic {

enum : uint8_t {
  F_ALIVE = GRPIC_FLAG_ALIVE,
  F_IMPLICIT = GRPIC_FLAG_IMPLICIT,
  F_NOCONV = GRPIC_FLAG_NOCONV,
  F_REMOVED = GRPIC_FLAG_REMOVED,
  F_REFLECTED = GRPIC_FLAG_REFLECTED,
  F_NONFINITE = GRPIC_FLAG_NONFINITE
};

struct PushArgs {
  GridView g;
  FieldView f;
  ParticleView p;
  double a, dt, thr, tol, ham_eps, r_min, r_max, th_lo, th_hi;
  double dt_im, t_end;  // implicit step and clock end (no grid only)
  int pusher, guess, kmax, reflect;
  double* gz[6];
  int* queue;       // kQueueSegs segments of seg_cap entries
  unsigned seg_cap;
  Stats* st;
  int use_gz;       // the implicit pass starts from gz (else from z^n)
  CollectView col;  // training-sample collection (col.T == nullptr: off)
};

// Step statistics.  Alive particles and their energy-violation histogram
// are not counted here: the diagnostics count them from the particle
// arrays when they are read (k_census).  The rest are counted by finalize
// through a sink: the block's LDS counters where lanes finalise many
// particles (the implicit pass), or direct global atomics for the rare
// events of the explicit pass (removal, reflection), which so needs no LDS
// counters, no barrier and no flush.
struct LocalStats {
  unsigned int iter_hist[kHistBins];
  unsigned int implicit_steps, noconv, removed, reflected, nonfinite;
};

__device__ __forceinline__ void stats_init(LocalStats& s) {
  for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) s.iter_hist[i] = 0;
  if (threadIdx.x == 0) s.implicit_steps = s.noconv = s.removed = s.reflected = s.nonfinite = 0;
}

__device__ __forceinline__ void stats_flush(const LocalStats& s, Stats* st) {
  StatRep* g = &st->rep[blockIdx.x % kStatReps];
  for (int i = threadIdx.x; i < kHistBins; i += blockDim.x)
    if (s.iter_hist[i]) atomicAdd(&g->iter_hist[i], (unsigned long long)s.iter_hist[i]);
  if (threadIdx.x == 0) {
    if (s.implicit_steps) atomicAdd(&g->implicit_steps, (unsigned long long)s.implicit_steps);
    if (s.noconv) atomicAdd(&g->noconv, (unsigned long long)s.noconv);
    if (s.removed) atomicAdd(&g->removed, (unsigned long long)s.removed);
    if (s.reflected) atomicAdd(&g->reflected, (unsigned long long)s.reflected);
    if (s.nonfinite) atomicAdd(&g->nonfinite, (unsigned long long)s.nonfinite);
  }
}

// what finalize counts, from the flags it wrote
__device__ __forceinline__ void record(LocalStats& s, uint8_t fl, int iters) {
  if (fl & F_REMOVED) {
    atomicAdd(&s.removed, 1u);
    if (fl & F_NONFINITE) atomicAdd(&s.nonfinite, 1u);
  }
  if (fl & F_REFLECTED) atomicAdd(&s.reflected, 1u);
  if (fl & F_IMPLICIT) {
    atomicAdd(&s.implicit_steps, 1u);
    atomicAdd(&s.iter_hist[iters < kHistBins ? iters : kHistBins - 1], 1u);
  }
  if (fl & F_NOCONV) atomicAdd(&s.noconv, 1u);
}

struct GlobalStats {
  StatRep* g;  // the block's replica
};

__device__ __forceinline__ void record(GlobalStats& s, uint8_t fl, int iters) {
  if (fl & F_REMOVED) {
    atomicAdd(&s.g->removed, 1ull);
    if (fl & F_NONFINITE) atomicAdd(&s.g->nonfinite, 1ull);
  }
  if (fl & F_REFLECTED) atomicAdd(&s.g->reflected, 1ull);
  if (fl & F_IMPLICIT) {
    atomicAdd(&s.g->implicit_steps, 1ull);
    atomicAdd(&s.g->iter_hist[iters < kHistBins ? iters : kHistBins - 1], 1ull);
  }
  if (fl & F_NOCONV) atomicAdd(&s.g->noconv, 1ull);
}

// --------------------------------------------------------------- F(z)
// F at z (eqs. p1, p2, O1, O2), with s, c = sin, cos of z[1]; *pw = the
// power (q/m) E_i dx^i/dt, *e (optional) = alpha Gamma - beta^r u_r.
// The metric derivatives enter the gravity force only contracted with the
// momenta, u_l u_m d_k gamma^lm; with P = rho^2, S = P + 2r, xi = S/P and
// s2 = sin^2 theta that contraction is
//   -dP_k / P^2 (a^2 s2 u_r^2 + u_th^2 + u_ph^2 / s2 + 2 a u_r u_ph)
//   + d(s2)_k / P (a^2 u_r^2 - u_ph^2 / s2^2) - d(xi)_k / xi^2 u_r^2,
// evaluated in that factored form (fewer live values than the twelve
// derivatives; equal to rounding).
// SPLIT: issue the field loads first and compute the gravity terms while
// they are in flight (more registers: pays where occupancy is already two
// waves per SIMD, the implicit pass)
// CACHE: gc holds the corners of the cells of an earlier evaluation and is
// reused without memory traffic while the point stays in those cells (the
// implicit iterates, whose points move by far less than a cell); a miss
// loads the new cells into gc, issued before the gravity terms.
// COEFS (with CACHE): the cache holds the corners as FP64 interpolation
// coefficients, converted once per loaded cell set instead of at every use
// (more registers; the explicit push has them to spare at two waves per SIMD)
template <bool GRID, bool SPLIT = false, bool CACHE = false, bool COEFS = false>
__device__ __forceinline__ void eval(const PushArgs& A, double qm,
                                     const double* z, double s, double c, double* f,
                                     double* pw, double* e = nullptr,
                                     GatherLoads* gc = nullptr, bool issued = false) {
  const double a = A.a, a2 = a * a, r = z[0], ur = z[3], ut = z[4], up = z[5];
  const double s2 = s * s, sc = s * c;
  // one inverse square root w = (rho2 S sin^2)^(-1/2) = 1/sqrt(gamma) gives
  // 1/sin^2 = rho2 S w^2, y = (rho2 S)^(-1/2) = |sin| w, alpha = sqrt(rho2 / S)
  // = rho2 y, sqrt(gamma) = rho2 S sin^2 w, 1/S = rho2 y^2 and 1/rho2 = S y^2
  const double rho2 = r * r + a2 * c * c, S = rho2 + 2.0 * r, P = rho2 * S;
  const double Q = P * s2, isg = frsq(Q), w2 = isg * isg;
  const double is2 = P * w2, y2 = s2 * w2, y = fabs(s) * isg;
  const double irho2 = S * y2, iS = rho2 * y2;
  const double ixi = rho2 * iS, alpha = rho2 * y, betar = 2.0 * r * iS;
  const double sg = Q * isg;
  double D[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
  const bool charged = GRID && qm != 0.0;
  GatherLoads gl;
  bool hit = false;
  if (charged) {
    if constexpr (CACHE) {
      // issued: the caller has issued this point's loads into gc already
      if (!issued) {
        hit = gather_hit(A.g, r, z[1], *gc);
        if (!hit) gather_issue(A.g, A.f, r, z[1], *gc);
      }
    } else if constexpr (SPLIT) {
      gather_issue(A.g, A.f, r, z[1], gl);
    } else {
      gather(A.g, A.f, r, z[1], isg, D, B);
    }
  }
  // contravariant momentum gamma^ij u_j and the Lorentz factor
  const double irp = a * irho2;
  const double Ur = (a2 * s2 * irho2 + ixi) * ur + irp * up;
  const double Ut = irho2 * ut;
  const double Up = irp * ur + irho2 * is2 * up;
  // u_i gamma^ij u_j = Aq / rho2 + u_r^2 / xi, with Aq = a^2 s2 u_r^2 + u_th^2
  // + u_ph^2 / s2 + 2 a u_r u_ph the quadratic form of the gravity terms
  const double q = ur * Ur + ut * Ut + up * Up;
  const double G2 = 1.0 + q;
  const double iG = frsq(G2), G = G2 * iG;  // 1/Gamma and Gamma
  const double aiG = alpha * iG;
  if (e) *e = alpha * G - betar * ur;
  f[0] = aiG * Ur - betar;
  f[1] = aiG * Ut;
  f[2] = aiG * Up;
  // gravity: -Gamma d_k alpha + u_r d_k beta^r - alpha/(2 Gamma) u u d_k gamma^-1
  const double i4 = irho2 * irho2, ixi2 = ixi * ixi, ur2 = ur * ur;
  const double Aq_r = fma(-ixi, ur2, q);  // Aq / rho2, from the sum above
  const double Bq = irho2 * (a2 * ur2 - up * up * is2 * is2);
  const double Cq = 0.5 * G * alpha * ixi + ur * ixi2 + 0.5 * aiG * ixi2 * ur2;
  const double dxr = 2.0 * irho2 * (1.0 - 2.0 * r * r * irho2);  // d_r xi
  const double dxt = 4.0 * r * a2 * sc * i4;                      // d_theta xi
  const double gr = dxr * Cq + aiG * r * irho2 * Aq_r;
  const double gt = dxt * Cq - aiG * sc * (a2 * irho2 * Aq_r + Bq);
  if constexpr (CACHE) {
    if (charged) {
      if constexpr (COEFS) {
        if (!hit) {
          gather_settle(A.g, A.f, r, *gc);
          gather_coefs(*gc);
          gather_bounds(A.g, *gc);
        }
        gather_interp_coefs(A.g, r, z[1], isg, *gc, D, B);
      } else {
        if (!hit) {
          gather_settle(A.g, A.f, r, *gc);
          gather_bounds(A.g, *gc);
        }
        gather_interp(A.g, r, z[1], isg, *gc, D, B);
      }
    }
  } else if constexpr (SPLIT) {
    if (charged) gather_finish(A.g, A.f, r, z[1], isg, gl, D, B);
  }
  if (qm != 0.0) {
    // Lorentz force: alpha (q/m) [gamma_ij D^j + sqrt(g) eta_ijk U^j B^k / Gamma]
    const double xi = S * irho2;
    const double Dl_r = xi * (D[0] - a * s2 * D[2]);
    const double Dl_t = rho2 * D[1];
    const double Dl_p = s2 * (-a * xi * D[0] + (rho2 + a2 * xi * s2) * D[2]);
    const double sgiG = sg * iG;
    const double cr = Ut * B[2] - Up * B[1];
    const double ct = Up * B[0] - Ur * B[2];
    const double cp = Ur * B[1] - Ut * B[0];
    const double qa = qm * alpha;
    f[3] = gr + qa * (Dl_r + sgiG * cr);
    f[4] = gt + qa * (Dl_t + sgiG * ct);
    f[5] = qa * (Dl_p + sgiG * cp);
    // E_i = alpha D_i + sqrt(g) eta_ijk beta^j B^k (eq. Ei)
    const double sgb = sg * betar;
    const double Er = alpha * Dl_r;
    const double Et = alpha * Dl_t - sgb * B[2];
    const double Ep = alpha * Dl_p + sgb * B[1];
    *pw = qm * (Er * f[0] + Et * f[1] + Ep * f[2]);
  } else {
    f[3] = gr;
    f[4] = gt;
    f[5] = 0.0;
    *pw = 0.0;
  }
}

// RK4; *e0 = energy e at z (from the first stage)
// classical RK4 with the fields re-gathered at every stage; s0, c0 (out):
// sin, cos of z[1], from which the stage angles are reached by short series
// CACHE: the stages reuse the field corners of the previous stage's cells,
// held as FP64 interpolation coefficients, while they stay in them (a step
// moves a particle by a fraction of a cell, so three of the four stage
// gathers mostly need no memory round trip; the cache raises the explicit
// push from 154 to 232 VGPRs, three to two waves per SIMD, and still takes
// 5 % off its time on 2^27 particles)
// gc (out): the gather cells of the last stage (pn = -1 without the cache)
template <bool GRID, bool CACHE = false>
__device__ __forceinline__ void rk4(const PushArgs& A, double dt, double qm,
                                    const double* z, double* out, double* Wq,
                                    double* e0, double* s0, double* c0, GatherLoads& gc) {
  const double hdt = 0.5 * dt;
  double k[6], acc[6], y[6], p, pacc, s, c;
  gc.pn = -1;
  // the first stage's field loads go out before the angle's sine and cosine
  // are computed, so that their latency overlaps that work
  const bool pre = CACHE && GRID && qm != 0.0;
  if (pre) gather_issue(A.g, A.f, z[0], z[1], gc);
  fsincos(z[1], s0, c0);
  eval<GRID, false, CACHE, CACHE>(A, qm, z, *s0, *c0, k, &p, e0, &gc, pre);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    acc[i] = k[i];
    y[i] = z[i] + hdt * k[i];
  }
  pacc = p;
  sincos_near(y[1], z[1], *s0, *c0, &s, &c);
  eval<GRID, false, CACHE, CACHE>(A, qm, y, s, c, k, &p, nullptr, &gc);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    acc[i] += 2.0 * k[i];
    y[i] = z[i] + hdt * k[i];
  }
  pacc += 2.0 * p;
  sincos_near(y[1], z[1], *s0, *c0, &s, &c);
  eval<GRID, false, CACHE, CACHE>(A, qm, y, s, c, k, &p, nullptr, &gc);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    acc[i] += 2.0 * k[i];
    y[i] = z[i] + dt * k[i];
  }
  pacc += 2.0 * p;
  sincos_near(y[1], z[1], *s0, *c0, &s, &c);
  eval<GRID, false, CACHE, CACHE>(A, qm, y, s, c, k, &p, nullptr, &gc);
  const double c6 = dt * (1.0 / 6.0);
#pragma unroll
  for (int i = 0; i < 6; ++i) out[i] = z[i] + c6 * (acc[i] + k[i]);
  *Wq = c6 * (pacc + p);
}

// max_i |zn_i - zo_i| / max(|zn_i|, 1) <= tol, tested without divisions as
// |zn_i - zo_i| <= tol max(|zn_i|, 1) for every i (the two differ only when
// a term lies within rounding of tol); a NaN term passes, as it does not
// raise that maximum
__device__ __forceinline__ bool small_change(const double* zn, const double* zo,
                                             double tol) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 6; ++i) ok = ok & !(fabs(zn[i] - zo[i]) > tol * fmax(fabs(zn[i]), 1.0));
  return ok;
}

// implicit midpoint rule by fixed-point iteration; zk: guess in, result out.
// The field corners of the midpoint's cells are kept across iterations and
// reloaded only when the midpoint leaves those cells.
// col (out): the node column of the last midpoint's gather (pn = -1: none)
template <bool GRID, bool SPLIT = false>
__device__ int imr(const PushArgs& A, double dt, double qm, const double* z, double s0,
                   double c0, double* zk, double* Wq, ColumnHint* col) {
  double p = 0.0;
  GatherLoads gc;
  gc.pn = -1;
  for (int k = 1; k <= A.kmax; ++k) {
    double zm[6], f[6], zn[6], sm, cm;
#pragma unroll
    for (int i = 0; i < 6; ++i) zm[i] = 0.5 * (z[i] + zk[i]);
    sincos_near(zm[1], z[1], s0, c0, &sm, &cm);
    eval<GRID, SPLIT, GRID>(A, qm, zm, sm, cm, f, &p, nullptr, &gc);
#pragma unroll
    for (int i = 0; i < 6; ++i) zn[i] = z[i] + dt * f[i];
    bool c = small_change(zn, zk, A.tol);
#pragma unroll
    for (int i = 0; i < 6; ++i) zk[i] = zn[i];
    if (c) {
      *Wq = dt * p;
      *col = column_hint(gc);
      return k;
    }
  }
  *Wq = dt * p;
  *col = column_hint(gc);
  return -A.kmax;
}

// Newton's method on the same equation (the solver the paper names; the
// Picard iteration above is the default): G(y) = y - z - dt F((z + y)/2),
// J = I - (dt/2) dF/dx at the midpoint by forward differences with steps
// 2^-26 max(|m_j|, 1) (the step taken, (m_j + h) - m_j, divides), then
// y -= J^{-1} G(y) by Gaussian elimination with partial pivoting; same
// stopping test; Wq from the last midpoint evaluation
// Every index into J is a compile-time constant (the column loop writes its
// column through selects, the pivot swap is a chain of selects), so the
// 6x7 system stays in registers.
template <bool GRID>
__device__ int imr_newton(const PushArgs& A, double dt, double qm, const double* z,
                          double s0, double c0, double* zk, double* Wq) {
  double p = 0.0;
  GatherLoads gc;  // corners of the midpoint's cells, as in imr
  gc.pn = -1;
  for (int k = 1; k <= A.kmax; ++k) {
    double m[6], f0[6], J[6][7] = {}, sm, cm;
#pragma unroll
    for (int i = 0; i < 6; ++i) m[i] = 0.5 * (z[i] + zk[i]);
    sincos_near(m[1], z[1], s0, c0, &sm, &cm);
    eval<GRID, false, GRID>(A, qm, m, sm, cm, f0, &p, nullptr, &gc);
#pragma unroll 1
    for (int j = 0; j < 6; ++j) {
      double mj[6], fj[6], pj, sj, cj, mv = m[0];
#pragma unroll
      for (int i = 1; i < 6; ++i) mv = i == j ? m[i] : mv;
      double h = 0x1p-26 * fmax(fabs(mv), 1.0);
      const double sv = mv + h;
      h = sv - mv;
#pragma unroll
      for (int i = 0; i < 6; ++i) mj[i] = i == j ? sv : m[i];
      sincos_near(mj[1], z[1], s0, c0, &sj, &cj);
      eval<GRID, false, GRID>(A, qm, mj, sj, cj, fj, &pj, nullptr, &gc);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const double v = (i == j ? 1.0 : 0.0) - 0.5 * dt * (fj[i] - f0[i]) / h;
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) J[i][jj] = jj == j ? v : J[i][jj];
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) J[i][6] = -(zk[i] - z[i] - dt * f0[i]);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      int piv = c;
      double best = fabs(J[c][c]);
#pragma unroll
      for (int i = c + 1; i < 6; ++i)
        if (fabs(J[i][c]) > best) {
          piv = i;
          best = fabs(J[i][c]);
        }
#pragma unroll
      for (int i = c + 1; i < 6; ++i)
#pragma unroll
        for (int j = c; j < 7; ++j) {
          const double t = J[c][j];
          J[c][j] = piv == i ? J[i][j] : t;
          J[i][j] = piv == i ? t : J[i][j];
        }
#pragma unroll
      for (int i = c + 1; i < 6; ++i) {
        double l = J[i][c] / J[c][c];
#pragma unroll
        for (int j = c; j < 7; ++j) J[i][j] -= l * J[c][j];
      }
    }
    double dy[6], zn[6];
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      double v = J[i][6];
#pragma unroll
      for (int j = i + 1; j < 6; ++j) v -= J[i][j] * dy[j];
      dy[i] = v / J[i][i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) zn[i] = zk[i] + dy[i];
    bool cv = small_change(zn, zk, A.tol);
#pragma unroll
    for (int i = 0; i < 6; ++i) zk[i] = zn[i];
    if (cv) {
      *Wq = dt * p;
      return k;
    }
  }
  *Wq = dt * p;
  return -A.kmax;
}

// ------------------------------------------- discrete-gradient scheme (DG)
// Variables 0 r, 1 theta, 2 phi, 3 u_r, 4 u_theta, 5 u_phi.  Six orderings
// (three cyclic orders with x before u and their reverses); at most four
// distinct positions (r^n or r^{n+1}) x (theta^n or theta^{n+1}) occur.
// Position quotients of the metric are cancellation-free divided
// differences (metric_dd); below |dx| = eps the analytic derivative at the
// midpoint replaces them.
// The table is a compile-time constant and both loops below unroll fully, so
// every step's variable and mask are literals: the four metric copies stay
// in registers instead of being indexed through scratch memory.
constexpr int8_t kDGOrder[6][6] = {{0, 3, 1, 4, 2, 5}, {1, 4, 2, 5, 0, 3},
                                    {2, 5, 0, 3, 1, 4}, {5, 2, 4, 1, 3, 0},
                                    {3, 0, 5, 2, 4, 1}, {4, 1, 3, 0, 5, 2}};

__device__ __forceinline__ double lorentz(const Met& m, double ur, double ut,
                                          double up) {
  return sqrt(1.0 + m.irr * ur * ur + m.itt * ut * ut + m.ipp * up * up +
              2.0 * m.irp * ur * up);
}

__device__ int ham_dg(const PushArgs& A, double dt, const double* z, double* zk) {
  for (int k = 1; k <= A.kmax; ++k) {
    Met M[4];  // index: bit0 = r updated, bit1 = theta updated
    metric(A.a, z[0], z[1], M[0]);
    metric(A.a, zk[0], z[1], M[1]);
    metric(A.a, z[0], zk[1], M[2]);
    metric(A.a, zk[0], zk[1], M[3]);
    double grad[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      int mask = 0;  // bit v set: variable v already at level n+1
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        int v = kDGOrder[o][s];
        double ur = (mask & 8) ? zk[3] : z[3];
        double ut = (mask & 16) ? zk[4] : z[4];
        double up = (mask & 32) ? zk[5] : z[5];
        double q = 0.0;
        if (v >= 3) {
          const Met& m = M[mask & 3];
          double ur1 = v == 3 ? zk[3] : ur, ut1 = v == 4 ? zk[4] : ut,
                 up1 = v == 5 ? zk[5] : up;
          double G0 = lorentz(m, ur, ut, up), G1 = lorentz(m, ur1, ut1, up1);
          double num;
          if (v == 3)
            num = m.irr * (ur1 + ur) + 2.0 * m.irp * up;
          else if (v == 4)
            num = m.itt * (ut1 + ut);
          else
            num = m.ipp * (up1 + up) + 2.0 * m.irp * ur;
          q = m.alpha * num / (G0 + G1) - (v == 3 ? m.betar : 0.0);
        } else if (v < 2) {
          const Met& m0 = M[mask & 3];
          const Met& m1 = M[(mask | (1 << v)) & 3];
          double G0 = lorentz(m0, ur, ut, up), G1 = lorentz(m1, ur, ut, up);
          double dx = zk[v] - z[v];
          double qa, qb, qrr, qtt, qpp, qrp;
          if (fabs(dx) >= A.ham_eps) {
            double q6[6];
            double r0 = (mask & 1) ? zk[0] : z[0];
            double r1 = v == 0 ? zk[0] : r0;
            metric_dd(A.a, v, r0, r1, dx, m0, m1, q6);
            qa = q6[0];
            qb = q6[1];
            qrr = q6[2];
            qtt = q6[3];
            qpp = q6[4];
            qrp = q6[5];
          } else {
            double rr = v == 0 ? 0.5 * (z[0] + zk[0]) : ((mask & 1) ? zk[0] : z[0]);
            double tt = v == 1 ? 0.5 * (z[1] + zk[1]) : ((mask & 2) ? zk[1] : z[1]);
            Met mm;
            DMet d;
            metric_d(A.a, rr, tt, mm, d);
            qa = d.da[v];
            qb = d.db[v];
            qrr = d.drr[v];
            qtt = d.dtt[v];
            qpp = d.dpp[v];
            qrp = d.drp[v];
          }
          double quad = qrr * ur * ur + qtt * ut * ut + qpp * up * up +
                        2.0 * qrp * ur * up;
          q = 0.5 * (G0 + G1) * qa + 0.5 * (m0.alpha + m1.alpha) * quad / (G0 + G1) -
              ur * qb;
        }
        grad[v] += q * (1.0 / 6.0);
        mask |= 1 << v;
      }
    }
    double zn[6];
    zn[0] = z[0] + dt * grad[3];
    zn[1] = z[1] + dt * grad[4];
    zn[2] = z[2] + dt * grad[5];
    zn[3] = z[3] - dt * grad[0];
    zn[4] = z[4] - dt * grad[1];
    zn[5] = z[5] - dt * grad[2];
    bool c = small_change(zn, zk, A.tol);
#pragma unroll
    for (int i = 0; i < 6; ++i) zk[i] = zn[i];
    if (c) return k;
  }
  return -A.kmax;
}

// ----------------------------------------------------------- switch value
// neutral: |e - H0| / |H0|; charged: |e' - e - W| / |e| (W: the scheme's
// quadrature of (q/m) E_i dx^i/dt)
// zn: the new state; s0, c0: sin, cos of the old angle z0
// (*sn, *cn: sin, cos of zn[1], for finalize)
// H0 (the particle's initial H) is read only for a neutral particle: the
// charged ones never wait for that load
__device__ __forceinline__ double switch_value(const PushArgs& A, double qm,
                                               const double* H0, double e0,
                                               const double* zn, double Wq,
                                               double z0, double s0, double c0,
                                               double* sn, double* cn) {
  double s, c;
  sincos_near(zn[1], z0, s0, c0, &s, &c);
  *sn = s;
  *cn = c;
  double e1 = energy_sc(A.a, zn, s, c);
  // (the quotients by one refined reciprocal: within an ulp of the division)
  if (qm == 0.0) {
    const double h0 = *H0;
    return fabs(e1 - h0) * frcp(fabs(h0));
  }
  return fabs(e1 - e0 - Wq) * frcp(fabs(e0));
}

// histogram bin b = floor(2 (log10 v + 30)) of an energy violation (a
// diagnostic: FP32 logarithm)
__device__ __forceinline__ int herr_bin(double v) {
  if (!(v >= 1e-30)) return 0;
  float l = __builtin_amdgcn_logf((float)fmin(v, 1e30)) * 0.30102999566398120f;
  int b = (int)floorf(2.0f * (l + 30.0f));
  return b < 0 ? 0 : (b >= kHistBins ? kHistBins - 1 : b);
}

// A particle array element: at(p, k) with a 64-bit index k, or with an
// Off32 index, whose byte offsets are 32-bit (particle counts below 2^28,
// so below 2^31 bytes): the explicit pass then addresses every array as a
// scalar base plus one 32-bit lane offset per element size, instead of a
// 64-bit address sum per array.
struct Off32 {
  uint32_t i;
};

template <class T>
__device__ __forceinline__ T& at(T* p, long k) {
  return p[k];
}

template <class Ix>
__device__ __forceinline__ Ix make_ix(long k);
template <>
__device__ __forceinline__ long make_ix<long>(long k) {
  return k;
}
template <>
__device__ __forceinline__ Off32 make_ix<Off32>(long k) {
  return Off32{(uint32_t)k};
}

template <class T>
__device__ __forceinline__ T& at(T* p, Off32 k) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + k.i * (uint32_t)sizeof(T));
}

// write the step result, apply the particle boundary conditions and (for a
// deposit) store the old position and the weights of the new one
// s0, c0: sin, cos of z[1]
template <bool EVOLVE, class Ix, class Sink>
// sn, cn: sin, cos of out[1] as pushed; hint: the last stage's node column
__device__ void finalize(const PushArgs& A, Ix k, const double* z,
                         double* out, double herr, int iters, uint8_t fl,
                         Sink& ls, double s0, double c0, double sn, double cn,
                         ColumnHint hint) {
  const ParticleView& P = A.p;
  bool finite = true;
#pragma unroll
  for (int i = 0; i < 6; ++i) finite = finite && isfinite(out[i]);
  if (!finite) {  // a state that is no number: taken out of the run
    fl = F_REMOVED | F_NONFINITE;
  } else if (out[0] < A.r_min || out[0] > A.r_max) {
    fl = F_REMOVED;
  } else if (A.reflect) {
    if (out[1] < A.th_lo) {
      out[1] = 2.0 * A.th_lo - out[1];
      out[4] = -out[4];
      fl |= F_REFLECTED;
    } else if (out[1] > A.th_hi) {
      out[1] = 2.0 * A.th_hi - out[1];
      out[4] = -out[4];
      fl |= F_REFLECTED;
    }
  }
  const bool moved = (fl & F_REFLECTED) != 0;
  at(P.r, k) = out[0];
  at(P.th, k) = out[1];
  at(P.ph, k) = out[2];
  at(P.ur, k) = out[3];
  at(P.uth, k) = out[4];
  at(P.uph, k) = out[5];
  at(P.herr, k) = herr;
  at(P.flags, k) = fl;
  at(P.iters, k) = (uint8_t)(iters < 255 ? iters : 255);  // a restart can take 2 kmax
  record(ls, fl, iters);
  if (EVOLVE) {
    at(P.r_old, k) = z[0];
    at(P.th_old, k) = z[1];
    at(P.dphi, k) = (float)(out[2] - z[2]);
    if (fl & F_ALIVE) {
      int p, q;
      double W[4], st = sn, ct = cn;
      if (moved) sincos_near(out[1], z[1], s0, c0, &st, &ct);
      cell_and_weights(A.g, out[0], out[1], st, ct, p, q, W, hint);
#pragma unroll
      for (int c = 1; c < 4; ++c) at(P.Wn[c], k) = wq_encode(W[c]);
      at(P.celln, k) = q * A.g.nr + p;
    }
  }
}

template <class Ix>
__device__ __forceinline__ void load_z(const ParticleView& P, Ix k, double* z) {
  z[0] = at(P.r, k);
  z[1] = at(P.th, k);
  z[2] = at(P.ph, k);
  z[3] = at(P.ur, k);
  z[4] = at(P.uth, k);
  z[5] = at(P.uph, k);
}

// ------------------------------------------------------- explicit pass
template <bool GRID, bool EVOLVE, int WPS, bool CACHE = false, bool OFF32 = false>
__global__ __launch_bounds__(kPushBlock) __attribute__((amdgpu_waves_per_eu(WPS)))
void k_push_explicit(PushArgs A) {
  const ParticleView& P = A.p;
  const long kg = (long)blockIdx.x * blockDim.x + threadIdx.x;
  using Ix = typename std::conditional<OFF32, Off32, long>::type;
  const Ix k = make_ix<Ix>(kg);
  // the state is loaded together with the flags, before the statistics are
  // set up (one memory round trip before the first stage's field loads,
  // overlapped with that set-up)
  const bool inr = kg < P.n;
  double z[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, qm = 0.0;
  uint8_t flg = 0;
  if (inr) {
    flg = at(P.flags, k);
    load_z(P, k, z);
    qm = (double)at(P.qm, k);
  }
  GlobalStats ls{&A.st->rep[blockIdx.x % kStatReps]};
  const bool act = inr && (flg & F_ALIVE);
  bool enq = false;
  double trial[6];
  if (act) {
    // without a grid each particle keeps its own time: the step is clipped
    // to the time left before t_end, and a particle at t_end stays
    double dt = A.dt, tk = 0.0;
    bool frozen = false, ends = false;
    if constexpr (!GRID) {
      tk = at(P.t, k);
      if (A.t_end > 0.0) {
        double left = A.t_end - tk;
        if (!(left > 0.0)) {
          frozen = true;
        } else if (left <= dt) {
          dt = left;
          ends = true;
        }
      }
    }
    if (frozen) {
      at(P.flags, k) = F_ALIVE;
      at(P.iters, k) = 0;
    } else if (A.pusher == GRPIC_PUSH_IMR || A.pusher == GRPIC_PUSH_HAM) {
      enq = true;
#pragma unroll
      for (int i = 0; i < 6; ++i) trial[i] = z[i];  // no RK4 trial: start at z^n
    } else {
      double Wq, e0, s0, c0, sn, cn;
      GatherLoads gc;
      rk4<GRID, CACHE && GRID>(A, dt, qm, z, trial, &Wq, &e0, &s0, &c0, gc);
      double v = switch_value(A, qm, &at(P.H0, k), e0, trial, Wq, z[1], s0, c0, &sn, &cn);
      bool accept = true;
      if (A.pusher == GRPIC_PUSH_HYB2) {
        accept = v < A.thr;
      } else if (A.pusher == GRPIC_PUSH_HYB1) {
        double prev = at(P.herr, k);
        accept = (v - prev) / (dt * fmax(prev, 0x1p-52)) < A.thr;
      }
      if (accept) {
        finalize<EVOLVE>(A, k, z, trial, v, 0, F_ALIVE, ls, s0, c0, sn, cn,
                         column_hint(gc));
        if constexpr (!GRID) at(P.t, k) = ends ? A.t_end : tk + dt;
      } else {
        enq = true;
      }
    }
  }
  // append the rejected particles to the implicit queue: one ballot and, when
  // a lane was rejected, one atomic on the block's queue segment
  static_assert(kPushBlock == 64, "the explicit push runs one wave per block");
  const int lane = threadIdx.x & 63;
  const unsigned long long mask = __ballot(enq);
  if (mask != 0ull) {
    const unsigned seg = blockIdx.x % kQueueSegs;
    unsigned base = 0u;
    if (lane == 0) base = atomicAdd(&A.st->seg_count[seg], (unsigned)__popcll(mask));
    base = __builtin_amdgcn_readfirstlane(base);
    if (enq) {
      const unsigned slot = seg * A.seg_cap + base +
                            (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
      A.queue[slot] = (int)kg;
      // first iterate (RK4 result; the base of the learned guess in the hybrid)
      if (A.use_gz && (A.guess == GRPIC_GUESS_RK4 || A.pusher == GRPIC_PUSH_HYB1 ||
                       A.pusher == GRPIC_PUSH_HYB2)) {
#pragma unroll
        for (int i = 0; i < 6; ++i) A.gz[i][slot] = trial[i];
      }
    }
  }
}

// ------------------------------------------------------- implicit pass
constexpr unsigned kGrab = 64;  // queue entries a wave takes at a time

template <bool GRID, bool EVOLVE, bool HAM, bool NEWTON>
__global__ __launch_bounds__(256) void k_push_implicit(PushArgs A) {
  __shared__ LocalStats ls;
  __shared__ unsigned pref[kQueueSegs + 1];
  stats_init(ls);
  const unsigned qn = segment_prefix(A.st, pref);
  const ParticleView& P = A.p;
  const int lane = threadIdx.x & 63;
  // wave w of nw takes queue groups w, w + nw, w + 2 nw, ...: fixed shares,
  // no shared work counter (every wave appending to one counter serialised
  // the grabs: 0.47 against 0.42 ms per step on 2^27 particles)
  const unsigned nw = gridDim.x * (blockDim.x >> 6);
  for (unsigned grp = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);; grp += nw) {
    const unsigned base = grp * kGrab;
    if (base >= qn) break;
    for (unsigned sub = 0; sub < kGrab; sub += 64) {
      unsigned v = base + sub + lane;
      if (v >= qn) break;
      unsigned slot = virtual_slot(pref, v, A.seg_cap);
      long k = A.queue[slot];
      double z[6], zk[6];
      load_z(P, k, z);
      double qm = (double)P.qm[k];
      if (!A.use_gz) {
#pragma unroll
        for (int i = 0; i < 6; ++i) zk[i] = z[i];
      } else {
#pragma unroll
        for (int i = 0; i < 6; ++i) zk[i] = A.gz[i][slot];
      }
      const bool ham = HAM && qm == 0.0 && A.pusher != GRPIC_PUSH_IMR;
      // the implicit step (no grid: its own length, clipped before t_end)
      double dt = A.dt, tk = 0.0;
      bool ends = false;
      if constexpr (!GRID) {
        dt = A.dt_im;
        tk = P.t[k];
        if (A.t_end > 0.0 && A.t_end - tk <= dt) {
          dt = A.t_end - tk;
          ends = true;
        }
      }
      double Wq = 0.0, s0, c0;
      ColumnHint col{-1, 0.0, 0.0, -1, 0.0, 0.0};  // Picard: the last midpoint's node column
      fsincos(z[1], &s0, &c0);
      int it;
      if constexpr (NEWTON)
        it = ham ? ham_dg(A, dt, z, zk) : imr_newton<GRID>(A, dt, qm, z, s0, c0, zk, &Wq);
      else
        it = ham ? ham_dg(A, dt, z, zk) : imr<GRID, EVOLVE>(A, dt, qm, z, s0, c0, zk, &Wq, &col);
      bool finite = true;
#pragma unroll
      for (int i = 0; i < 6; ++i) finite = finite && isfinite(zk[i]);
      if ((it < 0 || !finite) && A.guess == GRPIC_GUESS_MLP && !A.col.T) {
        // no convergence from the learned guess (a non-finite iterate passes
        // the stopping test, whose maximum skips NaN): restart from z^n
#pragma unroll
        for (int i = 0; i < 6; ++i) zk[i] = z[i];
        int it2;
        if constexpr (NEWTON)
          it2 = ham ? ham_dg(A, dt, z, zk) : imr_newton<GRID>(A, dt, qm, z, s0, c0, zk, &Wq);
        else
          it2 = ham ? ham_dg(A, dt, z, zk) : imr<GRID, EVOLVE>(A, dt, qm, z, s0, c0, zk, &Wq, &col);
        it = it2 < 0 ? it2 - A.kmax : it2 + A.kmax;
      }
      uint8_t fl = F_ALIVE | F_IMPLICIT;
      if (it < 0) {
        fl |= F_NOCONV;
        it = -it;
      }
      if (A.col.T) {  // training sample: converged step minus the Euler start
        unsigned long long row = *A.col.rows + v;
        if (row < (unsigned long long)A.col.cap) {
#pragma unroll
          for (int i = 0; i < 6; ++i) A.col.T[row * 6 + i] = (float)(zk[i] - A.gz[i][slot]);
          A.col.valid[row] = (fl & F_NOCONV) ? 0 : 1;
        }
      }
      double e0 = qm != 0.0 ? energy_sc(A.a, z, s0, c0) : 0.0;
      double sn, cn;
      double v2 = switch_value(A, qm, P.H0 + k, e0, zk, Wq, z[1], s0, c0, &sn, &cn);
      finalize<EVOLVE>(A, k, z, zk, v2, it, fl, ls, s0, c0, sn, cn, col);
      if constexpr (!GRID) P.t[k] = ends ? A.t_end : tk + dt;
    }
  }
  __syncthreads();
  stats_flush(ls, A.st);
}

// alive particles and the histogram of the energy violations their last
// step wrote (census[0]: alive, census[1 + b]: bin b of herr_bin)
__global__ __launch_bounds__(256) void k_census(ParticleView P, unsigned long long* census) {
  __shared__ unsigned int h[1 + kHistBins];
  for (int i = threadIdx.x; i <= kHistBins; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const long stride = (long)gridDim.x * blockDim.x;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < P.n; k += stride) {
    if (P.flags[k] & F_ALIVE) {
      atomicAdd(&h[0], 1u);
      atomicAdd(&h[1 + herr_bin(P.herr[k])], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= kHistBins; i += blockDim.x)
    if (h[i]) atomicAdd(&census[i], (unsigned long long)h[i]);
}

// per-step counters back to zero (cumulative counters are kept)
__global__ void k_reset_step(Stats* st) {
  const int t = threadIdx.x;
  for (int i = t; i < kQueueSegs; i += blockDim.x) st->seg_count[i] = 0;
}

static PushArgs make_args(grpic_ctx* c) {
  PushArgs A;
  A.g = make_grid_view(c);
  A.f.Dr = c->D[2].c[0];
  A.f.Dt = c->D[2].c[1];
  A.f.Dp = c->D[2].c[2];
  A.f.Br = c->B[2].c[0];
  A.f.Bt = c->B[2].c[1];
  A.f.Bp = c->B[2].c[2];
  A.p = c->pv;
  A.p.n = c->n;
  A.a = c->cfg.a;
  A.dt = c->cfg.dt;
  A.dt_im = c->cfg.dt_implicit > 0.0 ? c->cfg.dt_implicit : c->cfg.dt;
  A.t_end = c->cfg.t_end;
  A.thr = c->cfg.hyb_threshold;
  A.tol = c->cfg.tol;
  A.ham_eps = c->cfg.ham_eps;
  A.r_min = c->cfg.r_remove_in;
  A.r_max = c->cfg.r_remove_out;
  A.th_lo = c->cfg.theta0;
  A.th_hi = kPi - c->cfg.theta0;
  A.pusher = c->cfg.pusher;
  A.guess = c->cfg.guess;
  A.kmax = c->cfg.kmax;
  A.reflect = c->cfg.reflect;
  for (int i = 0; i < 6; ++i) A.gz[i] = c->gz[i];
  A.queue = c->queue;
  A.seg_cap = c->seg_cap;
  A.st = c->stats;
  A.col = mlp_collect_view(c);
  A.use_gz = (A.guess != GRPIC_GUESS_PLAIN || A.col.T) ? 1 : 0;
  return A;
}

template <bool GRID, bool EVOLVE>
static void push_impl(grpic_ctx* c, const PushArgs& A) {
  // one wave per block: a block ends with the queue append (one returning
  // atomic), which with four waves per block and a barrier held all four
  // until the slowest was done (12.39 ms per C5 step at 256 threads, 11.95
  // at 128, 11.49 at 64); a one-wave block frees its slot as soon as it is
  // done, and its append needs no barrier
  const int block = kPushBlock;
  hipEvent_t ev;
  time_begin(c, GRPIC_K_PUSH, &ev);
  if (c->cfg.push_waves_per_simd >= 4)
    hipLaunchKernelGGL((k_push_explicit<GRID, EVOLVE, 4>), dim3(grid_for(c->n, block)),
                       dim3(block), 0, c->stream, A);
  else if (c->n < (1L << 28))  // 32-bit byte offsets into the particle arrays
    hipLaunchKernelGGL((k_push_explicit<GRID, EVOLVE, 1, true, true>),
                       dim3(grid_for(c->n, block)), dim3(block), 0, c->stream, A);
  else
    hipLaunchKernelGGL((k_push_explicit<GRID, EVOLVE, 1, true>), dim3(grid_for(c->n, block)),
                       dim3(block), 0, c->stream, A);
  GRPIC_HIP(hipGetLastError());
  time_end(c, GRPIC_K_PUSH, ev);
  bool implicit = c->cfg.pusher != GRPIC_PUSH_RK4;
  if (!implicit) return;
  const bool collect = A.col.T != nullptr;
  if (c->cfg.guess == GRPIC_GUESS_MLP || collect) launch_guess(c);
  int dev_cus = c->num_cus;
  int waves = c->cfg.persistent_waves > 0 ? c->cfg.persistent_waves : 8;
  unsigned blocks = (unsigned)((long)dev_cus * waves / 4);
  long need = (c->n + 255) / 256;
  if ((long)blocks > need) blocks = (unsigned)(need < 1 ? 1 : need);
  time_begin(c, GRPIC_K_IMPLICIT, &ev);
  // the discrete-gradient code is only compiled into the variant used when
  // neutral particles are present (it needs many more registers)
  const bool ham = c->has_neutral && c->cfg.pusher != GRPIC_PUSH_IMR;
  if (c->cfg.solver == GRPIC_SOLVER_NEWTON) {
    if (ham)
      hipLaunchKernelGGL((k_push_implicit<GRID, EVOLVE, true, true>), dim3(blocks),
                         dim3(256), 0, c->stream, A);
    else
      hipLaunchKernelGGL((k_push_implicit<GRID, EVOLVE, false, true>), dim3(blocks),
                         dim3(256), 0, c->stream, A);
  } else if (ham) {
    hipLaunchKernelGGL((k_push_implicit<GRID, EVOLVE, true, false>), dim3(blocks), dim3(256),
                       0, c->stream, A);
  } else {
    hipLaunchKernelGGL((k_push_implicit<GRID, EVOLVE, false, false>), dim3(blocks),
                       dim3(256), 0, c->stream, A);
  }
  GRPIC_HIP(hipGetLastError());
  time_end(c, GRPIC_K_IMPLICIT, ev);
  if (collect) mlp_collect_advance(c);
}

void launch_census(grpic_ctx* c) {
  launch_fill(c, c->stats->census, sizeof(c->stats->census));
  if (c->n == 0) return;
  // a few blocks per CU; each block's LDS counts stay far below 2^32
  long blocks = (c->n + 255) / 256;
  if (blocks > 8L * c->num_cus) blocks = 8L * c->num_cus;
  ParticleView P = c->pv;
  P.n = c->n;
  hipLaunchKernelGGL(k_census, dim3((unsigned)blocks), dim3(256), 0, c->stream, P,
                     c->stats->census);
  GRPIC_HIP(hipGetLastError());
}

void launch_push(grpic_ctx* c) {
  if (c->n == 0) return;
  hipLaunchKernelGGL(k_reset_step, dim3(1), dim3(256), 0, c->stream, c->stats);
  GRPIC_HIP(hipGetLastError());
  PushArgs A = make_args(c);
  int mode = c->cfg.field_mode;
  if (mode == GRPIC_FIELDS_NONE)
    push_impl<false, false>(c, A);
  else if (mode == GRPIC_FIELDS_STATIC)
    push_impl<true, false>(c, A);
  else
    push_impl<true, true>(c, A);
}

// ------------------------------------------------------- initial energy
__global__ void k_energy_H0(ParticleView P, double a) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  double z[6];
  load_z(P, k, z);
  P.H0[k] = energy(a, z);
}

void launch_energy_H0(grpic_ctx* c) {
  if (c->n == 0) return;
  ParticleView P = c->pv;
  P.n = c->n;
  hipLaunchKernelGGL(k_energy_H0, dim3(grid_for(c->n, 256)), dim3(256), 0,
                     c->stream, P, c->cfg.a);
  GRPIC_HIP(hipGetLastError());
}

}  // namespace grpic
