// api.hip -- the C ABI of the GRPIC library (include/grpic.h): context and
// memory management, grid set-up, particle loading, the per-step sequence of
// Sec. 2.1 (sub-steps 1-4, push, deposit, 7-10), hipGraph replay, kernel
// timing and diagnostics.
#include <math.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "kerr_device.hpp"

using namespace grpic;

namespace {

std::mutex g_err_mu;
std::string g_create_err;

int fail(grpic_ctx* c, int code, const std::string& msg) {
  if (c) {
    c->err = msg;
  } else {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_create_err = msg;
  }
  return code;
}

template <class F>
int guarded(grpic_ctx* c, F&& f) {
  try {
    f();
    return GRPIC_OK;
  } catch (const Error& e) {
    return fail(c, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(c, GRPIC_E_OOM, "host allocation failed");
  } catch (...) {
    return fail(c, GRPIC_E_INVALID, "unexpected error");
  }
}


// Courant limit of the leapfrog on this grid: the smallest
// 1 / sqrt((c_r/dr)^2 + (c_th/dth)^2) over the nodes, with the coordinate
// light speeds c_r = alpha sqrt(gamma^rr) + |beta^r|, c_th = alpha
// sqrt(gamma^thth).
double cfl_limit(const grpic_config& cfg) {
  const double a = cfg.a;
  double dlnr = log(cfg.r_out / cfg.r_in) / cfg.nr;
  double dth = (kPi - 2.0 * cfg.theta0) / cfg.nth;
  double best = 1e300;
  for (int i = 0; i < cfg.nr; ++i) {
    double r0 = cfg.r_in * exp(i * dlnr), r1 = cfg.r_in * exp((i + 1) * dlnr);
    double dr = r1 - r0;
    for (int j = 0; j <= cfg.nth; j += std::max(1, cfg.nth / 64)) {
      double th = cfg.theta0 + j * dth;
      double s = sin(th), c = cos(th);
      double rho2 = r0 * r0 + a * a * c * c;
      double xi = 1.0 + 2.0 * r0 / rho2;
      double alpha = 1.0 / sqrt(xi), beta = (xi - 1.0) / xi;
      double irr = a * a * s * s / rho2 + 1.0 / xi, itt = 1.0 / rho2;
      double cr = alpha * sqrt(irr) + fabs(beta), ct = alpha * sqrt(itt);
      double lim = 1.0 / sqrt((cr / dr) * (cr / dr) + (ct / dth) * (ct / dth));
      best = std::min(best, lim);
    }
  }
  return best;
}

void validate(const grpic_config& c) {
  auto bad = [](const char* m) { throw Error(GRPIC_E_INVALID, m); };
  if (!(c.a >= 0.0 && c.a < 1.0)) bad("spin a must lie in [0, 1)");
  if (!(c.dt != 0.0 && std::isfinite(c.dt))) bad("dt must be finite and nonzero");
  if (c.field_mode < 0 || c.field_mode > 2) bad("unknown field_mode");
  if (c.pusher < 0 || c.pusher > 4) bad("unknown pusher");
  if (c.guess < 0 || c.guess > 2) bad("unknown guess");
  if (c.kmax < 1 || c.kmax > 255) bad("kmax must lie in [1, 255]");
  if (!(c.tol > 0.0)) bad("tol must be positive");
  if (c.max_particles < 0 || c.max_particles > (1L << 31) - 1)
    bad("max_particles must lie in [0, 2^31)");
  if (c.field_mode != GRPIC_FIELDS_NONE) {
    if (c.nr < 2 || c.nth < 2) bad("grid needs at least 2 x 2 cells");
    if ((long)(c.nr + 1) * (c.nth + 1) > (1L << 30) || c.nr > (1 << 22) - 2 ||
        c.nth > (1 << 22) - 2)
      bad("grid too large: (nr + 1)(nth + 1) must not exceed 2^30 and nr, nth 2^22 - 2");
    if (!(c.r_in > 0.0 && c.r_out > c.r_in)) bad("need 0 < r_in < r_out");
    if (!(c.theta0 > 0.0 && c.theta0 < 0.5 * kPi)) bad("theta0 must lie in (0, pi/2)");
    if (c.tile_r < 1 || c.tile_th < 1) bad("tile sizes must be positive");
    if ((long)((c.nr + c.tile_r - 1) / c.tile_r) * ((c.nth + c.tile_th - 1) / c.tile_th) > 16384)
      bad("too many sort tiles (at most 16384): enlarge tile_r / tile_th");
    if (c.dt < 0.0) bad("dt must be positive with a grid");
  }
  if (!(c.dt_implicit >= 0.0 && std::isfinite(c.dt_implicit)))
    bad("dt_implicit must be finite and >= 0");
  if (!(c.t_end >= 0.0 && std::isfinite(c.t_end))) bad("t_end must be finite and >= 0");
  if (c.deposit_mode != GRPIC_DEPOSIT_CONSERVING && c.deposit_mode != GRPIC_DEPOSIT_PAPER)
    bad("unknown deposit_mode");
  if (c.clean_every < 0) bad("clean_every must be >= 0");
  if (c.clean_every > 0 && c.clean_iters < 1) bad("clean_iters must be >= 1");
  if ((c.deposit_mode != GRPIC_DEPOSIT_CONSERVING || c.clean_every > 0) &&
      c.field_mode != GRPIC_FIELDS_EVOLVE)
    bad("deposit_mode and clean_every need field_mode EVOLVE");
  if (c.solver != GRPIC_SOLVER_PICARD && c.solver != GRPIC_SOLVER_NEWTON)
    bad("unknown solver");
  if (c.inj_every < 0) bad("inj_every must be >= 0");
  if (c.inj_every > 0 && c.field_mode != GRPIC_FIELDS_EVOLVE)
    bad("inj_every needs field_mode EVOLVE");
  if (!(c.inj_mult > 0.0 && c.inj_density > 0.0 && c.inj_theta > 0.0))
    bad("inj_mult, inj_density and inj_theta must be positive");
  if ((c.dt_implicit > 0.0 && c.dt_implicit != c.dt) || c.t_end > 0.0) {
    if (c.field_mode != GRPIC_FIELDS_NONE)
      bad("steps of their own length and t_end need field_mode NONE");
    if (!(c.dt > 0.0)) bad("steps of their own length need dt > 0");
    if (c.guess == GRPIC_GUESS_MLP) bad("the learned guess needs one common dt");
  }
}

void alloc_particles(grpic_ctx* c, long cap) {
  ParticleView& P = c->pv;
  ParticleView& Q = c->alt;
  size_t n = (size_t)std::max(cap, 1L);
  for (ParticleView* V : {&P, &Q}) {
    V->r = dalloc<double>(n);
    V->th = dalloc<double>(n);
    V->ph = dalloc<double>(n);
    V->ur = dalloc<double>(n);
    V->uth = dalloc<double>(n);
    V->uph = dalloc<double>(n);
    V->H0 = dalloc<double>(n);
    V->herr = dalloc<double>(n);
    V->w = dalloc<double>(n);
    V->qm = dalloc<int8_t>(n);
    V->flags = dalloc<uint8_t>(n);
    V->iters = dalloc<uint8_t>(n);
    V->id = dalloc<uint32_t>(n);
    bool grid = c->cfg.field_mode != GRPIC_FIELDS_NONE;
    // weights of nodes 1..3; node 0's is the complement 1 - W1 - W2 - W3
    for (int q = 1; q < 4; ++q) V->W[q] = grid ? dalloc<uint32_t>(n) : nullptr;
    V->cell = grid ? dalloc<int>(n) : nullptr;
  }
  bool evolve = c->cfg.field_mode == GRPIC_FIELDS_EVOLVE;
  for (int q = 1; q < 4; ++q) P.Wn[q] = evolve ? dalloc<uint32_t>(n) : nullptr;
  P.celln = evolve ? dalloc<int>(n) : nullptr;
  P.r_old = evolve ? dalloc<double>(n) : nullptr;
  P.th_old = evolve ? dalloc<double>(n) : nullptr;
  P.dphi = evolve ? dalloc<float>(n) : nullptr;
  c->xqueue = evolve ? dalloc<int>(n) : nullptr;
  P.t = c->cfg.field_mode == GRPIC_FIELDS_NONE ? dalloc<double>(n) : nullptr;
  if (c->cfg.pusher != GRPIC_PUSH_RK4) {
    // explicit-pass block b appends to segment b % kQueueSegs, so a segment
    // holds at most ceil(blocks / kQueueSegs) blocks of kPushBlock entries
    long blocks = (n + kPushBlock - 1) / kPushBlock;
    c->seg_cap = (unsigned)(((blocks + kQueueSegs - 1) / kQueueSegs) * kPushBlock);
    size_t qlen = (size_t)c->seg_cap * kQueueSegs;
    c->queue = dalloc<int>(qlen);
    // first iterates (RK4 result, learned or collected Euler guess)
    for (int i = 0; i < 6; ++i) c->gz[i] = dalloc<double>(qlen);
  }
  c->cap = cap;
}

void free_particles(grpic_ctx* c) {
  for (ParticleView* V : {&c->pv, &c->alt}) {
    dfree(V->r);
    dfree(V->th);
    dfree(V->ph);
    dfree(V->ur);
    dfree(V->uth);
    dfree(V->uph);
    dfree(V->H0);
    dfree(V->herr);
    dfree(V->w);
    dfree(V->qm);
    dfree(V->flags);
    dfree(V->iters);
    dfree(V->id);
    for (int q = 0; q < 4; ++q) {
      dfree(V->W[q]);
      dfree(V->Wn[q]);
    }
    dfree(V->cell);
    dfree(V->celln);
    dfree(V->r_old);
    dfree(V->th_old);
    dfree(V->dphi);
    dfree(V->t);
  }
  dfree(c->queue);
  dfree(c->xqueue);
  for (int i = 0; i < 6; ++i) dfree(c->gz[i]);
}

#pragma clang fp contract(off)
void setup_grid(grpic_ctx* c) {
  const grpic_config& g = c->cfg;
  c->nr = g.nr;
  c->nth = g.nth;
  c->dlnr = log(g.r_out / g.r_in) / g.nr;
  c->dth = (kPi - 2.0 * g.theta0) / g.nth;
  c->h_rn.resize(g.nr + 1);
  c->h_rh.resize(g.nr);
  c->h_tn.resize(g.nth + 1);
  c->h_th.resize(g.nth);
  for (int i = 0; i <= g.nr; ++i) c->h_rn[i] = g.r_in * exp(i * c->dlnr);
  for (int i = 0; i < g.nr; ++i) c->h_rh[i] = sqrt(c->h_rn[i] * c->h_rn[i + 1]);
  for (int j = 0; j <= g.nth; ++j) c->h_tn[j] = g.theta0 + j * c->dth;
  for (int j = 0; j < g.nth; ++j) c->h_th[j] = g.theta0 + (j + 0.5) * c->dth;
  std::vector<double> idrn(g.nr), idrh(std::max(g.nr - 1, 1));
  std::vector<float> fdrn(g.nr), fdrd(g.nr + 1, 0.0f);
  for (int i = 0; i < g.nr; ++i) {
    idrn[i] = 1.0 / (c->h_rn[i + 1] - c->h_rn[i]);
    fdrn[i] = (float)idrn[i];
  }
  for (int i = 0; i + 1 < g.nr; ++i) idrh[i] = 1.0 / (c->h_rh[i + 1] - c->h_rh[i]);
  for (int i = 1; i < g.nr; ++i) fdrd[i] = (float)(1.0 / (c->h_rh[i] - c->h_rh[i - 1]));
  c->rn = dalloc<double>(g.nr + 1);
  c->rh = dalloc<double>(g.nr);
  c->tn = dalloc<double>(g.nth + 1);
  c->th = dalloc<double>(g.nth);
  c->idrn = dalloc<double>(g.nr);
  c->idrh = dalloc<double>(idrh.size());
  c->tab.inv_drn = dalloc<float>(g.nr);
  c->tab.inv_drd = dalloc<float>(g.nr + 1);
  std::vector<double> st(g.nth + 1), ct(g.nth + 1);
  for (int j = 0; j <= g.nth; ++j) {
    st[j] = sin(c->h_tn[j]);
    ct[j] = cos(c->h_tn[j]);
  }
  c->stn = dalloc<double>(g.nth + 1);
  c->ctn = dalloc<double>(g.nth + 1);
  std::vector<double> sh(g.nth), ch(g.nth);
  for (int j = 0; j < g.nth; ++j) {
    sh[j] = sin(c->h_th[j]);
    ch[j] = cos(c->h_th[j]);
  }
  c->sth = dalloc<double>(g.nth);
  c->cth = dalloc<double>(g.nth);
  auto up = [&](void* d, const void* h, size_t b) {
    GRPIC_HIP(hipMemcpy(d, h, b, hipMemcpyHostToDevice));
  };
  up(c->rn, c->h_rn.data(), sizeof(double) * (g.nr + 1));
  up(c->rh, c->h_rh.data(), sizeof(double) * g.nr);
  up(c->tn, c->h_tn.data(), sizeof(double) * (g.nth + 1));
  up(c->th, c->h_th.data(), sizeof(double) * g.nth);
  up(c->idrn, idrn.data(), sizeof(double) * g.nr);
  up(c->idrh, idrh.data(), sizeof(double) * idrh.size());
  up(c->tab.inv_drn, fdrn.data(), sizeof(float) * g.nr);
  up(c->tab.inv_drd, fdrd.data(), sizeof(float) * (g.nr + 1));
  up(c->stn, st.data(), sizeof(double) * (g.nth + 1));
  up(c->ctn, ct.data(), sizeof(double) * (g.nth + 1));
  up(c->sth, sh.data(), sizeof(double) * g.nth);
  up(c->cth, ch.data(), sizeof(double) * g.nth);
}
#pragma clang fp contract(on)

size_t node_count(const grpic_ctx* c) { return (size_t)(c->nr + 1) * (c->nth + 1); }

void alloc_fields(grpic_ctx* c) {
  size_t nn = node_count(c);
  for (int t = 0; t < 4; ++t) {
    c->tab.krr[t] = dalloc<float>(nn);
    c->tab.ktt[t] = dalloc<float>(nn);
    c->tab.kpp[t] = dalloc<float>(nn);
    c->tab.krp[t] = dalloc<float>(nn);
    c->tab.beta[t] = dalloc<float>(nn);
    c->tab.sg[t] = dalloc<float>(nn);
  }
  c->tab.damp_n = dalloc<float>(c->nr + 1);
  c->tab.damp_h = dalloc<float>(c->nr + 1);
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 3; ++q) {
      c->D[l].c[q] = dalloc<float>(nn);
      c->B[l].c[q] = dalloc<float>(nn);
      launch_fill(c, c->D[l].c[q], nn * 4);
      launch_fill(c, c->B[l].c[q], nn * 4);
    }
  for (int q = 0; q < 3; ++q) {
    c->E.c[q] = dalloc<float>(nn);
    c->H.c[q] = dalloc<float>(nn);
  }
  for (int s = 0; s < 2; ++s)
    for (int q = 0; q < 4; ++q) {
      c->J[s][q] = dalloc<float>(nn);
      launch_fill(c, c->J[s][q], nn * 4);
    }
  c->acc.Q = dalloc<long long>(nn);
  c->acc.P = dalloc<long long>(nn);
  c->acc.Fr = dalloc<long long>(nn);
  c->acc.Ft = dalloc<long long>(nn);
  for (long long* p : {c->acc.Q, c->acc.P, c->acc.Fr, c->acc.Ft})
    launch_fill(c, p, nn * 8);
  c->acc.scale = 1.0;
  int ntr = (c->nr + c->cfg.tile_r - 1) / c->cfg.tile_r;
  int ntt = (c->nth + c->cfg.tile_th - 1) / c->cfg.tile_th;
  c->ntiles = ntr * ntt;
  c->tile_count = dalloc<int>(c->ntiles + 1);
  c->tile_offset = dalloc<int>(c->ntiles + 1);
  launch_fill(c, c->tile_count, sizeof(int) * (c->ntiles + 1));
}

void free_all(grpic_ctx* c) {
  free_particles(c);
  dfree(c->rn);
  dfree(c->rh);
  dfree(c->tn);
  dfree(c->th);
  dfree(c->idrn);
  dfree(c->idrh);
  dfree(c->stn);
  dfree(c->ctn);
  dfree(c->sth);
  dfree(c->cth);
  for (int t = 0; t < 4; ++t) {
    dfree(c->tab.krr[t]);
    dfree(c->tab.ktt[t]);
    dfree(c->tab.kpp[t]);
    dfree(c->tab.krp[t]);
    dfree(c->tab.beta[t]);
    dfree(c->tab.sg[t]);
  }
  dfree(c->tab.damp_n);
  dfree(c->tab.damp_h);
  dfree(c->tab.inv_drn);
  dfree(c->tab.inv_drd);
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 3; ++q) {
      dfree(c->D[l].c[q]);
      dfree(c->B[l].c[q]);
    }
  for (int q = 0; q < 3; ++q) {
    dfree(c->E.c[q]);
    dfree(c->H.c[q]);
  }
  for (int s = 0; s < 2; ++s)
    for (int q = 0; q < 4; ++q) dfree(c->J[s][q]);
  for (double* p : {c->clean_kr, c->clean_kt, c->clean_kp, c->clean_src, c->clean_phi[0],
                    c->clean_phi[1]})
    dfree(p);
  dfree(c->inj_wsum);
  dfree(c->inj_flag);
  dfree(c->inj_off);
  dfree(c->inj_tot);
  dfree(c->inj_mj);
  dfree(c->acc.Q);
  dfree(c->acc.P);
  dfree(c->acc.Fr);
  dfree(c->acc.Ft);
  dfree(c->tile_count);
  dfree(c->tile_offset);
  dfree(c->dep_plan);
  dfree(c->dep_plan_off);
  dfree(c->dep_plan_meta);
  dfree(c->dep_plan_box);
  dfree(c->stats);
  mlp_free(c);
}

void drop_graphs(grpic_ctx* c);

// device state after particles change: sort, weights, initial rho
void particles_loaded(grpic_ctx* c) {
  drop_graphs(c);
  invalidate_deposit_plan(c);  // a new particle order
  launch_fill(c, c->stats, sizeof(Stats));
  c->steps = 0;
  if (c->pv.t && c->n > 0) launch_fill(c, c->pv.t, sizeof(double) * (size_t)c->n);
  if (c->cfg.field_mode == GRPIC_FIELDS_NONE) return;
  launch_sort(c);
  if (c->cfg.field_mode == GRPIC_FIELDS_EVOLVE) {
    c->acc.scale = c->qw_max > 0.0 ? ldexp(1.0, 40) / c->qw_max : 1.0;
    launch_deposit_initial(c);
  }
}

// ---------------------------------------------------------------- step
// Host ranges for tracing tools (roctx): one per part of the step, named
// after the sub-steps of Sec. 2.1; they mark when the launches are issued
// (and, for a captured graph, when it is recorded).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
};

void step_kernels(grpic_ctx* c) {
  bool evolve = c->cfg.field_mode == GRPIC_FIELDS_EVOLVE;
  hipEvent_t ev;
  if (evolve) {
    TraceRange t("grpic sub-steps 1-4: E, Faraday on both chains");
    time_begin(c, GRPIC_K_FIELDS, &ev);
    launch_fields_step_pre(c);
    time_end(c, GRPIC_K_FIELDS, ev);
  }
  {
    TraceRange t("grpic sub-step 5: gather and push (RK4, switch, implicit queue)");
    launch_push(c);
  }
  if (evolve) {
    {
      TraceRange t("grpic sub-step 6: deposit");
      launch_deposit(c);
    }
    TraceRange t("grpic sub-steps 7-10: H, Ampere on both chains");
    time_begin(c, GRPIC_K_FIELDS, &ev);
    launch_fields_step_post(c);
    time_end(c, GRPIC_K_FIELDS, ev);
  }
}

// the host-side pointer rotation that closes a step
void advance_host_state(grpic_ctx* c) {
  if (c->cfg.field_mode == GRPIC_FIELDS_EVOLVE) {
    std::swap(c->B[0], c->B[1]);  // B^{n+1} -> B^n slot, B^{n+2} -> B^{n+1}
    std::swap(c->D[1], c->D[2]);  // D^{n+3/2} -> D^{n+1/2}, new -> D^{n+3/2}
    c->jcur ^= 1;
    for (int q = 0; q < 4; ++q) std::swap(c->pv.W[q], c->pv.Wn[q]);
    std::swap(c->pv.cell, c->pv.celln);
  }
  c->steps += 1;
}

void drop_graphs(grpic_ctx* c) {
  for (auto& g : c->graph_exec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

std::vector<double> mj_table(double theta, int K, double* h_out);

// pair injection after a step or on call; returns the particles added
long inject_now(grpic_ctx* c) {
  const long ncell = (long)c->nr * c->nth;
  if (!c->inj_tot) {
    long long* wsum = nullptr;
    int *flag = nullptr, *off = nullptr, *tot = nullptr;
    double* mj = nullptr;
    try {
      wsum = dalloc<long long>(ncell);
      flag = dalloc<int>(ncell);
      off = dalloc<int>(ncell);
      mj = dalloc<double>(kInjMjK + 1);
      tot = dalloc<int>(4);
    } catch (...) {
      dfree(wsum);
      dfree(flag);
      dfree(off);
      dfree(mj);
      dfree(tot);
      throw;
    }
    double h = 0.0;
    std::vector<double> C = mj_table(c->cfg.inj_theta, kInjMjK, &h);
    GRPIC_HIP(hipMemcpy(mj, C.data(), sizeof(double) * (kInjMjK + 1), hipMemcpyHostToDevice));
    launch_fill(c, wsum, sizeof(long long) * ncell);
    c->inj_wsum = wsum;
    c->inj_flag = flag;
    c->inj_off = off;
    c->inj_mj = mj;
    c->inj_mj_h = h;
    c->inj_tot = tot;
  }
  long added = launch_inject(c, c->inj_mj, kInjMjK, c->inj_mj_h);
  if (added > 0) {
    // the deposit's fixed-point unit follows the largest weight (the
    // accumulators are empty between steps); captured steps are stale
    c->acc.scale = ldexp(1.0, 40) / c->qw_max;
    drop_graphs(c);
  }
  return added;
}

void run_step(grpic_ctx* c) {
  TraceRange t(c->use_graph ? "grpic step (graph replay)" : "grpic step");
  if (!c->use_graph) {
    step_kernels(c);
    advance_host_state(c);
  } else {
    const int key = (int)(c->steps & 1) + 2 * c->sort_flip;
    if (c->graph_exec[key] == nullptr) {
      bool was_timing = c->timing;
      c->timing = false;
      hipGraph_t g = nullptr;
      GRPIC_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      try {
        step_kernels(c);
      } catch (...) {
        (void)hipStreamEndCapture(c->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        c->timing = was_timing;
        throw;
      }
      GRPIC_HIP(hipStreamEndCapture(c->stream, &g));
      c->timing = was_timing;
      hipError_t e = hipGraphInstantiate(&c->graph_exec[key], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      GRPIC_HIP(e);
    }
    GRPIC_HIP(hipGraphLaunch(c->graph_exec[key], c->stream));
    advance_host_state(c);
  }
  if (c->cfg.clean_every > 0 && c->steps % c->cfg.clean_every == 0) {
    TraceRange r("grpic divergence cleaning");
    launch_clean(c, c->cfg.clean_iters);  // eager, after the step
  }
  if (c->cfg.inj_every > 0 && c->steps % c->cfg.inj_every == 0) {
    TraceRange r("grpic pair injection");
    inject_now(c);
  }
  if (c->cfg.sort_every > 0 && c->cfg.field_mode != GRPIC_FIELDS_NONE &&
      c->steps % c->cfg.sort_every == 0) {
    TraceRange r("grpic tile sort");
    // swaps the buffer sets (the other cached graphs apply); the full cycle
    // keeps every particle's node cell, which gives its tile directly
    launch_sort(c, c->cfg.field_mode == GRPIC_FIELDS_EVOLVE);
  }
}

hipEvent_t take_event(grpic_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  GRPIC_HIP(hipEventCreate(&e));
  return e;
}

void harvest_timings(grpic_ctx* c) {
  if (c->pending.empty()) return;
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float ms = 0.0f;
    GRPIC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    c->t_ms[p.kid] += ms;
    c->t_count[p.kid] += 1;
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
}

std::vector<double> mj_table(double theta, int K, double* h_out) {
  // cumulative Maxwell-Juettner speed distribution f(u) ~ u^2
  // exp(-(gamma - 1)/Theta) on [0, u_max], gamma_max - 1 = 50 Theta,
  // trapezoidal rule on K equal intervals, normalised to 1
  double gm = 1.0 + 50.0 * theta;
  double umax = sqrt(gm * gm - 1.0);
  double h = umax / K;
  std::vector<double> C(K + 1, 0.0);
  double fprev = 0.0;
  for (int k = 1; k <= K; ++k) {
    double u = k * h;
    double f = u * u * exp(-(sqrt(1.0 + u * u) - 1.0) / theta);
    C[k] = C[k - 1] + 0.5 * (fprev + f) * h;
    fprev = f;
  }
  double tot = C[K];
  for (int k = 0; k <= K; ++k) C[k] /= tot;
  *h_out = h;
  return C;
}

void check_ctx(grpic_ctx* c) {
  if (!c) throw Error(GRPIC_E_INVALID, "null context");
  GRPIC_HIP(hipSetDevice(c->device));
}

float* level_ptr(grpic_ctx* c, int level, int comp) {
  if (level >= GRPIC_LEVEL_DN && level <= GRPIC_LEVEL_DH1) {
    if (comp < 0 || comp > 2) throw Error(GRPIC_E_INVALID, "comp must be 0..2");
    return c->D[level - GRPIC_LEVEL_DN].c[comp];
  }
  if (level >= GRPIC_LEVEL_BM && level <= GRPIC_LEVEL_BH) {
    if (comp < 0 || comp > 2) throw Error(GRPIC_E_INVALID, "comp must be 0..2");
    return c->B[level - GRPIC_LEVEL_BM].c[comp];
  }
  if (level == GRPIC_LEVEL_J || level == GRPIC_LEVEL_JPREV) {
    if (comp < 0 || comp > 3) throw Error(GRPIC_E_INVALID, "comp must be 0..3");
    return c->J[level == GRPIC_LEVEL_J ? c->jcur : c->jcur ^ 1][comp];
  }
  throw Error(GRPIC_E_INVALID, "unknown field level");
}

size_t comp_size(grpic_ctx* c, int level, int comp) {
  // shapes: r-half for D^r/J^r (comp 0 of D/J levels) and B^th, B^ph
  bool is_b = level >= GRPIC_LEVEL_BM && level <= GRPIC_LEVEL_BH;
  bool rh, thh;
  if (is_b) {
    rh = comp == 1 || comp == 2;
    thh = comp == 0 || comp == 2;
  } else {
    rh = comp == 0;
    thh = comp == 1;
  }
  size_t nR = rh ? c->nr : c->nr + 1, nT = thh ? c->nth : c->nth + 1;
  return nR * nT;
}

}  // namespace

// ---------------------------------------------------------------- timing
namespace grpic {
void time_begin(grpic_ctx* c, int kid, hipEvent_t* a) {
  (void)kid;
  *a = nullptr;
  if (!c->timing) return;
  *a = take_event(c);
  GRPIC_HIP(hipEventRecord(*a, c->stream));
}
void time_end(grpic_ctx* c, int kid, hipEvent_t a) {
  if (!c->timing || a == nullptr) return;
  hipEvent_t b = take_event(c);
  GRPIC_HIP(hipEventRecord(b, c->stream));
  c->pending.push_back({kid, a, b});
}
}  // namespace grpic

// ================================================================== ABI
extern "C" {

int grpic_config_default(grpic_config* cfg) {
  if (!cfg) return GRPIC_E_INVALID;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->a = 0.0;
  cfg->nr = cfg->nth = 0;
  cfg->r_in = 1.0;
  cfg->r_out = 20.0;
  cfg->theta0 = kPi / 200.0;
  cfg->dt = 0.01;
  cfg->field_mode = GRPIC_FIELDS_NONE;
  cfg->pusher = GRPIC_PUSH_RK4;
  cfg->guess = GRPIC_GUESS_PLAIN;
  cfg->hyb_threshold = 0.0;
  cfg->tol = 1e-13;
  cfg->kmax = 50;
  cfg->ham_eps = 1e-10;
  cfg->r_abs = 0.0;
  cfg->chi0 = 0.0;
  cfg->lambda_abs = 5.0;
  cfg->r_remove_in = 0.0;
  cfg->r_remove_out = 1e300;
  cfg->reflect = 0;
  cfg->max_particles = 0;
  cfg->sort_every = 0;
  cfg->tile_r = 32;
  cfg->tile_th = 16;
  cfg->block = 256;
  cfg->persistent_waves = 8;
  cfg->deposit_mode = GRPIC_DEPOSIT_CONSERVING;
  cfg->clean_every = 0;
  cfg->clean_iters = 500;
  cfg->inj_every = 0;
  cfg->inj_r0 = cfg->inj_r1 = 0.0;
  cfg->inj_mult = 3.0;
  cfg->inj_density = 5.0;
  cfg->inj_theta = 0.5;
  cfg->inj_seed = 0;
  return GRPIC_OK;
}

int grpic_cfl_dt(const grpic_config* cfg, double* dt_out) {
  if (!cfg || !dt_out) return GRPIC_E_INVALID;
  if (cfg->nr < 2 || cfg->nth < 2 || !(cfg->r_out > cfg->r_in) || cfg->r_in <= 0)
    return fail(nullptr, GRPIC_E_INVALID, "grid needed for a Courant limit");
  *dt_out = cfl_limit(*cfg);
  return GRPIC_OK;
}

int grpic_create(const grpic_config* cfg, grpic_ctx** out) {
  if (!cfg || !out) return fail(nullptr, GRPIC_E_INVALID, "null argument");
  *out = nullptr;
  grpic_ctx* c = nullptr;
  try {
    grpic_config cf = *cfg;
    // dt = 0 with a grid: half the Courant limit
    if (cf.dt == 0.0 && cf.field_mode != GRPIC_FIELDS_NONE && cf.nr >= 2 && cf.nth >= 2 &&
        cf.r_in > 0.0 && cf.r_out > cf.r_in && cf.theta0 > 0.0 && cf.theta0 < 0.5 * kPi)
      cf.dt = 0.5 * cfl_limit(cf);
    cfg = &cf;
    validate(*cfg);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      (void)hipGetLastError();
      return fail(nullptr, GRPIC_E_NODEVICE, "no HIP device available");
    }
    if (cfg->field_mode == GRPIC_FIELDS_EVOLVE) {
      double lim = cfl_limit(*cfg);
      if (cfg->dt > lim)
        return fail(nullptr, GRPIC_E_CFL,
                    "dt = " + std::to_string(cfg->dt) +
                        " exceeds the Courant limit " + std::to_string(lim));
    }
    c = new grpic_ctx();
    c->cfg = *cfg;
    GRPIC_HIP(hipGetDevice(&c->device));
    diag_scratch_init(c->device);
    GRPIC_HIP(hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount,
                                    c->device));
    GRPIC_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
    c->stream = c->own_stream;
    c->stats = dalloc<Stats>(1);
    launch_fill(c, c->stats, sizeof(Stats));
    if (cfg->field_mode != GRPIC_FIELDS_NONE) {
      setup_grid(c);
      alloc_fields(c);
      launch_metric_tables(c);
    }
    alloc_particles(c, cfg->max_particles);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    *out = c;
    return GRPIC_OK;
  } catch (const Error& e) {
    if (c) {
      free_all(c);
      if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
      delete c;
    }
    return fail(nullptr, e.code, e.msg);
  } catch (...) {
    if (c) {
      free_all(c);
      delete c;
    }
    return fail(nullptr, GRPIC_E_INVALID, "unexpected error in grpic_create");
  }
}

void grpic_destroy(grpic_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  free_all(c);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

const char* grpic_last_error(const grpic_ctx* c) {
  if (c) return c->err.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  return g_create_err.c_str();
}

int grpic_get_config(grpic_ctx* c, grpic_config* out) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!out) throw Error(GRPIC_E_INVALID, "null pointer");
    *out = c->cfg;
  });
}

int grpic_set_stream(grpic_ctx* c, void* s) {
  return guarded(c, [&] {
    check_ctx(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->stream = s ? (hipStream_t)s : c->own_stream;
  });
}

int grpic_sync(grpic_ctx* c) {
  return guarded(c, [&] {
    check_ctx(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
  });
}

int grpic_grid_coords(grpic_ctx* c, double* rn, double* rh, double* tn,
                      double* th) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->nr == 0) throw Error(GRPIC_E_STATE, "context has no grid");
    if (rn) std::memcpy(rn, c->h_rn.data(), sizeof(double) * (c->nr + 1));
    if (rh) std::memcpy(rh, c->h_rh.data(), sizeof(double) * c->nr);
    if (tn) std::memcpy(tn, c->h_tn.data(), sizeof(double) * (c->nth + 1));
    if (th) std::memcpy(th, c->h_th.data(), sizeof(double) * c->nth);
  });
}

int grpic_set_fields_wald(grpic_ctx* c, double B0, double a_field) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->nr == 0) throw Error(GRPIC_E_STATE, "context has no grid");
    if (!std::isfinite(B0)) throw Error(GRPIC_E_INVALID, "B0 must be finite");
    if (!(a_field >= 0.0 && a_field < 1.0))
      throw Error(GRPIC_E_INVALID, "a_field must lie in [0, 1)");
    drop_graphs(c);
    launch_wald(c, B0, a_field);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
  });
}

int grpic_set_fields_split_monopole(grpic_ctx* c, double B0, double zeta0) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->nr == 0) throw Error(GRPIC_E_STATE, "context has no grid");
    drop_graphs(c);
    launch_split_monopole(c, B0, zeta0);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
  });
}

int grpic_set_field(grpic_ctx* c, int level, int comp, const float* host) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->nr == 0) throw Error(GRPIC_E_STATE, "context has no grid");
    if (!host) throw Error(GRPIC_E_INVALID, "null host buffer");
    float* d = level_ptr(c, level, comp);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    GRPIC_HIP(hipMemcpy(d, host, sizeof(float) * comp_size(c, level, comp),
                        hipMemcpyHostToDevice));
  });
}

int grpic_get_field(grpic_ctx* c, int level, int comp, float* host) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->nr == 0) throw Error(GRPIC_E_STATE, "context has no grid");
    if (!host) throw Error(GRPIC_E_INVALID, "null host buffer");
    float* d = level_ptr(c, level, comp);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    GRPIC_HIP(hipMemcpy(host, d, sizeof(float) * comp_size(c, level, comp),
                        hipMemcpyDeviceToHost));
  });
}

int grpic_init_particles(grpic_ctx* c, const grpic_init_spec* s) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!s) throw Error(GRPIC_E_INVALID, "null spec");
    if (s->n < 0 || s->n > c->cap) throw Error(GRPIC_E_INVALID, "n exceeds max_particles");
    if (s->kind < 0 || s->kind > 2) throw Error(GRPIC_E_INVALID, "unknown init kind");
    if (s->kind == GRPIC_INIT_ORBITS && (c->cfg.a != 0.0 || s->r0 <= 3.0))
      throw Error(GRPIC_E_INVALID, "orbit initial data need a = 0 and r0 > 3");
    if (s->kind != GRPIC_INIT_ORBITS && !(s->r0 > 0.0 && s->r1 > s->r0))
      throw Error(GRPIC_E_INVALID, "need 0 < r0 < r1");
    if (s->kind == GRPIC_INIT_SHELL_MJ && !(s->p0 > 0.0))
      throw Error(GRPIC_E_INVALID, "temperature must be positive");
    drop_graphs(c);
    double* dmj = nullptr;
    int K = 4096;
    double h = 0.0;
    if (s->kind == GRPIC_INIT_SHELL_MJ) {
      std::vector<double> C = mj_table(s->p0, K, &h);
      dmj = dalloc<double>(K + 1);
      GRPIC_HIP(hipMemcpy(dmj, C.data(), sizeof(double) * (K + 1), hipMemcpyHostToDevice));
    }
    c->n = s->n;
    if (s->n > 0) launch_init_particles(c, s, dmj, K, h);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    dfree(dmj);
    c->qw_max = fabs(s->w);
    c->has_neutral = s->kind == GRPIC_INIT_ORBITS;
    particles_loaded(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
  });
}

int grpic_load_particles(grpic_ctx* c, long n, const double* r,
                         const double* th, const double* ph, const double* ur,
                         const double* uth, const double* uph,
                         const double* qm, const double* w, const double* H0,
                         const double* herr) {
  return guarded(c, [&] {
    check_ctx(c);
    if (n < 0 || n > c->cap) throw Error(GRPIC_E_INVALID, "n exceeds max_particles");
    if (n > 0 && (!r || !th || !ph || !ur || !uth || !uph || !qm || !w))
      throw Error(GRPIC_E_INVALID, "null particle array");
    drop_graphs(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    c->n = n;
    if (n > 0) {
      auto up = [&](void* d, const void* h, size_t b) {
        GRPIC_HIP(hipMemcpy(d, h, b, hipMemcpyHostToDevice));
      };
      size_t b = sizeof(double) * n;
      ParticleView& P = c->pv;
      up(P.r, r, b);
      up(P.th, th, b);
      up(P.ph, ph, b);
      up(P.ur, ur, b);
      up(P.uth, uth, b);
      up(P.uph, uph, b);
      up(P.w, w, b);
      std::vector<int8_t> q(n);
      std::vector<uint8_t> fl(n, GRPIC_FLAG_ALIVE), it(n, 0);
      std::vector<uint32_t> id(n);
      double qwm = 0.0;
      c->has_neutral = false;
      for (long k = 0; k < n; ++k) {
        if (!(qm[k] == 1.0 || qm[k] == -1.0 || qm[k] == 0.0))
          throw Error(GRPIC_E_INVALID, "q/m must be +1, -1 or 0");
        q[k] = (int8_t)qm[k];
        id[k] = (uint32_t)k;
        if (q[k] != 0) qwm = std::max(qwm, fabs(w[k]));
        else c->has_neutral = true;
      }
      up(P.qm, q.data(), n);
      up(P.flags, fl.data(), n);
      up(P.iters, it.data(), n);
      up(P.id, id.data(), sizeof(uint32_t) * n);
      if (herr)
        up(P.herr, herr, b);
      else
        launch_fill(c, P.herr, b);
      c->qw_max = qwm;
      if (H0)
        up(P.H0, H0, b);
      else
        launch_energy_H0(c);
    }
    particles_loaded(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
  });
}

int grpic_sample_particles(grpic_ctx* c, long m, const long* ids, double* rec,
                           int32_t* flags, int32_t* iters) {
  return guarded(c, [&] {
    check_ctx(c);
    if (m < 0 || (m > 0 && (!ids || !rec))) throw Error(GRPIC_E_INVALID, "bad arguments");
    if (m == 0) return;
    if (m > (1L << 24)) throw Error(GRPIC_E_INVALID, "sample larger than 2^24");
    std::vector<int> map((size_t)c->n, -1);
    for (long s = 0; s < m; ++s) {
      if (ids[s] < 0 || ids[s] >= c->n) throw Error(GRPIC_E_INVALID, "id out of range");
      if (map[(size_t)ids[s]] >= 0) throw Error(GRPIC_E_INVALID, "repeated id");
      map[(size_t)ids[s]] = (int)s;
    }
    int* dmap = dalloc<int>((size_t)c->n);
    double* dout = nullptr;
    int* dfl = nullptr;
    try {
      dout = dalloc<double>((size_t)m * 10);
      dfl = dalloc<int>((size_t)m * 2);
      GRPIC_HIP(hipMemcpyAsync(dmap, map.data(), sizeof(int) * (size_t)c->n,
                               hipMemcpyHostToDevice, c->stream));
      launch_sample(c, dmap, dout, dfl);
      GRPIC_HIP(hipMemcpyAsync(rec, dout, sizeof(double) * 10 * (size_t)m,
                               hipMemcpyDeviceToHost, c->stream));
      std::vector<int> fl((size_t)m * 2);
      GRPIC_HIP(hipMemcpyAsync(fl.data(), dfl, sizeof(int) * 2 * (size_t)m,
                               hipMemcpyDeviceToHost, c->stream));
      GRPIC_HIP(hipStreamSynchronize(c->stream));
      for (long s = 0; s < m; ++s) {
        if (flags) flags[s] = fl[2 * s];
        if (iters) iters[s] = fl[2 * s + 1];
      }
    } catch (...) {
      (void)hipStreamSynchronize(c->stream);
      dfree(dmap);
      dfree(dout);
      dfree(dfl);
      throw;
    }
    dfree(dmap);
    dfree(dout);
    dfree(dfl);
  });
}

int grpic_num_particles(grpic_ctx* c, long* n) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!n) throw Error(GRPIC_E_INVALID, "null pointer");
    *n = c->n;
  });
}

int grpic_get_times(grpic_ctx* c, long n, double* t) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!c->pv.t) throw Error(GRPIC_E_STATE, "particle clocks exist only without a grid");
    if (n != c->n) throw Error(GRPIC_E_INVALID, "n differs from the particle count");
    if (n > 0 && !t) throw Error(GRPIC_E_INVALID, "null host buffer");
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    if (n == 0) return;
    std::vector<uint32_t> id(n);
    std::vector<double> tmp(n);
    GRPIC_HIP(hipMemcpy(id.data(), c->pv.id, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
    GRPIC_HIP(hipMemcpy(tmp.data(), c->pv.t, sizeof(double) * n, hipMemcpyDeviceToHost));
    for (long k = 0; k < n; ++k) t[id[k]] = tmp[k];
  });
}

int grpic_get_particles(grpic_ctx* c, long n, double* r, double* th,
                        double* ph, double* ur, double* uth, double* uph,
                        double* qm, double* w, double* H0, double* herr,
                        int32_t* flags, int32_t* iters) {
  return guarded(c, [&] {
    check_ctx(c);
    if (n != c->n) throw Error(GRPIC_E_INVALID, "n differs from the particle count");
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    if (n == 0) return;
    std::vector<uint32_t> id(n);
    GRPIC_HIP(hipMemcpy(id.data(), c->pv.id, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
    std::vector<double> tmp(n);
    auto get_d = [&](double* out, const double* d) {
      if (!out) return;
      GRPIC_HIP(hipMemcpy(tmp.data(), d, sizeof(double) * n, hipMemcpyDeviceToHost));
      for (long k = 0; k < n; ++k) out[id[k]] = tmp[k];
    };
    const ParticleView& P = c->pv;
    get_d(r, P.r);
    get_d(th, P.th);
    get_d(ph, P.ph);
    get_d(ur, P.ur);
    get_d(uth, P.uth);
    get_d(uph, P.uph);
    get_d(w, P.w);
    get_d(H0, P.H0);
    get_d(herr, P.herr);
    std::vector<uint8_t> b8(n);
    if (qm) {
      GRPIC_HIP(hipMemcpy(b8.data(), P.qm, n, hipMemcpyDeviceToHost));
      for (long k = 0; k < n; ++k) qm[id[k]] = (double)(int8_t)b8[k];
    }
    if (flags) {
      GRPIC_HIP(hipMemcpy(b8.data(), P.flags, n, hipMemcpyDeviceToHost));
      for (long k = 0; k < n; ++k) flags[id[k]] = b8[k];
    }
    if (iters) {
      GRPIC_HIP(hipMemcpy(b8.data(), P.iters, n, hipMemcpyDeviceToHost));
      for (long k = 0; k < n; ++k) iters[id[k]] = b8[k];
    }
  });
}

int grpic_step(grpic_ctx* c, int nsteps) {
  return guarded(c, [&] {
    check_ctx(c);
    if (nsteps < 0) throw Error(GRPIC_E_INVALID, "nsteps must be >= 0");
    if (c->cfg.guess == GRPIC_GUESS_MLP && !c->mlp_ready && !mlp_collecting(c))
      throw Error(GRPIC_E_STATE, "learned guess selected but no network set");
    for (int s = 0; s < nsteps; ++s) run_step(c);
  });
}

int grpic_use_graph(grpic_ctx* c, int enable) {
  return guarded(c, [&] {
    check_ctx(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->use_graph = enable != 0;
  });
}

int grpic_get_diagnostics(grpic_ctx* c, grpic_diag* out) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!out) throw Error(GRPIC_E_INVALID, "null pointer");
    std::unique_ptr<Stats> sp(new Stats);
    const Stats& s = *sp;
    launch_census(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    GRPIC_HIP(hipMemcpy(sp.get(), c->stats, sizeof(Stats), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->steps = c->steps;
    out->alive = (long)s.census[0];
    for (int i = 0; i < GRPIC_HIST_BINS; ++i) out->herr_hist[i] = (long)s.census[1 + i];
    for (const StatRep& r : s.rep) {
      out->removed += (long)r.removed;
      out->implicit_steps += (long)r.implicit_steps;
      out->noconv += (long)r.noconv;
      out->reflected += (long)r.reflected;
      out->nonfinite += (long)r.nonfinite;
      for (int i = 0; i < GRPIC_HIST_BINS; ++i) out->iter_hist[i] += (long)r.iter_hist[i];
    }
    out->deposit_fallback = (long)s.deposit_fallback;
    out->deposit_outside = (long)s.deposit_outside;
  });
}

int grpic_field_diagnostics(grpic_ctx* c, double* gauss_max, double* divb_max,
                            double* pbz) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->nr == 0) throw Error(GRPIC_E_STATE, "context has no grid");
    launch_field_diag(c, gauss_max, divb_max, pbz);
  });
}

int grpic_field_diagnostics_noalloc(grpic_ctx* c, double* gauss_max, double* divb_max,
                                    double* pbz) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->nr == 0) throw Error(GRPIC_E_STATE, "context has no grid");
    field_diag_noalloc(c, gauss_max, divb_max, pbz);
  });
}

int grpic_clean(grpic_ctx* c, int iters) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->cfg.field_mode != GRPIC_FIELDS_EVOLVE)
      throw Error(GRPIC_E_STATE, "cleaning needs field_mode EVOLVE");
    if (iters < 1) throw Error(GRPIC_E_INVALID, "iters must be >= 1");
    launch_clean(c, iters);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
  });
}

int grpic_inject(grpic_ctx* c, long* added) {
  return guarded(c, [&] {
    check_ctx(c);
    if (c->cfg.field_mode != GRPIC_FIELDS_EVOLVE)
      throw Error(GRPIC_E_STATE, "injection needs field_mode EVOLVE");
    long n = inject_now(c);
    if (added) *added = n;
  });
}

int grpic_enable_timing(grpic_ctx* c, int enable) {
  return guarded(c, [&] {
    check_ctx(c);
    harvest_timings(c);
    c->timing = enable != 0;
  });
}

int grpic_get_timings(grpic_ctx* c, double* ms, long* count) {
  return guarded(c, [&] {
    check_ctx(c);
    harvest_timings(c);
    for (int k = 0; k < GRPIC_K_COUNT; ++k) {
      if (ms) ms[k] = c->t_ms[k];
      if (count) count[k] = c->t_count[k];
    }
  });
}

int grpic_reset_timings(grpic_ctx* c) {
  return guarded(c, [&] {
    check_ctx(c);
    harvest_timings(c);
    for (int k = 0; k < GRPIC_K_COUNT; ++k) {
      c->t_ms[k] = 0.0;
      c->t_count[k] = 0;
    }
  });
}

int grpic_mlp_set(grpic_ctx* c, const float* theta, const float* mean,
                  const float* inv_std, const float* scale) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!theta || !mean || !inv_std || !scale) throw Error(GRPIC_E_INVALID, "null pointer");
    drop_graphs(c);
    mlp_upload(c, theta, mean, inv_std, scale);
    c->mlp_ready = true;
  });
}

int grpic_mlp_get(grpic_ctx* c, float* theta, float* mean, float* inv_std, float* scale) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!theta || !mean || !inv_std || !scale) throw Error(GRPIC_E_INVALID, "null pointer");
    if (!c->mlp_ready) throw Error(GRPIC_E_STATE, "no network loaded");
    mlp_download(c, theta, mean, inv_std, scale);
  });
}

int grpic_mlp_collect(grpic_ctx* c, long max_rows) {
  return guarded(c, [&] {
    check_ctx(c);
    if (max_rows < 0) throw Error(GRPIC_E_INVALID, "negative sample count");
    if (max_rows > 0 && c->cfg.pusher == GRPIC_PUSH_RK4)
      throw Error(GRPIC_E_STATE, "the RK4 pusher has no implicit pass to sample");
    drop_graphs(c);
    mlp_collect_start(c, max_rows);
  });
}

int grpic_mlp_num_samples(grpic_ctx* c, long* n) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!n) throw Error(GRPIC_E_INVALID, "null pointer");
    *n = mlp_num_samples(c);
  });
}

int grpic_mlp_get_samples(grpic_ctx* c, long n, float* X, float* T, unsigned char* valid) {
  return guarded(c, [&] {
    check_ctx(c);
    if (n < 0) throw Error(GRPIC_E_INVALID, "negative sample count");
    mlp_get_samples(c, n, X, T, valid);
  });
}

int grpic_mlp_train(grpic_ctx* c, const grpic_mlp_train_config* tc, double* epoch_loss) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!tc) throw Error(GRPIC_E_INVALID, "null pointer");
    drop_graphs(c);
    mlp_train(c, tc, epoch_loss);
  });
}

int grpic_mlp_forward(grpic_ctx* c, long n, const float* X, float* Y) {
  return guarded(c, [&] {
    check_ctx(c);
    if (n < 0 || (n > 0 && (!X || !Y))) throw Error(GRPIC_E_INVALID, "bad arguments");
    mlp_forward_rows(c, n, X, Y);
  });
}

int grpic_mlp_loss_grad(grpic_ctx* c, long n, const float* X, const float* T, float* grad,
                        double* loss) {
  return guarded(c, [&] {
    check_ctx(c);
    if (n <= 0 || !X || !T || !grad || !loss) throw Error(GRPIC_E_INVALID, "bad arguments");
    mlp_loss_grad(c, n, X, T, grad, loss);
  });
}

}  // extern "C"

// ------------------------------------------------------------- autotuner
namespace {

double time_steps(grpic_ctx* c, int k) {
  run_step(c);  // untimed: graph capture, caches
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  hipEvent_t a, b;
  GRPIC_HIP(hipEventCreate(&a));
  GRPIC_HIP(hipEventCreate(&b));
  float ms = 0.0f;
  try {
    GRPIC_HIP(hipEventRecord(a, c->stream));
    for (int s = 0; s < k; ++s) run_step(c);
    GRPIC_HIP(hipEventRecord(b, c->stream));
    GRPIC_HIP(hipEventSynchronize(b));
    GRPIC_HIP(hipEventElapsedTime(&ms, a, b));
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return (double)ms / k;
}

bool set_tiles(grpic_ctx* c, int tr, int tt) {
  long ntr = (c->nr + tr - 1) / tr, ntt = (c->nth + tt - 1) / tt;
  if (ntr * ntt > 16384) return false;
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  dfree(c->tile_count);
  dfree(c->tile_offset);
  c->cfg.tile_r = tr;
  c->cfg.tile_th = tt;
  c->ntiles = (int)(ntr * ntt);
  c->tile_count = dalloc<int>(c->ntiles + 1);
  c->tile_offset = dalloc<int>(c->ntiles + 1);
  launch_fill(c, c->tile_count, sizeof(int) * (c->ntiles + 1));
  launch_sort(c);
  return true;
}

}  // namespace

int grpic_autotune(grpic_ctx* c, int trial_steps, grpic_tune_result* out) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!out || trial_steps < 1) throw Error(GRPIC_E_INVALID, "bad arguments");
    if (c->n == 0) throw Error(GRPIC_E_STATE, "no particles loaded");
    std::memset(out, 0, sizeof(*out));
    const long steps0 = c->steps;
    const int sort_every = c->cfg.sort_every;
    c->cfg.sort_every = 0;  // no re-sort inside the trials
    try {
      const bool grid = c->cfg.field_mode != GRPIC_FIELDS_NONE;
      const bool implicit = c->cfg.pusher != GRPIC_PUSH_RK4;
      if (grid) set_tiles(c, c->cfg.tile_r, c->cfg.tile_th);
      double best = time_steps(c, trial_steps);
      out->ms_start = best;
      out->trials = 1;
      if (grid) {
        const int cand[5][2] = {{16, 16}, {32, 16}, {32, 32}, {64, 16}, {64, 32}};
        int br = c->cfg.tile_r, bt = c->cfg.tile_th;
        for (auto& t : cand) {
          if (t[0] == br && t[1] == bt) continue;
          if (!set_tiles(c, t[0], t[1])) continue;
          double ms = time_steps(c, trial_steps);
          ++out->trials;
          if (ms < best) {
            best = ms;
            br = t[0];
            bt = t[1];
          }
        }
        set_tiles(c, br, bt);
      }
      if (implicit) {
        int bw = c->cfg.persistent_waves;
        for (int w : {4, 8, 16, 32}) {
          if (w == bw) continue;
          c->cfg.persistent_waves = w;
          drop_graphs(c);
          double ms = time_steps(c, trial_steps);
          ++out->trials;
          if (ms < best) {
            best = ms;
            bw = w;
          }
        }
        c->cfg.persistent_waves = bw;
      }
      {
        int bp = c->cfg.push_waves_per_simd;
        for (int p : {0, 4}) {
          if (p == bp) continue;
          c->cfg.push_waves_per_simd = p;
          drop_graphs(c);
          double ms = time_steps(c, trial_steps);
          ++out->trials;
          if (ms < best) {
            best = ms;
            bp = p;
          }
        }
        c->cfg.push_waves_per_simd = bp;
      }
      drop_graphs(c);
      out->tile_r = c->cfg.tile_r;
      out->tile_th = c->cfg.tile_th;
      out->persistent_waves = c->cfg.persistent_waves;
      out->push_waves_per_simd = c->cfg.push_waves_per_simd;
      out->ms_best = best;
      out->steps = (int)(c->steps - steps0);
    } catch (...) {
      c->cfg.sort_every = sort_every;
      throw;
    }
    c->cfg.sort_every = sort_every;
  });
}

int grpic_probe_peaks(grpic_ctx* c, double* fp64_fma_tflops, double* copy_tbs) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!fp64_fma_tflops || !copy_tbs) throw Error(GRPIC_E_INVALID, "null pointer");
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    probe_peaks(c, fp64_fma_tflops, copy_tbs);
  });
}

// ------------------------------------------------------ state snapshots
namespace {

struct StateItem {
  void* d;
  size_t bytes;
};

// the device arrays of a snapshot, in snapshot order, for n particles
std::vector<StateItem> state_items(grpic_ctx* c, long n) {
  std::vector<StateItem> v;
  if (c->nr > 0) {
    for (int lev = GRPIC_LEVEL_DN; lev <= GRPIC_LEVEL_JPREV; ++lev) {
      int nc = lev >= GRPIC_LEVEL_J ? 4 : 3;
      for (int q = 0; q < nc; ++q)
        v.push_back({level_ptr(c, lev, q), sizeof(float) * comp_size(c, lev, q)});
    }
  }
  const ParticleView& P = c->pv;
  size_t d = sizeof(double) * (size_t)n;
  for (double* a : {P.r, P.th, P.ph, P.ur, P.uth, P.uph, P.H0, P.herr, P.w})
    v.push_back({a, d});
  v.push_back({P.qm, (size_t)n});
  v.push_back({P.flags, (size_t)n});
  v.push_back({P.iters, (size_t)n});
  v.push_back({P.id, sizeof(uint32_t) * (size_t)n});
  if (P.cell) {
    for (int q = 1; q < 4; ++q) v.push_back({P.W[q], sizeof(uint32_t) * (size_t)n});
    v.push_back({P.cell, sizeof(int) * (size_t)n});
  }
  if (P.t) v.push_back({P.t, d});
  v.push_back({c->stats, sizeof(Stats)});
  return v;
}

size_t state_bytes(const std::vector<StateItem>& v) {
  size_t b = sizeof(grpic_state_header);
  for (const StateItem& s : v) b += s.bytes;
  return b;
}

const char kStateMagic[8] = {'G', 'R', 'P', 'I', 'C', 'S', 'T', 0};

}  // namespace

extern "C" {

int grpic_state_size(grpic_ctx* c, size_t* bytes) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!bytes) throw Error(GRPIC_E_INVALID, "null pointer");
    *bytes = state_bytes(state_items(c, c->n));
  });
}

int grpic_get_state(grpic_ctx* c, void* host, size_t bytes) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!host) throw Error(GRPIC_E_INVALID, "null host buffer");
    std::vector<StateItem> items = state_items(c, c->n);
    size_t need = state_bytes(items);
    if (bytes < need) throw Error(GRPIC_E_INVALID, "buffer smaller than the snapshot");
    grpic_state_header h{};
    std::memcpy(h.magic, kStateMagic, sizeof(h.magic));
    h.version = 2;
    h.field_mode = c->cfg.field_mode;
    h.nr = c->nr;
    h.nth = c->nth;
    h.a = c->cfg.a;
    h.r_in = c->cfg.r_in;
    h.r_out = c->cfg.r_out;
    h.theta0 = c->cfg.theta0;
    h.dt = c->cfg.dt;
    h.n = c->n;
    h.steps = c->steps;
    h.qw_max = c->qw_max;
    h.has_neutral = c->has_neutral ? 1 : 0;
    h.bytes = need;
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    char* out = static_cast<char*>(host);
    std::memcpy(out, &h, sizeof(h));
    size_t off = sizeof(h);
    for (const StateItem& s : items) {
      if (s.bytes) GRPIC_HIP(hipMemcpy(out + off, s.d, s.bytes, hipMemcpyDeviceToHost));
      off += s.bytes;
    }
  });
}

int grpic_set_state(grpic_ctx* c, const void* host, size_t bytes) {
  return guarded(c, [&] {
    check_ctx(c);
    if (!host) throw Error(GRPIC_E_INVALID, "null host buffer");
    grpic_state_header h;
    if (bytes < sizeof(h)) throw Error(GRPIC_E_INVALID, "block shorter than a snapshot header");
    std::memcpy(&h, host, sizeof(h));
    if (std::memcmp(h.magic, kStateMagic, sizeof(h.magic)) != 0 || h.version != 2)
      throw Error(GRPIC_E_INVALID, "not a snapshot of this library");
    if (h.field_mode != c->cfg.field_mode || h.nr != c->nr || h.nth != c->nth ||
        h.a != c->cfg.a || h.dt != c->cfg.dt ||
        (c->nr > 0 && (h.r_in != c->cfg.r_in || h.r_out != c->cfg.r_out ||
                       h.theta0 != c->cfg.theta0)))
      throw Error(GRPIC_E_INVALID, "snapshot taken on another grid, field mode or dt");
    if (h.n < 0 || h.n > c->cap) throw Error(GRPIC_E_INVALID, "snapshot exceeds max_particles");
    std::vector<StateItem> items = state_items(c, (long)h.n);
    size_t need = state_bytes(items);
    if (h.bytes != need || bytes < need)
      throw Error(GRPIC_E_INVALID, "snapshot size does not match its header");
    drop_graphs(c);
    GRPIC_HIP(hipStreamSynchronize(c->stream));
    const char* in = static_cast<const char*>(host);
    size_t off = sizeof(h);
    for (const StateItem& s : items) {
      if (s.bytes) GRPIC_HIP(hipMemcpy(s.d, in + off, s.bytes, hipMemcpyHostToDevice));
      off += s.bytes;
    }
    c->n = (long)h.n;
    c->steps = (long)h.steps;
    invalidate_deposit_plan(c);  // the snapshot's particle order
    c->qw_max = h.qw_max;
    c->has_neutral = h.has_neutral != 0;
    if (c->cfg.field_mode == GRPIC_FIELDS_EVOLVE)
      c->acc.scale = c->qw_max > 0.0 ? ldexp(1.0, 40) / c->qw_max : 1.0;
  });
}

}  // extern "C"
