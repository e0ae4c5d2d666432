// deposit.hip -- charge and current deposit (sub-step 6 of Sec. 2.1).
//
// Weights are the paper's volume fractions (Sec. 2.3); the current is the
// charge-conserving one: the straight move in (r, theta) is cut at node-cell
// boundaries, the weight change inside a cell becomes four face fluxes
//   S_r = W10 + W11, S_t = W01 + W11, Fr1 = dS_r (S_t + S_t')/2,
//   Fr0 = dS_r - Fr1, Ft1 = dW11 - Fr1, Ft0 = dS_t - Ft1,
// and the jump of the (cell-dependent) weights at a crossing point moves
// along the shared edge.  Sums are accumulated in 64-bit fixed point with
// integer atomics, so the result does not depend on the order in which
// particles are processed.  A finalize pass turns the sums into densitized
// FP32 sqrt(g) rho, sqrt(g) J^r, sqrt(g) J^theta, sqrt(g) J^phi and clears
// the accumulators.
#include "deposit_device.hpp"

namespace grpic {

struct DepArgs {
  GridView g;
  ParticleView p;
  DepositAcc acc;
  int nr, nth;
};

__device__ __forceinline__ void acc_add(long long* a, long idx, double v,
                                        double scale) {
  long long q = llrint(v * scale);
  if (q != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(a + idx),
              static_cast<unsigned long long>(q));
}

// face fluxes (in charge units) of a weight change inside node cell (p, q)
__device__ __forceinline__ void cell_flux(const DepArgs& A, int p, int q,
                                          const double* W0, const double* W1,
                                          double qw) {
  double dSr = (W1[1] + W1[3]) - (W0[1] + W0[3]);
  double St0 = W0[2] + W0[3], St1 = W1[2] + W1[3];
  double dSt = St1 - St0, dW11 = W1[3] - W0[3];
  double Fr1 = 0.5 * dSr * (St0 + St1);
  double Fr0 = dSr - Fr1;
  double Ft1 = dW11 - Fr1;
  double Ft0 = dSt - Ft1;
  double s = A.acc.scale;
  acc_add(A.acc.Fr, (long)q * A.nr + p, qw * Fr0, s);
  acc_add(A.acc.Fr, (long)(q + 1) * A.nr + p, qw * Fr1, s);
  acc_add(A.acc.Ft, (long)q * (A.nr + 1) + p, qw * Ft0, s);
  acc_add(A.acc.Ft, (long)q * (A.nr + 1) + p + 1, qw * Ft1, s);
}

__global__ __launch_bounds__(256) void k_deposit(DepArgs A) {
  const ParticleView& P = A.p;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  if (!(P.flags[k] & GRPIC_FLAG_ALIVE)) return;
  const int nrn = A.nr + 1;
  double qw = (double)P.qm[k] * P.w[k];
  if (qw == 0.0) return;
  int c0 = P.cell[k], c1 = P.celln[k];
  int p0 = c0 % A.nr, q0 = c0 / A.nr, p1 = c1 % A.nr, q1 = c1 / A.nr;
  double Wo[4], Wn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Wo[c] = P.W[c][k];
    Wn[c] = P.Wn[c][k];
  }
  const double s = A.acc.scale;
  const double hdphi = 0.5 * qw * P.dphi[k];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int di = c & 1, dj = c >> 1;
    long nn = (long)(q1 + dj) * nrn + p1 + di;
    long no = (long)(q0 + dj) * nrn + p0 + di;
    acc_add(A.acc.Q, nn, qw * Wn[c], s);
    acc_add(A.acc.P, no, hdphi * Wo[c], s);
    acc_add(A.acc.P, nn, hdphi * Wn[c], s);
  }
  if (c0 == c1) {
    cell_flux(A, p0, q0, Wo, Wn, qw);
    return;
  }
  // walk the move through the node cells it crosses
  const double r0 = P.r_old[k], t0 = P.th_old[k], r1 = P.r[k], t1 = P.th[k];
  int cp = p0, cq = q0;
  double Wa[4] = {Wo[0], Wo[1], Wo[2], Wo[3]};
  for (int guard = 0; guard < 16 && (cp != p1 || cq != q1); ++guard) {
    double tr = 2.0, tt = 2.0;
    int br = -1, bt = -1;
    if (p1 > cp) br = cp + 1;
    else if (p1 < cp) br = cp;
    if (q1 > cq) bt = cq + 1;
    else if (q1 < cq) bt = cq;
    if (br >= 0) tr = (A.g.rn[br] - r0) / (r1 - r0);
    if (bt >= 0) tt = (A.g.tn[bt] - t0) / (t1 - t0);
    double xr, xt, Wb[4], Wc[4], jump;
    if (tr <= tt) {
      xr = A.g.rn[br];
      xt = t0 + tr * (t1 - t0);
      dep_weights(A.g, xr, xt, cp, cq, Wb);
      cell_flux(A, cp, cq, Wa, Wb, qw);
      int np = (br > cp) ? cp + 1 : cp - 1;
      dep_weights(A.g, xr, xt, np, cq, Wc);
      // node (br, cq+1): slot 3 of the old cell if br = cp+1 else slot 2;
      // in the new cell slot 2 if br = np else slot 3
      double prev = (br == cp + 1) ? Wb[3] : Wb[2];
      double now = (br == np) ? Wc[2] : Wc[3];
      jump = now - prev;
      acc_add(A.acc.Ft, (long)cq * nrn + br, qw * jump, s);
      cp = np;
    } else {
      xr = r0 + tt * (r1 - r0);
      xt = A.g.tn[bt];
      dep_weights(A.g, xr, xt, cp, cq, Wb);
      cell_flux(A, cp, cq, Wa, Wb, qw);
      int nq = (bt > cq) ? cq + 1 : cq - 1;
      dep_weights(A.g, xr, xt, cp, nq, Wc);
      // node (cp+1, bt): slot 3 of the old cell if bt = cq+1 else slot 1
      double prev = (bt == cq + 1) ? Wb[3] : Wb[1];
      double now = (bt == nq) ? Wc[1] : Wc[3];
      jump = now - prev;
      acc_add(A.acc.Fr, (long)bt * A.nr + cp, qw * jump, s);
      cq = nq;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) Wa[c] = Wc[c];
  }
  cell_flux(A, cp, cq, Wa, Wn, qw);
}

// charge of the current positions only (initial rho)
__global__ __launch_bounds__(256) void k_deposit_rho(DepArgs A) {
  const ParticleView& P = A.p;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  if (!(P.flags[k] & GRPIC_FLAG_ALIVE)) return;
  double qw = (double)P.qm[k] * P.w[k];
  int c0 = P.cell[k];
  int p0 = c0 % A.nr, q0 = c0 / A.nr;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    long nn = (long)(q0 + (c >> 1)) * (A.nr + 1) + p0 + (c & 1);
    acc_add(A.acc.Q, nn, qw * P.W[c][k], A.acc.scale);
  }
}

// weights and node cell of the current positions
__global__ __launch_bounds__(256) void k_weights(GridView g, ParticleView P) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  if (!(P.flags[k] & GRPIC_FLAG_ALIVE)) return;
  int p, q;
  double r = P.r[k], th = P.th[k];
  node_cell(g, r, th, p, q);
  double W[4];
  dep_weights(g, r, th, p, q, W);
#pragma unroll
  for (int c = 0; c < 4; ++c) P.W[c][k] = W[c];
  P.cell[k] = q * g.nr + p;
}

// dual lengths of node (i, j): half cells on the edges
__device__ __forceinline__ double dual_r(const GridView& g, int i) {
  if (i == 0) return g.rh[0] - g.rn[0];
  if (i == g.nr) return g.rn[g.nr] - g.rh[g.nr - 1];
  return g.rh[i] - g.rh[i - 1];
}
__device__ __forceinline__ double dual_t(const GridView& g, int j) {
  return (j == 0 || j == g.nth) ? 0.5 * g.dth : g.dth;
}

__global__ __launch_bounds__(256) void k_deposit_finalize(
    GridView g, DepositAcc acc, double dt, float* Jr, float* Jt, float* Jp,
    float* rho) {
  const int nrn = g.nr + 1, ntn = g.nth + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long nn = (long)nrn * ntn;
  if (k >= nn) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  const double is = 1.0 / acc.scale, tp = 2.0 * kPi;
  double Lr = dual_r(g, i), Lt = dual_t(g, j);
  rho[k] = (float)((double)acc.Q[k] * is / (tp * Lr * Lt));
  Jp[k] = (float)((double)acc.P[k] * is / (dt * tp * Lr * Lt));
  acc.Q[k] = 0;
  acc.P[k] = 0;
  if (i < g.nr) {  // J^r at (i+1/2, j)
    long kk = (long)j * g.nr + i;
    Jr[kk] = (float)((double)acc.Fr[kk] * is / (dt * tp * Lt));
    acc.Fr[kk] = 0;
  }
  if (j < g.nth) {  // J^theta at (i, j+1/2)
    long kk = (long)j * nrn + i;
    Jt[kk] = (float)((double)acc.Ft[kk] * is / (dt * tp * Lr));
    acc.Ft[kk] = 0;
  }
}

static GridView grid_view(grpic_ctx* c) { return make_grid_view(c); }

static void finalize(grpic_ctx* c, int which) {
  long nn = (long)(c->nr + 1) * (c->nth + 1);
  float** J = c->J[which];
  hipLaunchKernelGGL(k_deposit_finalize, dim3(grid_for(nn, 256)), dim3(256), 0,
                     c->stream, grid_view(c), c->acc, c->cfg.dt, J[0], J[1],
                     J[2], J[3]);
  GRPIC_HIP(hipGetLastError());
}

void launch_deposit(grpic_ctx* c) {
  hipEvent_t ev;
  time_begin(c, GRPIC_K_DEPOSIT, &ev);
  if (c->n > 0) {
    DepArgs A;
    A.g = grid_view(c);
    A.p = c->pv;
    A.p.n = c->n;
    A.acc = c->acc;
    A.nr = c->nr;
    A.nth = c->nth;
    hipLaunchKernelGGL(k_deposit, dim3(grid_for(c->n, 256)), dim3(256), 0,
                       c->stream, A);
    GRPIC_HIP(hipGetLastError());
  }
  finalize(c, c->jcur ^ 1);  // this step's deposit goes to J[jnext]
  time_end(c, GRPIC_K_DEPOSIT, ev);
}

void launch_deposit_initial(grpic_ctx* c) {
  if (c->n > 0) {
    ParticleView P = c->pv;
    P.n = c->n;
    hipLaunchKernelGGL(k_weights, dim3(grid_for(c->n, 256)), dim3(256), 0,
                       c->stream, grid_view(c), P);
    GRPIC_HIP(hipGetLastError());
    DepArgs A;
    A.g = grid_view(c);
    A.p = P;
    A.acc = c->acc;
    A.nr = c->nr;
    A.nth = c->nth;
    hipLaunchKernelGGL(k_deposit_rho, dim3(grid_for(c->n, 256)), dim3(256), 0,
                       c->stream, A);
    GRPIC_HIP(hipGetLastError());
  }
  finalize(c, c->jcur);  // initial rho (and zero currents) in J[jcur]
}

}  // namespace grpic
