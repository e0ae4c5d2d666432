// maxwell.hip -- field side of the GRPIC step: metric tables at the Yee
// points (Sec. 2.1), the Wald and split-monopole initial fields (App. B),
// the constitutive relations E = alpha D + beta x B and H = alpha B -
// beta x D, the Faraday and Ampere curl updates (eqs. m3, m4) with the
// absorbing layer (eqs. abs0-abs2) and the boundary conditions (Sec. 2.5),
// sequenced as sub-steps 1-4 and 7-10 of the leapfrog; and the grid
// diagnostics (Gauss residual, div B, Poynting luminosity, eq. Pbz).
//
// Storage is FP32 and densitized, G = sqrt(gamma) F at the component's Yee
// point, so that the curl updates read
//   d_t G_B^i = -eta^ijk d_j E_k,   d_t G_D^i = eta^ijk d_j H_k - 4 pi G_J^i,
// and a component needed off its own point is the plain average of the two
// neighbouring G values (the metric-weighted average of the paper, times
// sqrt(gamma) of the target point).
#include <mutex>
#include <string>

#include "kerr_device.hpp"

namespace grpic {

// ------------------------------------------------------------------ tables
struct TabArgs {
  double a;
  int nr, nth;
  const double *rn, *rh, *tn, *th;
  float *krr, *ktt, *kpp, *krp, *beta, *sg;
  int rhalf, thalf;
};

__global__ void k_metric_table(TabArgs T) {
  int nR = T.rhalf ? T.nr : T.nr + 1;
  int nT = T.thalf ? T.nth : T.nth + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nR * nT) return;
  int i = (int)(k % nR), j = (int)(k / nR);
  double r = T.rhalf ? T.rh[i] : T.rn[i];
  double th = T.thalf ? T.th[j] : T.tn[j];
  Met m;
  metric(T.a, r, th, m);
  double ks = m.alpha / m.sg;
  T.krr[k] = (float)(ks * m.grr);
  T.ktt[k] = (float)(ks * m.gtt);
  T.kpp[k] = (float)(ks * m.gpp);
  T.krp[k] = (float)(ks * m.grp);
  T.beta[k] = (float)m.betar;
  T.sg[k] = (float)m.sg;
}

__global__ void k_damp(const double* rn, const double* rh, int nr, double dt,
                       double r_abs, double r_max, double chi0, double lam,
                       float* dn, float* dh) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nr) return;
  auto f = [&](double r) {
    if (chi0 <= 0.0 || r <= r_abs) return 1.0;
    double x = (r - r_abs) / (r_max - r_abs);
    return exp(-chi0 * pow(x, lam) * dt);
  };
  dn[i] = (float)f(rn[i]);
  if (i < nr) dh[i] = (float)f(rh[i]);
}

void launch_metric_tables(grpic_ctx* c) {
  for (int t = 0; t < 4; ++t) {
    TabArgs T;
    T.a = c->cfg.a;
    T.nr = c->nr;
    T.nth = c->nth;
    T.rn = c->rn;
    T.rh = c->rh;
    T.tn = c->tn;
    T.th = c->th;
    T.krr = c->tab.krr[t];
    T.ktt = c->tab.ktt[t];
    T.kpp = c->tab.kpp[t];
    T.krp = c->tab.krp[t];
    T.beta = c->tab.beta[t];
    T.sg = c->tab.sg[t];
    T.rhalf = (t == 0 || t == 3);  // hn, hh
    T.thalf = (t == 1 || t == 3);  // nh, hh
    long n = (long)(c->nr + 1) * (c->nth + 1);
    hipLaunchKernelGGL(k_metric_table, dim3(grid_for(n, 256)), dim3(256), 0,
                       c->stream, T);
    GRPIC_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_damp, dim3(grid_for(c->nr + 1, 256)), dim3(256), 0,
                     c->stream, c->rn, c->rh, c->nr, c->cfg.dt, c->cfg.r_abs,
                     c->cfg.r_out, c->cfg.chi0, c->cfg.lambda_abs,
                     c->tab.damp_n, c->tab.damp_h);
  GRPIC_HIP(hipGetLastError());
}

// -------------------------------------------------------------- Wald field
// App. B.1: B^i from the closed forms, E_r = d_r A_0, E_theta = d_theta A_0
// (one factor of a), E_phi = 0, A_0 = B0 a r (1 + cos^2) / rho^2;
// D_i = (E_i - sqrt(g) eta_ijk beta^j B^k) / alpha, D^i = gamma^ij D_j.
// The potential of eq. Amu carries its own spin af: the curl (sqrt(g) B^i,
// the stored densitized value) and E_i come from the af solution, alpha,
// beta, gamma from the spacetime.  af = 0 is the start of Sec. 3.3: E_i = 0,
// D = -beta x B / alpha.
__device__ void wald_point(double a, double af, double B0, double r, double th,
                           double* D, double* B, double& sg) {
  Met m;
  metric(a, r, th, m);
  double s = m.s, c = m.c;
  double a2 = af * af, r2 = r * r;
  double rho2 = r2 + a2 * c * c, irho4 = 1.0 / (rho2 * rho2);
  double isg = 1.0 / m.sg;
  B[0] = B0 * isg * (r2 + a2 - 2.0 * r + 2.0 * r * (r2 * r2 - a2 * a2) * irho4) * s * c;
  B[1] = -B0 * isg * (r + a2 * (1.0 + c * c) * (2.0 * r2 - rho2) * irho4) * s * s;
  B[2] = -B0 * isg * (2.0 * af * r * (a2 - r2) * irho4 - af) * s * c;
  double Er = B0 * af * (1.0 + c * c) * (a2 * c * c - r2) * irho4;
  double Et = B0 * af * 2.0 * r * (a2 - r2) * irho4 * s * c;
  double ia = 1.0 / m.alpha;
  double Dr = Er * ia;
  double Dt = (Et + m.sg * m.betar * B[2]) * ia;
  double Dp = (-m.sg * m.betar * B[1]) * ia;
  D[0] = m.irr * Dr + m.irp * Dp;
  D[1] = m.itt * Dt;
  D[2] = m.irp * Dr + m.ipp * Dp;
  sg = m.sg;
}

struct IcArgs {
  double a, a_field, B0, zeta0;
  int nr, nth;
  const double *rn, *rh, *tn, *th;
  float* D[3][3];  // [level][comp]
  float* B[3][3];
  double dth;
};

// component c at Yee type: 0 D^r hn, 1 D^th nh, 2 D^ph nn, 3 B^r nh,
// 4 B^th hn, 5 B^ph hh
__global__ void k_wald(IcArgs A, int comp) {
  int rhalf = (comp == 0 || comp == 4 || comp == 5);
  int thalf = (comp == 1 || comp == 3 || comp == 5);
  int nR = rhalf ? A.nr : A.nr + 1, nT = thalf ? A.nth : A.nth + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nR * nT) return;
  int i = (int)(k % nR), j = (int)(k / nR);
  double r = rhalf ? A.rh[i] : A.rn[i];
  double th = thalf ? A.th[j] : A.tn[j];
  double D[3], B[3], sg;
  wald_point(A.a, A.a_field, A.B0, r, th, D, B, sg);
  float v = (float)(sg * (comp < 3 ? D[comp] : B[comp - 3]));
  for (int l = 0; l < 3; ++l) {
    if (comp < 3)
      A.D[l][comp][k] = v;
    else
      A.B[l][comp - 3][k] = v;
  }
}

// App. B.2: densitized B^r = (Psi(theta_{j+1}) - Psi(theta_j)) / dtheta,
// everything else zero
__global__ void k_split_monopole(IcArgs A) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int nrn = A.nr + 1;
  if (k >= (long)nrn * A.nth) return;
  int j = (int)(k / nrn);
  auto psi = [&](double t) {
    double zeta = 2.0 / kPi * atan(A.zeta0 * (t - 0.5 * kPi));
    return 4.0 * A.B0 * zeta * (1.0 - cos(t));
  };
  float v = (float)((psi(A.tn[j + 1]) - psi(A.tn[j])) / A.dth);
  for (int l = 0; l < 3; ++l) A.B[l][0][k] = v;
}

static IcArgs ic_args(grpic_ctx* c) {
  IcArgs A;
  A.a = c->cfg.a;
  A.nr = c->nr;
  A.nth = c->nth;
  A.rn = c->rn;
  A.rh = c->rh;
  A.tn = c->tn;
  A.th = c->th;
  A.dth = c->dth;
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 3; ++q) {
      A.D[l][q] = c->D[l].c[q];
      A.B[l][q] = c->B[l].c[q];
    }
  return A;
}

void launch_wald(grpic_ctx* c, double B0, double a_field) {
  IcArgs A = ic_args(c);
  A.B0 = B0;
  A.a_field = a_field;
  long n = (long)(c->nr + 1) * (c->nth + 1);
  for (int comp = 0; comp < 6; ++comp) {
    hipLaunchKernelGGL(k_wald, dim3(grid_for(n, 256)), dim3(256), 0, c->stream,
                       A, comp);
    GRPIC_HIP(hipGetLastError());
  }
}

void launch_split_monopole(grpic_ctx* c, double B0, double zeta0) {
  IcArgs A = ic_args(c);
  A.B0 = B0;
  A.zeta0 = zeta0;
  long nn = (long)(c->nr + 1) * (c->nth + 1);
  for (int l = 0; l < 3; ++l)
    for (int q = 0; q < 3; ++q) {
      launch_fill(c, c->D[l].c[q], sizeof(float) * nn);
      launch_fill(c, c->B[l].c[q], sizeof(float) * nn);
    }
  hipLaunchKernelGGL(k_split_monopole, dim3(grid_for(nn, 256)), dim3(256), 0,
                     c->stream, A);
  GRPIC_HIP(hipGetLastError());
}

// ------------------------------------------------------------- stencils
struct FdArgs {
  int nr, nth;
  float dt, inv_dth;
  const float *inv_drn;   // 1/(r_{i+1} - r_i), i < nr
  const float *inv_drd;   // 1/(r_{i+1/2} - r_{i-1/2}), 0 < i < nr
  Tables tab;
};

// E at all three Yee points of node (i, j) from D = wa Da + wb Db and B
__global__ __launch_bounds__(256) void k_compute_E(FdArgs F, Level3 Da,
                                                   Level3 Db, float wa,
                                                   float wb, Level3 B,
                                                   Level3 E) {
  const int nr = F.nr, nth = F.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  auto D = [&](int c, long idx) { return wa * Da.c[c][idx] + wb * Db.c[c][idx]; };
  if (i < nr) {  // E_r at (i+1/2, j)
    long h = (long)j * nr + i;
    float Dp = 0.5f * (D(2, k) + D(2, k + 1));
    E.c[0][h] = F.tab.krr[0][h] * D(0, h) + F.tab.krp[0][h] * Dp;
  }
  if (j < nth) {  // E_theta at (i, j+1/2)
    long h = (long)j * nr;
    float Bp;
    if (i == 0) Bp = B.c[2][h];
    else if (i == nr) Bp = B.c[2][h + nr - 1];
    else Bp = 0.5f * (B.c[2][h + i - 1] + B.c[2][h + i]);
    E.c[1][k] = F.tab.ktt[1][k] * D(1, k) - F.tab.beta[1][k] * Bp;
  }
  // E_phi at (i, j): zero on the theta edges (axis condition)
  if (j == 0 || j == nth) {
    E.c[2][k] = 0.0f;
  } else {
    long h = (long)j * nr;
    float Dr, Bt;
    if (i == 0) {
      Dr = D(0, h);
      Bt = B.c[1][h];
    } else if (i == nr) {
      Dr = D(0, h + nr - 1);
      Bt = B.c[1][h + nr - 1];
    } else {
      Dr = 0.5f * (D(0, h + i - 1) + D(0, h + i));
      Bt = 0.5f * (B.c[1][h + i - 1] + B.c[1][h + i]);
    }
    E.c[2][k] = F.tab.krp[2][k] * Dr + F.tab.kpp[2][k] * D(2, k) +
                F.tab.beta[2][k] * Bt;
  }
}

// H at all three Yee points around node (i, j) from B and D
__global__ __launch_bounds__(256) void k_compute_H(FdArgs F, Level3 B,
                                                   Level3 D, Level3 H) {
  const int nr = F.nr, nth = F.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  if (j < nth) {  // H_r at (i, j+1/2)
    long h = (long)j * nr;
    float Bp;
    if (i == 0) Bp = B.c[2][h];
    else if (i == nr) Bp = B.c[2][h + nr - 1];
    else Bp = 0.5f * (B.c[2][h + i - 1] + B.c[2][h + i]);
    H.c[0][k] = F.tab.krr[1][k] * B.c[0][k] + F.tab.krp[1][k] * Bp;
  }
  if (i < nr) {  // H_theta at (i+1/2, j)
    long h = (long)j * nr + i;
    float Dp = 0.5f * (D.c[2][k] + D.c[2][k + 1]);
    H.c[1][h] = F.tab.ktt[0][h] * B.c[1][h] + F.tab.beta[0][h] * Dp;
  }
  if (i < nr && j < nth) {  // H_phi at (i+1/2, j+1/2)
    long h = (long)j * nr + i;
    float Br = 0.5f * (B.c[0][k] + B.c[0][k + 1]);
    float Dt = 0.5f * (D.c[1][k] + D.c[1][k + 1]);
    H.c[2][h] = F.tab.krp[3][h] * Br + F.tab.kpp[3][h] * B.c[2][h] -
                F.tab.beta[3][h] * Dt;
  }
}

// Bout = damp (wa Ba + wb Bb - dt curl E)
__global__ __launch_bounds__(256) void k_faraday(FdArgs F, Level3 Ba,
                                                 Level3 Bb, float wa, float wb,
                                                 Level3 E, Level3 Bout) {
  const int nr = F.nr, nth = F.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  const float dt = F.dt, idt = F.inv_dth;
  if (j < nth) {  // B^r at (i, j+1/2)
    float c = (E.c[2][k + nrn] - E.c[2][k]) * idt;
    float b = wa * Ba.c[0][k] + wb * Bb.c[0][k];
    Bout.c[0][k] = F.tab.damp_n[i] * (b - dt * c);
  }
  if (i < nr) {  // B^theta at (i+1/2, j)
    long h = (long)j * nr + i;
    float c = -(E.c[2][k + 1] - E.c[2][k]) * F.inv_drn[i];
    float b = wa * Ba.c[1][h] + wb * Bb.c[1][h];
    Bout.c[1][h] = F.tab.damp_h[i] * (b - dt * c);
  }
  if (i < nr && j < nth) {  // B^phi at (i+1/2, j+1/2)
    long h = (long)j * nr + i;
    float c = (E.c[1][k + 1] - E.c[1][k]) * F.inv_drn[i] -
              (E.c[0][h + nr] - E.c[0][h]) * idt;
    float b = wa * Ba.c[2][h] + wb * Bb.c[2][h];
    Bout.c[2][h] = F.tab.damp_h[i] * (b - dt * c);
  }
}

// Dout = damp (Din + dt (curl H - 4 pi (cj J + cp Jp)))
__global__ __launch_bounds__(256) void k_ampere(FdArgs F, Level3 Din,
                                                Level3 H, Level4 J, Level4 Jp,
                                                float cj, float cp,
                                                Level3 Dout) {
  const int nr = F.nr, nth = F.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  const float dt = F.dt, idt = F.inv_dth, fp = 4.0f * 3.14159265358979f;
  if (i < nr) {  // D^r at (i+1/2, j); H_phi = 0 on the axis edges
    long h = (long)j * nr + i;
    float c;
    if (j == 0) c = H.c[2][h] * (2.0f * idt);
    else if (j == nth) c = -H.c[2][h - nr] * (2.0f * idt);
    else c = (H.c[2][h] - H.c[2][h - nr]) * idt;
    float src = cj * J.c[0][h] + (cp != 0.0f ? cp * Jp.c[0][h] : 0.0f);
    Dout.c[0][h] = F.tab.damp_h[i] * (Din.c[0][h] + dt * (c - fp * src));
  }
  if (j < nth && i > 0 && i < nr) {  // D^theta at (i, j+1/2)
    long h = (long)j * nr + i;
    float c = -(H.c[2][h] - H.c[2][h - 1]) * F.inv_drd[i];
    float src = cj * J.c[1][k] + (cp != 0.0f ? cp * Jp.c[1][k] : 0.0f);
    Dout.c[1][k] = F.tab.damp_n[i] * (Din.c[1][k] + dt * (c - fp * src));
  }
  if (j == 0 || j == nth) {
    Dout.c[2][k] = 0.0f;  // D^phi = 0 on the axis edges
  } else if (i > 0 && i < nr) {  // D^phi at (i, j)
    long h = (long)j * nr + i;
    float c = (H.c[1][h] - H.c[1][h - 1]) * F.inv_drd[i] -
              (H.c[0][k] - H.c[0][k - nrn]) * idt;
    float src = cj * J.c[2][k] + (cp != 0.0f ? cp * Jp.c[2][k] : 0.0f);
    Dout.c[2][k] = F.tab.damp_n[i] * (Din.c[2][k] + dt * (c - fp * src));
  }
}

// zero radial gradient of D^theta and D^phi at the radial ends (applied to
// the non-densitized value: G_end = G_in sqrt(g)_end / sqrt(g)_in)
__global__ void k_radial_bc(FdArgs F, Level3 D) {
  const int nr = F.nr, nth = F.nth, nrn = nr + 1;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nth) return;
  long row = (long)j * nrn;
  if (j < nth) {
    D.c[1][row] = D.c[1][row + 1] * (F.tab.sg[1][row] / F.tab.sg[1][row + 1]);
    D.c[1][row + nr] =
        D.c[1][row + nr - 1] * (F.tab.sg[1][row + nr] / F.tab.sg[1][row + nr - 1]);
  }
  if (j > 0 && j < nth) {
    D.c[2][row] = D.c[2][row + 1] * (F.tab.sg[2][row] / F.tab.sg[2][row + 1]);
    D.c[2][row + nr] =
        D.c[2][row + nr - 1] * (F.tab.sg[2][row + nr] / F.tab.sg[2][row + nr - 1]);
  }
}

static FdArgs fd_args(grpic_ctx* c) {
  FdArgs F;
  F.nr = c->nr;
  F.nth = c->nth;
  F.dt = (float)c->cfg.dt;
  F.inv_dth = (float)(1.0 / c->dth);
  F.inv_drn = c->tab.inv_drn;
  F.inv_drd = c->tab.inv_drd;
  F.tab = c->tab;
  return F;
}

static Level4 jlevel(grpic_ctx* c, int which) {
  Level4 L;
  for (int q = 0; q < 4; ++q) L.c[q] = c->J[which][q];
  return L;
}

// sub-steps 1-4: E^{n+1} from <D>^{n+1} and B^{n+1}; B^{n+3/2} from
// <B>^{n+1/2}; E^{n+3/2}; B^{n+2} (written over B^n, which is no longer
// needed)
void launch_fields_step_pre(grpic_ctx* c) {
  FdArgs F = fd_args(c);
  long n = (long)(c->nr + 1) * (c->nth + 1);
  dim3 g(grid_for(n, 256)), b(256);
  hipLaunchKernelGGL(k_compute_E, g, b, 0, c->stream, F, c->D[1], c->D[2], 0.5f,
                     0.5f, c->B[1], c->E);
  hipLaunchKernelGGL(k_faraday, g, b, 0, c->stream, F, c->B[0], c->B[1], 0.5f,
                     0.5f, c->E, c->B[2]);
  hipLaunchKernelGGL(k_compute_E, g, b, 0, c->stream, F, c->D[2], c->D[2], 1.0f,
                     0.0f, c->B[2], c->E);
  hipLaunchKernelGGL(k_faraday, g, b, 0, c->stream, F, c->B[1], c->B[1], 1.0f,
                     0.0f, c->E, c->B[0]);
  GRPIC_HIP(hipGetLastError());
}

// sub-steps 7-10: H^{n+3/2}; D^{n+2} (in place) with J^{n+3/2}; H^{n+2};
// D^{n+5/2} (written over D^{n+1/2}) with 1.5 J^{n+3/2} - 0.5 J^{n+1/2}.
// The deposit of this step sits in J[jnext], the previous one in J[jcur].
void launch_fields_step_post(grpic_ctx* c) {
  FdArgs F = fd_args(c);
  long n = (long)(c->nr + 1) * (c->nth + 1);
  dim3 g(grid_for(n, 256)), b(256);
  dim3 gb(grid_for(c->nth + 1, 256));
  Level4 Jc = jlevel(c, c->jcur ^ 1), Jp = jlevel(c, c->jcur);
  // conserving deposit: J^{n+3/2}, then 1.5 J^{n+3/2} - 0.5 J^{n+1/2};
  // the paper's current: (J^{n+1} + J^{n+2}) / 2, then J^{n+2}
  const bool paper = c->cfg.deposit_mode == GRPIC_DEPOSIT_PAPER;
  const float c8 = paper ? 0.5f : 1.0f, p8 = paper ? 0.5f : 0.0f;
  const float c10 = paper ? 1.0f : 1.5f, p10 = paper ? 0.0f : -0.5f;
  hipLaunchKernelGGL(k_compute_H, g, b, 0, c->stream, F, c->B[2], c->D[2], c->H);
  hipLaunchKernelGGL(k_ampere, g, b, 0, c->stream, F, c->D[0], c->H, Jc, Jp,
                     c8, p8, c->D[0]);
  hipLaunchKernelGGL(k_radial_bc, gb, b, 0, c->stream, F, c->D[0]);
  hipLaunchKernelGGL(k_compute_H, g, b, 0, c->stream, F, c->B[0], c->D[0], c->H);
  hipLaunchKernelGGL(k_ampere, g, b, 0, c->stream, F, c->D[2], c->H, Jc, Jp,
                     c10, p10, c->D[1]);
  hipLaunchKernelGGL(k_radial_bc, gb, b, 0, c->stream, F, c->D[1]);
  GRPIC_HIP(hipGetLastError());
}

// ------------------------------------------------------------ diagnostics
__device__ __forceinline__ void atomic_max_pos(float* addr, float v) {
  atomicMax(reinterpret_cast<unsigned int*>(addr), __float_as_uint(v));
}

struct DiagArgs {
  int nr, nth;
  double dth;
  const double *rn, *rh;
  Level3 D, B;
  const float* rho;
  float* out;  // [0] gauss max, [1] div B max
};

__global__ void k_field_diag(DiagArgs A) {
  const int nr = A.nr, nth = A.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  if (i > 0 && i < nr && j > 0 && j < nth) {
    long h = (long)j * nr + i;
    double fr = (double)A.D.c[0][h] - (double)A.D.c[0][h - 1];
    double ft = (double)A.D.c[1][k] - (double)A.D.c[1][k - nrn];
    double g = fr / (A.rh[i] - A.rh[i - 1]) + ft / A.dth -
               4.0 * kPi * (double)A.rho[k];
    atomic_max_pos(&A.out[0], (float)fabs(g));
  }
  if (i < nr && j < nth) {
    long h = (long)j * nr + i;
    double fr = (double)A.B.c[0][k + 1] - (double)A.B.c[0][k];
    double ft = (double)A.B.c[1][h + nr] - (double)A.B.c[1][h];
    double d = fr / (A.rn[i + 1] - A.rn[i]) + ft / A.dth;
    atomic_max_pos(&A.out[1], (float)fabs(d));
  }
}

// Poynting luminosity through r_i: (1/2) sum_j (E_th H_ph - E_ph H_th) dth
// at theta_{j+1/2}, all factors brought there by densitized averages
__global__ void k_poynting(FdArgs F, Level3 E, Level3 H, double dth,
                           double* out) {
  const int nr = F.nr, nth = F.nth, nrn = nr + 1;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nr) return;
  int i0 = i > 0 ? i - 1 : -1, i1 = i < nr ? i : -1;
  double sum = 0.0;
  for (int j = 0; j < nth; ++j) {
    long k = (long)j * nrn + i;
    double s = F.tab.sg[1][k];
    double Et = E.c[1][k];
    double Hp = 0.0, Ht = 0.0;
    int n = 0;
    if (i0 >= 0) Hp += (double)F.tab.sg[3][(long)j * nr + i0] * H.c[2][(long)j * nr + i0], ++n;
    if (i1 >= 0) Hp += (double)F.tab.sg[3][(long)j * nr + i1] * H.c[2][(long)j * nr + i1], ++n;
    Hp /= (n * s);
    double Ep = 0.5 * ((double)F.tab.sg[2][k] * E.c[2][k] +
                       (double)F.tab.sg[2][k + nrn] * E.c[2][k + nrn]) / s;
    n = 0;
    for (int jj = j; jj <= j + 1; ++jj) {
      if (i0 >= 0) Ht += (double)F.tab.sg[0][(long)jj * nr + i0] * H.c[1][(long)jj * nr + i0], ++n;
      if (i1 >= 0) Ht += (double)F.tab.sg[0][(long)jj * nr + i1] * H.c[1][(long)jj * nr + i1], ++n;
    }
    Ht /= (n * s);
    sum += (Et * Hp - Ep * Ht) * dth;
  }
  out[i] = 0.5 * sum;
}

// the diagnostics into dmax[2] (FP32 maxima, cleared here) and dp[nr + 1]
// (device), then copied to the caller's host outputs; synchronises
static void field_diag_into(grpic_ctx* c, float* dmax, double* dp, double* gauss_max,
                            double* divb_max, double* pbz) {
  launch_fill(c, dmax, 2 * sizeof(float));
  DiagArgs A;
  A.nr = c->nr;
  A.nth = c->nth;
  A.dth = c->dth;
  A.rn = c->rn;
  A.rh = c->rh;
  A.D = c->D[0];
  A.B = c->B[1];
  A.rho = c->J[c->jcur][3];
  A.out = dmax;
  long n = (long)(c->nr + 1) * (c->nth + 1);
  hipLaunchKernelGGL(k_field_diag, dim3(grid_for(n, 256)), dim3(256), 0,
                     c->stream, A);
  // grid E and H of the integer chain (D^{n+1}, B^{n+1})
  FdArgs F = fd_args(c);
  hipLaunchKernelGGL(k_compute_E, dim3(grid_for(n, 256)), dim3(256), 0, c->stream,
                     F, c->D[0], c->D[0], 1.0f, 0.0f, c->B[1], c->E);
  hipLaunchKernelGGL(k_compute_H, dim3(grid_for(n, 256)), dim3(256), 0, c->stream,
                     F, c->B[1], c->D[0], c->H);
  hipLaunchKernelGGL(k_poynting, dim3(grid_for(c->nr + 1, 64)), dim3(64), 0,
                     c->stream, F, c->E, c->H, c->dth, dp);
  GRPIC_HIP(hipGetLastError());
  float hm[2];
  GRPIC_HIP(hipMemcpyAsync(hm, dmax, sizeof(hm), hipMemcpyDeviceToHost, c->stream));
  if (pbz)
    GRPIC_HIP(hipMemcpyAsync(pbz, dp, sizeof(double) * (c->nr + 1), hipMemcpyDeviceToHost,
                             c->stream));
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  if (gauss_max) *gauss_max = hm[0];
  if (divb_max) *divb_max = hm[1];
}

void launch_field_diag(grpic_ctx* c, double* gauss_max, double* divb_max,
                       double* pbz) {
  float* dmax = nullptr;
  double* dp = nullptr;
  GRPIC_HIP(hipMalloc(&dmax, 2 * sizeof(float)));
  hipError_t e = hipMalloc(&dp, sizeof(double) * (c->nr + 1));
  if (e != hipSuccess) {
    (void)hipFree(dmax);
    GRPIC_HIP(e);
  }
  try {
    field_diag_into(c, dmax, dp, gauss_max, divb_max, pbz);
  } catch (...) {
    (void)hipFree(dmax);
    (void)hipFree(dp);
    throw;
  }
  GRPIC_HIP(hipFree(dmax));
  GRPIC_HIP(hipFree(dp));
}

// ------------------------------------------- allocation-free diagnostics
// Scratch of grpic_field_diagnostics_noalloc: bytes [0, 8) hold the two FP32
// maxima, bytes [256, 256 + 8 (kDiagMaxNr + 1)) the luminosities P(r_i).
// Every device that runs the library holds its own copy until the process
// ends.  Host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in, not a device address).
constexpr size_t kDiagScratchBytes = 256 + sizeof(double) * (kDiagMaxNr + 1);
static __device__ __align__(256) unsigned char scratch[kDiagScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu[kScratchDevices];
static void* g_scratch_ptr[kScratchDevices] = {};

// once per device, with that device current (called by grpic_create)
void diag_scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu[device]);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  GRPIC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch_ptr[device] = p;
}

void field_diag_noalloc(grpic_ctx* c, double* gauss_max, double* divb_max, double* pbz) {
  if (c->nr > kDiagMaxNr)
    throw Error(GRPIC_E_INVALID, "grid has " + std::to_string(c->nr) +
                                     " radial cells: the allocation-free diagnostics hold "
                                     "at most " + std::to_string(kDiagMaxNr));
  if (c->device < 0 || c->device >= kScratchDevices || !g_scratch_ptr[c->device])
    throw Error(GRPIC_E_STATE, "diagnostics scratch not set up on this device");
  // calls on one device are serialised: each waits for its stream before
  // the next one may use the shared scratch
  std::lock_guard<std::mutex> lock(g_scratch_mu[c->device]);
  unsigned char* base = static_cast<unsigned char*>(g_scratch_ptr[c->device]);
  field_diag_into(c, reinterpret_cast<float*>(base), reinterpret_cast<double*>(base + 256),
                  gauss_max, divb_max, pbz);
}

}  // namespace grpic
