// clean.hip -- divergence cleaning (Sec. 2.4, eq. phi).  In densitized form
// on the nodes,
//   d_r(sqrt(g) g^rr d_r phi) + d_th(sqrt(g) g^thth d_th phi) = G,
// with G = div_h(sqrt(g) D) - 4 pi sqrt(g) rho the Gauss residual of eq. m1
// at the interior nodes (d_phi = 0 by axisymmetry, g^rth = 0).  d_r phi sits
// on the D^r faces and d_th phi on the D^theta faces, so the operator is the
// discrete divergence of the discrete gradient and a converged phi removes
// the residual exactly.  phi = 0 on the boundary nodes; Jacobi sweeps from
// phi = 0 in FP64; then sqrt(g) D^i -= sqrt(g) g^ij d_j phi.
#include "grpic_common.hpp"
#include "kerr_device.hpp"

namespace grpic {

namespace {

struct CleanArgs {
  int nr, nth;
  double dth;
  const double *rn, *rh;
  double *kr, *kt, *kp;  // face / node coefficients (see grpic_ctx)
};

// coefficients, once per context: kr on the D^r faces (r_{i+1/2}, th_j),
// kt on the D^theta faces (r_i, th_{j+1/2}), kp on the nodes
__global__ __launch_bounds__(256) void k_clean_coeffs(CleanArgs A, double a,
                                                      const double* tn,
                                                      const double* thh) {
  const int nr = A.nr, nth = A.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  Met m;
  if (i < nr) {
    metric(a, A.rh[i], tn[j], m);
    A.kr[(long)j * nr + i] = m.sg * m.irr / (A.rn[i + 1] - A.rn[i]);
  }
  if (j < nth) {
    metric(a, A.rn[i], thh[j], m);
    A.kt[k] = m.sg * m.itt / A.dth;
  }
  metric(a, A.rn[i], tn[j], m);
  A.kp[k] = m.sg * m.irp;
}

// G at the nodes from the densitized FP32 D^r, D^theta and the charge
// c0 rho0 + c1 rho1 (0 on the boundary nodes); phi[0] = phi[1] = 0
__global__ __launch_bounds__(256) void k_clean_source(CleanArgs A, const float* Dr,
                                                      const float* Dt, const float* rho0,
                                                      const float* rho1, double c0,
                                                      double c1, double* G, double* phi0,
                                                      double* phi1) {
  const int nr = A.nr, nth = A.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  double v = 0.0;
  if (i > 0 && i < nr && j > 0 && j < nth) {
    long h = (long)j * nr + i;
    double fr = (double)Dr[h] - (double)Dr[h - 1];
    double ft = (double)Dt[k] - (double)Dt[k - nrn];
    double rho = c0 * (double)rho0[k] + (c1 != 0.0 ? c1 * (double)rho1[k] : 0.0);
    v = fr / (A.rh[i] - A.rh[i - 1]) + ft / A.dth - 4.0 * kPi * rho;
  }
  G[k] = v;
  phi0[k] = 0.0;
  phi1[k] = 0.0;
}

// one Jacobi sweep: phi_out = (sum of neighbour couplings - G) / diagonal
__global__ __launch_bounds__(256) void k_clean_jacobi(CleanArgs A, const double* G,
                                                      const double* phi,
                                                      double* out) {
  const int nr = A.nr, nth = A.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  if (i == 0 || i == nr || j == 0 || j == nth) {
    out[k] = 0.0;
    return;
  }
  long h = (long)j * nr + i;
  const double iLr = 1.0 / (A.rh[i] - A.rh[i - 1]), idt = 1.0 / A.dth;
  const double aE = A.kr[h] * iLr, aW = A.kr[h - 1] * iLr;
  const double aN = A.kt[k] * idt, aS = A.kt[k - nrn] * idt;
  double nb = aE * phi[k + 1] + aW * phi[k - 1] + aN * phi[k + nrn] + aS * phi[k - nrn];
  out[k] = (nb - G[k]) / (aE + aW + aN + aS);
}

// sqrt(g) D^i -= sqrt(g) g^ij d_j phi on the faces (D^r, D^theta) and the
// interior nodes (D^phi, mean of the two radial differences)
__global__ __launch_bounds__(256) void k_clean_apply(CleanArgs A, const double* phi,
                                                     float* Dr, float* Dt, float* Dp) {
  const int nr = A.nr, nth = A.nth, nrn = nr + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nrn * (nth + 1)) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  if (i < nr) {
    long h = (long)j * nr + i;
    Dr[h] = (float)((double)Dr[h] - A.kr[h] * (phi[k + 1] - phi[k]));
  }
  if (j < nth) Dt[k] = (float)((double)Dt[k] - A.kt[k] * (phi[k + nrn] - phi[k]));
  if (i > 0 && i < nr && j > 0 && j < nth) {
    double dr = 0.5 * ((phi[k + 1] - phi[k]) / (A.rn[i + 1] - A.rn[i]) +
                       (phi[k] - phi[k - 1]) / (A.rn[i] - A.rn[i - 1]));
    Dp[k] = (float)((double)Dp[k] - A.kp[k] * dr);
  }
}

CleanArgs clean_args(grpic_ctx* c) {
  CleanArgs A;
  A.nr = c->nr;
  A.nth = c->nth;
  A.dth = c->dth;
  A.rn = c->rn;
  A.rh = c->rh;
  A.kr = c->clean_kr;
  A.kt = c->clean_kt;
  A.kp = c->clean_kp;
  return A;
}

void clean_chain(grpic_ctx* c, const CleanArgs& A, Level3 D, const float* rho0,
                 const float* rho1, double c0, double c1, int iters) {
  long nn = (long)(c->nr + 1) * (c->nth + 1);
  dim3 g(grid_for(nn, 256)), b(256);
  hipLaunchKernelGGL(k_clean_source, g, b, 0, c->stream, A, D.c[0], D.c[1], rho0, rho1,
                     c0, c1, c->clean_src, c->clean_phi[0], c->clean_phi[1]);
  int cur = 0;
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_clean_jacobi, g, b, 0, c->stream, A, c->clean_src,
                       c->clean_phi[cur], c->clean_phi[cur ^ 1]);
    cur ^= 1;
  }
  hipLaunchKernelGGL(k_clean_apply, g, b, 0, c->stream, A, c->clean_phi[cur], D.c[0],
                     D.c[1], D.c[2]);
  GRPIC_HIP(hipGetLastError());
}

}  // namespace

void launch_clean(grpic_ctx* c, int iters) {
  long nn = (long)(c->nr + 1) * (c->nth + 1);
  if (!c->clean_kr) {
    double* buf[6] = {};
    try {
      for (double*& b : buf) b = dalloc<double>(nn);
    } catch (...) {
      for (double*& b : buf) dfree(b);
      throw;
    }
    c->clean_kt = buf[1];
    c->clean_kp = buf[2];
    c->clean_src = buf[3];
    c->clean_phi[0] = buf[4];
    c->clean_phi[1] = buf[5];
    c->clean_kr = buf[0];
    hipLaunchKernelGGL(k_clean_coeffs, dim3(grid_for(nn, 256)), dim3(256), 0, c->stream,
                       clean_args(c), c->cfg.a, c->tn, c->th);
    GRPIC_HIP(hipGetLastError());
  }
  hipEvent_t ev;
  time_begin(c, GRPIC_K_CLEAN, &ev);
  const CleanArgs A = clean_args(c);
  const float* rho = c->J[c->jcur][3];        // rho of the last deposit
  const float* rho_prev = c->J[c->jcur ^ 1][3];
  // integer chain D^{n+2} against rho^{n+2}; half chain D^{n+5/2} against
  // the charge extrapolated half a step, 1.5 rho^{n+2} - 0.5 rho^{n+1}
  clean_chain(c, A, c->D[0], rho, rho_prev, 1.0, 0.0, iters);
  clean_chain(c, A, c->D[2], rho, rho_prev, 1.5, -0.5, iters);
  time_end(c, GRPIC_K_CLEAN, ev);
}

}  // namespace grpic
