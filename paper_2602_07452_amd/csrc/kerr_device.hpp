// kerr_device.hpp -- FP64 device math of the GRPIC pusher: Kerr-Schild 3+1
// metric and its analytic derivatives (App. A; Sec. 2.2), the particle
// equations of motion (eqs. p1, p2, O1, O2) and the metric-weighted gather
// of the staggered grid fields.
//
// Forms used here (M = 1): with S = rho^2 + 2r = rho^2 xi,
//   1/xi = rho^2/S, alpha = sqrt(rho^2/S), beta^r = 2r/S,
//   sqrt(gamma) = |sin theta| sqrt(rho^2 S),
// which avoid most divisions; gamma_{r phi} = -a xi sin^2 theta (the value
// that inverts the printed gamma^{ij}).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastmath.hpp"
#include "grpic_common.hpp"

namespace grpic {

struct Met {
  double s, c;                 // sin, cos theta
  double alpha, betar;         // lapse, radial shift
  double grr, gtt, gpp, grp;   // gamma_ij
  double irr, itt, ipp, irp;   // gamma^ij
  double sg;                   // sqrt(gamma)
};

struct DMet {  // [0] = d/dr, [1] = d/dtheta
  double da[2], db[2], drr[2], dtt[2], dpp[2], drp[2];
};

__device__ __forceinline__ double rcp(double x) { return frcp(x); }

// metric at (r, theta) given s = sin theta, c = cos theta
__device__ __forceinline__ void metric_sc(double a, double r, double s, double c, Met& m) {
  double a2 = a * a, s2 = s * s;
  double rho2 = r * r + a2 * c * c;
  double S = rho2 + 2.0 * r, P = rho2 * S;
  // y = (rho2 S)^(-1/2): 1/rho2 = S y^2, 1/S = rho2 y^2, alpha = rho2 y,
  // sqrt(gamma) = |sin| rho2 S y
  double y = frsq(P), y2 = y * y;
  double irho2 = S * y2, iS = rho2 * y2;
  double ixi = rho2 * iS, xi = S * irho2;
  m.s = s;
  m.c = c;
  m.alpha = rho2 * y;
  m.betar = 2.0 * r * iS;
  m.grr = xi;
  m.gtt = rho2;
  m.grp = -a * xi * s2;
  m.gpp = s2 * (rho2 + a2 * xi * s2);
  m.irr = a2 * s2 * irho2 + ixi;
  m.itt = irho2;
  m.irp = a * irho2;
  m.ipp = irho2 * rcp(s2);
  m.sg = fabs(s) * (P * y);
}

__device__ __forceinline__ void metric(double a, double r, double th, Met& m) {
  double s, c;
  fsincos(th, &s, &c);
  metric_sc(a, r, s, c, m);
}

// metric plus derivatives of alpha, beta^r and gamma^ij
__device__ __forceinline__ void metric_d_sc(double a, double r, double s, double c,
                                            Met& m, DMet& d) {
  double a2 = a * a, s2 = s * s, sc = s * c;
  double rho2 = r * r + a2 * c * c;
  double S = rho2 + 2.0 * r, P = rho2 * S;
  double y = frsq(P), y2 = y * y;  // as in metric_sc
  double irho2 = S * y2, iS = rho2 * y2, is2 = rcp(s2);
  double ixi = rho2 * iS, xi = S * irho2;
  double alpha = rho2 * y;
  m.s = s;
  m.c = c;
  m.alpha = alpha;
  m.betar = 2.0 * r * iS;
  m.grr = xi;
  m.gtt = rho2;
  m.grp = -a * xi * s2;
  m.gpp = s2 * (rho2 + a2 * xi * s2);
  m.irr = a2 * s2 * irho2 + ixi;
  m.itt = irho2;
  m.irp = a * irho2;
  m.ipp = irho2 * is2;
  m.sg = fabs(s) * (P * y);
  double i4 = irho2 * irho2, ixi2 = ixi * ixi;
  double dr2[2] = {2.0 * r, -2.0 * a2 * sc};
  double dxi[2] = {2.0 * irho2 * (1.0 - 2.0 * r * r * irho2),
                   4.0 * r * a2 * sc * i4};
  double ds2[2] = {0.0, 2.0 * sc};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    d.da[k] = -0.5 * dxi[k] * alpha * ixi;
    d.db[k] = dxi[k] * ixi2;
    d.drr[k] = a2 * (ds2[k] * irho2 - s2 * dr2[k] * i4) - dxi[k] * ixi2;
    d.dtt[k] = -dr2[k] * i4;
    d.dpp[k] = -(dr2[k] * s2 + rho2 * ds2[k]) * (i4 * is2 * is2);
    d.drp[k] = -a * dr2[k] * i4;
  }
}

__device__ __forceinline__ void metric_d(double a, double r, double th, Met& m,
                                         DMet& d) {
  double s, c;
  fsincos(th, &s, &c);
  metric_d_sc(a, r, s, c, m, d);
}

// Divided differences [f(x1) - f(x0)] / (x1^k - x0^k) of f = alpha, beta^r,
// gamma^rr, gamma^thth, gamma^phph, gamma^rph for positions that differ in
// coordinate k only (0 = r, 1 = theta), free of cancellation: with
// P = rho^2 and S = rho^2 + 2r,
//   k = r:     dP = r0 + r1, dS = dP + 2;
//   k = theta: d(cos^2) = -sin(t0 + t1) sin(t1 - t0) / (t1 - t0) = -d(sin^2),
//              dP = dS = a^2 d(cos^2);
// then d(1/g) = -dg / (g0 g1), d(g h) = g1 dh + h0 dg, d(sqrt g) = dg /
// (sqrt g0 + sqrt g1).  m0, m1 are the metrics at x0, x1.
__device__ __forceinline__ void metric_dd(double a, int k, double r0,
                                          double r1, double dx, const Met& m0,
                                          const Met& m1, double* q) {
  const double A = a * a;
  double C0 = m0.c * m0.c, C1 = m1.c * m1.c;
  double Ss0 = m0.s * m0.s, Ss1 = m1.s * m1.s;
  double P0 = r0 * r0 + A * C0, P1 = r1 * r1 + A * C1;
  double S0 = P0 + 2.0 * r0, S1 = P1 + 2.0 * r1;
  double dP, dS, dSs;
  if (k == 0) {
    dP = r0 + r1;
    dS = dP + 2.0;
    dSs = 0.0;
  } else {
    double sinc = fabs(dx) < 1e-4 ? 1.0 - dx * dx * (1.0 / 6.0) : sin(dx) / dx;
    double s01 = m0.s * m1.c + m0.c * m1.s;  // sin(t0 + t1)
    double dC = -s01 * sinc;
    dSs = -dC;
    dP = A * dC;
    dS = dP;
  }
  double iP01 = 1.0 / (P0 * P1);
  double d_irho2 = -dP * iP01;
  double d_ixi = (dP * S0 - P0 * dS) / (S0 * S1);
  q[0] = d_ixi / (m0.alpha + m1.alpha);
  q[1] = -d_ixi;
  q[2] = A * (Ss1 * d_irho2 + dSs / P0) + d_ixi;
  q[3] = d_irho2;
  q[4] = -(P1 * dSs + Ss0 * dP) * iP01 / (Ss0 * Ss1);
  q[5] = a * d_irho2;
}

// e = alpha Gamma - beta^r u_r, with s, c = sin, cos of z[1]
__device__ __forceinline__ double energy_sc(double a, const double* z, double s, double c) {
  Met m;
  metric_sc(a, z[0], s, c, m);
  double ur = z[3], ut = z[4], up = z[5];
  double q = m.irr * ur * ur + m.itt * ut * ut + m.ipp * up * up +
             2.0 * m.irp * ur * up;
  return m.alpha * fsqrt(1.0 + q) - m.betar * ur;
}

__device__ __forceinline__ double energy(double a, const double* z) {
  double s, c;
  fsincos(z[1], &s, &c);
  return energy_sc(a, z, s, c);
}

// ---------------------------------------------------------------- gather
struct GridView {
  int nr, nth;
  double a, r_in, th0, dth, inv_dlnr, inv_dth;
  const double *rn, *rh, *tn, *th;  // coordinates
  const double *idrn, *idrh;        // 1/(rn[i+1]-rn[i]), 1/(rh[i+1]-rh[i])
  const double *stn, *ctn;          // sin, cos of the node angles
  const double *sth, *cth;          // sin, cos of the half angles
  float inv_rin_f, l2_dlnr_f;       // 1/r_in, ln(2)/dlnr for the estimate
};

// radial cell coordinate log(r/r_in)/dlnr to within far less than a cell
// (FP32 log2); callers refine the index against the FP64 node table
__device__ __forceinline__ float radial_coord(const GridView& g, double r) {
  return __log2f((float)r * g.inv_rin_f) * g.l2_dlnr_f;
}

struct FieldView {  // densitized FP32 components at their Yee points
  const float *Dr, *Dt, *Dp, *Br, *Bt, *Bp;
};

inline GridView make_grid_view(const grpic_ctx* c) {
  GridView g;
  g.nr = c->nr;
  g.nth = c->nth;
  g.a = c->cfg.a;
  g.r_in = c->cfg.r_in;
  g.th0 = c->cfg.theta0;
  g.dth = c->dth;
  g.inv_dlnr = c->dlnr > 0 ? 1.0 / c->dlnr : 0.0;
  g.inv_dth = c->dth > 0 ? 1.0 / c->dth : 0.0;
  g.rn = c->rn;
  g.rh = c->rh;
  g.tn = c->tn;
  g.th = c->th;
  g.idrn = c->idrn;
  g.idrh = c->idrh;
  g.stn = c->stn;
  g.ctn = c->ctn;
  g.sth = c->sth;
  g.cth = c->cth;
  g.inv_rin_f = (float)(1.0 / c->cfg.r_in);
  g.l2_dlnr_f = c->dlnr > 0 ? (float)(0.6931471805599453 / c->dlnr) : 0.0f;
  return g;
}

// cell index p in [0, n-2] with x[p] <= v < x[p+1] (clamped), from a first
// estimate that may be off by one
__device__ __forceinline__ int refine(const double* x, int n, double v, int p) {
  p = p < 0 ? 0 : (p > n - 2 ? n - 2 : p);
  if (p > 0 && v < x[p]) --p;
  else if (p < n - 2 && v >= x[p + 1]) ++p;
  return p;
}

// f clamped to [0, 1]: two FP64 max/min instructions (a NaN comes out as 0;
// a particle with a NaN coordinate is removed by its step anyway)
__device__ __forceinline__ double clamp01(double f) {
  return fmin(fmax(f, 0.0), 1.0);
}

// theta nodes of the uniform grid, bit-identical to the host tables
// (theta0 + j dth and theta0 + (j + 1/2) dth: rounded product, then sum)
__device__ __forceinline__ double theta_node(const GridView& g, int j) {
  return __dadd_rn(g.th0, __dmul_rn((double)j, g.dth));
}
__device__ __forceinline__ double theta_half(const GridView& g, int j) {
  return __dadd_rn(g.th0, __dmul_rn((double)j + 0.5, g.dth));
}

// cell j in [0, n-2] of the n theta points (nodes, or half points if HALF)
// with x_j <= th < x_{j+1} (clamped); lt = (th - theta0) / dth
template <bool HALF>
__device__ __forceinline__ int theta_cell(const GridView& g, double th, double lt, int n) {
  int j = (int)floor(HALF ? lt - 0.5 : lt);
  j = j < 0 ? 0 : (j > n - 2 ? n - 2 : j);
  const double x0 = HALF ? theta_half(g, j) : theta_node(g, j);
  const double x1 = HALF ? theta_half(g, j + 1) : theta_node(g, j + 1);
  if (j > 0 && th < x0) --j;
  else if (j < n - 2 && th >= x1) ++j;
  return j;
}


// the two adjacent values at byte offset b of a field array.  Offsets are
// 32-bit: a field array holds at most 2^30 values and a grid dimension is
// below 2^22 cells (both checked when the context is created), so that row
// offsets are 24-bit products and the loads take a scalar base address plus
// a 32-bit vector offset.
__device__ __forceinline__ float2 ld2(const float* base, uint32_t b) {
  const float* p = reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + b);
  return make_float2(p[0], p[1]);
}

// the two adjacent values of a row and of the next row of each component
__device__ __forceinline__ void corner_loads(const FieldView& F, int nrn, int nrh, int pn,
                                             int ph, int qn, int qh, float2* c) {
  const uint32_t sn = 4u * (uint32_t)nrn, sh = 4u * (uint32_t)nrh;  // row strides
  const uint32_t bn = 4u * (uint32_t)pn, bh = 4u * (uint32_t)ph;
  uint32_t b = __umul24((uint32_t)qn, sh) + bh;  // r-half columns, node rows
  c[0] = ld2(F.Dr, b);
  c[1] = ld2(F.Dr, b + sh);
  c[8] = ld2(F.Bt, b);
  c[9] = ld2(F.Bt, b + sh);
  b = __umul24((uint32_t)qh, sn) + bn;  // node columns, theta-half rows
  c[2] = ld2(F.Dt, b);
  c[3] = ld2(F.Dt, b + sn);
  c[6] = ld2(F.Br, b);
  c[7] = ld2(F.Br, b + sn);
  b = __umul24((uint32_t)qn, sn) + bn;  // node columns, node rows
  c[4] = ld2(F.Dp, b);
  c[5] = ld2(F.Dp, b + sn);
  b = __umul24((uint32_t)qh, sh) + bh;  // r-half columns, theta-half rows
  c[10] = ld2(F.Bp, b);
  c[11] = ld2(F.Bp, b + sh);
}

// bilinear form of the corners v_ij (i radial, j angular) as
// c00 + fr c10 + ft (c01 + fr c11); lerp2 and the cached coefficients of
// gather_coefs share this arithmetic, so both give the same bits
struct Bilin {
  double c00, c10, c01, c11;
};

__device__ __forceinline__ Bilin bilin(float2 r0, float2 r1) {
  const double v00 = r0.x, v10 = r0.y, v01 = r1.x, v11 = r1.y;
  return Bilin{v00, v10 - v00, v01 - v00, (v11 - v01) - (v10 - v00)};
}

__device__ __forceinline__ double bilin_eval(double c00, double c10, double c01, double c11,
                                             double fr, double ft) {
  return fma(ft, fma(fr, c11, c01), fma(fr, c10, c00));
}

__device__ __forceinline__ double lerp2(float2 r0, float2 r1, double fr, double ft) {
  const Bilin b = bilin(r0, r1);
  return bilin_eval(b.c00, b.c10, b.c01, b.c11, fr, ft);
}

// D^i, B^i at (r, theta): sum_c w_c (sqrt(g) F)_c / sqrt(g)(x).  The theta
// cells come from the uniform-grid formula; the radial cells from an FP32
// estimate checked against the node tables.  The field corners of the
// estimated cells are loaded together with those node values (one memory
// round trip) and reloaded only when the estimate was one cell off.  Split
// in two so that a caller can compute between issuing the loads
// (gather_issue) and using them (gather_finish).
struct GatherLoads {
  float2 c[12];
  double rn0, rn1, irn, rh0, rh1, irh;
  // theta_node(qn), theta_node(qn + 1), theta_half(qn), theta_half(qh)
  double tn0, tn1, thq, thh;
  // with gather_bounds: a point with rlo <= r < rhi and tlo <= th < thi lies
  // in all four cells (node and half, in r and in theta)
  double rlo, rhi, tlo, thi;
  int pn, ph, qn, qh;
  // with gather_coefs: each component's corners v_ij (i radial, j angular)
  // in FP64 as the bilinear form's coefficients v00, v10 - v00, v01 - v00
  // and (v11 - v01) - (v10 - v00); the order of gather_interp's D, B
  double c00[6], c10[6], c01[6], c11[6];
};

// the radial node and half values bounding cells pn and ph and their
// inverse widths (32-bit byte offsets, as in corner_loads)
__device__ __forceinline__ double ldd(const double* base, uint32_t b) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + b);
}

__device__ __forceinline__ void radial_loads(const GridView& g, int pn, int ph,
                                             GatherLoads& L) {
  const uint32_t bn = 8u * (uint32_t)pn, bh = 8u * (uint32_t)ph;
  L.rn0 = ldd(g.rn, bn);
  L.rn1 = ldd(g.rn, bn + 8u);
  L.irn = ldd(g.idrn, bn);
  L.rh0 = ldd(g.rh, bh);
  L.rh1 = ldd(g.rh, bh + 8u);
  L.irh = ldd(g.idrh, bh);
}

__device__ __forceinline__ void gather_issue(const GridView& g, const FieldView& F,
                                             double r, double th, GatherLoads& L) {
  const int nr = g.nr, nrn = nr + 1, nrh = nr;
  const double lt = (th - g.th0) * g.inv_dth;
  L.qn = theta_cell<false>(g, th, lt, g.nth + 1);
  // the half-angle cell from the node cell: th lies in [theta_qn,
  // theta_qn+1), so its half cell is qn at or above theta_{qn+1/2} and
  // qn - 1 below (clamped to [0, nth - 2] like the search it replaces)
  L.tn0 = theta_node(g, L.qn);
  L.tn1 = theta_node(g, L.qn + 1);
  L.thq = theta_half(g, L.qn);
  const int qh = th >= L.thq ? L.qn : L.qn - 1;
  L.qh = qh < 0 ? 0 : (qh > g.nth - 2 ? g.nth - 2 : qh);
  L.thh = L.qh == L.qn ? L.thq : theta_half(g, L.qh);
  const float lr = radial_coord(g, r);
  int pn = (int)floorf(lr), ph = (int)floorf(lr - 0.5f);
  L.pn = pn < 0 ? 0 : (pn > nr - 1 ? nr - 1 : pn);
  L.ph = ph < 0 ? 0 : (ph > nr - 2 ? nr - 2 : ph);
  corner_loads(F, nrn, nrh, L.pn, L.ph, L.qn, L.qh, L.c);
  radial_loads(g, L.pn, L.ph, L);
}

// Refine the estimated radial cells against the node values loaded with
// them (one cell either way) and reload the corners when a cell changed:
// afterwards L holds the corners, cells and radial bounds (rn0, rn1, irn,
// rh0, rh1, irh) of the cells of (r, th).
__device__ __forceinline__ void gather_settle(const GridView& g, const FieldView& F,
                                              double r, GatherLoads& L) {
  const int nr = g.nr, nrn = nr + 1, nrh = nr;
  int pn = L.pn, ph = L.ph, pn2 = pn, ph2 = ph;
  if (pn > 0 && r < L.rn0) --pn2;
  else if (pn < nr - 1 && r >= L.rn1) ++pn2;
  if (ph > 0 && r < L.rh0) --ph2;
  else if (ph < nr - 2 && r >= L.rh1) ++ph2;
  if (pn2 != pn || ph2 != ph) {
    L.pn = pn2;
    L.ph = ph2;
    corner_loads(F, nrn, nrh, pn2, ph2, L.qn, L.qh, L.c);
    radial_loads(g, pn2, ph2, L);
  }
}

// the interpolation itself, from settled loads
__device__ __forceinline__ void gather_interp(const GridView& g, double r, double th,
                                              double isg, const GatherLoads& L, double* D,
                                              double* B) {
  const float2* c = L.c;
  const double frn = clamp01((r - L.rn0) * L.irn), frh = clamp01((r - L.rh0) * L.irh);
  const double ftn = clamp01((th - L.tn0) * g.inv_dth);
  const double fth = clamp01((th - L.thh) * g.inv_dth);
  D[0] = lerp2(c[0], c[1], frh, ftn) * isg;
  D[1] = lerp2(c[2], c[3], frn, fth) * isg;
  D[2] = lerp2(c[4], c[5], frn, ftn) * isg;
  B[0] = lerp2(c[6], c[7], frn, fth) * isg;
  B[1] = lerp2(c[8], c[9], frh, ftn) * isg;
  B[2] = lerp2(c[10], c[11], frh, fth) * isg;
}

// the FP64 coefficients of the settled corners (once per loaded cell set;
// interpolating from them takes three FMAs per component and gives exactly
// what gather_interp gives)
__device__ __forceinline__ void gather_coefs(GatherLoads& L) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const Bilin b = bilin(L.c[2 * j], L.c[2 * j + 1]);
    L.c00[j] = b.c00;
    L.c10[j] = b.c10;
    L.c01[j] = b.c01;
    L.c11[j] = b.c11;
  }
}

__device__ __forceinline__ double lerp2c(const GatherLoads& L, int j, double fr, double ft) {
  return bilin_eval(L.c00[j], L.c10[j], L.c01[j], L.c11[j], fr, ft);
}

// gather_interp from the coefficients of gather_coefs
__device__ __forceinline__ void gather_interp_coefs(const GridView& g, double r, double th,
                                                    double isg, const GatherLoads& L,
                                                    double* D, double* B) {
  const double frn = clamp01((r - L.rn0) * L.irn), frh = clamp01((r - L.rh0) * L.irh);
  const double ftn = clamp01((th - L.tn0) * g.inv_dth);
  const double fth = clamp01((th - L.thh) * g.inv_dth);
  D[0] = lerp2c(L, 0, frh, ftn) * isg;
  D[1] = lerp2c(L, 1, frn, fth) * isg;
  D[2] = lerp2c(L, 2, frn, ftn) * isg;
  B[0] = lerp2c(L, 3, frn, fth) * isg;
  B[1] = lerp2c(L, 4, frh, ftn) * isg;
  B[2] = lerp2c(L, 5, frh, fth) * isg;
}

__device__ __forceinline__ void gather_finish(const GridView& g, const FieldView& F,
                                              double r, double th, double isg,
                                              GatherLoads& L, double* D, double* B) {
  gather_settle(g, F, r, L);
  gather_interp(g, r, th, isg, L, D, B);
}

// the hit bounds of the settled cells: each cell is the unique one with
// x_lo <= v < x_hi, open towards the clamped grid edges (an infinite bound
// there); the half theta cell is qn at or above theta_half(qn), else
// qn - 1 (L.qh != L.qn only as L.qh = L.qn - 1).  In the half theta cells
// next to the two axes, where the clamp acts, a point of the same cells can
// fall outside these bounds: it then takes the full gather, which finds
// them again.
__device__ __forceinline__ void gather_bounds(const GridView& g, GatherLoads& L) {
  const double inf = __builtin_huge_val();
  const double rnl = L.pn == 0 ? -inf : L.rn0, rnh = L.pn == g.nr - 1 ? inf : L.rn1;
  const double rhl = L.ph == 0 ? -inf : L.rh0, rhh = L.ph == g.nr - 2 ? inf : L.rh1;
  L.rlo = fmax(rnl, rhl);
  L.rhi = fmin(rnh, rhh);
  const double tnl = L.qn == 0 ? -inf : L.tn0, tnh = L.qn == g.nth - 1 ? inf : L.tn1;
  L.tlo = L.qh == L.qn ? fmax(tnl, L.thq) : tnl;
  L.thi = L.qh == L.qn ? tnh : fmin(tnh, L.thq);
}

// True only when (r, th) lies in the cells whose corners L holds (L.pn < 0:
// none yet), i.e. when a full gather would find exactly these cells: each
// cell is the unique one with x_lo <= v < x_hi, open towards the clamped
// edges.  (A false answer is always safe: the caller gathers in full.)
// Arithmetic only; lets an iteration whose point stays in its cells reuse
// the corners it loaded.
__device__ __forceinline__ bool gather_hit(const GridView& g, double r, double th,
                                           const GatherLoads& L) {
  return L.pn >= 0 && r >= L.rlo && r < L.rhi && th >= L.tlo && th < L.thi;
}

__device__ __forceinline__ void gather(const GridView& g, const FieldView& F,
                                       double r, double th, double isg,
                                       double* D, double* B) {
  GatherLoads L;
  gather_issue(g, F, r, th, L);
  gather_finish(g, F, r, th, isg, L, D, B);
}

// ------------------------------------------------------- equations of motion
// f = (dx^i/dt, du_i/dt); *pw = (q/m) E_i dx^i/dt with
// E_i = alpha D_i + sqrt(g) eta_ijk beta^j B^k (eq. Ei).
__device__ __forceinline__ void rhs(double qm, const double* z, const Met& m,
                                    const DMet& d, const double* D,
                                    const double* B, double* f, double* pw,
                                    double* e = nullptr) {
  double ur = z[3], ut = z[4], up = z[5];
  double Ur = m.irr * ur + m.irp * up;
  double Ut = m.itt * ut;
  double Up = m.irp * ur + m.ipp * up;
  double G = fsqrt(1.0 + ur * Ur + ut * Ut + up * Up);
  double iG = rcp(G);
  double aiG = m.alpha * iG;
  if (e) *e = m.alpha * G - m.betar * ur;
  f[0] = aiG * Ur - m.betar;
  f[1] = aiG * Ut;
  f[2] = aiG * Up;
  double half_aiG = 0.5 * aiG;
  double q_r = ur * ur * d.drr[0] + ut * ut * d.dtt[0] + up * up * d.dpp[0] +
               2.0 * ur * up * d.drp[0];
  double q_t = ur * ur * d.drr[1] + ut * ut * d.dtt[1] + up * up * d.dpp[1] +
               2.0 * ur * up * d.drp[1];
  double gr = -G * d.da[0] + ur * d.db[0] - half_aiG * q_r;
  double gt = -G * d.da[1] + ur * d.db[1] - half_aiG * q_t;
  if (qm != 0.0) {
    double Dl_r = m.grr * D[0] + m.grp * D[2];
    double Dl_t = m.gtt * D[1];
    double Dl_p = m.grp * D[0] + m.gpp * D[2];
    double sgiG = m.sg * iG;
    double cr = Ut * B[2] - Up * B[1];
    double ct = Up * B[0] - Ur * B[2];
    double cp = Ur * B[1] - Ut * B[0];
    double qa = qm * m.alpha;
    f[3] = gr + qa * (Dl_r + sgiG * cr);
    f[4] = gt + qa * (Dl_t + sgiG * ct);
    f[5] = qa * (Dl_p + sgiG * cp);
    double sgb = m.sg * m.betar;
    double Er = m.alpha * Dl_r;
    double Et = m.alpha * Dl_t - sgb * B[2];
    double Ep = m.alpha * Dl_p + sgb * B[1];
    *pw = qm * (Er * f[0] + Et * f[1] + Ep * f[2]);
  } else {
    f[3] = gr;
    f[4] = gt;
    f[5] = 0.0;
    *pw = 0.0;
  }
}

}  // namespace grpic
