// deposit_device.hpp -- volume weights of the charge deposit (Sec. 2.3,
// eqs. v1-v5): a node receives the fraction V_opp / V of the particle's
// charge, V_opp the proper sub-volume (integral of sqrt(gamma) dr dtheta)
// of the sub-rectangle opposite to it and V the sum of the four
// sub-volumes; each sub-volume uses the 2-D trapezoidal rule on 4 x 4 points.
#pragma once
#include "kerr_device.hpp"

namespace grpic {

// node cell (p, q) with rn[p] <= r < rn[p+1], tn[q] <= th < tn[q+1]
// (clamped to the grid)
__device__ __forceinline__ void node_cell(const GridView& g, double r,
                                          double th, int& p, int& q) {
  float lr = radial_coord(g, r);
  double lt = (th - g.th0) * g.inv_dth;
  p = refine(g.rn, g.nr + 1, r, (int)floorf(lr));
  q = theta_cell<false>(g, th, lt, g.nth + 1);
}

// sin and cos of t0 + j h, j = 0..3, from those of t0 and of the small step
// h (Taylor series to h^9 and h^8, exact to rounding for |h| < 0.05) by the
// angle-addition recurrence
__device__ __forceinline__ void sincos_steps(double s0, double c0, double h,
                                             double* S, double* C) {
  double h2 = h * h;
  double sh = h * (1.0 - h2 * (1.0 / 6.0) * (1.0 - h2 * (1.0 / 20.0) *
                   (1.0 - h2 * (1.0 / 42.0) * (1.0 - h2 * (1.0 / 72.0)))));
  double ch = 1.0 - h2 * 0.5 * (1.0 - h2 * (1.0 / 12.0) *
                   (1.0 - h2 * (1.0 / 30.0) * (1.0 - h2 * (1.0 / 56.0))));
  S[0] = s0;
  C[0] = c0;
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    S[j] = S[j - 1] * ch + C[j - 1] * sh;
    C[j] = C[j - 1] * ch - S[j - 1] * sh;
  }
}

// W[0..3] for the corners (ra,ta), (rb,ta), (ra,tb), (rb,tb) of any cell;
// st, ct = sin, cos of th; sq, cq: sin, cos of ta
__device__ __forceinline__ void dep_weights_box(const GridView& g, double r, double th,
                                                double st, double ct, double ra, double rb,
                                                double ta, double tb, double sq, double cq,
                                                double* W) {
  const double a2 = g.a * g.a;
  double h1r = (r - ra) * (1.0 / 3.0), h2r = (rb - r) * (1.0 / 3.0);
  double h1t = (th - ta) * (1.0 / 3.0), h2t = (tb - th) * (1.0 / 3.0);
  // 7 radii ra + i h1r (i = 0..2), r, r + i h2r (i = 1..3), and 7 angles the
  // same way; the rows are visited in order and their angles advanced by the
  // angle-addition recurrence of sincos_steps (few values live at a time;
  // both loops unroll, so each row's trapezoid weights are constants)
  const double h1t2 = h1t * h1t, h2t2 = h2t * h2t;
  const double sh1 = h1t * (1.0 - h1t2 * (1.0 / 6.0) * (1.0 - h1t2 * (1.0 / 20.0) *
                     (1.0 - h1t2 * (1.0 / 42.0) * (1.0 - h1t2 * (1.0 / 72.0)))));
  const double ch1 = 1.0 - h1t2 * 0.5 * (1.0 - h1t2 * (1.0 / 12.0) *
                     (1.0 - h1t2 * (1.0 / 30.0) * (1.0 - h1t2 * (1.0 / 56.0))));
  const double sh2 = h2t * (1.0 - h2t2 * (1.0 / 6.0) * (1.0 - h2t2 * (1.0 / 20.0) *
                     (1.0 - h2t2 * (1.0 / 42.0) * (1.0 - h2t2 * (1.0 / 72.0)))));
  const double ch2 = 1.0 - h2t2 * 0.5 * (1.0 - h2t2 * (1.0 / 12.0) *
                     (1.0 - h2t2 * (1.0 / 30.0) * (1.0 - h2t2 * (1.0 / 56.0))));
  // trapezoid weights along each half: (1/2, 1, 1, 1/2)
  double Vaa = 0.0, Vba = 0.0, Vab = 0.0, Vbb = 0.0;
  double Sj = sq, Cj = cq;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    if (j == 3) {
      Sj = st;
      Cj = ct;
    }
    const double Sabs = fabs(Sj), C2 = a2 * Cj * Cj;
    double wa_t = (j == 0 || j == 3) ? 0.5 : (j < 3 ? 1.0 : 0.0);
    double wb_t = (j == 3 || j == 6) ? 0.5 : (j > 3 ? 1.0 : 0.0);
    double rowa = 0.0, rowb = 0.0;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const double rr = i < 3 ? ra + i * h1r : (i == 3 ? r : r + (i - 3) * h2r);
      const double rho2 = rr * rr + C2, X = rho2 * (rho2 + 2.0 * rr);
      // sqrt(X) = s (1 + e / 2) to about 2^-48 relative, from the hardware
      // estimate y of 1/sqrt(X), s = X y and e = 1 - s y (one Goldschmidt
      // step; the weights end in FP32 sums).  A trapezoid weight w enters
      // through the factor, w sqrt(X) = s (w + (w / 2) e), so that each
      // term is one FMA.  A sample outside a sub-rectangle has weight 0
      // there (its term would add +0 exactly): only the nonzero terms are
      // formed
      const double y = __builtin_amdgcn_rsq(X), sx = X * y, e = fma(-sx, y, 1.0);
      if (i <= 3) {
        const double w = (i == 0 || i == 3) ? 0.5 : 1.0;
        rowa = fma(sx, fma(e, 0.5 * w, w), rowa);
      }
      if (i >= 3) {
        const double w = (i == 3 || i == 6) ? 0.5 : 1.0;
        rowb = fma(sx, fma(e, 0.5 * w, w), rowb);
      }
    }
    if (j <= 3) {
      Vaa += wa_t * Sabs * rowa;  // [ra, r] x [ta, th]
      Vba += wa_t * Sabs * rowb;  // [r, rb] x [ta, th]
    }
    if (j >= 3) {
      Vab += wb_t * Sabs * rowa;  // [ra, r] x [th, tb]
      Vbb += wb_t * Sabs * rowb;  // [r, rb] x [th, tb]
    }
    if (j < 2 || (j >= 3 && j < 6)) {
      const double ch = j < 3 ? ch1 : ch2, sh = j < 3 ? sh1 : sh2;
      const double Sn = Sj * ch + Cj * sh;
      Cj = Cj * ch - Sj * sh;
      Sj = Sn;
    }
  }
  Vaa *= h1r * h1t;
  Vba *= h2r * h1t;
  Vab *= h1r * h2t;
  Vbb *= h2r * h2t;
  double iV = frcp(Vaa + Vba + Vab + Vbb);
  W[0] = Vbb * iV;
  W[1] = Vab * iV;
  W[2] = Vba * iV;
  W[3] = Vaa * iV;
}

// W[0..3] for nodes (p,q), (p+1,q), (p,q+1), (p+1,q+1) of node cell row q;
// ra, rb: radii of the cell's node columns; sq, cq: sin, cos of its lower
// node angle
__device__ __forceinline__ void dep_weights_at(const GridView& g, double r, double th,
                                               double st, double ct, double ra, double rb,
                                               double sq, double cq, int q, double* W) {
  dep_weights_box(g, r, th, st, ct, ra, rb, theta_node(g, q), theta_node(g, q + 1), sq, cq,
                  W);
}

__device__ __forceinline__ void dep_weights(const GridView& g, double r,
                                            double th, double st, double ct,
                                            int p, int q, double* W) {
  dep_weights_at(g, r, th, st, ct, g.rn[p], g.rn[p + 1], g.stn[q], g.ctn[q], q, W);
}

// The node cell of a nearby gather: rn[pn] = rn0, rn[pn + 1] = rn1 and
// theta_node(qn) = tn0, theta_node(qn + 1) = tn1 (pn < 0: none; then the
// other fields are undefined).
struct ColumnHint {
  int pn;
  double rn0, rn1;
  int qn;
  double tn0, tn1;
};

__device__ __forceinline__ ColumnHint column_hint(const GatherLoads& L) {
  return ColumnHint{L.pn, L.rn0, L.rn1, L.qn, L.tn0, L.tn1};
}

// node cell (p, q) of (r, th) and its weights.  hint: the node cell of a
// nearby gather (the last RK4 stage); when r lies in its column the radii
// come from it, else the node values are loaded in one memory round trip
// (the FP32 radial estimate is checked against them); when th lies in its
// row, so do q and the row's angles.
// The sin and cos of the cell's lower node angle follow from those of th by
// the short series of sincos_near when the two are close, else from the
// node tables.
__device__ __forceinline__ void cell_and_weights(const GridView& g, double r, double th,
                                                 double st, double ct, int& p, int& q,
                                                 double* W,
                                                 ColumnHint hint = ColumnHint{-1, 0.0, 0.0,
                                                                              -1, 0.0, 0.0}) {
  const int nr = g.nr;
  double tq, tq1;
  if (hint.pn >= 0 && (hint.qn == 0 || th >= hint.tn0) &&
      (hint.qn == g.nth - 1 || th < hint.tn1)) {
    q = hint.qn;
    tq = hint.tn0;
    tq1 = hint.tn1;
  } else {
    q = theta_cell<false>(g, th, (th - g.th0) * g.inv_dth, g.nth + 1);
    tq = theta_node(g, q);
    tq1 = theta_node(g, q + 1);
  }
  double r0, r1;
  if (hint.pn >= 0 && (hint.pn == 0 || r >= hint.rn0) && (hint.pn == nr - 1 || r < hint.rn1)) {
    p = hint.pn;
    r0 = hint.rn0;
    r1 = hint.rn1;
  } else {
    int p0 = (int)floorf(radial_coord(g, r));
    p0 = p0 < 0 ? 0 : (p0 > nr - 1 ? nr - 1 : p0);
    r0 = g.rn[p0];
    r1 = g.rn[p0 + 1];
    p = p0;
    if (p0 > 0 && r < r0) {
      p = p0 - 1;
      r1 = r0;
      r0 = g.rn[p];
    } else if (p0 < nr - 1 && r >= r1) {
      p = p0 + 1;
      r0 = r1;
      r1 = g.rn[p + 1];
    }
  }
  double sq, cq;
  if (fabs(tq - th) <= 0.01) {
    sincos_near(tq, th, st, ct, &sq, &cq);
  } else {
    sq = g.stn[q];
    cq = g.ctn[q];
  }
  dep_weights_box(g, r, th, st, ct, r0, r1, tq, tq1, sq, cq, W);
}

__device__ __forceinline__ void dep_weights(const GridView& g, double r,
                                            double th, int p, int q,
                                            double* W) {
  double st, ct;
  fsincos(th, &st, &ct);
  dep_weights(g, r, th, st, ct, p, q, W);
}

}  // namespace grpic
