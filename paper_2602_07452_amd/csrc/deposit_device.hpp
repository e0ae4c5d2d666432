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
  double lr = log(r / g.r_in) * g.inv_dlnr;
  double lt = (th - g.th0) * g.inv_dth;
  p = refine(g.rn, g.nr + 1, r, (int)floor(lr));
  q = refine(g.tn, g.nth + 1, th, (int)floor(lt));
}

// W[0..3] for nodes (p,q), (p+1,q), (p,q+1), (p+1,q+1)
__device__ __forceinline__ void dep_weights(const GridView& g, double r,
                                            double th, int p, int q,
                                            double* W) {
  const double a2 = g.a * g.a;
  double ra = g.rn[p], rb = g.rn[p + 1], ta = g.tn[q], tb = g.tn[q + 1];
  double h1r = (r - ra) * (1.0 / 3.0), h2r = (rb - r) * (1.0 / 3.0);
  double h1t = (th - ta) * (1.0 / 3.0), h2t = (tb - th) * (1.0 / 3.0);
  // 7 radii: ra + i h1r (i = 0..2), r, r + i h2r (i = 1..3); same for theta
  double R[7], S[7], C2[7];
#pragma unroll
  for (int i = 0; i < 3; ++i) R[i] = ra + i * h1r;
  R[3] = r;
#pragma unroll
  for (int i = 1; i < 4; ++i) R[3 + i] = r + i * h2r;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double t = j < 3 ? ta + j * h1t : (j == 3 ? th : th + (j - 3) * h2t);
    double s, c;
    sincos(t, &s, &c);
    S[j] = fabs(s);
    C2[j] = a2 * c * c;
  }
  // trapezoid weights along each half: (1/2, 1, 1, 1/2)
  double Vaa = 0.0, Vba = 0.0, Vab = 0.0, Vbb = 0.0;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double wa_t = (j == 0 || j == 3) ? 0.5 : (j < 3 ? 1.0 : 0.0);
    double wb_t = (j == 3 || j == 6) ? 0.5 : (j > 3 ? 1.0 : 0.0);
    double rowa = 0.0, rowb = 0.0;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      double rr = R[i];
      double rho2 = rr * rr + C2[j];
      double f = S[j] * sqrt(rho2 * (rho2 + 2.0 * rr));
      double wa_r = (i == 0 || i == 3) ? 0.5 : (i < 3 ? 1.0 : 0.0);
      double wb_r = (i == 3 || i == 6) ? 0.5 : (i > 3 ? 1.0 : 0.0);
      rowa += wa_r * f;
      rowb += wb_r * f;
    }
    Vaa += wa_t * rowa;  // [ra, r] x [ta, th]
    Vba += wa_t * rowb;  // [r, rb] x [ta, th]
    Vab += wb_t * rowa;  // [ra, r] x [th, tb]
    Vbb += wb_t * rowb;  // [r, rb] x [th, tb]
  }
  Vaa *= h1r * h1t;
  Vba *= h2r * h1t;
  Vab *= h1r * h2t;
  Vbb *= h2r * h2t;
  double iV = 1.0 / (Vaa + Vba + Vab + Vbb);
  W[0] = Vbb * iV;
  W[1] = Vab * iV;
  W[2] = Vba * iV;
  W[3] = Vaa * iV;
}

}  // namespace grpic
