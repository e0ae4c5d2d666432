/* Internal declarations of the reference oracle (test infrastructure). */
#ifndef OM_INTERNAL_H
#define OM_INTERNAL_H
#include "grpic_oracle.h"

struct om_grid {
  double a;
  int nr, nth;
  double r_in, r_out, th0, dth, dlnr;
  double *rn; /* nr+1 node radii                                        */
  double *rh; /* nr half radii r_{i+1/2} = sqrt(r_i r_{i+1})             */
  double *tn; /* nth+1 node angles                                       */
  double *th; /* nth half angles                                         */
};

/* position types: r half? theta half? */
static inline int om_comp_rhalf(int c) {
  /* D^r, B^theta, B^phi live at half-integer radii */
  return c == 0 || c == 4 || c == 5;
}
static inline int om_comp_thalf(int c) {
  /* D^theta, B^r, B^phi live at half-integer angles */
  return c == 1 || c == 3 || c == 5;
}

double om_sqrtg(double a, double r, double th);
/* cell index lo of v in the increasing table x[0..n-1], clamped to [0, n-2] */
int om_locate(const double *x, int n, double v);

#endif
