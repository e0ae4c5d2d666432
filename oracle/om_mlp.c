/*
 * om_mlp.c -- reference oracle (TEST INFRASTRUCTURE ONLY): FP64 forward and
 * backward pass of the 14 -> 64 -> 64 -> 6 GELU network that supplies the
 * implicit pusher's initial guess (a project extension, not in the paper).
 * GELU is the exact form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.
 * Loss = mean over rows and outputs of (y - t)^2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "om_internal.h"

#define NI 14
#define NH 64
#define NO 6

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }
static double gelu_d(double x) {
  double pdf = exp(-0.5 * x * x) / sqrt(2.0 * 3.14159265358979323846);
  return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * pdf;
}

typedef struct {
  const double *W1, *b1, *W2, *b2, *W3, *b3;
} params;

static params unpack(const double *t) {
  params p;
  p.W1 = t;
  p.b1 = p.W1 + NH * NI;
  p.W2 = p.b1 + NH;
  p.b2 = p.W2 + NH * NH;
  p.W3 = p.b2 + NH;
  p.b3 = p.W3 + NO * NH;
  return p;
}

static void forward_row(const params *p, const double *x, double *a1,
                        double *h1, double *a2, double *h2, double *y) {
  for (int o = 0; o < NH; ++o) {
    double s = p->b1[o];
    for (int i = 0; i < NI; ++i) s += p->W1[o * NI + i] * x[i];
    a1[o] = s;
    h1[o] = gelu(s);
  }
  for (int o = 0; o < NH; ++o) {
    double s = p->b2[o];
    for (int i = 0; i < NH; ++i) s += p->W2[o * NH + i] * h1[i];
    a2[o] = s;
    h2[o] = gelu(s);
  }
  for (int o = 0; o < NO; ++o) {
    double s = p->b3[o];
    for (int i = 0; i < NH; ++i) s += p->W3[o * NH + i] * h2[i];
    y[o] = s;
  }
}

void om_mlp_forward(const double *theta, long n, const double *X, double *Y) {
  params p = unpack(theta);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < n; ++k) {
    double a1[NH], h1[NH], a2[NH], h2[NH];
    forward_row(&p, X + k * NI, a1, h1, a2, h2, Y + k * NO);
  }
}

double om_mlp_loss_grad(const double *theta, long n, const double *X,
                        const double *T, double *grad) {
  params p = unpack(theta);
  memset(grad, 0, sizeof(double) * OM_MLP_NPARAM);
  double *gW1 = grad, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH,
         *gb2 = gW2 + NH * NH, *gW3 = gb2 + NH, *gb3 = gW3 + NO * NH;
  double loss = 0.0, scale = 1.0 / ((double)n * NO);
  /* sequential over rows: the plain definition of the summed gradient */
  for (long k = 0; k < n; ++k) {
    double a1[NH], h1[NH], a2[NH], h2[NH], y[NO], dy[NO], dh2[NH], da2[NH],
        dh1[NH], da1[NH];
    const double *x = X + k * NI;
    forward_row(&p, x, a1, h1, a2, h2, y);
    for (int o = 0; o < NO; ++o) {
      double e = y[o] - T[k * NO + o];
      loss += e * e * scale;
      dy[o] = 2.0 * e * scale;
    }
    for (int i = 0; i < NH; ++i) dh2[i] = 0.0;
    for (int o = 0; o < NO; ++o) {
      gb3[o] += dy[o];
      for (int i = 0; i < NH; ++i) {
        gW3[o * NH + i] += dy[o] * h2[i];
        dh2[i] += p.W3[o * NH + i] * dy[o];
      }
    }
    for (int i = 0; i < NH; ++i) da2[i] = dh2[i] * gelu_d(a2[i]);
    for (int i = 0; i < NH; ++i) dh1[i] = 0.0;
    for (int o = 0; o < NH; ++o) {
      gb2[o] += da2[o];
      for (int i = 0; i < NH; ++i) {
        gW2[o * NH + i] += da2[o] * h1[i];
        dh1[i] += p.W2[o * NH + i] * da2[o];
      }
    }
    for (int i = 0; i < NH; ++i) da1[i] = dh1[i] * gelu_d(a1[i]);
    for (int o = 0; o < NH; ++o) {
      gb1[o] += da1[o];
      for (int i = 0; i < NI; ++i) gW1[o * NI + i] += da1[o] * x[i];
    }
  }
  return loss;
}
