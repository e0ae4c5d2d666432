// flopcount.cpp -- FP64 operation counts of the particle step, measured by
// compiling the oracle's own sources (om_core.c, om_grid.c, om_init.c) with
// every `double` replaced by a counting scalar type.
//
// TEST INFRASTRUCTURE: like the rest of oracle/, this program is not part of
// the product path.  Its output (per-particle operation counts of the pieces
// of one particle step: the RK4 step with its four field gathers, the energy
// of the switch, one implicit-midpoint (Picard) iteration and the deposit
// weights of a position) gives the algorithmic FLOPs against which the GPU
// push's roofline fraction is stated.
//
// Counting: an addition, subtraction or multiplication is one operation, a
// fused multiply-add would be two (the oracle writes none); divisions, square
// roots and transcendental functions (sin, cos, exp, log, atan, ...) are
// counted separately; comparisons, negations, fabs, floor and conversions
// are not counted.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <cstdio>

namespace opc {
struct Counts {
  unsigned long long add = 0, mul = 0, div = 0, sqrt = 0, trans = 0;
};
Counts c;
}  // namespace opc

struct fd {
  double v;
  fd() = default;
  constexpr fd(double x) : v(x) {}
  explicit operator double() const { return v; }
  explicit operator int() const { return (int)v; }
  explicit operator long() const { return (long)v; }
  explicit operator long long() const { return (long long)v; }
  explicit operator unsigned long long() const { return (unsigned long long)v; }
  explicit operator float() const { return (float)v; }
  explicit operator bool() const { return v != 0.0; }
  fd& operator+=(fd o) { ++opc::c.add; v += o.v; return *this; }
  fd& operator-=(fd o) { ++opc::c.add; v -= o.v; return *this; }
  fd& operator*=(fd o) { ++opc::c.mul; v *= o.v; return *this; }
  fd& operator/=(fd o) { ++opc::c.div; v /= o.v; return *this; }
};
static_assert(sizeof(fd) == sizeof(double), "layout");

inline fd operator+(fd a, fd b) { ++opc::c.add; return fd(a.v + b.v); }
inline fd operator-(fd a, fd b) { ++opc::c.add; return fd(a.v - b.v); }
inline fd operator*(fd a, fd b) { ++opc::c.mul; return fd(a.v * b.v); }
inline fd operator/(fd a, fd b) { ++opc::c.div; return fd(a.v / b.v); }
inline fd operator-(fd a) { return fd(-a.v); }
inline fd operator+(fd a) { return a; }
inline bool operator<(fd a, fd b) { return a.v < b.v; }
inline bool operator>(fd a, fd b) { return a.v > b.v; }
inline bool operator<=(fd a, fd b) { return a.v <= b.v; }
inline bool operator>=(fd a, fd b) { return a.v >= b.v; }
inline bool operator==(fd a, fd b) { return a.v == b.v; }
inline bool operator!=(fd a, fd b) { return a.v != b.v; }
inline bool operator!(fd a) { return !a.v; }
inline bool operator&&(fd a, bool b) { return a.v != 0.0 && b; }

inline fd sqrt(fd a) { ++opc::c.sqrt; return fd(std::sqrt(a.v)); }
inline fd sin(fd a) { ++opc::c.trans; return fd(std::sin(a.v)); }
inline fd cos(fd a) { ++opc::c.trans; return fd(std::cos(a.v)); }
inline fd tan(fd a) { ++opc::c.trans; return fd(std::tan(a.v)); }
inline fd exp(fd a) { ++opc::c.trans; return fd(std::exp(a.v)); }
inline fd log(fd a) { ++opc::c.trans; return fd(std::log(a.v)); }
inline fd atan(fd a) { ++opc::c.trans; return fd(std::atan(a.v)); }
inline fd atan2(fd a, fd b) { ++opc::c.trans; return fd(std::atan2(a.v, b.v)); }
inline fd asin(fd a) { ++opc::c.trans; return fd(std::asin(a.v)); }
inline fd acos(fd a) { ++opc::c.trans; return fd(std::acos(a.v)); }
inline fd pow(fd a, fd b) { ++opc::c.trans; return fd(std::pow(a.v, b.v)); }
inline fd cbrt(fd a) { ++opc::c.trans; return fd(std::cbrt(a.v)); }
inline fd erf(fd a) { ++opc::c.trans; return fd(std::erf(a.v)); }
inline fd fabs(fd a) { return fd(std::fabs(a.v)); }
inline fd floor(fd a) { return fd(std::floor(a.v)); }
inline fd ceil(fd a) { return fd(std::ceil(a.v)); }
inline fd fmax(fd a, fd b) { return fd(std::fmax(a.v, b.v)); }
inline fd fmin(fd a, fd b) { return fd(std::fmin(a.v, b.v)); }
inline fd copysign(fd a, fd b) { return fd(std::copysign(a.v, b.v)); }
inline fd ldexp(fd a, int e) { return fd(std::ldexp(a.v, e)); }
inline bool isfinite(fd a) { return std::isfinite(a.v); }
inline bool isnan(fd a) { return std::isnan(a.v); }
inline long lround(fd a) { return std::lround(a.v); }

#define double fd
#include "om_core.c"
#include "om_grid.c"
#include "om_init.c"
#undef double

namespace {

struct Tally {
  unsigned long long add = 0, mul = 0, div = 0, sqrt = 0, trans = 0;
  long units = 0;
  void take(const opc::Counts& a, const opc::Counts& b) {
    add += b.add - a.add;
    mul += b.mul - a.mul;
    div += b.div - a.div;
    sqrt += b.sqrt - a.sqrt;
    trans += b.trans - a.trans;
    ++units;
  }
  void print(const char* name, bool last) const {
    double u = units > 0 ? (double)units : 1.0;
    std::printf(
        "  \"%s\": {\"units\": %ld, \"add_sub\": %.2f, \"mul\": %.2f, \"div\": %.2f, "
        "\"sqrt\": %.2f, \"transcendental\": %.2f, \"flop\": %.2f}%s\n",
        name, units, add / u, mul / u, div / u, sqrt / u, trans / u,
        (add + mul + div + sqrt + trans) / u, last ? "" : ",");
  }
};

}  // namespace

// Workload: the full-cycle split-monopole magnetosphere (Kerr a = 0.9,
// positions uniform in proper volume over [r_+, 90], Maxwell-Juettner
// Theta = 0.05) in the grid fields of the split monopole on a 256 x 256 grid
// over [0.9 r_+, 100] (the counts per particle do not depend on the grid
// size), time step 1e-3; argv[1] = particles (default 4096).
int main(int argc, char** argv) {
  const long n = argc > 1 ? std::atol(argv[1]) : 4096;
  const double a = 0.9, rp = 1.0 + std::sqrt(1.0 - a * a);
  const int nr = 256, nth = 256;
  const double th0 = 3.14159265358979323846 / 200.0;
  om_grid* g = om_grid_new(fd(a), nr, nth, fd(0.9 * rp), fd(100.0), fd(th0));
  // split-monopole grid fields, densitized as the push reads them
  fd* D[3];
  fd* B[3];
  fd* G[6];
  for (int c = 0; c < 6; ++c) {
    int nR, nT;
    om_comp_shape(g, c, &nR, &nT);
    fd* arr = (fd*)calloc((size_t)nR * nT, sizeof(fd));
    (c < 3 ? D[c] : B[c - 3]) = arr;
    G[c] = (fd*)calloc((size_t)nR * nT, sizeof(fd));
  }
  om_split_monopole_grid(g, fd(1.0), fd(1e3), D, B);
  for (int c = 0; c < 6; ++c) om_densitize(g, c, 1, c < 3 ? D[c] : B[c - 3], G[c]);
  // particles
  om_particles p;
  memset(&p, 0, sizeof(p));
  p.n = n;
  fd** arrs[] = {&p.r, &p.th, &p.ph, &p.ur, &p.uth, &p.uph, &p.qm, &p.w, &p.H0, &p.herr,
                 &p.crit};
  for (fd** q : arrs) *q = (fd*)calloc((size_t)n, sizeof(fd));
  p.flags = (int*)calloc((size_t)n, sizeof(int));
  p.iters = (int*)calloc((size_t)n, sizeof(int));
  om_init_particles(2, fd(a), 2602074525ull, n, fd(rp), fd(90.0), fd(th0),
                    fd(3.14159265358979323846 - th0), fd(0.05), fd(1.0), &p);
  om_push_params P;
  memset(&P, 0, sizeof(P));
  P.a = a;
  P.dt = 1e-3;
  P.pusher = OM_IMR;
  P.tol = 1e-13;
  P.kmax = 50;
  P.field_kind = OM_FIELDS_GRID;
  P.r_min = rp;
  P.r_max = 100.0;
  P.th_lo = th0;
  P.th_hi = 3.14159265358979323846 - th0;
  P.ham_eps = 1e-10;

  Tally rk4, energy, weights, imr2, imr3, gather, metric, metric_d, rhs;
  for (long k = 0; k < n; ++k) {
    if (!(p.flags[k] & OM_ALIVE) || p.qm[k] == fd(0.0)) continue;
    fd z[6] = {p.r[k], p.th[k], p.ph[k], p.ur[k], p.uth[k], p.uph[k]};
    fd out[6], Wq, Dg[3], Bg[3], m[13], d[12], f[6];
    opc::Counts c0 = opc::c;
    om_step_rk4(&P, g, G, p.qm[k], z, out, &Wq);
    rk4.take(c0, opc::c);
    c0 = opc::c;
    (void)om_energy(fd(a), out);
    energy.take(c0, opc::c);
    // deposit weights of the new position (its node cell by the table search)
    int pc = om_locate(g->rn, nr + 1, out[0]), qc = om_locate(g->tn, nth + 1, out[1]);
    fd W[4];
    c0 = opc::c;
    om_dep_weights(g, out[0], out[1], pc, qc, 0, W);
    weights.take(c0, opc::c);
    // one Picard iteration: the count of two iterations minus one
    om_push_params Pk = P;
    fd o2[6], o3[6], w2, w3;
    Pk.kmax = 2;
    c0 = opc::c;
    int i2 = om_step_imr(&Pk, g, G, p.qm[k], z, nullptr, o2, &w2);
    imr2.take(c0, opc::c);
    Pk.kmax = 3;
    c0 = opc::c;
    int i3 = om_step_imr(&Pk, g, G, p.qm[k], z, nullptr, o3, &w3);
    imr3.take(c0, opc::c);
    (void)i3;
    if (i2 > 0) return 2;  // converged in two from z^n: no third iteration counted
    // pieces of one evaluation of the equations of motion
    c0 = opc::c;
    om_gather(g, G, z[0], z[1], Dg, Bg);
    gather.take(c0, opc::c);
    c0 = opc::c;
    om_metric(fd(a), z[0], z[1], m);
    metric.take(c0, opc::c);
    c0 = opc::c;
    om_metric_deriv(fd(a), z[0], z[1], d);
    metric_d.take(c0, opc::c);
    c0 = opc::c;
    om_rhs(fd(a), p.qm[k], z, Dg, Bg, f);
    rhs.take(c0, opc::c);
  }
  // Newton's method for the same equation: one iteration likewise
  Tally nw2, nw3;
  om_push_params Pn = P;
  Pn.solver = OM_SOLVER_NEWTON;
  for (long k = 0; k < n && nw3.units < 512; ++k) {
    if (!(p.flags[k] & OM_ALIVE) || p.qm[k] == fd(0.0)) continue;
    fd z[6] = {p.r[k], p.th[k], p.ph[k], p.ur[k], p.uth[k], p.uph[k]};
    fd o[6], w;
    Pn.kmax = 1;
    opc::Counts c0 = opc::c;
    int i1 = om_step_imr(&Pn, g, G, p.qm[k], z, nullptr, o, &w);
    nw2.take(c0, opc::c);
    Pn.kmax = 2;
    c0 = opc::c;
    int i2 = om_step_imr(&Pn, g, G, p.qm[k], z, nullptr, o, &w);
    nw3.take(c0, opc::c);
    (void)i2;
    if (i1 > 0) return 3;  // Newton converged in one: no second iteration counted
  }

  // Neutral test particles without fields (Schwarzschild orbits, r in
  // [6, 20], theta in [pi/4, 3 pi/4], dt = 0.01): the explicit step, and one
  // iteration of the discrete-gradient scheme
  om_particles q;
  memset(&q, 0, sizeof(q));
  q.n = 1024;
  fd** qarrs[] = {&q.r, &q.th, &q.ph, &q.ur, &q.uth, &q.uph, &q.qm, &q.w, &q.H0, &q.herr,
                  &q.crit};
  for (fd** x : qarrs) *x = (fd*)calloc((size_t)q.n, sizeof(fd));
  q.flags = (int*)calloc((size_t)q.n, sizeof(int));
  q.iters = (int*)calloc((size_t)q.n, sizeof(int));
  const double pi = 3.14159265358979323846;
  om_init_particles(0, fd(0.0), 2602074521ull, q.n, fd(6.0), fd(20.0), fd(0.25 * pi),
                    fd(0.75 * pi), fd(0.1), fd(1.0), &q);
  om_push_params Q;
  memset(&Q, 0, sizeof(Q));
  Q.a = 0.0;
  Q.dt = 0.01;
  Q.pusher = OM_HAM;
  Q.tol = 1e-13;
  Q.field_kind = OM_FIELDS_NONE;
  Q.r_min = 2.0;
  Q.r_max = 1e30;
  Q.th_lo = -1.0;
  Q.th_hi = 10.0;
  Q.ham_eps = 1e-10;
  Tally rk4n, ham2, ham3;
  for (long k = 0; k < q.n; ++k) {
    if (!(q.flags[k] & OM_ALIVE)) continue;
    fd z[6] = {q.r[k], q.th[k], q.ph[k], q.ur[k], q.uth[k], q.uph[k]};
    fd o[6], w;
    opc::Counts c0 = opc::c;
    om_step_rk4(&Q, g, nullptr, fd(0.0), z, o, &w);
    rk4n.take(c0, opc::c);
    Q.kmax = 2;
    c0 = opc::c;
    int i2 = om_step_ham(&Q, z, nullptr, o);
    ham2.take(c0, opc::c);
    Q.kmax = 3;
    c0 = opc::c;
    int i3 = om_step_ham(&Q, z, nullptr, o);
    ham3.take(c0, opc::c);
    (void)i3;
    if (i2 > 0) return 4;
  }

  // one iteration = difference of the counts with one more iteration allowed
  auto diff = [](const Tally& hi, const Tally& lo) {
    Tally t;
    t.add = hi.add - lo.add;
    t.mul = hi.mul - lo.mul;
    t.div = hi.div - lo.div;
    t.sqrt = hi.sqrt - lo.sqrt;
    t.trans = hi.trans - lo.trans;
    t.units = hi.units;
    return t;
  };
  std::printf("{\n  \"particles\": %ld,\n", rk4.units);
  rk4.print("rk4_step", false);
  energy.print("energy", false);
  weights.print("deposit_weights", false);
  diff(imr3, imr2).print("imr_iteration", false);
  diff(nw3, nw2).print("newton_iteration", false);
  gather.print("gather", false);
  metric.print("metric", false);
  metric_d.print("metric_derivatives", false);
  rhs.print("equations_of_motion", false);
  rk4n.print("rk4_step_no_fields", false);
  diff(ham3, ham2).print("ham_iteration", true);
  std::printf("}\n");
  return 0;
}
