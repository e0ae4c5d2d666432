// inject.hip -- pair injection (Sec. 3.3).  Every node cell (p, q) whose
// centre (r_{p+1/2}, theta_{q+1/2}) lies in the injection shell receives one
// co-located e+/e- pair while its plasma density n (the weights of its
// charged particles over V_cell) is below mult * n_GJ:
//   n_GJ = Omega_H |cos(theta) B^r - r sin(theta) B^theta| / (4 pi)
// (the rotation axis taken as the gradient of r cos(theta)), Omega_H =
// a / (2 r_+), B at the cell centre from the mean of the densitized values
// on the cell's two faces; V_cell = 2 pi sqrt(g)(centre) dr dtheta.  Each
// particle of the pair weighs density * n_GJ * V_cell / 2.  Cells are taken
// in index order q n_r + p while there is room for a pair (prefix sum over
// the eligible cells), so the result does not depend on thread order; the
// pair's position and momenta come from the seeded draws of
// sampling_device.hpp (stream c = q n_r + p for the position, 2c and 2c + 1
// for the momenta) with the seed of the injection event.
#include <cstring>

#include "deposit_device.hpp"
#include "sampling_device.hpp"

namespace grpic {

namespace {

struct InjArgs {
  GridView g;
  ParticleView p;        // the particles before the injection (p.n of them)
  const float *Br, *Bt;  // densitized B^r at (r_i, th_{j+1/2}), B^th at (r_{i+1/2}, th_j)
  long long* wsum;       // per node cell: weights in units of 1 / scale
  int *flag, *off, *tot; // eligibility, prefix sums, tot[0] = eligible cells
  unsigned long long* wmax;  // bits of the largest injected weight
  double scale, mult, density, OmH;
  int p0, p1;            // cell columns whose centre radius is in the shell
  uint64_t seed;         // seed of this injection event
  const double* mj;
  int mj_k;
  double mj_h;
  long room;             // particles that still fit
};

__global__ __launch_bounds__(256) void k_inj_count(InjArgs A) {
  const ParticleView& P = A.p;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  if (!(P.flags[k] & GRPIC_FLAG_ALIVE) || P.qm[k] == 0) return;
  long long v = llrint(P.w[k] * A.scale);
  if (v != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(A.wsum + P.cell[k]),
              static_cast<unsigned long long>(v));
}

// n_GJ and V_cell of cell (p, q)
__device__ __forceinline__ void cell_gj(const InjArgs& A, int p, int q, double& ngj,
                                        double& V) {
  const GridView& g = A.g;
  const int nr = g.nr, nrn = nr + 1;
  const double rc = g.rh[p], tc = g.th[q];
  Met m;
  metric(g.a, rc, tc, m);
  const double br = 0.5 * ((double)A.Br[(long)q * nrn + p] + (double)A.Br[(long)q * nrn + p + 1]) / m.sg;
  const double bt = 0.5 * ((double)A.Bt[(long)q * nr + p] + (double)A.Bt[(long)(q + 1) * nr + p]) / m.sg;
  ngj = A.OmH * fabs(m.c * br - rc * m.s * bt) / (4.0 * kPi);
  V = 2.0 * kPi * m.sg * (g.rn[p + 1] - g.rn[p]) * g.dth;
}

__global__ __launch_bounds__(256) void k_inj_decide(InjArgs A) {
  const int nr = A.g.nr;
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)nr * A.g.nth) return;
  int q = (int)(c / nr), p = (int)(c - (long)q * nr);
  int f = 0;
  if (p >= A.p0 && p <= A.p1) {
    double ngj, V;
    cell_gj(A, p, q, ngj, V);
    double n = (double)A.wsum[c] / A.scale / V;
    f = n < A.mult * ngj ? 1 : 0;
  }
  A.flag[c] = f;
  A.wsum[c] = 0;  // ready for the next injection
}

// exclusive prefix sum of flag over all cells, one block of 1024 threads
// (each a contiguous range); tot[0] = the sum
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_inj_scan(InjArgs A, long ncell) {
  __shared__ long part[kScanThreads];
  const int t = threadIdx.x;
  const long per = (ncell + kScanThreads - 1) / kScanThreads;
  const long b = (long)t * per, e = min(b + per, ncell);
  long s = 0;
  for (long c = b; c < e; ++c) s += A.flag[c];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    long run = 0;
    for (int i = 0; i < kScanThreads; ++i) {
      long v = part[i];
      part[i] = run;
      run += v;
    }
    A.tot[0] = (int)run;
  }
  __syncthreads();
  long run = part[t];
  for (long c = b; c < e; ++c) {
    A.off[c] = (int)run;
    run += A.flag[c];
  }
}

__global__ __launch_bounds__(256) void k_inj_write(InjArgs A) {
  const GridView& g = A.g;
  const int nr = g.nr;
  long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long)nr * g.nth) return;
  if (!A.flag[c]) return;
  const long k = A.off[c];
  if (2 * (k + 1) > A.room) return;
  int q = (int)(c / nr), p = (int)(c - (long)q * nr);
  double ngj, V;
  cell_gj(A, p, q, ngj, V);
  const double w = 0.5 * A.density * ngj * V;
  double z[6];
  sample_position(g.a, A.seed, c, g.rn[p], g.rn[p + 1], theta_node(g, q),
                  theta_node(g, q + 1), z);
  double st, ct;
  fsincos(z[1], &st, &ct);
  int cp, cq;
  double W[4];
  cell_and_weights(g, z[0], z[1], st, ct, cp, cq, W);
  const ParticleView& P = A.p;
  for (int s = 0; s < 2; ++s) {
    const long id = 2 * c + s, slot = P.n + 2 * k + s;
    const double mag = mj_speed(A.mj, A.mj_k, A.mj_h, draw(A.seed, id, 200));
    fido_momentum(g.a, A.seed, id, mag, z[0], z[1], z + 3);
    P.r[slot] = z[0];
    P.th[slot] = z[1];
    P.ph[slot] = z[2];
    P.ur[slot] = z[3];
    P.uth[slot] = z[4];
    P.uph[slot] = z[5];
    P.qm[slot] = s == 0 ? 1 : -1;
    P.w[slot] = w;
    P.H0[slot] = energy(g.a, z);
    P.herr[slot] = 0.0;
    P.flags[slot] = GRPIC_FLAG_ALIVE;
    P.iters[slot] = 0;
    P.id[slot] = (uint32_t)slot;
#pragma unroll
    for (int i = 1; i < 4; ++i) P.W[i][slot] = wq_encode(W[i]);
    P.cell[slot] = cq * nr + cp;
  }
  atomicMax(A.wmax, (unsigned long long)__double_as_longlong(w));
}

}  // namespace

long launch_inject(grpic_ctx* c, const double* mj, int mj_k, double mj_h) {
  const int nr = c->nr, nth = c->nth;
  const long ncell = (long)nr * nth;
  InjArgs A;
  A.g = make_grid_view(c);
  A.p = c->pv;
  A.p.n = c->n;
  A.Br = c->B[1].c[0];  // the integer chain: B^{n+2} after the step
  A.Bt = c->B[1].c[1];
  A.wsum = c->inj_wsum;
  A.flag = c->inj_flag;
  A.off = c->inj_off;
  A.tot = c->inj_tot;
  A.wmax = reinterpret_cast<unsigned long long*>(c->inj_tot + 2);
  A.scale = c->qw_max > 0.0 ? ldexp(1.0, 40) / c->qw_max : 1.0;
  A.mult = c->cfg.inj_mult;
  A.density = c->cfg.inj_density;
  const double a = c->cfg.a, rp = 1.0 + sqrt(1.0 - a * a);
  A.OmH = a / (2.0 * rp);
  A.p0 = nr;
  A.p1 = -1;
  for (int p = 0; p < nr; ++p)
    if (c->h_rh[p] >= c->cfg.inj_r0 && c->h_rh[p] <= c->cfg.inj_r1) {
      A.p0 = std::min(A.p0, p);
      A.p1 = std::max(A.p1, p);
    }
  A.seed = c->cfg.inj_seed + (uint64_t)c->steps * 0x9E3779B97F4A7C15ull;
  A.mj = mj;
  A.mj_k = mj_k;
  A.mj_h = mj_h;
  A.room = c->cap - c->n;
  launch_fill(c, c->inj_tot, 4 * sizeof(int));
  if (c->n > 0)
    hipLaunchKernelGGL(k_inj_count, dim3(grid_for(c->n, 256)), dim3(256), 0, c->stream, A);
  hipLaunchKernelGGL(k_inj_decide, dim3(grid_for(ncell, 256)), dim3(256), 0, c->stream, A);
  hipLaunchKernelGGL(k_inj_scan, dim3(1), dim3(kScanThreads), 0, c->stream, A, ncell);
  hipLaunchKernelGGL(k_inj_write, dim3(grid_for(ncell, 256)), dim3(256), 0, c->stream, A);
  GRPIC_HIP(hipGetLastError());
  int tot[4];
  GRPIC_HIP(hipMemcpyAsync(tot, c->inj_tot, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  const long pairs = std::min<long>(tot[0], A.room / 2);
  if (pairs > 0) {
    unsigned long long bits;
    std::memcpy(&bits, tot + 2, sizeof(bits));
    double wmax;
    std::memcpy(&wmax, &bits, sizeof(wmax));
    c->n += 2 * pairs;
    c->qw_max = std::max(c->qw_max, wmax);
  }
  return 2 * pairs;
}

}  // namespace grpic
