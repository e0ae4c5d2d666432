// particles.hip -- particle initial data, tile sort and small utilities.
//
// Initial data: the seeded draws of sampling_device.hpp (positions uniform
// in proper volume over a shell; FIDO-frame momenta isotropic with
// |u| ~ U[0, p0], or Maxwell-Juettner), or circular/eccentric orbits.
//
// Tile sort: counting sort of the particles by node-cell tile (32 x 16 cells
// by default, tiles in serpentine order), dead particles last; keeps a
// block's particles in a few neighbouring cells for the gather and the
// deposit.
#include <algorithm>

#include "deposit_device.hpp"
#include "sampling_device.hpp"

namespace grpic {

// ------------------------------------------------------------------- fill
__global__ void k_fill(uint32_t* p, long n) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0u;
}

void launch_fill(grpic_ctx* c, void* p, size_t bytes) {
  long n = (long)(bytes / 4);
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, c->stream,
                     (uint32_t*)p, n);
  GRPIC_HIP(hipGetLastError());
}

struct InitArgs {
  ParticleView p;
  grpic_init_spec s;
  double a;
  const double* mj;  // cumulative table, mj_k + 1 entries
  int mj_k;
  double mj_h;
};

__global__ void k_init(InitArgs A) {
  long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= A.s.n) return;
  const grpic_init_spec& s = A.s;
  const double a = A.a;
  double z[6];
  int8_t qm;
  if (s.kind == GRPIC_INIT_ORBITS) {
    double r = s.r0 + (s.r1 - s.r0) * draw(s.seed, id, 0);
    double th = s.t0 + (s.t1 - s.t0) * draw(s.seed, id, 1);
    double E = (1.0 - 2.0 / r) / sqrt(1.0 - 3.0 / r);
    double L = sqrt(r) / sqrt(1.0 - 3.0 / r);
    z[0] = r;
    z[1] = th;
    z[2] = 0.0;
    z[3] = 2.0 * E / (r - 2.0);
    if (id & 1) z[3] += -s.p0 + 2.0 * s.p0 * draw(s.seed, id, 2);
    z[4] = 0.0;
    z[5] = L * sin(th);
    qm = 0;
  } else {
    long pid = (s.kind == GRPIC_INIT_SHELL_MJ) ? id / 2 : id;
    sample_position(a, s.seed, pid, s.r0, s.r1, s.t0, s.t1, z);
    double mag = s.kind == GRPIC_INIT_SHELL_MJ
                     ? mj_speed(A.mj, A.mj_k, A.mj_h, draw(s.seed, id, 200))
                     : s.p0 * draw(s.seed, id, 200);
    fido_momentum(a, s.seed, id, mag, z[0], z[1], z + 3);
    qm = (id & 1) ? -1 : 1;
  }
  ParticleView& P = A.p;
  P.r[id] = z[0];
  P.th[id] = z[1];
  P.ph[id] = z[2];
  P.ur[id] = z[3];
  P.uth[id] = z[4];
  P.uph[id] = z[5];
  P.qm[id] = qm;
  P.w[id] = s.w;
  P.H0[id] = energy(a, z);
  P.herr[id] = 0.0;
  P.flags[id] = GRPIC_FLAG_ALIVE;
  P.iters[id] = 0;
  P.id[id] = (uint32_t)id;
}

void launch_init_particles(grpic_ctx* c, const grpic_init_spec* s,
                           const double* mj_table, int mj_k, double mj_h) {
  InitArgs A;
  A.p = c->pv;
  A.s = *s;
  A.a = c->cfg.a;
  A.mj = mj_table;
  A.mj_k = mj_k;
  A.mj_h = mj_h;
  hipLaunchKernelGGL(k_init, dim3(grid_for(s->n, 256)), dim3(256), 0,
                     c->stream, A);
  GRPIC_HIP(hipGetLastError());
}

// -------------------------------------------------------------- tile sort
struct SortArgs {
  GridView g;
  ParticleView p, q;  // source, destination
  int tile_r, tile_th, ntr, ntiles;
  int* count;
  int* offset;
  const int* cell;  // node cells of the current positions (nullptr: from r, theta)
};

__device__ __forceinline__ int tile_key(const SortArgs& A, long k) {
  if (!(A.p.flags[k] & GRPIC_FLAG_ALIVE)) return A.ntiles;
  int p, q;
  if (A.cell) {
    const unsigned c = (unsigned)A.cell[k];
    q = (int)(c / (unsigned)A.g.nr);
    p = (int)(c - (unsigned)q * (unsigned)A.g.nr);
  } else {
    node_cell(A.g, A.p.r[k], A.p.th[k], p, q);
  }
  // serpentine order: odd tile rows run backwards in r, so consecutive
  // tiles are always neighbours
  int tq = q / A.tile_th, tp = p / A.tile_r;
  return tq * A.ntr + ((tq & 1) ? A.ntr - 1 - tp : tp);
}

constexpr int kSortChunk = 4096;

// per-block histogram of the chunk's tile keys in LDS, one global add per
// non-empty bin
__global__ __launch_bounds__(256) void k_tile_count(SortArgs A) {
  extern __shared__ int hist[];
  const int nb = A.ntiles + 1;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  long beg = (long)blockIdx.x * kSortChunk, end = min(beg + (long)kSortChunk, A.p.n);
  for (long k = beg + threadIdx.x; k < end; k += blockDim.x)
    atomicAdd(&hist[tile_key(A, k)], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (hist[i]) atomicAdd(&A.count[i], hist[i]);
}

// exclusive scan of ntiles + 1 counts in one block
__global__ void k_tile_scan(int* count, int* offset, int n) {
  __shared__ int part[256];
  int t = threadIdx.x;
  int per = (n + 255) / 256;
  int lo = t * per, hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += count[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int i = 0; i < 256; ++i) {
      int v = part[i];
      part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int acc = part[t];
  for (int i = lo; i < hi; ++i) {
    offset[i] = acc;
    acc += count[i];
    count[i] = 0;
  }
}

// scatter: the block reserves one range per non-empty bin with a single
// global add, then ranks its particles inside the range with LDS atomics
__global__ __launch_bounds__(256) void k_tile_scatter(SortArgs A) {
  extern __shared__ int sh[];
  const int nb = A.ntiles + 1;
  int* hist = sh;
  int* base = sh + nb;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  long beg = (long)blockIdx.x * kSortChunk, end = min(beg + (long)kSortChunk, A.p.n);
  for (long k = beg + threadIdx.x; k < end; k += blockDim.x)
    atomicAdd(&hist[tile_key(A, k)], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    base[i] = hist[i] ? atomicAdd(&A.offset[i], hist[i]) : 0;
    hist[i] = 0;
  }
  __syncthreads();
  // four particles per thread at a time, all their loads issued before the
  // stores (one scattered particle at a time kept too few loads in flight)
  const ParticleView &S = A.p, &D = A.q;
  constexpr int U = 4;
  for (long k0 = beg + threadIdx.x; k0 < end; k0 += U * (long)blockDim.x) {
    long kk[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      kk[u] = k0 + u * (long)blockDim.x;
      d[u] = -1;
      if (kk[u] < end) {
        const int key = tile_key(A, kk[u]);
        d[u] = base[key] + atomicAdd(&hist[key], 1);
      }
    }
    double x[U][9];
    uint32_t wq[U][3];
    int8_t qm[U];
    uint8_t fl[U], it[U];
    uint32_t id[U];
    int cl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (d[u] < 0) continue;
      const long k = kk[u];
      x[u][0] = S.r[k];
      x[u][1] = S.th[k];
      x[u][2] = S.ph[k];
      x[u][3] = S.ur[k];
      x[u][4] = S.uth[k];
      x[u][5] = S.uph[k];
      x[u][6] = S.H0[k];
      x[u][7] = S.herr[k];
      x[u][8] = S.w[k];
      wq[u][0] = S.W[1][k];
      wq[u][1] = S.W[2][k];
      wq[u][2] = S.W[3][k];
      qm[u] = S.qm[k];
      fl[u] = S.flags[k];
      it[u] = S.iters[k];
      id[u] = S.id[k];
      cl[u] = S.cell[k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (d[u] < 0) continue;
      const long t = d[u];
      D.r[t] = x[u][0];
      D.th[t] = x[u][1];
      D.ph[t] = x[u][2];
      D.ur[t] = x[u][3];
      D.uth[t] = x[u][4];
      D.uph[t] = x[u][5];
      D.H0[t] = x[u][6];
      D.herr[t] = x[u][7];
      D.w[t] = x[u][8];
      D.W[1][t] = wq[u][0];
      D.W[2][t] = wq[u][1];
      D.W[3][t] = wq[u][2];
      D.qm[t] = qm[u];
      D.flags[t] = fl[u];
      D.iters[t] = it[u];
      D.id[t] = id[u];
      D.cell[t] = cl[u];
    }
  }
}

// ------------------------------------------------------------ sampling
// records of the particles whose id has a slot in the map (map[id] = slot
// of the sample, -1 otherwise); out holds 10 doubles per slot (r, theta,
// phi, u_r, u_theta, u_phi, q/m, w, H0, herr) and fl 2 ints (flags, iters)
__global__ __launch_bounds__(256) void k_sample(ParticleView P, const int* map, double* out,
                                                int* fl) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  int s = map[P.id[k]];
  if (s < 0) return;
  double* o = out + (long)s * 10;
  o[0] = P.r[k];
  o[1] = P.th[k];
  o[2] = P.ph[k];
  o[3] = P.ur[k];
  o[4] = P.uth[k];
  o[5] = P.uph[k];
  o[6] = (double)P.qm[k];
  o[7] = P.w[k];
  o[8] = P.H0[k];
  o[9] = P.herr[k];
  fl[2 * s] = P.flags[k];
  fl[2 * s + 1] = P.iters[k];
}

void launch_sample(grpic_ctx* c, const int* map, double* out, int* fl) {
  ParticleView P = c->pv;
  P.n = c->n;
  hipLaunchKernelGGL(k_sample, dim3(grid_for(c->n, 256)), dim3(256), 0, c->stream, P, map, out,
                     fl);
  GRPIC_HIP(hipGetLastError());
}

// ---------------------------------------------------- deposit chunk plan
// After a sort the deposit takes its particles by runs of consecutive tiles:
// groups of tiles covering about kPlanCells cells (their node box, plus the
// drift until the next sort, fits the deposit's LDS bins), each group cut
// every kDepChunk particles.  Near the inner boundary, where the
// log-spaced cells are small and hold few particles, a chunk of kDepChunk
// particles in sort order would span hundreds of tiles and miss the LDS
// bins; there the groups become small chunks of their own.
constexpr int kPlanCells = 1024;

int plan_group_tiles(const grpic_ctx* c) {
  return std::max(1, kPlanCells / (c->cfg.tile_r * c->cfg.tile_th));
}

// chunks of each group (tile_end: end offsets of the tiles after the
// scatter); nch[ngroups] = 0 closes the scan
__global__ __launch_bounds__(256) void k_plan_count(const int* tile_end, int ntiles, int K,
                                                    int ngroups, int* nch) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g > ngroups) return;
  if (g == ngroups) {
    nch[g] = 0;
    return;
  }
  const int t0 = g * K, t1 = min(t0 + K, ntiles);
  const int s = t0 == 0 ? 0 : tile_end[t0 - 1], e = tile_end[t1 - 1];
  nch[g] = (e - s + kDepChunk - 1) / kDepChunk;
}

// The node box of a group: its tiles' cells (serpentine order keeps them
// together), widened on every side by the largest margin of at most
// kPlanMargin cells for which the box still fits the deposit's LDS bins,
// so that particles which drift until the next sort mostly stay inside.
// {p0, q0, bw, bh} in nodes; bw = 0 when even the bare tiles do not fit.
constexpr int kPlanMargin = 8;

struct PlanGeom {
  int tile_r, tile_th, ntr, nr, nth;
};

__device__ int4 group_box(const PlanGeom& G, int t0, int t1) {
  int p0 = 1 << 30, p1 = -1, q0 = 1 << 30, q1 = -1;
  for (int t = t0; t < t1; ++t) {
    const int tq = t / G.ntr, tc = t - tq * G.ntr;
    const int tp = (tq & 1) ? G.ntr - 1 - tc : tc;
    p0 = min(p0, tp * G.tile_r);
    p1 = max(p1, min((tp + 1) * G.tile_r, G.nr) - 1);
    q0 = min(q0, tq * G.tile_th);
    q1 = max(q1, min((tq + 1) * G.tile_th, G.nth) - 1);
  }
  for (int m = kPlanMargin; m >= 0; --m) {
    const int a0 = max(p0 - m, 0), a1 = min(p1 + m, G.nr - 1);
    const int b0 = max(q0 - m, 0), b1 = min(q1 + m, G.nth - 1);
    const int bw = a1 - a0 + 2, bh = b1 - b0 + 2;  // nodes of cells a0..a1, b0..b1
    if (bw * bh <= kDepBins) return make_int4(a0, b0, bw, bh);
  }
  return make_int4(0, 0, 0, 0);
}

// chunk starts from the groups' chunk offsets; start[total] = end of the
// particles alive at the sort; meta = {total, n, 1}; box: each chunk's
// group box
__global__ __launch_bounds__(256) void k_plan_write(const int* tile_end, int ntiles, int K,
                                                    int ngroups, const int* off, int n,
                                                    int* start, int* meta, PlanGeom G,
                                                    int4* box) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g > ngroups) return;
  if (g == ngroups) {
    const int total = off[ngroups];
    start[total] = tile_end[ntiles - 1];
    meta[0] = total;
    meta[1] = n;
    meta[2] = 1;
    return;
  }
  const int t0 = g * K;
  const int s = t0 == 0 ? 0 : tile_end[t0 - 1];
  const int4 b = group_box(G, t0, min(t0 + K, ntiles));
  for (int i = off[g]; i < off[g + 1]; ++i) {
    start[i] = s + (i - off[g]) * kDepChunk;
    box[i] = b;
  }
}

void plan_deposit_chunks(grpic_ctx* c) {
  const int K = plan_group_tiles(c);
  const int ngroups = (c->ntiles + K - 1) / K;
  const long need = ngroups + (c->cap + kDepChunk - 1) / kDepChunk + 2;
  if (need > c->dep_plan_cap || !c->dep_plan_meta) {
    dfree(c->dep_plan);
    dfree(c->dep_plan_off);
    dfree(c->dep_plan_box);
    if (!c->dep_plan_meta) c->dep_plan_meta = dalloc<int>(3);
    c->dep_plan_cap = 0;
    c->dep_plan = dalloc<int>(need);
    c->dep_plan_off = dalloc<int>(need);
    c->dep_plan_box = dalloc<int4>(need);
    c->dep_plan_cap = need;
  }
  c->plan_groups = ngroups;
  // tile_count is all zero between sorts; it holds the per-group counts
  // here and the scan leaves it zero again
  const unsigned gb = (unsigned)((ngroups + 1 + 255) / 256);
  hipLaunchKernelGGL(k_plan_count, dim3(gb), dim3(256), 0, c->stream, c->tile_offset,
                     c->ntiles, K, ngroups, c->tile_count);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(256), 0, c->stream, c->tile_count,
                     c->dep_plan_off, ngroups + 1);
  PlanGeom G{c->cfg.tile_r, c->cfg.tile_th, (c->nr + c->cfg.tile_r - 1) / c->cfg.tile_r,
             c->nr, c->nth};
  hipLaunchKernelGGL(k_plan_write, dim3(gb), dim3(256), 0, c->stream, c->tile_offset,
                     c->ntiles, K, ngroups, c->dep_plan_off, (int)c->n, c->dep_plan,
                     c->dep_plan_meta, G, c->dep_plan_box);
  GRPIC_HIP(hipGetLastError());
}

long deposit_blocks(const grpic_ctx* c) {
  // plan chunks <= groups + ceil(n_sort / kDepChunk); appended particles
  // need ceil((n - n_sort) / kDepChunk) more
  return (long)c->plan_groups + (c->n + kDepChunk - 1) / kDepChunk + 1;
}

void invalidate_deposit_plan(grpic_ctx* c) {
  if (c->dep_plan_meta) launch_fill(c, c->dep_plan_meta, 3 * sizeof(int));
}

void launch_sort(grpic_ctx* c, bool from_cells) {
  if (c->n == 0 || c->nr == 0) return;
  hipEvent_t ev;
  time_begin(c, GRPIC_K_SORT, &ev);
  SortArgs A;
  A.g = make_grid_view(c);
  A.p = c->pv;
  A.p.n = c->n;
  A.q = c->alt;
  A.tile_r = c->cfg.tile_r;
  A.tile_th = c->cfg.tile_th;
  A.ntr = (c->nr + A.tile_r - 1) / A.tile_r;
  A.ntiles = c->ntiles;
  A.count = c->tile_count;
  A.offset = c->tile_offset;
  A.cell = from_cells ? c->pv.cell : nullptr;
  dim3 g(grid_for(c->n, kSortChunk)), b(256);
  size_t sh = sizeof(int) * (c->ntiles + 1);
  hipLaunchKernelGGL(k_tile_count, g, b, sh, c->stream, A);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(256), 0, c->stream,
                     c->tile_count, c->tile_offset, c->ntiles + 1);
  hipLaunchKernelGGL(k_tile_scatter, g, b, 2 * sh, c->stream, A);
  GRPIC_HIP(hipGetLastError());
  plan_deposit_chunks(c);
  ParticleView& P = c->pv;
  ParticleView& Q = c->alt;
  c->sort_flip ^= 1;
  std::swap(P.r, Q.r);
  std::swap(P.th, Q.th);
  std::swap(P.ph, Q.ph);
  std::swap(P.ur, Q.ur);
  std::swap(P.uth, Q.uth);
  std::swap(P.uph, Q.uph);
  std::swap(P.H0, Q.H0);
  std::swap(P.herr, Q.herr);
  std::swap(P.w, Q.w);
  std::swap(P.qm, Q.qm);
  std::swap(P.flags, Q.flags);
  std::swap(P.iters, Q.iters);
  std::swap(P.id, Q.id);
  for (int q = 1; q < 4; ++q) std::swap(P.W[q], Q.W[q]);
  std::swap(P.cell, Q.cell);
  time_end(c, GRPIC_K_SORT, ev);
}

}  // namespace grpic
