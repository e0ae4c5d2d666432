// deposit.hip -- charge and current deposit (sub-step 6 of Sec. 2.1).
//
// Weights are the paper's volume fractions (Sec. 2.3); the current is the
// charge-conserving one: the straight move in (r, theta) is cut at node-cell
// boundaries, the weight change inside a cell becomes four face fluxes
//   S_r = W10 + W11, S_t = W01 + W11, Fr1 = dS_r (S_t + S_t')/2,
//   Fr0 = dS_r - Fr1, Ft1 = dW11 - Fr1, Ft0 = dS_t - Ft1,
// and the jump of the (cell-dependent) weights at a crossing point moves
// along the shared edge.  Sums are accumulated in 64-bit fixed point with
// integer atomics, so the result does not depend on the order in which
// particles are processed.  A finalize pass turns the sums into densitized
// FP32 sqrt(g) rho, sqrt(g) J^r, sqrt(g) J^theta, sqrt(g) J^phi and clears
// the accumulators.
#include <algorithm>

#include "deposit_device.hpp"

namespace grpic {

struct DepArgs {
  GridView g;
  ParticleView p;
  DepositAcc acc;
  int nr, nth;
  double inv_nr;       // 1 / nr, to split a cell index without an integer division
  unsigned* fallback;  // blocks that used global atomics (diagnostic)
  unsigned long long* outside;  // particles outside their planned box (diagnostic)
  int* xqueue;         // particles whose move crosses a node-cell boundary
  unsigned* xcount;
  const int* plan;       // chunk starts of the last sort (see chunk_range)
  const int* plan_meta;  // {chunks, particles at the sort, valid}; null: no plan
  const int4* plan_box;  // node box {p0, q0, bw, bh} of each planned chunk
};

// Particle range [beg, end) of deposit chunk b (false: past the last
// chunk; a chunk may be empty).  With a valid plan the first chunks are its
// runs of tiles whose node box fits the LDS bins (the dead particles the
// sort put last need no deposit) and the rest are the particles appended
// since, kDepChunk at a time; without one, equal chunks of the whole array.
// Blocks stride over the chunks, so any grid size covers them all.  box:
// the planned node box of the chunk (bw = 0: none, the chunk's own box is
// measured).
__device__ __forceinline__ bool chunk_range(const DepArgs& A, long b, long& beg, long& end,
                                            int4& box) {
  long first = 0;
  box = make_int4(0, 0, 0, 0);
  if (A.plan_meta && A.plan_meta[2]) {
    const long total = A.plan_meta[0];
    if (b < total) {
      beg = A.plan[b];
      end = min((long)A.plan[b + 1], A.p.n);
      box = A.plan_box[b];
      return true;
    }
    b -= total;
    first = A.plan_meta[1];
  }
  beg = first + b * kDepChunk;
  end = min(beg + (long)kDepChunk, A.p.n);
  return beg < A.p.n;
}

// node cell c = q nr + p -> (p, q); (c + 1/2) / nr in FP64 is exact enough to
// floor correctly for any grid that fits in memory
__device__ __forceinline__ void split_cell(const DepArgs& A, int c, int& p, int& q) {
  q = (int)(((double)c + 0.5) * A.inv_nr);
  p = c - q * A.nr;
}

// Where contributions go: the global accumulators, or a block's LDS bins
// covering node columns [p0, p0 + bw) and rows [q0, q0 + bh).  The four
// arrays use the node indexing of their own sub-grid (Fr: r-half column i
// for i + 1/2, Ft: theta-half row j for j + 1/2).
struct GlobalSink {
  const DepositAcc* acc;
  int nr;
  __device__ __forceinline__ long long* slot(int a, int i, int j) const {
    switch (a) {
      case 0: return acc->Q + (long)j * (nr + 1) + i;
      case 1: return acc->P + (long)j * (nr + 1) + i;
      case 2: return acc->Fr + (long)j * nr + i;
      default: return acc->Ft + (long)j * (nr + 1) + i;
    }
  }
};

struct LdsSink {
  long long* bins;  // 4 arrays of bw * bh
  int p0, q0, bw, bh, n;  // n = bw * bh
  __device__ __forceinline__ long long* slot(int a, int i, int j) const {
    return bins + a * n + (j - q0) * bw + (i - p0);
  }
};

template <class Sink>
__device__ __forceinline__ void sink_add(const Sink& S, int a, int i, int j,
                                         double v, double scale) {
  long long q = llrint(v * scale);
  if (q != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(S.slot(a, i, j)),
              static_cast<unsigned long long>(q));
}

// face fluxes (in charge units) of a weight change inside node cell (p, q)
template <class Sink>
__device__ __forceinline__ void cell_flux(const Sink& S, double s, int p, int q,
                                          const double* W0, const double* W1,
                                          double qw) {
  double dSr = (W1[1] + W1[3]) - (W0[1] + W0[3]);
  double St0 = W0[2] + W0[3], St1 = W1[2] + W1[3];
  double dSt = St1 - St0, dW11 = W1[3] - W0[3];
  double Fr1 = 0.5 * dSr * (St0 + St1);
  double Fr0 = dSr - Fr1;
  double Ft1 = dW11 - Fr1;
  double Ft0 = dSt - Ft1;
  sink_add(S, 2, p, q, qw * Fr0, s);
  sink_add(S, 2, p, q + 1, qw * Fr1, s);
  sink_add(S, 3, p, q, qw * Ft0, s);
  sink_add(S, 3, p + 1, q, qw * Ft1, s);
}

// what the deposit reads of one particle: raw loads only, so that nothing
// waits for them until the record is used (the loads of the next records
// stay in flight meanwhile)
struct PRec {
  double w;
  float dphi;
  uint32_t W1, W2, W3, N1, N2, N3;  // fixed-point weights (wq_decode)
  int c0, c1;
  uint8_t fl;
  int8_t qm;
};

// k must be a valid particle index (callers clamp it)
__device__ __forceinline__ void load_rec(const ParticleView& P, long k, PRec& d) {
  d.fl = P.flags[k];
  d.qm = P.qm[k];
  d.w = P.w[k];
  d.c0 = P.cell[k];
  d.c1 = P.celln[k];
  d.W1 = P.W[1][k];
  d.W2 = P.W[2][k];
  d.W3 = P.W[3][k];
  d.N1 = P.Wn[1][k];
  d.N2 = P.Wn[2][k];
  d.N3 = P.Wn[3][k];
  d.dphi = P.dphi[k];
}

// the deposit's view of a record
struct PDep {
  double Wo[4], Wn[4], dphi, qw;
  int c0, c1;
  bool act;
};

__device__ __forceinline__ void unpack_rec(const PRec& r, PDep& d) {
  d.Wo[1] = wq_decode(r.W1);
  d.Wo[2] = wq_decode(r.W2);
  d.Wo[3] = wq_decode(r.W3);
  d.Wn[1] = wq_decode(r.N1);
  d.Wn[2] = wq_decode(r.N2);
  d.Wn[3] = wq_decode(r.N3);
  d.Wo[0] = 1.0 - d.Wo[1] - d.Wo[2] - d.Wo[3];
  d.Wn[0] = 1.0 - d.Wn[1] - d.Wn[2] - d.Wn[3];
  d.dphi = (double)r.dphi;
  d.c0 = r.c0;
  d.c1 = r.c1;
  d.qw = (double)r.qm * r.w;
  d.act = (r.fl & GRPIC_FLAG_ALIVE) && d.qw != 0.0;
}

// charge and J^phi of a particle, and its face fluxes when the move stays in
// one node cell (returns false for a crossing move: fluxes left to
// deposit_crossing)
template <class Sink>
__device__ bool deposit_particle(const DepArgs& A, const Sink& S, const PDep& d) {
  const double s = A.acc.scale;
  const double qw = d.qw;
  int p0, q0, p1, q1;
  split_cell(A, d.c0, p0, q0);
  split_cell(A, d.c1, p1, q1);
  const double hdphi = 0.5 * qw * d.dphi;
  const bool same = d.c0 == d.c1;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int di = c & 1, dj = c >> 1;
    sink_add(S, 0, p1 + di, q1 + dj, qw * d.Wn[c], s);
    if (same) {  // old and new J^phi shares land on the same nodes
      sink_add(S, 1, p1 + di, q1 + dj, hdphi * (d.Wo[c] + d.Wn[c]), s);
    } else {
      sink_add(S, 1, p0 + di, q0 + dj, hdphi * d.Wo[c], s);
      sink_add(S, 1, p1 + di, q1 + dj, hdphi * d.Wn[c], s);
    }
  }
  if (same) {
    cell_flux(S, s, p0, q0, d.Wo, d.Wn, qw);
    return true;
  }
  return false;
}

// what the walk of a crossing move reads of its particle
struct XRec {
  double Wo[4], Wn[4], r0, t0, r1, t1, qw;
  int p0, q0, p1, q1;
};

// k must be a valid particle index (callers clamp it)
__device__ __forceinline__ void load_xrec(const DepArgs& A, long k, XRec& x) {
  const ParticleView& P = A.p;
#pragma unroll
  for (int c = 1; c < 4; ++c) {
    x.Wo[c] = wq_decode(P.W[c][k]);
    x.Wn[c] = wq_decode(P.Wn[c][k]);
  }
  x.r0 = P.r_old[k];
  x.t0 = P.th_old[k];
  x.r1 = P.r[k];
  x.t1 = P.th[k];
  x.qw = (double)P.qm[k] * P.w[k];
  split_cell(A, P.cell[k], x.p0, x.q0);
  split_cell(A, P.celln[k], x.p1, x.q1);
}

// face fluxes of a move that crosses node-cell boundaries: the straight move
// is walked cell by cell.  Each step loads the node values it may need in
// one burst (radii of the cell and of both radial neighbours, sin and cos
// of the cell's lower angle and of the angular neighbour toward the end
// cell) and evaluates sin, cos of the crossing point once for both cells.
template <class Sink>
__device__ void deposit_crossing(const DepArgs& A, const Sink& S, const XRec& x) {
  const GridView& g = A.g;
  double Wo[4], Wn[4];
#pragma unroll
  for (int c = 1; c < 4; ++c) {
    Wo[c] = x.Wo[c];
    Wn[c] = x.Wn[c];
  }
  Wo[0] = 1.0 - Wo[1] - Wo[2] - Wo[3];
  Wn[0] = 1.0 - Wn[1] - Wn[2] - Wn[3];
  const double s = A.acc.scale, qw = x.qw;
  const double r0 = x.r0, t0 = x.t0, r1 = x.r1, t1 = x.t1;
  const int p1 = x.p1, q1 = x.q1;
  int cp = x.p0, cq = x.q0;
  double Wa[4] = {Wo[0], Wo[1], Wo[2], Wo[3]};
  for (int guard = 0; guard < 16 && (cp != p1 || cq != q1); ++guard) {
    int br = -1, bt = -1;
    if (p1 > cp) br = cp + 1;
    else if (p1 < cp) br = cp;
    if (q1 > cq) bt = cq + 1;
    else if (q1 < cq) bt = cq;
    const int qo = q1 > cq ? cq + 1 : (cq > 0 ? cq - 1 : 0);
    const double rm = g.rn[cp > 0 ? cp - 1 : 0], ra = g.rn[cp], rb = g.rn[cp + 1],
                 rc = g.rn[cp + 2 <= A.nr ? cp + 2 : A.nr];
    const double sq = g.stn[cq], cqs = g.ctn[cq], so = g.stn[qo], co = g.ctn[qo];
    const double tb = g.tn[bt >= 0 ? bt : cq];
    const double tr = br >= 0 ? ((br > cp ? rb : ra) - r0) / (r1 - r0) : 2.0;
    const double tt = bt >= 0 ? (tb - t0) / (t1 - t0) : 2.0;
    double Wb[4], Wc[4];
    if (tr <= tt) {
      const double xr = br > cp ? rb : ra, xt = t0 + tr * (t1 - t0);
      double st, ct;
      fsincos(xt, &st, &ct);
      dep_weights_at(g, xr, xt, st, ct, ra, rb, sq, cqs, cq, Wb);
      cell_flux(S, s, cp, cq, Wa, Wb, qw);
      const int np = (br > cp) ? cp + 1 : cp - 1;
      dep_weights_at(g, xr, xt, st, ct, np > cp ? rb : rm, np > cp ? rc : ra, sq, cqs, cq, Wc);
      // node (br, cq+1): slot 3 of the old cell if br = cp+1 else slot 2;
      // in the new cell slot 2 if br = np else slot 3
      double prev = (br == cp + 1) ? Wb[3] : Wb[2];
      double now = (br == np) ? Wc[2] : Wc[3];
      sink_add(S, 3, br, cq, qw * (now - prev), s);
      cp = np;
    } else {
      const double xr = r0 + tt * (r1 - r0), xt = tb;
      double st, ct;
      fsincos(xt, &st, &ct);
      dep_weights_at(g, xr, xt, st, ct, ra, rb, sq, cqs, cq, Wb);
      cell_flux(S, s, cp, cq, Wa, Wb, qw);
      const int nq = (bt > cq) ? cq + 1 : cq - 1;  // = qo
      dep_weights_at(g, xr, xt, st, ct, ra, rb, so, co, nq, Wc);
      // node (cp+1, bt): slot 3 of the old cell if bt = cq+1 else slot 1
      double prev = (bt == cq + 1) ? Wb[3] : Wb[1];
      double now = (bt == nq) ? Wc[1] : Wc[3];
      sink_add(S, 2, cp, bt, qw * (now - prev), s);
      cq = nq;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) Wa[c] = Wc[c];
  }
  cell_flux(S, s, cp, cq, Wa, Wn, qw);
}

constexpr int kDepBlock = 512;
constexpr int kDepSub = 2048;     // segment length when the chunk box is too big

// Bounding box (node-cell columns box[0..1], rows box[2..3]) of the old and
// new cells of the charged particles in [beg, end); block-uniform result.
__device__ __forceinline__ void segment_box(const DepArgs& A, long beg, long end,
                                            int* box) {
  const ParticleView& P = A.p;
  __syncthreads();  // previous users of box / bins are done
  if (threadIdx.x == 0) {
    box[0] = 1 << 30;
    box[1] = -1;
    box[2] = 1 << 30;
    box[3] = -1;
  }
  __syncthreads();
  int pmin = 1 << 30, pmax = -1, qmin = 1 << 30, qmax = -1;
  // four particles per round, loads at clamped indices issued together and
  // used through selects (no branch for the compiler to sink them into)
  const long last = end - 1;
  for (long k0 = beg + threadIdx.x; k0 < end; k0 += 4 * kDepBlock) {
    uint8_t fl[4];
    int8_t qm[4];
    int c0[4], c1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long k = min(k0 + u * kDepBlock, last);
      fl[u] = P.flags[k];
      qm[u] = P.qm[k];
      c0[u] = P.cell[k];
      c1[u] = P.celln[k];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = k0 + u * kDepBlock < end && (fl[u] & GRPIC_FLAG_ALIVE) && qm[u] != 0;
      int p0, q0, p1, q1;
      split_cell(A, c0[u], p0, q0);
      split_cell(A, c1[u], p1, q1);
      pmin = ok ? min(pmin, min(p0, p1)) : pmin;
      pmax = ok ? max(pmax, max(p0, p1)) : pmax;
      qmin = ok ? min(qmin, min(q0, q1)) : qmin;
      qmax = ok ? max(qmax, max(q0, q1)) : qmax;
    }
  }
  if (pmax >= 0) {
    atomicMin(&box[0], pmin);
    atomicMax(&box[1], pmax);
    atomicMin(&box[2], qmin);
    atomicMax(&box[3], qmax);
  }
  __syncthreads();
}

// Crossing moves are collected per wave in LDS (kXList entries) and
// appended to the global crossing queue with one atomic per flush.
constexpr int kXList = 256;

struct WaveList {
  int* e;  // this wave's LDS list
  int n;   // entries held (uniform across the wave)
};

__device__ __forceinline__ void flush_list(const DepArgs& A, WaveList& X) {
  if (X.n == 0) return;
  const int lane = threadIdx.x & 63;
  __threadfence_block();  // the wave's LDS appends are visible to all lanes
  unsigned base = 0;
  if (lane == 0) base = atomicAdd(A.xcount, (unsigned)X.n);
  base = __shfl(base, 0, 64);
  for (int i = lane; i < X.n; i += 64) A.xqueue[base + i] = X.e[i];
  __threadfence_block();  // reads done before the list is refilled
  X.n = 0;
}

// the planned box holds both node cells of the move (the four nodes of each)
__device__ __forceinline__ bool in_box(const DepArgs& A, const LdsSink& L, int c0, int c1) {
  int p0, q0, p1, q1;
  split_cell(A, c0, p0, q0);
  split_cell(A, c1, p1, q1);
  const int pl = L.p0, ph = L.p0 + L.bw - 2, ql = L.q0, qh = L.q0 + L.bh - 2;
  return min(p0, p1) >= pl && max(p0, p1) <= ph && min(q0, q1) >= ql && max(q0, q1) <= qh;
}

// CHECKED (an LDS sink over a planned box): a particle whose cells left
// the box since the sort goes to the global accumulators instead
template <bool CHECKED = false, class Sink>
__device__ __forceinline__ void deposit_one(const DepArgs& A, const Sink& S, WaveList& X,
                                            const PRec& r, long k, long end) {
  const int lane = threadIdx.x & 63;
  bool cross = false;
  if (k < end) {
    PDep d;
    unpack_rec(r, d);
    if (d.act) {
      if constexpr (CHECKED) {
        const bool inside = in_box(A, S, d.c0, d.c1);
        if (inside) cross = !deposit_particle(A, S, d);
        else cross = !deposit_particle(A, GlobalSink{&A.acc, A.nr}, d);
        const unsigned long long o = __ballot(!inside);
        if (o && lane == (int)__ffsll((long long)o) - 1)
          atomicAdd(A.outside, (unsigned long long)__popcll(o));
      } else {
        cross = !deposit_particle(A, S, d);
      }
    }
  }
  unsigned long long m = __ballot(cross);
  if (m) {
    if (X.n + 64 > kXList) flush_list(A, X);
    if (cross) X.e[X.n + __popcll(m & ((1ull << lane) - 1ull))] = (int)k;
    X.n += __popcll(m);
  }
}

// Three records rotate (no register copies, which would wait for their
// loads): while one is accumulated the next two are in flight.  Loads use
// clamped indices; slots past the end are skipped.
template <bool CHECKED = false, class Sink>
__device__ __forceinline__ void deposit_range(const DepArgs& A, long beg, long end,
                                              const Sink& S, WaveList& X) {
  const ParticleView& P = A.p;
  const long last = end - 1, t = threadIdx.x, B = kDepBlock;
  PRec a, b, c;
  load_rec(P, min(beg + t, last), a);
  load_rec(P, min(beg + B + t, last), b);
  for (long kb = beg; kb < end; kb += 3 * B) {  // uniform trip count
    load_rec(P, min(kb + 2 * B + t, last), c);
    deposit_one<CHECKED>(A, S, X, a, kb + t, end);
    load_rec(P, min(kb + 3 * B + t, last), a);
    deposit_one<CHECKED>(A, S, X, b, kb + B + t, end);
    load_rec(P, min(kb + 4 * B + t, last), b);
    deposit_one<CHECKED>(A, S, X, c, kb + 2 * B + t, end);
  }
}

// face fluxes of the queued crossing moves (grid-stride over the queue,
// global atomics).  Loading the next move's record while one is walked was
// measured slower (223 VGPRs, two waves per SIMD).
__global__ __launch_bounds__(256) void k_deposit_crossing(DepArgs A) {
  GlobalSink Gs{&A.acc, A.nr};
  const unsigned nq = *A.xcount;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < nq;
       i += gridDim.x * blockDim.x) {
    XRec x;
    load_xrec(A, A.xqueue[i], x);
    deposit_crossing(A, Gs, x);
  }
}

__global__ void k_reset_xcount(unsigned* x) { *x = 0u; }

// the block's LDS bins into the global accumulators (nonzero bins only)
__device__ __forceinline__ void flush_bins(const DepArgs& A, const LdsSink& L) {
  GlobalSink Gs{&A.acc, A.nr};
  for (int i = threadIdx.x; i < 4 * L.n; i += kDepBlock) {
    long long v = L.bins[i];
    if (v == 0) continue;
    int a = i / L.n, r = i - a * L.n;
    int jj = r / L.bw, ii = r - jj * L.bw;
    // r-flux lives on cells (i < nr), theta-flux on rows j < nth
    if ((a == 2 && L.p0 + ii >= A.nr) || (a == 3 && L.q0 + jj >= A.nth)) continue;
    atomicAdd(reinterpret_cast<unsigned long long*>(Gs.slot(a, L.p0 + ii, L.q0 + jj)),
              static_cast<unsigned long long>(v));
  }
}

// Per chunk of (tile-sorted) particles (chunk_range), summed in LDS bins
// over a node box and flushed once.  A chunk of the sort's plan comes with
// its group's box: one pass, and the few particles that have drifted out
// of it since the sort go to the global accumulators.  Other chunks
// (particles appended since the sort, no plan) first measure the box of
// their old and new cells; a chunk whose box does not fit is redone in
// segments of kDepSub particles with their own boxes, and a segment that
// still does not fit uses global atomics.
__global__ __launch_bounds__(kDepBlock) void k_deposit(DepArgs A) {
  __shared__ long long bins[4 * kDepBins];
  __shared__ int box[4];
  __shared__ int xlist[(kDepBlock / 64) * kXList];
  WaveList X{xlist + (threadIdx.x >> 6) * kXList, 0};
  for (long b = blockIdx.x;; b += gridDim.x) {  // uniform over the block
    long beg, end;
    int4 pb;
    if (!chunk_range(A, b, beg, end, pb)) break;
    if (pb.z > 0) {
      if (beg >= end) continue;
      LdsSink L{bins, pb.x, pb.y, pb.z, pb.w, pb.z * pb.w};
      __syncthreads();  // the previous chunk's flush is done with the bins
      for (int i = threadIdx.x; i < 4 * L.n; i += kDepBlock) bins[i] = 0;
      __syncthreads();
      deposit_range<true>(A, beg, end, L, X);
      __syncthreads();
      flush_bins(A, L);
      continue;
    }
    for (int pass = 0; pass < 2; ++pass) {
      const long seg = pass == 0 ? kDepChunk : kDepSub;
      bool redo = false;
      for (long sb = beg; sb < end; sb += seg) {
        const long se = min(sb + seg, end);
        segment_box(A, sb, se, box);
        if (box[1] < 0) continue;  // nothing charged in this segment
        const int bp0 = box[0], bq0 = box[2];
        const int bw = box[1] - bp0 + 2, bh = box[3] - bq0 + 2;
        const bool fits = bw * bh <= kDepBins;
        if (!fits && pass == 0) {
          redo = true;
          break;
        }
        if (!fits) {
          if (threadIdx.x == 0) atomicAdd(A.fallback, 1u);
          deposit_range(A, sb, se, GlobalSink{&A.acc, A.nr}, X);
          continue;
        }
        LdsSink L{bins, bp0, bq0, bw, bh, bw * bh};
        for (int i = threadIdx.x; i < 4 * L.n; i += kDepBlock) bins[i] = 0;
        __syncthreads();
        deposit_range(A, sb, se, L, X);
        __syncthreads();
        flush_bins(A, L);
      }
      if (!redo) break;
    }
  }
  flush_list(A, X);
}

// charge of the current positions only (initial rho)
__global__ __launch_bounds__(256) void k_deposit_rho(DepArgs A) {
  const ParticleView& P = A.p;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  if (!(P.flags[k] & GRPIC_FLAG_ALIVE)) return;
  double qw = (double)P.qm[k] * P.w[k];
  int c0 = P.cell[k];
  int p0, q0;
  split_cell(A, c0, p0, q0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    long nn = (long)(q0 + (c >> 1)) * (A.nr + 1) + p0 + (c & 1);
    const double w1 = wq_decode(P.W[1][k]), w2 = wq_decode(P.W[2][k]),
                 w3 = wq_decode(P.W[3][k]);
    const double wc = c == 0 ? 1.0 - w1 - w2 - w3 : (c == 1 ? w1 : (c == 2 ? w2 : w3));
    long long q = llrint(qw * wc * A.acc.scale);
    if (q != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(A.acc.Q + nn),
                static_cast<unsigned long long>(q));
  }
}

// ---------------------------------------------------- the paper's current
// Sec. 2.3 as a deposit mode of its own: every particle alive after the push
// deposits at its state (x, u): rho and J^phi with the node weights (W1..W3
// and the node cell given), J^r on (r_{i+1/2}, th_j) and J^theta on
// (r_i, th_{j+1/2}) with the volume weights of that subgrid's cell, each
// carried by the coordinate velocity dx^i/dt = alpha g^ij u_j / Gamma -
// beta^i (the grid current alpha j - rho beta of eq. m3).  A position off a
// half subgrid is moved onto its edge for that component.  The integers
// accumulated are the finalize kernel's units: charge for rho, charge times
// dt (and over the subgrid spacing for J^r, J^theta) for the currents.
template <class Sink>
__device__ void paper_particle(const DepArgs& A, const Sink& S, long k, const uint32_t* W1,
                               const uint32_t* W2, const uint32_t* W3, const int* cell,
                               double dt) {
  const ParticleView& P = A.p;
  const GridView& g = A.g;
  const double qw = (double)P.qm[k] * P.w[k], s = A.acc.scale;
  const double r = P.r[k], th = P.th[k];
  const double ur = P.ur[k], ut = P.uth[k], up = P.uph[k];
  Met m;
  metric(g.a, r, th, m);
  const double Gam = fsqrt(1.0 + m.irr * ur * ur + m.itt * ut * ut + m.ipp * up * up +
                           2.0 * m.irp * ur * up);
  const double aG = m.alpha / Gam;
  const double vr = aG * (m.irr * ur + m.irp * up) - m.betar;
  const double vt = aG * m.itt * ut;
  const double vp = aG * (m.irp * ur + m.ipp * up);
  int p, q;
  split_cell(A, cell[k], p, q);
  // rho and J^phi on the nodes
  {
    const double w1 = wq_decode(W1[k]), w2 = wq_decode(W2[k]), w3 = wq_decode(W3[k]);
    const double W[4] = {1.0 - w1 - w2 - w3, w1, w2, w3};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = p + (c & 1), j = q + (c >> 1);
      sink_add(S, 0, i, j, qw * W[c], s);
      sink_add(S, 1, i, j, qw * W[c] * vp * dt, s);
    }
  }
  double st, ct;
  fsincos(th, &st, &ct);
  // J^r on (r_{i+1/2}, th_j): the half-radius cell of r, row q
  {
    const double rc = fmin(fmax(r, g.rh[0]), g.rh[A.nr - 1]);
    int pr = rc >= g.rh[p] ? p : p - 1;
    pr = pr < 0 ? 0 : (pr > A.nr - 2 ? A.nr - 2 : pr);
    double W[4];
    dep_weights_box(g, rc, th, st, ct, g.rh[pr], g.rh[pr + 1], theta_node(g, q),
                    theta_node(g, q + 1), g.stn[q], g.ctn[q], W);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = pr + (c & 1), j = q + (c >> 1);
      sink_add(S, 2, i, j, qw * W[c] * vr * dt * g.idrn[i], s);
    }
  }
  // J^theta on (r_i, th_{j+1/2}): the half-angle cell of th, column p
  {
    const double tc = fmin(fmax(th, g.th[0]), g.th[A.nth - 1]);
    int qt = tc >= g.th[q] ? q : q - 1;
    qt = qt < 0 ? 0 : (qt > A.nth - 2 ? A.nth - 2 : qt);
    double sc = st, cc = ct;  // tc is th unless th lies outside the half angles
    if (tc != th) fsincos(tc, &sc, &cc);
    const double sa = g.sth[qt], ca = g.cth[qt];
    double W[4];
    dep_weights_box(g, r, tc, sc, cc, g.rn[p], g.rn[p + 1], g.th[qt], g.th[qt + 1], sa, ca,
                    W);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = p + (c & 1), j = qt + (c >> 1);
      sink_add(S, 3, i, j, qw * W[c] * vt * dt * g.inv_dth, s);
    }
  }
}

// per chunk of sorted particles (chunk_range): the chunk's node box
// (widened one node down, where the half-subgrid cells start) is summed in
// LDS and flushed with one global atomic per touched entry; a chunk whose
// box does not fit goes to global atomics directly
__global__ __launch_bounds__(kDepBlock) void k_deposit_paper(DepArgs A, const uint32_t* W1,
                                                             const uint32_t* W2,
                                                             const uint32_t* W3,
                                                             const int* cell, double dt) {
  __shared__ long long bins[4 * kDepBins];
  __shared__ int box[4];
  const ParticleView& P = A.p;
  for (long b = blockIdx.x;; b += gridDim.x) {  // uniform over the block
    long beg, end;
    int4 unused_box;  // equal chunks (no plan): always zero
    if (!chunk_range(A, b, beg, end, unused_box)) break;
    __syncthreads();  // the previous chunk is done with box and bins
    if (threadIdx.x == 0) {
      box[0] = 1 << 30;
      box[1] = -1;
      box[2] = 1 << 30;
      box[3] = -1;
    }
    __syncthreads();
    int pmin = 1 << 30, pmax = -1, qmin = 1 << 30, qmax = -1;
    for (long k = beg + threadIdx.x; k < end; k += kDepBlock) {
      if (!(P.flags[k] & GRPIC_FLAG_ALIVE) || P.qm[k] == 0) continue;
      int p, q;
      split_cell(A, cell[k], p, q);
      pmin = min(pmin, p);
      pmax = max(pmax, p);
      qmin = min(qmin, q);
      qmax = max(qmax, q);
    }
    if (pmax >= 0) {
      atomicMin(&box[0], pmin);
      atomicMax(&box[1], pmax);
      atomicMin(&box[2], qmin);
      atomicMax(&box[3], qmax);
    }
    __syncthreads();
    if (box[1] < 0) continue;  // nothing charged in this chunk
    const int bp0 = max(box[0] - 1, 0), bq0 = max(box[2] - 1, 0);
    const int bw = box[1] + 2 - bp0, bh = box[3] + 2 - bq0;
    if (bw * bh > kDepBins) {
      if (threadIdx.x == 0) atomicAdd(A.fallback, 1u);
      GlobalSink Gs{&A.acc, A.nr};
      for (long k = beg + threadIdx.x; k < end; k += kDepBlock)
        if ((P.flags[k] & GRPIC_FLAG_ALIVE) && P.qm[k] != 0)
          paper_particle(A, Gs, k, W1, W2, W3, cell, dt);
      continue;
    }
    LdsSink L{bins, bp0, bq0, bw, bh, bw * bh};
    for (int i = threadIdx.x; i < 4 * L.n; i += kDepBlock) bins[i] = 0;
    __syncthreads();
    for (long k = beg + threadIdx.x; k < end; k += kDepBlock)
      if ((P.flags[k] & GRPIC_FLAG_ALIVE) && P.qm[k] != 0)
        paper_particle(A, L, k, W1, W2, W3, cell, dt);
    __syncthreads();
    GlobalSink Gs{&A.acc, A.nr};
    for (int i = threadIdx.x; i < 4 * L.n; i += kDepBlock) {
      long long v = bins[i];
      if (v == 0) continue;
      int a = i / L.n, rr = i - a * L.n;
      int jj = rr / bw, ii = rr - jj * bw;
      atomicAdd(reinterpret_cast<unsigned long long*>(Gs.slot(a, bp0 + ii, bq0 + jj)),
                static_cast<unsigned long long>(v));
    }
  }
}

static void launch_deposit_paper(grpic_ctx* c, const uint32_t* const* W, const int* cell) {
  DepArgs A;
  A.g = make_grid_view(c);
  A.p = c->pv;
  A.p.n = c->n;
  A.acc = c->acc;
  A.nr = c->nr;
  A.nth = c->nth;
  A.inv_nr = 1.0 / c->nr;
  A.fallback = &c->stats->deposit_fallback;
  A.outside = nullptr;  // no planned boxes here
  // equal chunks: its per-particle work is large, so the few chunks whose
  // box misses the LDS bins cost less than the plan's many small chunks
  A.plan = nullptr;
  A.plan_meta = nullptr;
  A.plan_box = nullptr;
  hipLaunchKernelGGL(k_deposit_paper, dim3(deposit_blocks(c)), dim3(kDepBlock), 0,
                     c->stream, A, W[1], W[2], W[3], cell, c->cfg.dt);
  GRPIC_HIP(hipGetLastError());
}

// weights and node cell of the current positions
__global__ __launch_bounds__(256) void k_weights(GridView g, ParticleView P) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  if (!(P.flags[k] & GRPIC_FLAG_ALIVE)) return;
  int p, q;
  double r = P.r[k], th = P.th[k];
  node_cell(g, r, th, p, q);
  double W[4];
  dep_weights(g, r, th, p, q, W);
#pragma unroll
  for (int c = 1; c < 4; ++c) P.W[c][k] = wq_encode(W[c]);
  P.cell[k] = q * g.nr + p;
}

// dual lengths of node (i, j): half cells on the edges
__device__ __forceinline__ double dual_r(const GridView& g, int i) {
  if (i == 0) return g.rh[0] - g.rn[0];
  if (i == g.nr) return g.rn[g.nr] - g.rh[g.nr - 1];
  return g.rh[i] - g.rh[i - 1];
}
__device__ __forceinline__ double dual_t(const GridView& g, int j) {
  return (j == 0 || j == g.nth) ? 0.5 * g.dth : g.dth;
}

__global__ __launch_bounds__(256) void k_deposit_finalize(
    GridView g, DepositAcc acc, double dt, float* Jr, float* Jt, float* Jp,
    float* rho) {
  const int nrn = g.nr + 1, ntn = g.nth + 1;
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long nn = (long)nrn * ntn;
  if (k >= nn) return;
  int i = (int)(k % nrn), j = (int)(k / nrn);
  const double is = 1.0 / acc.scale, tp = 2.0 * kPi;
  double Lr = dual_r(g, i), Lt = dual_t(g, j);
  rho[k] = (float)((double)acc.Q[k] * is / (tp * Lr * Lt));
  Jp[k] = (float)((double)acc.P[k] * is / (dt * tp * Lr * Lt));
  acc.Q[k] = 0;
  acc.P[k] = 0;
  if (i < g.nr) {  // J^r at (i+1/2, j)
    long kk = (long)j * g.nr + i;
    Jr[kk] = (float)((double)acc.Fr[kk] * is / (dt * tp * Lt));
    acc.Fr[kk] = 0;
  }
  if (j < g.nth) {  // J^theta at (i, j+1/2)
    long kk = (long)j * nrn + i;
    Jt[kk] = (float)((double)acc.Ft[kk] * is / (dt * tp * Lr));
    acc.Ft[kk] = 0;
  }
}

static GridView grid_view(grpic_ctx* c) { return make_grid_view(c); }

static void finalize(grpic_ctx* c, int which) {
  long nn = (long)(c->nr + 1) * (c->nth + 1);
  float** J = c->J[which];
  hipLaunchKernelGGL(k_deposit_finalize, dim3(grid_for(nn, 256)), dim3(256), 0,
                     c->stream, grid_view(c), c->acc, c->cfg.dt, J[0], J[1],
                     J[2], J[3]);
  GRPIC_HIP(hipGetLastError());
}

void launch_deposit(grpic_ctx* c) {
  hipEvent_t ev;
  time_begin(c, GRPIC_K_DEPOSIT, &ev);
  if (c->n > 0 && c->cfg.deposit_mode == GRPIC_DEPOSIT_PAPER) {
    // J^{n+2} at the pushed state (new weights and cells)
    launch_deposit_paper(c, c->pv.Wn, c->pv.celln);
  } else if (c->n > 0) {
    DepArgs A;
    A.g = grid_view(c);
    A.p = c->pv;
    A.p.n = c->n;
    A.acc = c->acc;
    A.nr = c->nr;
    A.nth = c->nth;
    A.inv_nr = 1.0 / c->nr;
    A.fallback = &c->stats->deposit_fallback;
    A.outside = &c->stats->deposit_outside;
    A.xqueue = c->xqueue;
    A.xcount = &c->stats->cross_count;
    A.plan = c->dep_plan;
    A.plan_meta = c->dep_plan_meta;
    A.plan_box = c->dep_plan_box;
    hipLaunchKernelGGL(k_reset_xcount, dim3(1), dim3(1), 0, c->stream, A.xcount);
    hipLaunchKernelGGL(k_deposit, dim3(deposit_blocks(c)), dim3(kDepBlock), 0,
                       c->stream, A);
    unsigned xb = (unsigned)std::min<long>(grid_for(c->n, 256), 4L * c->num_cus);
    hipLaunchKernelGGL(k_deposit_crossing, dim3(xb), dim3(256), 0, c->stream, A);
    GRPIC_HIP(hipGetLastError());
  }
  finalize(c, c->jcur ^ 1);  // this step's deposit goes to J[jnext]
  time_end(c, GRPIC_K_DEPOSIT, ev);
}

void launch_deposit_initial(grpic_ctx* c) {
  if (c->n > 0) {
    ParticleView P = c->pv;
    P.n = c->n;
    hipLaunchKernelGGL(k_weights, dim3(grid_for(c->n, 256)), dim3(256), 0,
                       c->stream, grid_view(c), P);
    GRPIC_HIP(hipGetLastError());
    DepArgs A;
    A.g = grid_view(c);
    A.p = P;
    A.acc = c->acc;
    A.nr = c->nr;
    A.nth = c->nth;
    A.inv_nr = 1.0 / c->nr;
    A.plan = nullptr;
    A.plan_meta = nullptr;
    A.plan_box = nullptr;
    if (c->cfg.deposit_mode == GRPIC_DEPOSIT_PAPER)
      launch_deposit_paper(c, P.W, P.cell);  // rho and J at the loaded state
    else
      hipLaunchKernelGGL(k_deposit_rho, dim3(grid_for(c->n, 256)), dim3(256), 0,
                         c->stream, A);
    GRPIC_HIP(hipGetLastError());
  }
  // initial rho (conserving: zero currents; paper: J^{n+1}) in J[jcur]
  finalize(c, c->jcur);
}

}  // namespace grpic
