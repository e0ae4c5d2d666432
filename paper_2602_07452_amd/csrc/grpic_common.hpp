// grpic_common.hpp -- shared declarations of the GRPIC HIP library: device
// views of the particle and field storage, the context, and the launchers
// implemented in each translation unit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/grpic.h"

namespace grpic {

constexpr double kPi = 3.14159265358979323846;
constexpr int kHistBins = GRPIC_HIST_BINS;

// ------------------------------------------------------------ particle views
struct ParticleView {
  long n;
  double *r, *th, *ph, *ur, *uth, *uph;  // state z
  double *H0, *herr, *w;
  int8_t* qm;                            // q/m in {+1, -1, 0}
  uint8_t *flags, *iters;
  uint32_t* id;
  // deposit weights of the cell's nodes 1..3 at x, stored in 31-bit fixed
  // point (wq_encode / wq_decode; W[0] unused: node 0's weight is
  // 1 - W1 - W2 - W3 of the decoded values, so the four sum to one)
  uint32_t* W[4];
  int* cell;                             // node cell index q * nr + p
  uint32_t* Wn[4];                       // the same at the pushed position
  int* celln;
  double *r_old, *th_old;                // previous position
  float* dphi;  // phi change of the step (FP32: it only scales J^phi, an FP32 output)
  double* t;                             // own time (field mode NONE only)
};

// device counters written by the particle kernels.  Counters that many
// blocks update are replicated (a block uses replica blockIdx % kStatReps)
// so that no single address takes more than a few thousand atomics a step;
// the host sums the replicas.
constexpr int kStatReps = 64;
constexpr int kQueueSegs = 256;  // the implicit queue is split in segments
constexpr int kPushBlock = 64;   // threads per block of the explicit push

struct StatRep {
  unsigned long long implicit_steps, noconv, removed, reflected;
  unsigned long long iter_hist[kHistBins];
  unsigned long long nonfinite;
  unsigned long long pad[3];
};

struct Stats {
  StatRep rep[kStatReps];
  // alive particles and the histogram of their energy violations, counted
  // from the particle arrays when the diagnostics are read (census[0]:
  // alive, census[1 + b]: bin b)
  unsigned long long census[1 + kHistBins];
  unsigned int seg_count[kQueueSegs];  // entries in each queue segment
  unsigned int deposit_fallback; // deposit segments that used global atomics
  unsigned int cross_count;      // crossing moves queued by the deposit
  unsigned long long deposit_outside;  // particles outside their planned box
};

// Stored deposit weights: W in [0, 1] as round(W 2^31) in a uint32 (an
// absolute error below 2^-32, 2^7 below the FP32 rounding of the densities
// and currents they make, and half the bytes of an FP64 weight).  Every
// user decodes the same stored values, so charge conservation, which needs
// the deposit's old and new weights to be the ones rho was made of, holds
// exactly.
constexpr double kWScale = 2147483648.0;  // 2^31
__device__ __forceinline__ uint32_t wq_encode(double w) {
  return (uint32_t)__double2uint_rn(fmin(fmax(w, 0.0), 1.0) * kWScale);
}
__device__ __forceinline__ double wq_decode(uint32_t q) { return (double)q * (1.0 / kWScale); }

// fixed-point charge accumulators (int64, deterministic under atomics)
struct DepositAcc {
  long long *Q, *P, *Fr, *Ft;  // rho (nodes), J^phi (nodes), r-flux (hn),
                               // theta-flux (nh)
  double scale;                // value -> integer units
};

struct Level3 {
  float* c[3];
};

struct Level4 {
  float* c[4];
};

struct Tables {
  // per Yee position type t (0 hn, 1 nh, 2 nn, 3 hh) FP32 coefficients
  // k_rr = alpha g_rr / sqrt(g), k_tt = alpha g_thth / sqrt(g),
  // k_pp = alpha g_phph / sqrt(g), k_rp = alpha g_rph / sqrt(g), beta^r,
  // sqrt(g)
  float *krr[4], *ktt[4], *kpp[4], *krp[4], *beta[4], *sg[4];
  float *damp_n, *damp_h;  // absorber factor exp(-chi dt) at r_i, r_{i+1/2}
  float *inv_drn;          // 1/(r_{i+1} - r_i), i < nr
  float *inv_drd;          // 1/(r_{i+1/2} - r_{i-1/2}), 0 < i < nr
};

}  // namespace grpic

// ------------------------------------------------------------------ context
struct grpic_ctx {
  grpic_config cfg;
  int device = 0;
  int num_cus = 256;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  std::string err;
  // grid
  int nr = 0, nth = 0;
  double dlnr = 0, dth = 0;
  std::vector<double> h_rn, h_rh, h_tn, h_th;
  double *rn = nullptr, *rh = nullptr, *tn = nullptr, *th = nullptr;
  double *idrn = nullptr, *idrh = nullptr;
  double *stn = nullptr, *ctn = nullptr;  // sin, cos of the node angles
  double *sth = nullptr, *cth = nullptr;  // sin, cos of the half angles
  grpic::Tables tab{};
  // field levels
  grpic::Level3 D[3]{};  // index: 0 = Dn, 1 = Dh0, 2 = Dh1
  grpic::Level3 B[3]{};  // 0 = Bm, 1 = Bn, 2 = Bh
  grpic::Level3 E{}, H{};
  float* J[2][4]{};      // [cur/prev][J^r, J^th, J^phi, rho]
  int jcur = 0;
  grpic::DepositAcc acc{};
  // particles
  long n = 0, cap = 0;
  bool has_neutral = false;  // some particle has q/m = 0
  grpic::ParticleView pv{};
  grpic::ParticleView alt{};  // second buffers of the sorted arrays
  double* gz[6]{};       // implicit guesses by queue slot
  int* queue = nullptr;
  unsigned seg_cap = 0;  // entries per implicit-queue segment
  int* xqueue = nullptr;  // crossing moves of the deposit
  grpic::Stats* stats = nullptr;
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  int* tile_count = nullptr;
  int* tile_offset = nullptr;
  int ntiles = 0;
  // deposit chunk plan of the last sort: chunk starts, their prefix by tile
  // group, and {chunks, particles at the sort, valid}
  int* dep_plan = nullptr;
  int* dep_plan_off = nullptr;
  int* dep_plan_meta = nullptr;
  int4* dep_plan_box = nullptr;  // node box of each planned chunk (see plan)
  long dep_plan_cap = 0;  // entries of dep_plan
  int plan_groups = 0;    // tile groups of the current plan layout
  double qw_max = 0;
  long steps = 0;
  // divergence cleaning (allocated on first use): coefficients
  // sqrt(g) g^rr / dr on the D^r faces, sqrt(g) g^thth / dth on the D^theta
  // faces, sqrt(g) g^phir on the nodes; the Gauss residual; phi ping-pong
  double *clean_kr = nullptr, *clean_kt = nullptr, *clean_kp = nullptr;
  double *clean_src = nullptr, *clean_phi[2]{};
  // pair injection (allocated on first use): per node cell weight sums,
  // eligibility and prefix sums; counters; the Maxwell-Juettner table
  long long* inj_wsum = nullptr;
  int *inj_flag = nullptr, *inj_off = nullptr, *inj_tot = nullptr;
  double* inj_mj = nullptr;
  double inj_mj_h = 0.0;
  // learned guess
  bool mlp_ready = false;
  void* mlp = nullptr;
  // graph
  bool use_graph = false;
  // captured steps, one per (step parity, particle buffer set): the step
  // alternates its level pointers every step and the sort swaps the two
  // particle buffer sets
  hipGraphExec_t graph_exec[4]{};
  int sort_flip = 0;
  // timing
  bool timing = false;
  double t_ms[GRPIC_K_COUNT]{};
  long t_count[GRPIC_K_COUNT]{};
  std::vector<hipEvent_t> ev_pool;
  struct Pending {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
};

#define GRPIC_HIP(call)                                                   \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      throw grpic::Error(GRPIC_E_HIP, std::string(#call) + ": " +         \
                                          hipGetErrorString(e_));         \
    }                                                                     \
  } while (0)

namespace grpic {

struct Error {
  int code;
  std::string msg;
  Error(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// launchers (defined in the .hip translation units)
void launch_metric_tables(grpic_ctx* c);
void launch_wald(grpic_ctx* c, double B0, double a_field);
void launch_split_monopole(grpic_ctx* c, double B0, double zeta0);
void launch_fields_step_pre(grpic_ctx* c);   // sub-steps 1-4
void launch_fields_step_post(grpic_ctx* c);  // sub-steps 7-10
void launch_fill(grpic_ctx* c, void* p, size_t bytes);
void launch_push(grpic_ctx* c);              // sub-step 5
void launch_census(grpic_ctx* c);            // alive count, energy histogram
void launch_deposit(grpic_ctx* c);           // sub-step 6
void launch_deposit_initial(grpic_ctx* c);
void launch_init_particles(grpic_ctx* c, const grpic_init_spec* s,
                           const double* mj_table, int mj_k, double mj_h);
void launch_energy_H0(grpic_ctx* c);
void launch_clean(grpic_ctx* c, int iters);  // Sec. 2.4, both D chains
constexpr int kInjMjK = 4096;                 // intervals of the MJ table
long launch_inject(grpic_ctx* c, const double* mj, int mj_k, double mj_h);
constexpr int kDepChunk = 8192;  // particles per deposit block at most
constexpr int kDepBins = 2048;   // LDS nodes per deposit array
// deposit blocks to launch for the current particle count and plan layout
long deposit_blocks(const grpic_ctx* c);
void invalidate_deposit_plan(grpic_ctx* c);
// measured FP64 FMA rate (TFLOP/s) and streaming copy rate (TB/s)
void probe_peaks(grpic_ctx* c, double* fma_tflops, double* copy_tbs);
// from_cells: the tile keys come from the stored node cells of the current
// positions (kept by every full-cycle step) instead of r and theta
void launch_sort(grpic_ctx* c, bool from_cells = false);
void launch_sample(grpic_ctx* c, const int* map, double* out, int* fl);
void launch_field_diag(grpic_ctx* c, double* gauss_max, double* divb_max,
                       double* pbz);
// allocation-free variant: the scratch is a static device array of the
// Maxwell translation unit; diag_scratch_init takes its address per device
constexpr int kDiagMaxNr = 16384;  // radial cells the scratch holds at most
void diag_scratch_init(int device);
void field_diag_noalloc(grpic_ctx* c, double* gauss_max, double* divb_max, double* pbz);
void launch_guess(grpic_ctx* c);
void mlp_upload(grpic_ctx* c, const float* theta, const float* mean,
                const float* inv_std, const float* scale);
void mlp_download(grpic_ctx* c, float* theta, float* mean, float* inv_std,
                  float* scale);
void mlp_free(grpic_ctx* c);
// training-sample collection by the implicit pass
struct CollectView {
  float* T = nullptr;  // targets, cap x 6 (nullptr: not collecting)
  uint8_t* valid = nullptr;
  const unsigned long long* rows = nullptr;  // rows collected before this step
  long cap = 0;
};
bool mlp_collecting(grpic_ctx* c);
CollectView mlp_collect_view(grpic_ctx* c);
void mlp_collect_start(grpic_ctx* c, long max_rows);
void mlp_collect_advance(grpic_ctx* c);
long mlp_num_samples(grpic_ctx* c);
void mlp_get_samples(grpic_ctx* c, long n, float* X, float* T, uint8_t* valid);
void mlp_train(grpic_ctx* c, const grpic_mlp_train_config* tc, double* epoch_loss);
void mlp_forward_rows(grpic_ctx* c, long n, const float* X, float* Y);
void mlp_loss_grad(grpic_ctx* c, long n, const float* X, const float* T, float* grad,
                   double* loss);

// timing helpers (api.hip)
void time_begin(grpic_ctx* c, int kid, hipEvent_t* a);
void time_end(grpic_ctx* c, int kid, hipEvent_t a);

template <class T>
T* dalloc(size_t n) {
  if (n == 0) n = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(GRPIC_E_OOM, std::string("hipMalloc of ") +
                                 std::to_string(n * sizeof(T)) + " bytes: " +
                                 hipGetErrorString(e));
  }
  return static_cast<T*>(p);
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

inline unsigned grid_for(long n, int block) {
  long g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace grpic
