// mlp.hip -- learned initial guess for the implicit pusher (a project
// extension; the paper's method starts the iteration from the old state).
//
// A 14 -> 64 -> 64 -> 6 network with GELU activations predicts the part of
// the converged implicit step that a cheap base predictor misses:
//   guess = base + s (.) MLP((x - mean) * inv_std),
// base = the RK4 result when the hybrid pusher computed one, else the
// explicit Euler step z^n + dt F(z^n),
//   x = (r, theta, phi, u_r, u_theta, u_phi, (q/m) D^r, (q/m) D^theta,
//        (q/m) D^phi, (q/m) B^r, (q/m) B^theta, (q/m) B^phi, alpha, beta^r)
// at step n, with the fields gathered as in the push (the charge-to-mass
// ratio enters the equations of motion only through these products).  The Picard iteration still decides
// the result, so the guess only changes the number of iterations; a particle
// whose iteration from the learned guess does not converge is restarted from
// the old state.
//
// Parameters are FP32 master values (layout W1[64][14], b1[64], W2[64][64],
// b2[64], W3[6][64], b3[6]); a block rounds the weights to BF16 (nearest
// even) when it stages them in LDS, the biases stay FP32.  Products run on
// the 16x16x16 BF16 matrix cores with FP32 accumulation, one wavefront per 64
// rows.  Training minimises the mean squared error of the scaled residual with
// Adam; the backward pass uses the same tiles, and the per-block gradients are
// summed in a fixed order, so a training run is deterministic.
#include <algorithm>
#include <cmath>

#include "kerr_device.hpp"
#include "queue_device.hpp"

namespace grpic {

namespace {

constexpr int NI = 14, NH = 64, NO = 6;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NH * NI;
constexpr int OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + NO * NH;
constexpr int NPARAM = OFF_B3 + NO;
static_assert(NPARAM == GRPIC_MLP_NPARAM, "parameter count");
constexpr int NNORM = 2 * NI + NO;  // feature mean, feature 1/std, output scale

constexpr int LDX = 20;  // LDS row length (BF16) of 16-wide tiles
constexpr int LDW = 72;  // LDS row length (BF16) of 64-wide tiles
constexpr int LDY = 17;  // LDS row length (FP32) of the output tile

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

__device__ __forceinline__ bf16 to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (bf16)(u >> 16);
}

// GELU x Phi(x) with Phi the normal distribution function, and its
// derivative Phi(x) + x phi(x).  erf by Abramowitz & Stegun 7.1.26 (Hastings'
// rational approximation, absolute error below 1.5e-7: far below the BF16
// rounding that follows).
__device__ __forceinline__ void gelu_parts(float x, float& Phi, float& pdf) {
  const float y = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * y);
  const float poly =
      t * (0.254829592f +
           t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float e = __expf(-y * y);  // exp(-x^2 / 2)
  const float erf_y = 1.0f - poly * e;
  Phi = 0.5f * (1.0f + copysignf(erf_y, x));
  pdf = 0.39894228040143268f * e;
}
__device__ __forceinline__ float gelu(float x) {
  float P, d;
  gelu_parts(x, P, d);
  return x * P;
}
__device__ __forceinline__ float gelu_d(float x) {
  float P, d;
  gelu_parts(x, P, d);
  return P + x * d;
}

// the wave's LDS writes are complete and visible to all its lanes
__device__ __forceinline__ void wave_sync() {
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ s4 ld4(const bf16* p) {
  return *reinterpret_cast<const s4*>(p);
}
__device__ __forceinline__ s4 ld4s(const bf16* p, int stride) {
  s4 v;
  v.x = (short)p[0];
  v.y = (short)p[stride];
  v.z = (short)p[2 * stride];
  v.w = (short)p[3 * stride];
  return v;
}

// acc[mt][nt] += sum_k A(m, k) B(k, n) for an (16 MT) x (16 NT) tile with
// K = 16 KT, on one wavefront:
//   A(m, k) = TA ? SA[k lda + m] : SA[m lda + k]
//   B(k, n) = TB ? SB[k ldb + n] : SB[n ldb + k]
// Operand lanes of the 16x16x16 instruction: lane l holds A(l % 16, 4 (l/16)
// + j) and B(4 (l/16) + j, l % 16), j = 0..3; the result element v of lane l
// is C(4 (l/16) + v, l % 16).
template <int MT, int NT, int KT, bool TA, bool TB>
__device__ __forceinline__ void mma(const bf16* SA, int lda, const bf16* SB,
                                    int ldb, f4 (&acc)[MT][NT]) {
  const int l = threadIdx.x & 63, i = l & 15, g = (l >> 4) * 4;
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    const int k = kt * 16 + g;
    s4 b[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + i;
      b[nt] = TB ? ld4s(SB + k * ldb + n, ldb) : ld4(SB + n * ldb + k);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int m = mt * 16 + i;
      s4 a = TA ? ld4s(SA + k * lda + m, lda) : ld4(SA + m * lda + k);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[nt], acc[mt][nt], 0, 0, 0);
    }
  }
}

template <int MT, int NT>
__device__ __forceinline__ void zero(f4 (&acc)[MT][NT]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
}

// weights of one block in LDS (BF16) and biases (FP32)
struct alignas(16) WeightsLds {
  bf16 W1[NH * LDX];  // [out][in], in padded to 16 with zeros
  bf16 W2[NH * LDW];  // [out][in]
  bf16 W3[16 * LDW];  // [out][in], out padded to 16 with zeros
  float b1[NH], b2[NH], b3[16];
};

__device__ void stage_weights(const float* th, WeightsLds& S) {
  for (int t = threadIdx.x; t < NH * 16; t += blockDim.x) {
    int o = t >> 4, i = t & 15;
    S.W1[o * LDX + i] = i < NI ? to_bf16(th[OFF_W1 + o * NI + i]) : (bf16)0;
  }
  for (int t = threadIdx.x; t < NH * NH; t += blockDim.x) {
    int o = t >> 6, i = t & 63;
    S.W2[o * LDW + i] = to_bf16(th[OFF_W2 + t]);
  }
  for (int t = threadIdx.x; t < 16 * NH; t += blockDim.x) {
    int o = t >> 6, i = t & 63;
    S.W3[o * LDW + i] = o < NO ? to_bf16(th[OFF_W3 + o * NH + i]) : (bf16)0;
  }
  for (int t = threadIdx.x; t < NH; t += blockDim.x) {
    S.b1[t] = th[OFF_B1 + t];
    S.b2[t] = th[OFF_B2 + t];
  }
  for (int t = threadIdx.x; t < 16; t += blockDim.x) S.b3[t] = t < NO ? th[OFF_B3 + t] : 0.f;
}

// Forward pass of 64 rows on one wavefront.  X: [64][LDX] BF16 inputs;
// H1, H2: [64][LDW] BF16 activations (may be the same buffer when the
// pre-activations are not kept); y: output tile in registers (column l % 16,
// rows 16 mt + 4 (l/16) + v).  a1, a2 (optional): FP32 pre-activations in the
// same register layout.
__device__ __forceinline__ void forward(const WeightsLds& W, const bf16* X,
                                        bf16* H1, bf16* H2, f4 (&y)[4][1],
                                        f4 (*a1)[4] = nullptr,
                                        f4 (*a2)[4] = nullptr) {
  const int l = threadIdx.x & 63, i = l & 15, g = (l >> 4) * 4;
  f4 acc[4][4];
  zero(acc);
  mma<4, 4, 1, false, false>(X, LDX, W.W1, LDX, acc);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float s = acc[mt][nt][v] + W.b1[nt * 16 + i];
        if (a1) a1[mt][nt][v] = s;
        H1[(mt * 16 + g + v) * LDW + nt * 16 + i] = to_bf16(gelu(s));
      }
  wave_sync();
  zero(acc);
  mma<4, 4, 4, false, false>(H1, LDW, W.W2, LDW, acc);
  wave_sync();  // every lane has read H1 before H2 (possibly H1) is written
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float s = acc[mt][nt][v] + W.b2[nt * 16 + i];
        if (a2) a2[mt][nt][v] = s;
        H2[(mt * 16 + g + v) * LDW + nt * 16 + i] = to_bf16(gelu(s));
      }
  wave_sync();
  zero(y);
  mma<4, 1, 4, false, false>(H2, LDW, W.W3, LDW, y);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) y[mt][0][v] += W.b3[i];
}

// ------------------------------------------- inference (guess, checks)
// GELU by the tanh form x sigma(2 sqrt(2/pi) (x + 0.044715 x^3)) (Hendrycks
// & Gimpel), at most 4.7e-4 from x Phi(x) (at x = 2.7): below the BF16
// rounding of the activations that follows.  Two hardware estimates (exp2,
// reciprocal) and five FP32 operations.
__device__ __forceinline__ float gelu_fast(float x) {
  constexpr float k0 = -2.0f * 0.79788456080286536f * 1.4426950408889634f;
  constexpr float k1 = k0 * 0.044715f;
  const float t = x * __builtin_fmaf(k1, x * x, k0);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));

// four FP32 values as one BF16 operand (hardware round to nearest even)
__device__ __forceinline__ s4 pack_bf16(float a, float b, float c, float d) {
  const bf2v lo = __builtin_convertvector((f2v){a, b}, bf2v);
  const bf2v hi = __builtin_convertvector((f2v){c, d}, bf2v);
  return __builtin_bit_cast(s4, (u2v){__builtin_bit_cast(unsigned, lo),
                                       __builtin_bit_cast(unsigned, hi)});
}

// Forward pass of 64 rows on one wavefront, transposed: each layer computes
// H^T = W H_prev^T (hidden units x rows), so the accumulator a lane holds
// after one layer (rows 4 (l/16) + v of a 16-unit block, column l % 16) is
// exactly its B operand of the next layer's 16x16x16 product; activations
// never leave the registers.  X: [64][LDX] BF16 inputs in LDS (row = one
// network input row); Y: [64][LDY] FP32 outputs in LDS (columns 0..5).
__device__ __forceinline__ void forward_chained(const WeightsLds& W, const bf16* X, float* Y) {
  const int l = threadIdx.x & 63, i = l & 15, g = (l >> 4) * 4;
  s4 hb[4][4];  // [unit block][row block] BF16 activations, B operands
  {
    f4 acc[4][4];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
      const s4 b = ld4(X + (pb * 16 + i) * LDX + g);
#pragma unroll
      for (int ho = 0; ho < 4; ++ho) {
        const s4 a = ld4(W.W1 + (ho * 16 + i) * LDX + g);
        acc[ho][pb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, f4{0.f, 0.f, 0.f, 0.f},
                                                               0, 0, 0);
      }
    }
#pragma unroll
    for (int ho = 0; ho < 4; ++ho) {
      const f4 bias = *reinterpret_cast<const f4*>(W.b1 + ho * 16 + g);
#pragma unroll
      for (int pb = 0; pb < 4; ++pb)
        hb[ho][pb] = pack_bf16(gelu_fast(acc[ho][pb][0] + bias[0]),
                               gelu_fast(acc[ho][pb][1] + bias[1]),
                               gelu_fast(acc[ho][pb][2] + bias[2]),
                               gelu_fast(acc[ho][pb][3] + bias[3]));
    }
  }
  {
    f4 acc[4][4];
#pragma unroll
    for (int ho = 0; ho < 4; ++ho)
#pragma unroll
      for (int pb = 0; pb < 4; ++pb) acc[ho][pb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int hi = 0; hi < 4; ++hi)
#pragma unroll
      for (int ho = 0; ho < 4; ++ho) {
        const s4 a = ld4(W.W2 + (ho * 16 + i) * LDW + hi * 16 + g);
#pragma unroll
        for (int pb = 0; pb < 4; ++pb)
          acc[ho][pb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, hb[hi][pb], acc[ho][pb],
                                                                 0, 0, 0);
      }
#pragma unroll
    for (int ho = 0; ho < 4; ++ho) {
      const f4 bias = *reinterpret_cast<const f4*>(W.b2 + ho * 16 + g);
#pragma unroll
      for (int pb = 0; pb < 4; ++pb)
        hb[ho][pb] = pack_bf16(gelu_fast(acc[ho][pb][0] + bias[0]),
                               gelu_fast(acc[ho][pb][1] + bias[1]),
                               gelu_fast(acc[ho][pb][2] + bias[2]),
                               gelu_fast(acc[ho][pb][3] + bias[3]));
    }
  }
  f4 y[4];
#pragma unroll
  for (int pb = 0; pb < 4; ++pb) y[pb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int hi = 0; hi < 4; ++hi) {
    const s4 a = ld4(W.W3 + i * LDW + hi * 16 + g);
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
      y[pb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, hb[hi][pb], y[pb], 0, 0, 0);
  }
  // y[pb][v] = output g + v of row pb * 16 + i (outputs 0..5 in lanes 0..31)
  if (g < 8) {
    const f4 bias = *reinterpret_cast<const f4*>(W.b3 + g);
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (g + v < NO) Y[(pb * 16 + i) * LDY + g + v] = y[pb][v] + bias[v];
  }
}

// ------------------------------------------------------------ guess kernel
struct GuessArgs {
  GridView g;
  FieldView f;
  ParticleView p;
  double a, dt;
  double* gz[6];
  const int* queue;
  unsigned seg_cap;
  Stats* st;
  const float* theta;
  const float* norm;
  int use_net;  // add the network's correction to the base
  int base_gz;  // base = gz (the RK4 result of the hybrid) instead of Euler
  int grid;     // fields live on the grid (else no electromagnetic force)
  // sample collection (X == nullptr: off)
  float* X;
  const unsigned long long* rows;
  long cap;
};

constexpr int kGuessWaves = 4;

__global__ __launch_bounds__(64 * kGuessWaves) void k_mlp_guess(GuessArgs A) {
  __shared__ WeightsLds W;
  __shared__ float nrm[NNORM];
  __shared__ unsigned pref[kQueueSegs + 1];
  __shared__ __attribute__((aligned(16))) bf16 Xs[kGuessWaves][64 * LDX];
  __shared__ float Ys[kGuessWaves][64 * LDY];
  if (A.use_net) stage_weights(A.theta, W);
  for (int t = threadIdx.x; t < NNORM; t += blockDim.x) nrm[t] = A.use_net ? A.norm[t] : 0.f;
  const unsigned qn = segment_prefix(A.st, pref);  // ends with a barrier
  const unsigned long long base = A.X ? *A.rows : 0ull;
  const ParticleView& P = A.p;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  bf16* xs = Xs[w];
  float* ys = Ys[w];
  // wave w of nw takes queue groups of 64 w, w + nw, ...: the work per group
  // is the same, so fixed shares balance it without a shared work counter
  // (whose serialised atomics made this kernel take twice as long)
  const unsigned nw = gridDim.x * kGuessWaves;
  for (unsigned grp = blockIdx.x * kGuessWaves + w;; grp += nw) {
    const unsigned v0 = grp * 64u;
    if (v0 >= qn) break;
    const unsigned v = v0 + l;
    const bool act = v < qn;
    unsigned slot = 0;
    double z[6], ze[6];
    float x[NI];
    if (act) {
      slot = virtual_slot(pref, v, A.seg_cap);
      const long k = A.queue[slot];
      z[0] = P.r[k];
      z[1] = P.th[k];
      z[2] = P.ph[k];
      z[3] = P.ur[k];
      z[4] = P.uth[k];
      z[5] = P.uph[k];
      const double qm = (double)P.qm[k];
      Met m;
      double D[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
      if (A.base_gz) {
        metric(A.a, z[0], z[1], m);
        if (A.grid && qm != 0.0) gather(A.g, A.f, z[0], z[1], rcp(m.sg), D, B);
#pragma unroll
        for (int i = 0; i < 6; ++i) ze[i] = A.gz[i][slot];
      } else {
        DMet d;
        metric_d(A.a, z[0], z[1], m, d);
        if (A.grid && qm != 0.0) gather(A.g, A.f, z[0], z[1], rcp(m.sg), D, B);
        double f[6], pw;
        rhs(qm, z, m, d, D, B, f, &pw);
#pragma unroll
        for (int i = 0; i < 6; ++i) ze[i] = z[i] + A.dt * f[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) x[i] = (float)z[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        x[6 + i] = (float)(qm * D[i]);
        x[9 + i] = (float)(qm * B[i]);
      }
      x[12] = (float)m.alpha;
      x[13] = (float)m.betar;
    }
    if (A.use_net) {
      // this lane's normalised features as row l of the input tile
      auto feat = [&](int f) { return (act && f < NI) ? (x[f] - nrm[f]) * nrm[NI + f] : 0.f; };
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<s4*>(xs + l * LDX + 4 * q) =
            pack_bf16(feat(4 * q), feat(4 * q + 1), feat(4 * q + 2), feat(4 * q + 3));
      wave_sync();
      forward_chained(W, xs, ys);
      wave_sync();
      if (act) {
#pragma unroll
        for (int o = 0; o < NO; ++o) ze[o] += (double)(nrm[2 * NI + o] * ys[l * LDY + o]);
      }
      wave_sync();  // all reads of xs / ys done before the next group
    }
    if (act) {
#pragma unroll
      for (int i = 0; i < 6; ++i) A.gz[i][slot] = ze[i];
      if (A.X) {
        unsigned long long row = base + v;
        if (row < (unsigned long long)A.cap) {
#pragma unroll
          for (int i = 0; i < NI; ++i) A.X[row * NI + i] = x[i];
        }
      }
    }
  }
}

// rows collected so far += this step's queue length (capped)
__global__ void k_collect_advance(const Stats* st, unsigned long long* rows, long cap) {
  if (threadIdx.x != 0) return;
  unsigned long long n = 0;
  for (int s = 0; s < kQueueSegs; ++s) n += st->seg_count[s];
  unsigned long long r = *rows + n;
  *rows = r < (unsigned long long)cap ? r : (unsigned long long)cap;
}

// ------------------------------------------------------------ training
struct TrainArgs {
  const float* X;  // features, n x 14
  const float* T;  // targets, n x 6
  const uint8_t* valid;
  long n;
  int raw;              // X, T raw: normalise features, divide targets by scale
  const float* norm;    // used when raw
  const float* theta;
  long first;           // first batch position of this launch
  long count;           // rows in the batch
  unsigned long long mul, add, mask;  // batch position -> row permutation
  double inv_count;     // 1 / (count * 6)
  float* part;          // per-block gradients, blocks x NPARAM
  double* part_loss;    // per-block sum of squared errors
};

__device__ __forceinline__ long batch_row(const TrainArgs& A, long j) {
  unsigned long long s = (unsigned long long)j;
  if (A.mul == 1 && A.add == 0) return j;  // identity
  do {
    s = (A.mul * s + A.add) & A.mask;
  } while (s >= (unsigned long long)A.n);
  return (long)s;
}

// sum over the 64 rows held in C layout (rows 16 mt + 4 (l/16) + v) for
// column l % 16; the total lands in lanes 0..15
template <int MT>
__device__ __forceinline__ float col_sum(const f4 (&c)[MT]) {
  float s = 0.f;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) s += (c[mt][0] + c[mt][1]) + (c[mt][2] + c[mt][3]);
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  return s;
}

__global__ __launch_bounds__(64) void k_mlp_train(TrainArgs A) {
  __shared__ WeightsLds W;
  __shared__ __attribute__((aligned(16))) bf16 Xs[64 * LDX];
  __shared__ __attribute__((aligned(16))) bf16 H1[64 * LDW];
  __shared__ __attribute__((aligned(16))) bf16 H2[64 * LDW];
  __shared__ __attribute__((aligned(16))) bf16 DA[64 * LDW];
  __shared__ __attribute__((aligned(16))) bf16 DY[64 * LDX];
  __shared__ float Ts[64 * 8];
  stage_weights(A.theta, W);
  const int l = threadIdx.x, i = l & 15, g = (l >> 4) * 4;
  const long j = A.first + (long)blockIdx.x * 64 + l;
  const bool act = j < A.first + A.count;
  long row = act ? batch_row(A, j) : 0;
  const bool use = act && (!A.valid || A.valid[row]);
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    float v = 0.f;
    if (use && c < NI) {
      v = A.X[row * NI + c];
      if (A.raw) v = (v - A.norm[c]) * A.norm[NI + c];
    }
    Xs[l * LDX + c] = to_bf16(v);
  }
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    float t = 0.f;
    if (use && o < NO) {
      t = A.T[row * NO + o];
      if (A.raw) t = t / A.norm[2 * NI + o];
    }
    Ts[l * 8 + o] = t;
  }
  Ts[l * 8 + 7] = use ? 1.f : 0.f;  // row mask
  __syncthreads();
  f4 a1[4][4], a2[4][4], y[4][1];
  forward(W, Xs, H1, H2, y, a1, a2);
  // dL/dy = 2 (y - t) / (count * 6) on used rows and real outputs
  float sq = 0.f;
  f4 dy[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = mt * 16 + g + v;
      float d = 0.f;
      if (i < NO && Ts[r * 8 + 7] != 0.f) {
        float e = y[mt][0][v] - Ts[r * 8 + i];
        sq += e * e;
        d = 2.0f * e * (float)A.inv_count;
      }
      dy[mt][v] = d;
      DY[r * LDX + i] = to_bf16(d);
    }
  wave_sync();
  float* gp = A.part + (long)blockIdx.x * NPARAM;
  {  // b3 and W3
    float s = col_sum<4>(dy);
    if (l < NO) gp[OFF_B3 + l] = s;
    f4 gw[1][4];
    zero(gw);
    mma<1, 4, 4, true, true>(DY, LDX, H2, LDW, gw);  // (o, i) = sum_r dy[r][o] h2[r][i]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (g + v < NO) gp[OFF_W3 + (g + v) * NH + nt * 16 + i] = gw[0][nt][v];
  }
  {  // da2 = (dy W3) * gelu'(a2)
    f4 dh[4][4];
    zero(dh);
    mma<4, 4, 1, false, true>(DY, LDX, W.W3, LDW, dh);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float d = dh[mt][nt][v] * gelu_d(a2[mt][nt][v]);
          a2[mt][nt][v] = d;  // a2 now holds da2
          DA[(mt * 16 + g + v) * LDW + nt * 16 + i] = to_bf16(d);
        }
  }
  wave_sync();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {  // b2
    f4 c[4] = {a2[0][nt], a2[1][nt], a2[2][nt], a2[3][nt]};
    float s = col_sum<4>(c);
    if (l < 16) gp[OFF_B2 + nt * 16 + l] = s;
  }
  {  // W2
    f4 gw[4][4];
    zero(gw);
    mma<4, 4, 4, true, true>(DA, LDW, H1, LDW, gw);  // (o, i) = sum_r da2[r][o] h1[r][i]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          gp[OFF_W2 + (mt * 16 + g + v) * NH + nt * 16 + i] = gw[mt][nt][v];
  }
  {  // da1 = (da2 W2) * gelu'(a1)
    f4 dh[4][4];
    zero(dh);
    mma<4, 4, 4, false, true>(DA, LDW, W.W2, LDW, dh);
    wave_sync();  // every lane has read DA before it is overwritten
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float d = dh[mt][nt][v] * gelu_d(a1[mt][nt][v]);
          a1[mt][nt][v] = d;
          DA[(mt * 16 + g + v) * LDW + nt * 16 + i] = to_bf16(d);
        }
  }
  wave_sync();
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {  // b1
    f4 c[4] = {a1[0][nt], a1[1][nt], a1[2][nt], a1[3][nt]};
    float s = col_sum<4>(c);
    if (l < 16) gp[OFF_B1 + nt * 16 + l] = s;
  }
  {  // W1
    f4 gw[4][1];
    zero(gw);
    mma<4, 1, 4, true, true>(DA, LDW, Xs, LDX, gw);  // (o, i) = sum_r da1[r][o] x[r][i]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (i < NI) gp[OFF_W1 + (mt * 16 + g + v) * NI + i] = gw[mt][0][v];
  }
  // squared error of the block (lanes hold disjoint elements)
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
  if (l == 0) A.part_loss[blockIdx.x] = (double)sq;
}

// sums the block gradients in block order; optional Adam step
struct AdamArgs {
  const float* part;
  const double* part_loss;
  int blocks;
  float* grad;
  double* loss;       // += (sum of squared errors) * inv_count
  double inv_count;
  float* theta;
  float *m, *v;
  int update;
  float lr, b1, b2, eps, c1, c2;  // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
};

__global__ __launch_bounds__(256) void k_mlp_reduce(AdamArgs A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    double s = 0.0;
    for (int b = 0; b < A.blocks; ++b) s += A.part_loss[b];
    *A.loss += s * A.inv_count;
  }
  if (p >= NPARAM) return;
  double s = 0.0;
  for (int b = 0; b < A.blocks; ++b) s += (double)A.part[(long)b * NPARAM + p];
  float gr = (float)s;
  A.grad[p] = gr;
  if (!A.update) return;
  float m = A.b1 * A.m[p] + (1.f - A.b1) * gr;
  float v = A.b2 * A.v[p] + (1.f - A.b2) * gr * gr;
  A.m[p] = m;
  A.v[p] = v;
  A.theta[p] -= A.lr * (m * A.c1) / (sqrtf(v * A.c2) + A.eps);
}

// network outputs for given (normalised) inputs
__global__ __launch_bounds__(64) void k_mlp_forward_rows(const float* theta, const float* X,
                                                         long n, float* Y) {
  __shared__ WeightsLds W;
  __shared__ __attribute__((aligned(16))) bf16 Xs[64 * LDX];
  __shared__ float Ys[64 * LDY];
  stage_weights(theta, W);
  const int l = threadIdx.x;
  const long r0 = (long)blockIdx.x * 64;
  auto feat = [&](int c) { return (r0 + l < n && c < NI) ? X[(r0 + l) * NI + c] : 0.f; };
#pragma unroll
  for (int q = 0; q < 4; ++q)
    *reinterpret_cast<s4*>(Xs + l * LDX + 4 * q) =
        pack_bf16(feat(4 * q), feat(4 * q + 1), feat(4 * q + 2), feat(4 * q + 3));
  __syncthreads();
  forward_chained(W, Xs, Ys);
  __syncthreads();
  if (r0 + l < n) {
#pragma unroll
    for (int o = 0; o < NO; ++o) Y[(r0 + l) * NO + o] = Ys[l * LDY + o];
  }
}

// feature / target moments: per block partial sums of x and x^2 (20 columns)
__global__ __launch_bounds__(256) void k_mlp_moments(const float* X, const float* T,
                                                     const uint8_t* valid, long n,
                                                     double* part) {
  __shared__ double red[256];
  for (int c = 0; c < NI + NO; ++c) {
    double s = 0.0, s2 = 0.0, cnt = 0.0;
    for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (long)gridDim.x * blockDim.x) {
      if (valid && !valid[r]) continue;
      double x = c < NI ? X[r * NI + c] : T[r * NO + (c - NI)];
      s += x;
      s2 += x * x;
      cnt += 1.0;
    }
    double vals[3] = {s, s2, cnt};
    for (int q = 0; q < 3; ++q) {
      red[threadIdx.x] = vals[q];
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[((long)blockIdx.x * (NI + NO) + c) * 3 + q] = red[0];
      __syncthreads();
    }
  }
}

// mean and 1/std of the features; RMS of the targets (output scale)
__global__ void k_mlp_norm(const double* part, int blocks, float* norm) {
  const int c = threadIdx.x;
  if (c >= NI + NO) return;
  double s = 0.0, s2 = 0.0, cnt = 0.0;
  for (int b = 0; b < blocks; ++b) {
    const double* q = part + ((long)b * (NI + NO) + c) * 3;
    s += q[0];
    s2 += q[1];
    cnt += q[2];
  }
  if (cnt <= 0.0) cnt = 1.0;
  double mean = s / cnt, var = s2 / cnt - mean * mean;
  if (c < NI) {
    norm[c] = (float)mean;
    norm[NI + c] = var > 1e-30 ? (float)(1.0 / sqrt(var)) : 1.f;
  } else {
    double rms = sqrt(s2 / cnt);
    norm[2 * NI + (c - NI)] = rms > 1e-300 ? (float)rms : 1.f;
  }
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// uniform initialisation in +-1/sqrt(fan_in) from a counter-based generator
__global__ void k_mlp_init(float* theta, float* m, float* v, unsigned long long seed) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const int fan = p < OFF_W2 ? NI : NH;
  unsigned long long r = mix64(seed * 0x9e3779b97f4a7c15ull + (unsigned long long)p + 1ull);
  double u = (double)(r >> 11) * 0x1p-53;
  theta[p] = (float)((2.0 * u - 1.0) / sqrt((double)fan));
  m[p] = 0.f;
  v[p] = 0.f;
}

}  // namespace

// ------------------------------------------------------------ host side
struct MlpState {
  float* theta = nullptr;  // FP32 master parameters
  float* norm = nullptr;   // mean[14], 1/std[14], scale[6]
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  double* loss = nullptr;
  // collected samples
  long cap = 0;
  bool collect = false;
  float* X = nullptr;
  float* T = nullptr;
  uint8_t* valid = nullptr;
  unsigned long long* rows = nullptr;
  // training scratch
  int part_blocks = 0;
  float* part = nullptr;
  double* part_loss = nullptr;
  double* moments = nullptr;
  // staging for the forward / gradient entry points
  long io_cap = 0;
  float* io_X = nullptr;
  float* io_T = nullptr;
};

constexpr int kMomentBlocks = 512;

static MlpState* state(grpic_ctx* c) {
  if (!c->mlp) {
    auto* s = new MlpState;
    c->mlp = s;
    s->theta = dalloc<float>(NPARAM);
    s->norm = dalloc<float>(NNORM);
    s->m = dalloc<float>(NPARAM);
    s->v = dalloc<float>(NPARAM);
    s->grad = dalloc<float>(NPARAM);
    s->loss = dalloc<double>(1);
    s->rows = dalloc<unsigned long long>(1);
    s->moments = dalloc<double>((size_t)kMomentBlocks * (NI + NO) * 3);
    launch_fill(c, s->rows, sizeof(unsigned long long));
  }
  return static_cast<MlpState*>(c->mlp);
}

static void ensure_part(grpic_ctx* c, MlpState* s, int blocks) {
  if (blocks <= s->part_blocks) return;
  dfree(s->part);
  dfree(s->part_loss);
  s->part = dalloc<float>((size_t)blocks * NPARAM);
  s->part_loss = dalloc<double>((size_t)blocks);
  s->part_blocks = blocks;
  (void)c;
}

static void ensure_io(MlpState* s, long n) {
  if (n <= s->io_cap) return;
  dfree(s->io_X);
  dfree(s->io_T);
  s->io_X = dalloc<float>((size_t)n * NI);
  s->io_T = dalloc<float>((size_t)n * NO);
  s->io_cap = n;
}

void mlp_free(grpic_ctx* c) {
  auto* s = static_cast<MlpState*>(c->mlp);
  if (!s) return;
  for (float** p : {&s->theta, &s->norm, &s->m, &s->v, &s->grad, &s->X, &s->T, &s->part,
                    &s->io_X, &s->io_T})
    dfree(*p);
  dfree(s->loss);
  dfree(s->valid);
  dfree(s->rows);
  dfree(s->part_loss);
  dfree(s->moments);
  delete s;
  c->mlp = nullptr;
}

void mlp_upload(grpic_ctx* c, const float* theta, const float* mean, const float* inv_std,
                const float* scale) {
  MlpState* s = state(c);
  GRPIC_HIP(hipMemcpyAsync(s->theta, theta, NPARAM * sizeof(float), hipMemcpyHostToDevice,
                           c->stream));
  float h[NNORM];
  for (int i = 0; i < NI; ++i) {
    h[i] = mean[i];
    h[NI + i] = inv_std[i];
  }
  for (int o = 0; o < NO; ++o) h[2 * NI + o] = scale[o];
  GRPIC_HIP(hipMemcpyAsync(s->norm, h, sizeof(h), hipMemcpyHostToDevice, c->stream));
  GRPIC_HIP(hipStreamSynchronize(c->stream));
}

void mlp_download(grpic_ctx* c, float* theta, float* mean, float* inv_std, float* scale) {
  MlpState* s = state(c);
  float h[NNORM];
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  GRPIC_HIP(hipMemcpy(theta, s->theta, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  GRPIC_HIP(hipMemcpy(h, s->norm, sizeof(h), hipMemcpyDeviceToHost));
  for (int i = 0; i < NI; ++i) {
    mean[i] = h[i];
    inv_std[i] = h[NI + i];
  }
  for (int o = 0; o < NO; ++o) scale[o] = h[2 * NI + o];
}

bool mlp_collecting(grpic_ctx* c) {
  auto* s = static_cast<MlpState*>(c->mlp);
  return s && s->collect;
}

CollectView mlp_collect_view(grpic_ctx* c) {
  CollectView v{};
  auto* s = static_cast<MlpState*>(c->mlp);
  if (!s || !s->collect) return v;
  v.T = s->T;
  v.valid = s->valid;
  v.rows = s->rows;
  v.cap = s->cap;
  return v;
}

void mlp_collect_start(grpic_ctx* c, long max_rows) {
  MlpState* s = state(c);
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  if (max_rows <= 0) {
    s->collect = false;
    return;
  }
  if (max_rows != s->cap) {
    dfree(s->X);
    dfree(s->T);
    dfree(s->valid);
    s->X = dalloc<float>((size_t)max_rows * NI);
    s->T = dalloc<float>((size_t)max_rows * NO);
    s->valid = dalloc<uint8_t>((size_t)max_rows);
    s->cap = max_rows;
  }
  launch_fill(c, s->rows, sizeof(unsigned long long));
  s->collect = true;
}

long mlp_num_samples(grpic_ctx* c) {
  auto* s = static_cast<MlpState*>(c->mlp);
  if (!s || !s->X) return 0;
  unsigned long long n = 0;
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  GRPIC_HIP(hipMemcpy(&n, s->rows, sizeof(n), hipMemcpyDeviceToHost));
  return (long)n;
}

void mlp_get_samples(grpic_ctx* c, long n, float* X, float* T, uint8_t* valid) {
  auto* s = static_cast<MlpState*>(c->mlp);
  long have = mlp_num_samples(c);
  if (n > have) throw Error(GRPIC_E_INVALID, "more samples requested than collected");
  if (n <= 0) return;
  if (X) GRPIC_HIP(hipMemcpy(X, s->X, (size_t)n * NI * sizeof(float), hipMemcpyDeviceToHost));
  if (T) GRPIC_HIP(hipMemcpy(T, s->T, (size_t)n * NO * sizeof(float), hipMemcpyDeviceToHost));
  if (valid) GRPIC_HIP(hipMemcpy(valid, s->valid, (size_t)n, hipMemcpyDeviceToHost));
}

void launch_guess(grpic_ctx* c) {
  MlpState* s = static_cast<MlpState*>(c->mlp);
  const bool net = c->cfg.guess == GRPIC_GUESS_MLP;
  if (net && !c->mlp_ready && !(s && s->collect))
    throw Error(GRPIC_E_STATE, "learned guess has no network");
  GuessArgs A;
  A.g = make_grid_view(c);
  A.f.Dr = c->D[2].c[0];
  A.f.Dt = c->D[2].c[1];
  A.f.Dp = c->D[2].c[2];
  A.f.Br = c->B[2].c[0];
  A.f.Bt = c->B[2].c[1];
  A.f.Bp = c->B[2].c[2];
  A.p = c->pv;
  A.p.n = c->n;
  A.a = c->cfg.a;
  A.dt = c->cfg.dt;
  for (int i = 0; i < 6; ++i) A.gz[i] = c->gz[i];
  A.queue = c->queue;
  A.seg_cap = c->seg_cap;
  A.st = c->stats;
  // while collecting, the iteration starts from the Euler predictor alone
  const bool coll = s && s->collect;
  A.theta = net ? s->theta : nullptr;
  A.norm = net ? s->norm : nullptr;
  A.use_net = (net && !coll) ? 1 : 0;
  // the hybrid pushers leave their RK4 result in gz
  A.base_gz = (c->cfg.pusher == GRPIC_PUSH_HYB1 || c->cfg.pusher == GRPIC_PUSH_HYB2) ? 1 : 0;
  A.grid = c->cfg.field_mode != GRPIC_FIELDS_NONE ? 1 : 0;
  A.X = coll ? s->X : nullptr;
  A.rows = coll ? s->rows : nullptr;
  A.cap = coll ? s->cap : 0;
  long need = (c->n + 64 * kGuessWaves - 1) / (64 * kGuessWaves);
  // two blocks per CU: with 149 VGPRs and 96 accumulation registers the
  // kernel holds two waves per SIMD
  long blocks = std::min<long>(2L * c->num_cus, std::max<long>(need, 1));
  hipEvent_t ev;
  time_begin(c, GRPIC_K_GUESS, &ev);
  hipLaunchKernelGGL(k_mlp_guess, dim3((unsigned)blocks), dim3(64 * kGuessWaves), 0,
                     c->stream, A);
  GRPIC_HIP(hipGetLastError());
  time_end(c, GRPIC_K_GUESS, ev);
}

void mlp_collect_advance(grpic_ctx* c) {
  MlpState* s = state(c);
  hipLaunchKernelGGL(k_collect_advance, dim3(1), dim3(64), 0, c->stream, c->stats, s->rows,
                     s->cap);
  GRPIC_HIP(hipGetLastError());
}

// one gradient evaluation over positions [first, first + count) of the batch order
static void gradient(grpic_ctx* c, MlpState* s, TrainArgs T, int update, float lr, int t,
                     const grpic_mlp_train_config* tc) {
  int blocks = (int)((T.count + 63) / 64);
  ensure_part(c, s, blocks);
  T.part = s->part;
  T.part_loss = s->part_loss;
  T.inv_count = 1.0 / ((double)T.count * NO);
  hipLaunchKernelGGL(k_mlp_train, dim3(blocks), dim3(64), 0, c->stream, T);
  GRPIC_HIP(hipGetLastError());
  AdamArgs A;
  A.part = s->part;
  A.part_loss = s->part_loss;
  A.blocks = blocks;
  A.grad = s->grad;
  A.loss = s->loss;
  A.inv_count = T.inv_count;
  A.theta = s->theta;
  A.m = s->m;
  A.v = s->v;
  A.update = update;
  A.lr = lr;
  A.b1 = tc ? (float)tc->beta1 : 0.9f;
  A.b2 = tc ? (float)tc->beta2 : 0.999f;
  A.eps = tc ? (float)tc->eps : 1e-8f;
  A.c1 = (float)(1.0 / (1.0 - std::pow((double)A.b1, t)));
  A.c2 = (float)(1.0 / (1.0 - std::pow((double)A.b2, t)));
  hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(NPARAM, 256)), dim3(256), 0, c->stream, A);
  GRPIC_HIP(hipGetLastError());
}

void mlp_forward_rows(grpic_ctx* c, long n, const float* X, float* Y) {
  MlpState* s = state(c);
  if (!c->mlp_ready) throw Error(GRPIC_E_STATE, "no network loaded");
  if (n <= 0) return;
  ensure_io(s, n);
  GRPIC_HIP(hipMemcpyAsync(s->io_X, X, (size_t)n * NI * sizeof(float), hipMemcpyHostToDevice,
                           c->stream));
  hipLaunchKernelGGL(k_mlp_forward_rows, dim3(grid_for(n, 64)), dim3(64), 0, c->stream,
                     s->theta, s->io_X, n, s->io_T);
  GRPIC_HIP(hipGetLastError());
  GRPIC_HIP(hipMemcpyAsync(Y, s->io_T, (size_t)n * NO * sizeof(float), hipMemcpyDeviceToHost,
                           c->stream));
  GRPIC_HIP(hipStreamSynchronize(c->stream));
}

void mlp_loss_grad(grpic_ctx* c, long n, const float* X, const float* T, float* grad,
                   double* loss) {
  MlpState* s = state(c);
  if (!c->mlp_ready) throw Error(GRPIC_E_STATE, "no network loaded");
  if (n <= 0) throw Error(GRPIC_E_INVALID, "empty batch");
  ensure_io(s, n);
  GRPIC_HIP(hipMemcpyAsync(s->io_X, X, (size_t)n * NI * sizeof(float), hipMemcpyHostToDevice,
                           c->stream));
  GRPIC_HIP(hipMemcpyAsync(s->io_T, T, (size_t)n * NO * sizeof(float), hipMemcpyHostToDevice,
                           c->stream));
  launch_fill(c, s->loss, sizeof(double));
  {
    TrainArgs A{};
    A.X = s->io_X;
    A.T = s->io_T;
    A.valid = nullptr;
    A.n = n;
    A.raw = 0;
    A.norm = s->norm;
    A.theta = s->theta;
    A.first = 0;
    A.count = n;
    A.mul = 1;
    A.add = 0;
    A.mask = ~0ull;
    gradient(c, s, A, 0, 0.f, 1, nullptr);
    GRPIC_HIP(hipMemcpyAsync(grad, s->grad, NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                             c->stream));
    GRPIC_HIP(hipMemcpyAsync(loss, s->loss, sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    GRPIC_HIP(hipStreamSynchronize(c->stream));
  }
}

static unsigned long long splitmix(unsigned long long& x) {
  unsigned long long z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

void mlp_train(grpic_ctx* c, const grpic_mlp_train_config* tc, double* epoch_loss) {
  MlpState* s = state(c);
  long n = mlp_num_samples(c);
  if (n < 64) throw Error(GRPIC_E_STATE, "fewer than 64 collected samples");
  if (tc->epochs <= 0 || tc->batch < 64 || tc->lr <= 0.0)
    throw Error(GRPIC_E_INVALID, "invalid training configuration");
  // normalisation from the samples
  hipLaunchKernelGGL(k_mlp_moments, dim3(kMomentBlocks), dim3(256), 0, c->stream, s->X, s->T,
                     s->valid, n, s->moments);
  hipLaunchKernelGGL(k_mlp_norm, dim3(1), dim3(64), 0, c->stream, s->moments, kMomentBlocks,
                     s->norm);
  hipLaunchKernelGGL(k_mlp_init, dim3(grid_for(NPARAM, 256)), dim3(256), 0, c->stream,
                     s->theta, s->m, s->v, (unsigned long long)tc->seed);
  GRPIC_HIP(hipGetLastError());
  int bits = 1;
  while ((1L << bits) < n) ++bits;
  const unsigned long long mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1ull);
  const long batch = std::min<long>(tc->batch, n);
  const long per_epoch = (n + batch - 1) / batch;
  const long total = per_epoch * tc->epochs;
  unsigned long long rng = (unsigned long long)tc->seed ^ 0x5deece66dull;
  int t = 0;
  std::vector<double> losses((size_t)tc->epochs);
  for (long e = 0; e < tc->epochs; ++e) {
    launch_fill(c, s->loss, sizeof(double));
    TrainArgs A{};
    A.X = s->X;
    A.T = s->T;
    A.valid = s->valid;
    A.n = n;
    A.raw = 1;
    A.norm = s->norm;
    A.theta = s->theta;
    A.mul = (splitmix(rng) & mask) | 1ull;
    A.add = splitmix(rng) & mask;
    A.mask = mask;
    if (A.mul == 1 && A.add == 0) A.add = 1;
    for (long b = 0; b < per_epoch; ++b) {
      ++t;
      // cosine decay from lr to lr_final over the run
      double f = 0.5 * (1.0 + std::cos(kPi * (double)(t - 1) / (double)std::max<long>(total, 1)));
      float lr = (float)(tc->lr_final + (tc->lr - tc->lr_final) * f);
      A.first = b * batch;
      A.count = std::min(batch, n - A.first);
      gradient(c, s, A, 1, lr, t, tc);
    }
    GRPIC_HIP(hipMemcpyAsync(&losses[(size_t)e], s->loss, sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  }
  GRPIC_HIP(hipStreamSynchronize(c->stream));
  if (epoch_loss)
    for (long e = 0; e < tc->epochs; ++e) epoch_loss[e] = losses[(size_t)e] / (double)per_epoch;
  c->mlp_ready = true;
}

}  // namespace grpic
