// probe.hip -- the two ceilings the kernels are measured against, timed on
// the device the context runs on: the FP64 vector fused-multiply-add rate
// (independent FMA chains, no memory traffic) and the streaming HBM rate (a
// copy between two buffers far larger than the last-level cache).
#include "grpic_common.hpp"

namespace grpic {

namespace {

constexpr int kFmaChains = 8;

// each thread runs kFmaChains independent chains a <- a m + c; the sums are
// stored so that the chains cannot be removed
__global__ __launch_bounds__(256) void k_probe_fma(double* out, int iters, double x0) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double a[kFmaChains];
#pragma unroll
  for (int j = 0; j < kFmaChains; ++j) a[j] = x0 + 1e-9 * (double)(t + j);
  const double m = 0.9999999, c = 1e-7;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kFmaChains; ++j) a[j] = fma(a[j], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kFmaChains; ++j) s += a[j];
  out[t] = s;
}

// dst = src, grid-stride, four 16-byte loads in flight per thread
__global__ __launch_bounds__(256) void k_probe_copy(const double2* __restrict__ src,
                                                    double2* __restrict__ dst, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const double2 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride],
                  v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

template <class Launch>
double mean_ms(hipStream_t s, int warm, int reps, Launch&& launch) {
  for (int i = 0; i < warm; ++i) launch();
  hipEvent_t e0, e1;
  GRPIC_HIP(hipEventCreate(&e0));
  GRPIC_HIP(hipEventCreate(&e1));
  GRPIC_HIP(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) launch();
  GRPIC_HIP(hipEventRecord(e1, s));
  GRPIC_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  GRPIC_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / reps;
}

}  // namespace

void probe_peaks(grpic_ctx* c, double* fma_tflops, double* copy_tbs) {
  const hipStream_t s = c->stream;
  // FMA: 8 waves per SIMD on every compute unit
  const unsigned blocks = (unsigned)c->num_cus * 8;
  const long threads = (long)blocks * 256;
  const int iters = 4096;
  double* out = dalloc<double>(threads);
  double ms = 0.0;
  try {
    ms = mean_ms(s, 2, 10, [&] {
      hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, s, out, iters, 1.0);
    });
    GRPIC_HIP(hipGetLastError());
  } catch (...) {
    dfree(out);
    throw;
  }
  dfree(out);
  *fma_tflops = 2.0 * kFmaChains * (double)iters * threads / (ms * 1e-3) / 1e12;
  // copy: 2 x 1 GiB buffers, read + write counted
  const long n = (1L << 30) / (long)sizeof(double2);
  double2* a = dalloc<double2>(n);
  double2* b = nullptr;
  try {
    b = dalloc<double2>(n);
    const unsigned cb = (unsigned)c->num_cus * 8;
    GRPIC_HIP(hipMemsetAsync(a, 0, n * sizeof(double2), s));
    ms = mean_ms(s, 2, 10, [&] {
      hipLaunchKernelGGL(k_probe_copy, dim3(cb), dim3(256), 0, s, a, b, n);
    });
    GRPIC_HIP(hipGetLastError());
  } catch (...) {
    dfree(a);
    dfree(b);
    throw;
  }
  dfree(a);
  dfree(b);
  *copy_tbs = 2.0 * (double)n * sizeof(double2) / (ms * 1e-3) / 1e12;
}

}  // namespace grpic
