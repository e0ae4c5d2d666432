// probe.hip -- the two ceilings the kernels are measured against, timed on
// the device the context runs on: the FP64 vector fused-multiply-add rate
// (independent FMA chains, no memory traffic) and the streaming HBM rate (a
// copy between two buffers far larger than the last-level cache).
#include <algorithm>

#include "grpic_common.hpp"

namespace grpic {

namespace {

// each thread runs CHAINS independent chains a <- a m + c; the sums are
// stored so that the chains cannot be removed
template <int CHAINS>
__global__ __launch_bounds__(256) void k_probe_fma(double* out, int iters, double x0) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double a[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) a[j] = x0 + 1e-9 * (double)(t + j);
  const double m = 0.9999999, c = 1e-7;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < CHAINS; ++j) a[j] = fma(a[j], m, c);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < CHAINS; ++j) s += a[j];
  out[t] = s;
}

// dst = src, grid-stride, four 16-byte loads in flight per thread; NT:
// nontemporal loads and stores (no cache allocation)
typedef double dvec2 __attribute__((ext_vector_type(2)));

template <bool NT>
__global__ __launch_bounds__(256) void k_probe_copy(const dvec2* __restrict__ src,
                                                    dvec2* __restrict__ dst, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  auto ld = [](const dvec2* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
  };
  auto st = [](dvec2* p, dvec2 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
  };
  for (; i + 3 * stride < n; i += 4 * stride) {
    const dvec2 v0 = ld(src + i), v1 = ld(src + i + stride), v2 = ld(src + i + 2 * stride),
                v3 = ld(src + i + 3 * stride);
    st(dst + i, v0);
    st(dst + i + stride, v1);
    st(dst + i + 2 * stride, v2);
    st(dst + i + 3 * stride, v3);
  }
  for (; i < n; i += stride) st(dst + i, ld(src + i));
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
  // FMA: 8 or 16 waves per SIMD on every compute unit, 8 or 16 chains per
  // thread; the best of the four
  const int iters = 4096;
  const long max_threads = (long)c->num_cus * 16 * 256;
  double* out = dalloc<double>(max_threads);
  double best = 0.0;
  try {
    for (int wps : {8, 16}) {
      const unsigned blocks = (unsigned)c->num_cus * wps;
      const long threads = (long)blocks * 256;
      for (int chains : {8, 16}) {
        const double ms = mean_ms(s, 2, 10, [&] {
          if (chains == 8)
            hipLaunchKernelGGL(k_probe_fma<8>, dim3(blocks), dim3(256), 0, s, out, iters, 1.0);
          else
            hipLaunchKernelGGL(k_probe_fma<16>, dim3(blocks), dim3(256), 0, s, out, iters,
                               1.0);
        });
        GRPIC_HIP(hipGetLastError());
        best = std::max(best, 2.0 * chains * (double)iters * threads / (ms * 1e-3) / 1e12);
      }
    }
  } catch (...) {
    dfree(out);
    throw;
  }
  dfree(out);
  *fma_tflops = best;
  // copy: 2 x 1 GiB buffers, read + write counted; 4, 8 or 16 blocks per
  // compute unit, cached or nontemporal, and the runtime's copy; the best
  const long n = (1L << 30) / (long)sizeof(dvec2);
  dvec2* a = dalloc<dvec2>(n);
  dvec2* b = nullptr;
  best = 0.0;
  try {
    b = dalloc<dvec2>(n);
    GRPIC_HIP(hipMemsetAsync(a, 0, n * sizeof(dvec2), s));
    for (int bpc : {4, 8, 16})
      for (int nt = 0; nt < 2; ++nt) {
        const unsigned cb = (unsigned)c->num_cus * bpc;
        const double ms = mean_ms(s, 2, 10, [&] {
          if (nt)
            hipLaunchKernelGGL(k_probe_copy<true>, dim3(cb), dim3(256), 0, s, a, b, n);
          else
            hipLaunchKernelGGL(k_probe_copy<false>, dim3(cb), dim3(256), 0, s, a, b, n);
        });
        GRPIC_HIP(hipGetLastError());
        best = std::max(best, 2.0 * (double)n * sizeof(dvec2) / (ms * 1e-3) / 1e12);
      }
    // and the HIP runtime's own device-to-device copy
    const double ms = mean_ms(s, 2, 10, [&] {
      GRPIC_HIP(hipMemcpyAsync(b, a, n * sizeof(dvec2), hipMemcpyDeviceToDevice, s));
    });
    best = std::max(best, 2.0 * (double)n * sizeof(dvec2) / (ms * 1e-3) / 1e12);
  } catch (...) {
    dfree(a);
    dfree(b);
    throw;
  }
  dfree(a);
  dfree(b);
  *copy_tbs = best;
}

}  // namespace grpic
