// queue_device.hpp -- reading the segmented implicit queue.  The explicit
// push appends block b's rejected particles to segment b % kQueueSegs; the
// consumers see the segments concatenated and address entry v of that
// sequence through the exclusive prefix of the segment lengths.
#pragma once
#include "grpic_common.hpp"

namespace grpic {

// exclusive prefix of the queue-segment lengths in LDS (blockDim == kQueueSegs)
__device__ __forceinline__ unsigned segment_prefix(const Stats* st, unsigned* pref) {
  const int t = threadIdx.x;
  pref[t + 1] = st->seg_count[t];
  if (t == 0) pref[0] = 0;
  __syncthreads();
  for (int d = 1; d < kQueueSegs; d <<= 1) {
    unsigned v = (t + 1 > d) ? pref[t + 1 - d] : 0u;
    __syncthreads();
    pref[t + 1] += v;
    __syncthreads();
  }
  return pref[kQueueSegs];
}

// queue slot of the v-th entry counted across segments
__device__ __forceinline__ unsigned virtual_slot(const unsigned* pref, unsigned v,
                                                 unsigned seg_cap) {
  int lo = 0, hi = kQueueSegs;  // pref[lo] <= v < pref[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (pref[mid] <= v) lo = mid;
    else hi = mid;
  }
  return (unsigned)lo * seg_cap + (v - pref[lo]);
}

}  // namespace grpic
