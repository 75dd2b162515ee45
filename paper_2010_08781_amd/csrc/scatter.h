// scatter.h -- load-balanced expansion of senders' out-edges for the push
// exchange (Section 4.3.2, push side).
//
// Each thread of a workgroup holds at most one sender (its edge range
// [beg, end) and a payload).  Out-edges are expanded in three tiers so that
// lanes stay busy whatever the degree skew:
//   1. senders with >= 256 edges are taken one at a time by the whole
//      workgroup (coalesced, 256 edges per pass);
//   2. senders with >= 64 edges are taken one at a time by their wavefront;
//   3. the remaining short lists of a wavefront are concatenated by a
//      wave-wide prefix sum and processed 64 edges per pass, each lane
//      locating its sender by binary search over the prefix (LDS).
// `emit(edge_index, payload)` is called exactly once per out-edge.  Every
// thread of the workgroup must call twc_scatter (it contains barriers).
#pragma once

#include "common.h"

namespace ipg {

template <class Payload, class Emit>
__device__ __forceinline__ void twc_scatter(bool has, uint64_t beg, uint64_t end, Payload pay, Emit&& emit) {
  __shared__ uint64_t sb_beg, sb_end;
  __shared__ Payload sb_pay;
  __shared__ int sb_owner;
  __shared__ uint64_t s_beg[kBlock];
  __shared__ uint32_t s_ex[kBlock];
  __shared__ Payload s_pay[kBlock];

  const uint32_t lane = lane_id();
  const uint32_t tid = threadIdx.x;

  // Tier 1: workgroup-cooperative.
  bool big = has && (end - beg) >= (uint64_t)kBlock;
  while (__syncthreads_or(big)) {
    if (big) sb_owner = static_cast<int>(tid);
    __syncthreads();
    if (sb_owner == static_cast<int>(tid)) {
      sb_beg = beg;
      sb_end = end;
      sb_pay = pay;
      big = false;
      has = false;
    }
    __syncthreads();
    const uint64_t b = sb_beg, e = sb_end;
    const Payload p = sb_pay;
    for (uint64_t x = b + tid; x < e; x += kBlock) emit(x, p);
    __syncthreads();
  }

  // Tier 2: wavefront-cooperative.
  for (;;) {
    const uint64_t mask = __ballot(has && (end - beg) >= (uint64_t)kWave);
    if (mask == 0) break;
    const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
    const uint64_t b = __shfl(beg, leader), e = __shfl(end, leader);
    const Payload p = __shfl(pay, leader);
    if (static_cast<int>(lane) == leader) has = false;
    for (uint64_t x = b + lane; x < e; x += kWave) emit(x, p);
  }

  // Tier 3: wave-wide prefix sum over the short lists.
  const uint32_t cnt = has ? static_cast<uint32_t>(end - beg) : 0u;
  uint32_t inc = cnt;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= static_cast<uint32_t>(o)) inc += t;
  }
  const uint32_t total = __shfl(inc, kWave - 1);
  const uint32_t wbase = tid & ~static_cast<uint32_t>(kWave - 1);
  s_beg[tid] = beg;
  s_ex[tid] = inc - cnt;
  s_pay[tid] = pay;
  __syncthreads();
  for (uint32_t k = 0; k < total; k += kWave) {
    const uint32_t j = k + lane;
    if (j < total) {
      int lo = 0, hi = kWave - 1;  // last lane L with s_ex[L] <= j
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_ex[wbase + mid] <= j) lo = mid;
        else hi = mid - 1;
      }
      emit(s_beg[wbase + lo] + (j - s_ex[wbase + lo]), s_pay[wbase + lo]);
    }
  }
  __syncthreads();
}

}  // namespace ipg
