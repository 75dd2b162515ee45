// common.h -- internal definitions shared by the library's HIP sources.
//
// Target: gfx950 (CDNA4), 64-lane wavefronts, 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ipregel.h"

namespace ipg {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kInf = 0xFFFFFFFFu;  // INF distance and identity of the min mailbox

// Pull tiling of the CSC: rows are grouped by the edge chunk of width
// kPullTile that contains their first in-edge; a group's edges are staged
// through LDS.  Rows with more than kPullTile in-edges get a workgroup each.
constexpr uint32_t kPullTile = 1024;

// ---------------------------------------------------------------- status --
void set_error(const std::string& msg);
ipg_status fail(ipg_status st, const std::string& msg);
ipg_status hip_fail(hipError_t e, const char* what);

#define IPG_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::ipg::hip_fail(e_, #call); \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves a caller-provided device workspace into 256-byte-aligned arrays.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    used = align_up(used, 256);
    T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
    used += count * sizeof(T);
    return p;
  }
};

// ---------------------------------------------------------- graph handle --
struct GraphTables {
  uint32_t* outdeg;     // [n] out-degree (u32)
  uint32_t* pull_rb;    // [nb+1] first CSC row of each pull row-group
  uint32_t* long_rows;  // [nl] rows with in-degree > kPullTile, ascending
  uint32_t* flags;      // [4] validation flags
};

}  // namespace ipg

struct ipg_graph {
  uint32_t n;
  uint64_t e;
  uint32_t flags;
  const uint64_t* csr_off;
  const int32_t* csr_dst;
  const uint64_t* csc_off;
  const int32_t* csc_src;
  const uint32_t* csr_w;
  const uint32_t* csc_w;
  ipg::GraphTables t;
  uint32_t nb;  // number of pull row-groups
  uint32_t nl;  // number of long rows
  int device;
  // last run
  int has_values;
  int last_app;
  const void* last_values;
};

namespace ipg {

// ------------------------------------------------------------ wave tools --
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Frontier compaction: every lane with `pred` appends `item` to `list`; one
// atomic per wave reserves the slots (ballot -> popcount -> atomicAdd by the
// lowest voting lane -> per-lane offset from mbcnt).  Safe in divergent code:
// only active lanes vote and the leader is always an active voter.
__device__ __forceinline__ void wave_append(bool pred, uint32_t item, uint32_t* list, uint32_t* counter) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(mask)) - 1);
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, static_cast<uint32_t>(__popcll(mask)));
  base = __shfl(base, static_cast<int>(leader));
  if (pred) list[base + lanes_below(mask)] = item;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
  unsigned long long v = x;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Block-wide sum of per-thread counters, then one atomicAdd per block.  Must
// be reached by every thread of the block.
__device__ __forceinline__ void block_add_u64(uint64_t x, unsigned long long* dst) {
  __shared__ uint64_t part[kWavesPerBlock];
  x = wave_sum_u64(x);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) part[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t s = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) s += part[i];
    if (s) atomicAdd(dst, static_cast<unsigned long long>(s));
  }
  __syncthreads();
}

// Per-superstep counters written by the kernels and read back by the host.
struct StepCounters {
  uint32_t next_count;           // vertices appended to the next frontier
  uint32_t overflow;             // an SSSP message would reach INF
  unsigned long long senders;    // vertices that broadcast
  unsigned long long messages;   // sum of senders' out-degrees
  unsigned long long examined;   // edges read by the exchange
  unsigned long long next_deg;   // sum of out-degrees of the next frontier
  unsigned long long pad[3];
};
static_assert(sizeof(StepCounters) == 64, "one cache line");

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v);
__global__ void fill_f64_kernel(double* p, uint64_t n, double v);
hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t fill_f64(double* p, uint64_t n, double v, hipStream_t s);

inline uint32_t grid_for(uint64_t items, uint32_t per_block = kBlock, uint32_t cap = 1u << 20) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<uint32_t>(g);
}

}  // namespace ipg
