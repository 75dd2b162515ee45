// common.h -- internal definitions shared by the library's HIP sources.
//
// Target: gfx950 (CDNA4), 64-lane wavefronts, 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ipregel.h"
#include "blocked_layout.h"

namespace ipg {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kInf = 0xFFFFFFFFu;  // INF distance and identity of the min mailbox

// Pull tiling of the CSC: rows are grouped by the edge chunk of width
// kPullTile that contains their first in-edge, so a group's in-edges (rows
// of at most kPullTile in-edges) span fewer than kWaveTile = 2*kPullTile
// edges and fit one wavefront's LDS tile.  Rows with more in-edges ("long
// rows") are cut into chunks of kWaveTile in-edges.
constexpr uint32_t kPullTile = 256;
constexpr uint32_t kWaveTile = 2 * kPullTile;

// A pull work item holds at most kItemRows rows (runs of vertices without
// in-edges would otherwise pile into one item).
constexpr uint32_t kItemRows = 64;

inline uint32_t num_pull_groups(uint64_t e) { return static_cast<uint32_t>(e / kPullTile + 1); }
// Rows with more than kPullTile in-edges: fewer than E / (kPullTile + 1) + 1.
inline uint64_t long_rows_cap(uint64_t e) { return e / (kPullTile + 1) + 1; }
// Chunks of the long rows: sum of ceil(deg / kWaveTile) <= E/kWaveTile + (long rows).
inline uint64_t chunks_cap(uint64_t e) { return e / kWaveTile + long_rows_cap(e) + 1; }
// Pull items: row pieces (at most groups + N / kItemRows) and long-row chunks.
inline uint64_t items_cap(uint32_t n, uint64_t e) { return num_pull_groups(e) + n / kItemRows + 1 + chunks_cap(e); }

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
// One unit of pull work for one wavefront: either rows [r0, r1) whose
// in-edges are [e0, e0 + ne) (fewer than kWaveTile edges, at most kItemRows
// rows), or chunk `slot` of a long row r0 (ne <= kWaveTile edges from e0).
struct PullItem {
  uint64_t e0;
  uint32_t ne;
  uint32_t r0;
  uint32_t r1;
  uint32_t slot;  // kNoSlot for a row item
};
static_assert(sizeof(PullItem) == 24, "packed item");
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

// Pull tiling of one CSC: device tables and their lengths.
struct TilingTables {
  uint32_t* pull_rb;    // [nb+1] first CSC row of each pull row-group
  uint32_t* long_rows;  // [nl] rows with in-degree > kPullTile, ascending
  uint32_t* lr_first;   // [nl+1] first chunk of each long row (chunks of kWaveTile in-edges)
  uint32_t* ch_row;     // [nc] index into long_rows of each chunk
  PullItem* items;      // [ni] pull work items: the nc chunks first, then the row pieces
  uint32_t nb, nl, nc, ni;
};

struct BlockedTables {
  uint32_t* edges;    // [e] packed edges (see above)
  BlkChunk* chunks;
  BlkSlice* slices;
  BlkGroup* groups;   // 64-row groups of the multi-slice blocks
  double* partial;    // partial sums of the multi-slice blocks
  uint32_t nchunks, nslices, ngroups;
  // binned cold sources (IPG_GRAPH_BINNED; hot == 0: none)
  double* slots;        // [nslots] one cold source's outbox per (block, source) pair
  uint16_t* bin_src;    // window lists: source offset of every slot
  BinRun* bin_runs;
  uint64_t* bin_wflat;  // [bin_nwin + 1]
  uint32_t* bin_wrun;   // [bin_nwin + 1]
  uint64_t* bin_wgroup; // [bin_nwin + 1]
  uint32_t* bin_group;
  BinUnit* bin_units;   // [bin_nunits] the bin launch's workgroups
  uint32_t hot, bin_w0, bin_nwin, bin_nunits;
  uint64_t nslots;
};

struct GraphTables {
  uint32_t* outdeg;     // [n] out-degree (u32)
  uint32_t* flags;      // [4] validation flags (+ a counter)
  TilingTables pull;    // tiling of the caller's CSC
  // Hot-first store (IPG_GRAPH_RENAME), else null: every vertex renamed by
  // descending out-degree, and the CSC rebuilt under the new names (rows in
  // the new order, each row's sources in their original order).
  uint32_t* perm;       // [n] new name of every vertex
  uint32_t* iperm;      // [n] the vertex of every new name
  uint32_t* outdeg_hot; // [n] out-degree by new name
  uint64_t* off_hot;    // [n+1] CSC offsets by new name
  int32_t* src_hot;     // [e] CSC sources, new names
  TilingTables pull_hot;
  // IPG_GRAPH_BLOCKED: the blocked in-edges of the CSC PageRank's pull uses
  // (the hot-first one when present), else edges == null; with a hot-first
  // store also those of the caller's CSC (blk_ids), for the CC/SSSP pull,
  // which works on the caller's vertex ids -- except on a symmetric store,
  // where CC and SSSP run under the new names on `blk` (min_space).
  BlockedTables blk;
  BlockedTables blk_ids;
};

// Pull-side view of the CSC handed to the gather kernels.  A launch has nc
// chunk workgroups (long rows, kPullTile in-edges each) followed by nb
// row-group workgroups.
struct PullTiling {
  const uint64_t* off;
  const int32_t* src;
  const uint32_t* rb;
  const uint32_t* long_rows;
  const uint32_t* lr_first;
  const uint32_t* ch_row;
  const PullItem* items;
  uint32_t nl, nc, nb, ni;
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
  int device;
  // last run
  int has_values;
  int last_app;
  const void* last_values;
  // PageRank superstep sequence captured as a hipGraph (IPG_RUN_GRAPH) and
  // the run it was captured for
  hipStream_t cap_stream;
  hipGraph_t pr_graph;
  hipGraphExec_t pr_exec;
  struct {
    uint32_t T;
    int push;
    const void* ws;
    const uint32_t* parts;
    uint32_t num_parts;
    uint32_t hot, grid, blocked;
    double damp;
  } pr_key;
  // HIP events reused by every run's timing (created on first use)
  std::vector<hipEvent_t> events;
  int wall_khz;  // device wall-clock rate, queried on first use (0 until then)
  uint32_t dd_steps[4];  // supersteps of the last device-driven run of each application (0: none yet)
  std::vector<uint32_t> perm_host;  // hot-first store: the new name of every vertex (host copy)
  void* mirror;      // pinned host block the decide kernels write (created on first use)
  void* mirror_dev;  // its device address
};

namespace ipg {

// ------------------------------------------------------------ wave tools --
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Bit v of a bitmap.
__device__ __forceinline__ bool bit_of(const uint32_t* bm, uint32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

// Set bit v of bitmap `bm` for every lane with `pred`, one atomic OR per
// distinct 32-bit word of the wavefront.  All 64 lanes must call it
// together (it reads other lanes' registers).
__device__ __forceinline__ void wave_set_bits(bool pred, uint32_t v, uint32_t* bm) {
  uint64_t pending = __ballot(pred);
  while (pending) {
    const int leader = __ffsll(static_cast<unsigned long long>(pending)) - 1;
    const uint32_t word = static_cast<uint32_t>(__shfl(static_cast<int>(v), leader)) >> 5;
    const bool mine = pred && (v >> 5) == word;
    uint32_t bits = mine ? (1u << (v & 31)) : 0u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) bits |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(bits), o));
    if (static_cast<int>(lane_id()) == leader) atomicOr(bm + word, bits);
    pending &= ~__ballot(mine);
  }
}

// Whether source u's row is to be read: always without a bitmap, else when
// its bit is set.
__device__ __forceinline__ bool row_live(const uint32_t* nz, int32_t u) {
  return nz == nullptr || ((nz[static_cast<uint32_t>(u) >> 5] >> (u & 31)) & 1u);
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

// Per-superstep counters.  Same-address device-scope atomics serialize
// device-wide (about 11 ns each on MI355X), so every workgroup adds into one
// of kCtrSlots slots (its own 128-byte line, chosen by blockIdx % kCtrSlots)
// and the host sums the slots.
constexpr int kCtrSlots = 64;
struct alignas(128) CtrSlot {
  uint32_t next_count;          // vertices with a message for the next superstep
  uint32_t overflow;            // an SSSP message would reach INF
  unsigned long long senders;   // vertices that broadcast
  unsigned long long messages;  // sum of the senders' out-degrees
  unsigned long long next_deg;  // sum of out-degrees of the next frontier
  unsigned long long active;    // (batched SSSP) query-vertex pairs that received a message
  uint32_t list_len;            // (push) recipients appended to this slot's segment of the next-frontier list
  uint32_t pieces;              // (push) pieces queued in this slot's segment of the piece queue
  unsigned long long pad[10];
};
static_assert(sizeof(CtrSlot) == 128, "one slot per 128-byte line");

// Host-side sum of the slots of one superstep.
struct StepCounters {
  uint64_t next_count, senders, messages, next_deg;
  uint32_t overflow;
};

__device__ __forceinline__ CtrSlot* my_slot(CtrSlot* base) { return base + (blockIdx.x % kCtrSlots); }

// Zero the kCtrSlots slots at `c` (called by workgroup 0 only).
__device__ __forceinline__ void clear_slots(CtrSlot* c) {
  if (c && blockIdx.x == 0) {
    uint32_t* w = reinterpret_cast<uint32_t*>(c);
    for (uint32_t i = threadIdx.x; i < kCtrSlots * sizeof(CtrSlot) / 4; i += blockDim.x) w[i] = 0;
  }
}

// Workgroup-wide sum of per-thread counters, then at most one atomic per
// non-zero field into the workgroup's slot.  Every thread must call it.
__device__ __forceinline__ void flush_counters(CtrSlot* base, uint64_t senders, uint64_t messages, uint64_t next_count,
                                               uint64_t next_deg, uint32_t overflow, uint64_t active = 0) {
  __shared__ unsigned long long part[5][kWavesPerBlock];
  __shared__ uint32_t ovf;
  if (threadIdx.x == 0) ovf = 0;
  senders = wave_sum_u64(senders);
  messages = wave_sum_u64(messages);
  next_count = wave_sum_u64(next_count);
  next_deg = wave_sum_u64(next_deg);
  active = wave_sum_u64(active);
  const bool any_ovf = __ballot(overflow != 0) != 0;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    part[0][w] = senders;
    part[1][w] = messages;
    part[2][w] = next_count;
    part[3][w] = next_deg;
    part[4][w] = active;
    if (any_ovf) ovf = 1;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    unsigned long long t = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) t += part[threadIdx.x][i];
    CtrSlot* c = my_slot(base);
    if (t) {
      if (threadIdx.x == 0) atomicAdd(&c->senders, t);
      if (threadIdx.x == 1) atomicAdd(&c->messages, t);
      if (threadIdx.x == 2) atomicAdd(&c->next_count, static_cast<uint32_t>(t));
      if (threadIdx.x == 3) atomicAdd(&c->next_deg, t);
      if (threadIdx.x == 4) atomicAdd(&c->active, t);
    }
    if (threadIdx.x == 0 && ovf) atomicOr(&c->overflow, 1u);
  }
  __syncthreads();
}

// Fixed grid for the grid-stride exchange kernels: enough resident
// workgroups to cover the chip (256 CUs) several times over, few enough that
// per-workgroup counter flushes stay cheap.
constexpr uint32_t kExchangeGrid = 4096;
// Grid of the pull item kernels: 8 resident workgroups (32 wavefronts, each
// working on its own items) on each of 256 CUs.
constexpr uint32_t kPullGrid = 2048;

// Wavefront-local LDS ordering: make this lane's LDS writes visible to the
// other lanes of its wavefront (LDS operations of one wavefront execute in
// order; this also stops the compiler from moving LDS accesses across it).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
