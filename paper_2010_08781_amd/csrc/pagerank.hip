// pagerank.hip -- PageRank (Fig. 8) on the superstep engine, FP64.
//
// Superstep 0 sets every rank to 1/N; superstep s >= 1 sets
//   rank(v) = (1 - d)/N + d * (sum of the messages v received),
// with the damping d a run parameter (0.85 in Fig. 8), and while s < T every
// vertex broadcasts rank / out-degree (a vertex without out-edges reaches
// nobody).  At s = T all vertices halt.  Messages are combined by '+=' (the
// sum combiner of Fig. 8).
//
// Every kernel that runs compute on a vertex counts it (active), and, when
// the vertex broadcasts, counts it as a sender and adds its out-degree
// (messages): the trace of the run is counted on the device (PrTrace).
//
// Pull form (Section 4.3.2): a broadcast writes one outbox value per vertex,
// contrib(u) = rank(u)/outdeg(u) (0 when outdeg is 0), and every vertex
// reduces the outboxes of its in-neighbours over the CSC.  Race-free, and the
// summation order is fixed, so results are bitwise reproducible.
//
// Push form: every vertex adds its contribution into its out-neighbours'
// one-slot mailboxes with FP64 atomic adds (the lock-free combiner the paper
// lists as future work, Section 4.3.2 and Section 9); summation order varies
// from run to run within rounding.
#include <algorithm>
#include <vector>

#include "common.h"
#include "blocked.h"
#include "engine.h"
#include "scatter.h"

namespace ipg {

// Per-superstep counts of a PageRank run (PrCntSlot): the first launch of
// superstep s + 1 (and a one-wavefront launch after the last superstep)
// folds the slots of superstep s into record s and clears them; the slot
// sets alternate by superstep parity.
static_assert(kCtrSlots == kWave, "one slot per lane of the folding wavefront");
struct PrTrace {
  PrCntSlot* add;            // the slots this superstep's kernels add into
  PrCntSlot* fold;           // the previous superstep's slots, or null (superstep 0)
  unsigned long long* rec;   // [kPrTraceCap][3]: active, senders, messages
  uint32_t fold_step;        // the superstep whose slots `fold` holds
};

// Per-thread counts of the vertices a thread finished.
struct PrTally {
  unsigned long long rows = 0, senders = 0, messages = 0;
};

// Workgroup 0, wavefront 0: record superstep t.fold_step and clear its slots.
// Called at the start of a kernel; no barrier (the slots it reads and
// clears are not those the kernel adds into).
__device__ __forceinline__ void pr_trace_fold(const PrTrace& t) {
  if (!t.fold || blockIdx.x != 0 || threadIdx.x >= kWave) return;
  PrCntSlot* sl = t.fold + threadIdx.x;
  unsigned long long a = sl->active, b = sl->senders, c = sl->messages;
  sl->active = 0;
  sl->senders = 0;
  sl->messages = 0;
  a = wave_sum_u64(a);
  b = wave_sum_u64(b);
  c = wave_sum_u64(c);
  if (threadIdx.x == 0 && t.fold_step < kPrTraceCap) {
    t.rec[3 * t.fold_step + 0] = a;
    t.rec[3 * t.fold_step + 1] = b;
    t.rec[3 * t.fold_step + 2] = c;
  }
}

// Workgroup sum of the threads' tallies added to the workgroup's slot
// (every thread must call; at most 1024 threads).
__device__ __forceinline__ void pr_tally_flush(const PrTrace& t, const PrTally& x) {
  __shared__ unsigned long long part[3][1024 / kWave];
  const unsigned long long a = wave_sum_u64(x.rows), b = wave_sum_u64(x.senders), c = wave_sum_u64(x.messages);
  const uint32_t w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    part[0][w] = a;
    part[1][w] = b;
    part[2][w] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long sum = 0;
    for (uint32_t i = 0; i < blockDim.x / kWave; ++i) sum += part[threadIdx.x][i];
    PrCntSlot* sl = t.add + (blockIdx.x % kCtrSlots);
    if (sum) atomicAdd(threadIdx.x == 0 ? &sl->active : threadIdx.x == 1 ? &sl->senders : &sl->messages, sum);
  }
}

// Folds the slots of the last superstep of a run (one wavefront).
__global__ void pr_trace_last_kernel(PrTrace t) { pr_trace_fold(t); }

struct PrPullArgs {
  PullTiling t;
  const uint32_t* outdeg;
  const double* contrib_in;
  double* contrib_out;
  double* value;
  double* partial;        // per long-row chunk
  double ratio;           // (1 - d) / N
  double damp;            // d
  double teleport;        // 1 - d (divided by the part's vertex count with part_n)
  const uint32_t* part_n; // vertex count of each vertex's part, or null (one part)
  PrTrace tr;
  double* l1;             // convergence run: rank stored every update, its L1 change added here (else null)
  int last;               // superstep == T: store the rank, no broadcast
};

// Counts of a vertex that ran compute, and broadcast unless `last`.
__device__ __forceinline__ void pr_tally(PrTally& t, int last, uint32_t d) {
  ++t.rows;
  if (!last) {
    ++t.senders;
    t.messages += d;
  }
}

// The rank of v after this update: the outbox for the next update, the
// stored rank when this is the last update, and both (plus the change of
// the rank) in a convergence run.
__device__ __forceinline__ void pr_store(const PrPullArgs& a, uint32_t v, double rank, uint32_t d, double& l1,
                                         PrTally& tl) {
  pr_tally(tl, a.last, d);
  if (a.l1) {
    l1 += fabs(rank - a.value[v]);
    a.value[v] = rank;
  } else if (a.last) {
    a.value[v] = rank;
    return;
  }
  a.contrib_out[v] = d ? rank / static_cast<double>(d) : 0.0;
}

// Workgroup sum of the threads' L1 changes added to one of kCtrSlots
// 128-byte slots (every thread must call).
__device__ __forceinline__ void flush_l1(double* slots, double x) {
  __shared__ double part[1024 / kWave];
  x = wave_sum(x);
  if (lane_id() == 0) part[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (uint32_t i = 0; i < blockDim.x / kWave; ++i) t += part[i];
    if (t != 0.0) unsafeAtomicAdd(slots + (blockIdx.x % kCtrSlots) * 16, t);
  }
}

// (1 - d) / N for the part that holds v.
__device__ __forceinline__ double pr_ratio(double ratio, double teleport, const uint32_t* part_n, uint32_t v) {
  return part_n ? teleport / static_cast<double>(part_n[v]) : ratio;
}

__device__ __forceinline__ void pr_finish(const PrPullArgs& a, uint32_t v, double sum, double& l1, PrTally& tl) {
  const double rank = pr_ratio(a.ratio, a.teleport, a.part_n, v) + a.damp * sum;
  pr_store(a, v, rank, a.outdeg[v], l1, tl);
}

// One pull item held in registers ahead of its gathers: its metadata, its
// CSC sources and, for a row item, the in-edge offsets and out-degrees of
// its rows.
struct ItemRegs {
  PullItem it;
  uint32_t ne;       // edges of the item (<= kWaveTile)
  uint32_t nrows;    // rows of a row item, 0 for a long-row chunk
  int32_t u[kWaveTile / kWave];
  uint32_t off_lane; // low word of the CSC offset of row min(lane, nrows)
  uint32_t off_end;  // low word of the CSC offset of row nrows (the item's end)
  uint32_t deg;      // out-degree of row `lane` (lane < nrows)
};
static_assert(kItemRows == kWave, "one row per lane");

__device__ __forceinline__ PullItem no_item() {
  PullItem it;
  it.e0 = 0;
  it.ne = 0;
  it.r0 = it.r1 = 0;
  it.slot = kNoSlot;
  return it;
}

// Every load is unconditional, from an index clamped into the item (an item
// without edges reads a dummy word of the item table), so that no lane
// branches around a load: a load under a branch is followed by a wait for
// every load before it, the gathers of the previous item included.  Every
// item has r0 < N (row items hold at least one row, a chunk names its long
// row), so the clamped row indices are in range.
__device__ __forceinline__ void load_item(const PrPullArgs& a, const PullItem& it, ItemRegs& R) {
  constexpr int kPer = kWaveTile / kWave;
  const uint32_t lane = lane_id();
  R.it = it;
  R.ne = it.ne < kWaveTile ? it.ne : kWaveTile;  // ne > kWaveTile only with bad offsets
  R.nrows = it.slot != kNoSlot ? 0 : it.r1 - it.r0;
  const int32_t* base = R.ne ? a.t.src + it.e0 : reinterpret_cast<const int32_t*>(a.t.items);
  const uint32_t last = R.ne ? R.ne - 1 : 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t i = lane + k * kWave;
    R.u[k] = __builtin_nontemporal_load(base + (i < last ? i : last));
  }
  R.off_lane = static_cast<uint32_t>(a.t.off[it.r0 + (lane < R.nrows ? lane : R.nrows)]);
  R.off_end = static_cast<uint32_t>(a.t.off[it.r0 + R.nrows]);
  R.deg = a.outdeg[it.r0 + (lane < R.nrows ? lane : 0)];
}

// Pull superstep, first launch.  Every wavefront works through its own pull
// items (grid-stride over wavefronts), with its own LDS tile and no
// workgroup barrier.  The item loop is software-pipelined so that one
// memory round trip per item is exposed instead of three: while the
// outboxes of item i are gathered, the CSC sources, row offsets and
// out-degrees of item i+1 and the metadata of item i+2 are in flight.
//  * row item: the gathered outboxes are staged in LDS and each row is
//    summed by G lanes (G from the item's row count), then finished here;
//  * long-row chunk: a fixed-order wavefront sum stored as the chunk's
//    partial (added up by the second launch).
// With a hot cache (hot > 0, hot-first store) the workgroup first copies the
// outbox entries of the `hot` most-read sources -- names 0 .. hot-1 -- into
// LDS, and gathers from those sources read LDS instead of the memory
// hierarchy (the L1 miss rate of the random gathers is the bound).
template <int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void pr_items_kernel(PrPullArgs a, uint32_t hot) {
  constexpr int kPer = kWaveTile / kWave;
  constexpr uint32_t kThreads = WAVES * kWave;
  constexpr int kHotBatch = 12;  // outbox loads in flight per thread while the cache fills
  __shared__ double s_tile[WAVES][kWaveTile];
  __shared__ uint32_t s_off[WAVES][kItemRows + 1];
  __shared__ uint32_t s_deg[WAVES][kItemRows];
  extern __shared__ double s_hot[];
  pr_trace_fold(a.tr);
  const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
  double* tile = s_tile[wv];
  uint32_t* soff = s_off[wv];
  uint32_t* sdeg = s_deg[wv];
  const uint64_t ni = a.t.ni, nw = static_cast<uint64_t>(gridDim.x) * WAVES;
  uint64_t item = static_cast<uint64_t>(blockIdx.x) * WAVES + wv;
  PullItem m_next = item + nw < ni ? a.t.items[item + nw] : no_item();
  ItemRegs cur;
  load_item(a, item < ni ? a.t.items[item] : no_item(), cur);
  if (hot) {
    for (uint32_t b = 0; b < hot; b += kHotBatch * kThreads) {
      double h[kHotBatch];
#pragma unroll
      for (int k = 0; k < kHotBatch; ++k) {
        const uint32_t i = b + threadIdx.x + k * kThreads;
        h[k] = i < hot ? a.contrib_in[i] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kHotBatch; ++k) {
        const uint32_t i = b + threadIdx.x + k * kThreads;
        if (i < hot) s_hot[i] = h[k];
      }
    }
    __syncthreads();
  }
  double l1 = 0.0;
  PrTally tl;
  for (; item < ni; item += nw) {
    const PullItem m2 = item + 2 * nw < ni ? a.t.items[item + 2 * nw] : no_item();
    // Cold sources are gathered from memory and hot ones from LDS into
    // separate registers, merged only where the values are used: a shared
    // destination register would make every LDS read wait for all the
    // gathers before it.
    double xg[kPer], xh[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t uk = static_cast<uint32_t>(cur.u[k]);
      xg[k] = 0.0;
      if (cur.ne && uk >= hot) xg[k] = a.contrib_in[uk];
    }
    if (hot) {
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const uint32_t uk = static_cast<uint32_t>(cur.u[k]);
        xh[k] = s_hot[uk < hot ? uk : 0];
      }
    }
    ItemRegs nxt;
    load_item(a, m_next, nxt);
    double x[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) x[k] = static_cast<uint32_t>(cur.u[k]) < hot ? xh[k] : xg[k];
    if (cur.nrows == 0) {  // long-row chunk
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (lane + k * kWave < cur.ne) s += x[k];
      s = wave_sum(s);
      if (lane == 0 && cur.it.slot != kNoSlot) a.partial[cur.it.slot] = s;
    } else {
      const uint32_t nrows = cur.nrows, ne = cur.ne, e0 = static_cast<uint32_t>(cur.it.e0);
      if (lane < nrows) {  // offsets relative to the item: differences of the low words
        soff[lane] = cur.off_lane - e0;
        sdeg[lane] = cur.deg;
      }
      if (lane == 0) soff[nrows] = cur.off_end - e0;
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const uint32_t i = lane + k * kWave;
        if (i < ne) tile[i] = x[k];
      }
      wave_lds_sync();
      uint32_t G = kWave;
      while (G > 1 && G * nrows > kWave) G >>= 1;
      const uint32_t groups = kWave / G, gi = lane / G, li = lane % G;
      for (uint32_t rb = 0; rb < nrows; rb += groups) {
        const uint32_t row = rb + gi;
        double s = 0.0;
        if (row < nrows) {
          uint32_t lo = soff[row], hi = soff[row + 1];
          if (hi > ne) hi = ne;
          for (uint32_t j = lo + li; j < hi; j += G) s += tile[j];
        }
        for (uint32_t o = G >> 1; o >= 1; o >>= 1) s += __shfl_xor(s, static_cast<int>(o));
        if (li == 0 && row < nrows) {
          const uint32_t v = cur.it.r0 + row;
          const double rank = pr_ratio(a.ratio, a.teleport, a.part_n, v) + a.damp * s;
          pr_store(a, v, rank, sdeg[row], l1, tl);
        }
      }
      wave_lds_sync();  // the tile is rewritten by the next item
    }
    cur = nxt;
    m_next = m2;
  }
  if (a.l1) flush_l1(a.l1, l1);
  pr_tally_flush(a.tr, tl);
}

// What finishing a row reads besides its sum: loaded for a batch of rows
// before any is finished, so that the loads are in flight together.
struct RowIn {
  uint32_t deg;   // out-degree
  uint32_t pn;    // vertex count of the row's part (part_n), else 0
  double old;     // previous rank (convergence run), else 0
};
__device__ __forceinline__ RowIn pr_row_load(const PrPullArgs& a, uint32_t v) {
  RowIn in;
  in.deg = a.outdeg[v];
  in.pn = a.part_n ? a.part_n[v] : 0u;
  in.old = a.l1 ? a.value[v] : 0.0;
  return in;
}
// pr_finish with the row's inputs already loaded.
__device__ __forceinline__ void pr_row_finish(const PrPullArgs& a, uint32_t v, double sum, const RowIn& in, double& l1,
                                              PrTally& tl) {
  const double ratio = a.part_n ? a.teleport / static_cast<double>(in.pn) : a.ratio;
  const double rank = ratio + a.damp * sum;
  pr_tally(tl, a.last, in.deg);
  if (a.l1) {
    l1 += fabs(rank - in.old);
    a.value[v] = rank;
  } else if (a.last) {
    a.value[v] = rank;
    return;
  }
  a.contrib_out[v] = in.deg ? rank / static_cast<double>(in.deg) : 0.0;
}

// Pull superstep, second launch: each long row adds its chunk partials in
// chunk order (one wavefront per row; a fixed order, so results are
// bitwise reproducible).
__global__ __launch_bounds__(kBlock) void pr_longrow_kernel(PrPullArgs a) {
  pr_trace_fold(a.tr);
  const uint32_t l = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  double l1 = 0.0;
  PrTally tl;
  if (l < a.t.nl) {  // wave-uniform
    const uint32_t f = a.t.lr_first[l], nch = a.t.lr_first[l + 1] - f;
    double s = 0.0;
    for (uint32_t i = lane_id(); i < nch; i += kWave) s += a.partial[f + i];
    s = wave_sum(s);
    if (lane_id() == 0) pr_finish(a, a.t.long_rows[l], s, l1, tl);
  }
  if (a.l1) flush_l1(a.l1, l1);
  pr_tally_flush(a.tr, tl);
}

// Blocked pull (IPG_GRAPH_BLOCKED): the in-edges of each block of at most
// kBlkRows destinations, sorted by source, streamed through one workgroup
// per slice (blocked.h).
struct PrBlkArgs {
  BlkView v;
  const double* slots;  // binned cold sources' outboxes, one per (block, source) pair (null: no binning)
  uint32_t n;
};

// Bin launch of the binned layout (IPG_GRAPH_BINNED): every cold source's
// outbox copied into its slots (bin_unit).
__global__ __launch_bounds__(kBlkThreads) void pr_bin_kernel(const double* contrib, uint32_t n, BinTables bv,
                                                             double* slots) {
  bin_unit<double>(bv, slots, n, [&](uint32_t u) { return contrib[u]; });
}

// Blocked pull, first launch: workgroup = slice.  The block's sums start at
// zero in LDS; the workgroup streams the slice's chunks, adding each edge's
// outbox into its destination's sum with an LDS atomic.  A block's only
// slice then finishes the block's vertices; a slice of a larger block
// stores its sums as a partial.
__global__ __launch_bounds__(kBlkThreads) void pr_blocked_kernel(PrPullArgs a, PrBlkArgs b) {
  // + one pad slot per lane (see blk_stream)
  __shared__ double part[kBlkRows + kWave];
  pr_trace_fold(a.tr);
  const BlkSlice sl = b.v.slices[blockIdx.x];
  for (uint32_t r = threadIdx.x; r < sl.rows; r += kBlkThreads) part[r] = 0.0;
  if (threadIdx.x < kWave) part[kBlkRows + threadIdx.x] = 0.0;
  __syncthreads();
  const double* contrib = a.contrib_in;
  const double* slots = b.slots;
  blk_stream<double>(
      b.v, sl, 0.0,
      [&](uint32_t wbase, uint32_t q, uint32_t cold) {
        return (cold ? slots : contrib)[static_cast<uint64_t>(wbase) + (q >> 16)];
      },
      [&](uint32_t slot, double x) { atomicAdd(&part[slot], x); });
  __syncthreads();
  const uint32_t r0 = sl.row0, rows = sl.rows;
  double l1 = 0.0;
  PrTally tl;
  if (sl.poff == kNoPartial) {
    // rows in batches of kFinBatch per thread, every batch's inputs loaded
    // first (indices clamped into the block: the loads are unconditional)
    constexpr uint32_t kFinBatch = 5;
    for (uint32_t r = threadIdx.x; r < rows; r += kFinBatch * kBlkThreads) {
      RowIn in[kFinBatch];
#pragma unroll
      for (uint32_t j = 0; j < kFinBatch; ++j) {
        const uint32_t rj = r + j * kBlkThreads;
        in[j] = pr_row_load(a, r0 + (rj < rows ? rj : rows - 1));
      }
#pragma unroll
      for (uint32_t j = 0; j < kFinBatch; ++j) {
        const uint32_t rj = r + j * kBlkThreads;
        if (rj < rows) pr_row_finish(a, r0 + rj, part[rj], in[j], l1, tl);
      }
    }
  } else {
    double* dst = static_cast<double*>(b.v.partial) + sl.poff;
    for (uint32_t r = threadIdx.x; r < rows; r += kBlkThreads) dst[r] = part[r];
  }
  if (a.l1) flush_l1(a.l1, l1);
  pr_tally_flush(a.tr, tl);
}

// Blocked pull, second launch: the rows of every block with several slices
// add the slices' partial sums in slice order (and the rows of blocks
// without in-edges, with no partials, get 0.15/N).  A wavefront takes one group
// of 64 rows at a time (lane = row): one record load, then every partial
// (eight at a time) and the row's inputs in flight together.
__global__ __launch_bounds__(kBlock) void pr_blocked_finish_kernel(PrPullArgs a, PrBlkArgs b) {
  pr_trace_fold(a.tr);
  const uint32_t lane = lane_id();
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  double l1 = 0.0;
  PrTally tl;
  for (uint32_t w = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; w < b.v.ngroups; w += nw) {  // wave-uniform
    const BlkGroup gr = b.v.groups[w];
    const uint32_t rr = lane < gr.nrows ? lane : gr.nrows - 1;
    const RowIn in = pr_row_load(a, gr.row0 + rr);
    const double* p = static_cast<const double*>(b.v.partial) + gr.poff + rr;
    double sum = 0.0;
    for (uint32_t k = 0; k < gr.k; k += 8) {
      double x[8];
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        const uint32_t kk = k + j < gr.k ? k + j : gr.k - 1;
        x[j] = p[static_cast<uint64_t>(kk) * gr.stride];
      }
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j)
        if (k + j < gr.k) sum += x[j];
    }
    if (lane < gr.nrows) pr_row_finish(a, gr.row0 + lane, sum, in, l1, tl);
  }
  if (a.l1) flush_l1(a.l1, l1);
  pr_tally_flush(a.tr, tl);
}

// 1 / N for the part that holds v.
__device__ __forceinline__ double pr_init(double init, const uint32_t* part_n, uint32_t v) {
  return part_n ? 1.0 / static_cast<double>(part_n[v]) : init;
}

// Superstep 0 of the pull form: rank 1/N, outbox 1/N/outdeg (and the rank
// itself when a convergence run tracks its changes).
__global__ __launch_bounds__(kBlock) void pr_pull_init_kernel(uint32_t n, const uint32_t* outdeg, double init,
                                                               const uint32_t* part_n, double* contrib, double* value,
                                                               int last, int track, PrTrace tr) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  PrTally tl;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const double x = pr_init(init, part_n, static_cast<uint32_t>(v));
    if (last || track) value[v] = x;
    const uint32_t d = outdeg[v];
    pr_tally(tl, last, d);
    if (!last) contrib[v] = d ? x / static_cast<double>(d) : 0.0;
  }
  pr_tally_flush(tr, tl);
}

// Vertex count of the part of every vertex: part p holds [off[p], off[p+1]);
// stored under the vertex's hot-first name when `perm` is given.
__global__ void pr_part_n_kernel(const uint32_t* off, uint32_t parts, uint32_t n, const uint32_t* perm,
                                 uint32_t* part_n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    uint32_t lo = 0, hi = parts - 1;  // last part p with off[p] <= v
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= v) lo = mid;
      else hi = mid - 1;
    }
    part_n[perm ? perm[v] : v] = off[lo + 1] - off[lo];
  }
}

// Ranks back to the caller's vertex ids: value[v] = value_hot[perm[v]].
__global__ void pr_unrename_kernel(const double* value_hot, const uint32_t* perm, uint32_t n, double* value) {
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
    value[v] = value_hot[perm[v]];
}

struct PrPushArgs {
  uint32_t n;
  const uint64_t* off;   // CSR offsets
  const int32_t* dst;    // CSR destinations
  double* mail_in;       // consumed and reset to 0.0
  double* mail_out;      // atomically accumulated
  double* value;
  double ratio, init;
  double damp, teleport; // d and 1 - d
  const uint32_t* part_n;
  PrTrace tr;
  double* l1;            // convergence run: rank stored every superstep, its L1 change added here
  int first, last;
  PrPiece* pieces;       // piece queue (see kPieceMin)
  uint64_t piece_seg;
  CtrSlot* ctr;          // this superstep's slots (piece counts)
  CtrSlot* ctr_clear;    // the next superstep's, cleared here
};

// Queue the out-edges of this wavefront's senders that have at least
// kPieceMin of them as pieces in the workgroup's segment (one atomic per
// wavefront, on the slot's counter); returns whether the lane still expands
// its sender itself (also when the segment is full: its entries are then
// marked unused).  All lanes of the wavefront call it together.
__device__ __forceinline__ bool pr_queue_pieces(const PrPushArgs& a, bool has, uint64_t beg, uint64_t end, double c) {
  const uint64_t d = has ? end - beg : 0;
  const uint32_t np = d >= kPieceMin ? static_cast<uint32_t>((d + kPiece - 1) / kPiece) : 0u;
  if (__ballot(np != 0) == 0) return has;  // uniform
  const uint32_t lane = lane_id();
  uint32_t inc = np;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= static_cast<uint32_t>(o)) inc += t;
  }
  const uint32_t total = __shfl(inc, kWave - 1);
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(&my_slot(a.ctr)->pieces, total);
  base = __shfl(base, 0);
  if (np == 0) return has;
  const uint64_t first = static_cast<uint64_t>(base) + (inc - np);
  const bool fits = first + np <= a.piece_seg;
  PrPiece* seg = a.pieces + static_cast<uint64_t>(blockIdx.x % kCtrSlots) * a.piece_seg;
  for (uint32_t k = 0; k < np && first + k < a.piece_seg; ++k) {
    const uint64_t b = beg + static_cast<uint64_t>(k) * kPiece;
    PrPiece p;
    p.beg = b;
    p.n = fits ? static_cast<uint32_t>(min(static_cast<uint64_t>(kPiece), end - b)) : 0u;
    p.pad = 0;
    p.c = c;
    seg[first + k] = p;
  }
  return !fits;
}

// Fused compute + push for one superstep: every vertex consumes its mailbox,
// updates its rank and (unless last) adds rank/outdeg into each
// out-neighbour's next mailbox.
__global__ __launch_bounds__(kBlock) void pr_push_kernel(PrPushArgs a) {
  clear_slots(a.ctr_clear);
  pr_trace_fold(a.tr);
  const uint64_t v = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
  double l1 = 0.0;
  PrTally tl;
  bool has = false;
  uint64_t beg = 0, end = 0;
  double c = 0.0;
  if (v < a.n) {
    double rank;
    if (a.first) {
      rank = pr_init(a.init, a.part_n, static_cast<uint32_t>(v));
    } else {
      const double m = a.mail_in[v];
      a.mail_in[v] = 0.0;
      rank = pr_ratio(a.ratio, a.teleport, a.part_n, static_cast<uint32_t>(v)) + a.damp * m;
      if (a.l1) l1 += fabs(rank - a.value[v]);
    }
    if (a.last || a.l1) a.value[v] = rank;
    beg = a.off[v];
    end = a.off[v + 1];
    pr_tally(tl, a.last, static_cast<uint32_t>(end - beg));
    if (!a.last) {
      has = end > beg;
      if (has) c = rank / static_cast<double>(end - beg);
    }
  }
  if (!a.last) has = pr_queue_pieces(a, has, beg, end, c);  // uniform condition
  double* mail = a.mail_out;
  const int32_t* dst = a.dst;
  twc_scatter(has, beg, end, c, [&](uint64_t e, double p) { unsafeAtomicAdd(mail + dst[e], p); });
  if (a.l1) flush_l1(a.l1, l1);
  pr_tally_flush(a.tr, tl);
}

// Second launch of a push superstep: the queued pieces dealt over the grid
// (piece g, counted over the segments in slot order, to workgroup
// g mod grid), kPiece / kBlock edges per thread with their loads issued
// together.
__global__ __launch_bounds__(kBlock) void pr_push_piece_kernel(PrPushArgs a) {
  __shared__ uint32_t s_pre[kCtrSlots + 1];
  if (threadIdx.x < kWave) {  // prefix of the segments' lengths (one wavefront)
    const uint32_t lane = lane_id();
    const uint32_t cnt = static_cast<uint32_t>(min(static_cast<uint64_t>(a.ctr[lane].pieces), a.piece_seg));
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(inc, o);
      if (lane >= static_cast<uint32_t>(o)) inc += t;
    }
    s_pre[lane + 1] = inc;
    if (lane == 0) s_pre[0] = 0;
  }
  __syncthreads();
  const uint32_t total = s_pre[kCtrSlots];
  double* mail = a.mail_out;
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {  // uniform over the workgroup
    uint32_t lo = 0, hi = kCtrSlots - 1;  // the last segment k with s_pre[k] <= g
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    const PrPiece pc = a.pieces[static_cast<uint64_t>(lo) * a.piece_seg + (g - s_pre[lo])];
    constexpr int kPer = kPiece / kBlock;
    uint32_t x[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t j = threadIdx.x + k * kBlock;
      x[k] = j < pc.n ? static_cast<uint32_t>(a.dst[pc.beg + j]) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (threadIdx.x + k * kBlock < pc.n) unsafeAtomicAdd(mail + x[k], pc.c);
  }
}

// Grid of the piece launch.
constexpr uint32_t kPrPieceGrid = 2048;

// One push superstep: the compute + scatter launch, then (unless it is the
// last, which sends nothing) the piece launch.  The counter slots
// alternate by superstep parity; each superstep clears the next one's.
static hipError_t launch_pr_push(PrPushArgs a, const RunWs& w, uint64_t e, uint32_t grid, uint32_t step,
                                 hipStream_t s) {
  a.pieces = w.pr_pieces;
  a.piece_seg = piece_seg(e);
  a.ctr = w.ctr + (step & 1) * kCtrSlots;
  a.ctr_clear = w.ctr + ((step + 1) & 1) * kCtrSlots;
  hipLaunchKernelGGL(pr_push_kernel, dim3(grid), dim3(kBlock), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || a.last) return err;
  hipLaunchKernelGGL(pr_push_piece_kernel, dim3(kPrPieceGrid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ host --

// First launch of a pull superstep: the hot-cache form (16-wavefront
// workgroups, one per CU with the cache in LDS) on a hot-first store, else
// the plain form.
// Largest LDS outbox cache of the 16-wavefront form: the device's LDS per
// workgroup minus the kernel's static tiles (a larger request is rejected
// by the runtime when the kernel is dispatched).  Queried once.
static hipError_t max_hot_entries(uint32_t* out) {
  static uint32_t cached = 0;
  if (!cached) {
    hipFuncAttributes attr;
    hipError_t err = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&pr_items_kernel<16>));
    if (err != hipSuccess) return err;
    int dev = 0, lds = 0;
    if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
    if ((err = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return err;
    const size_t room = static_cast<size_t>(lds) > attr.sharedSizeBytes ? lds - attr.sharedSizeBytes : 0;
    cached = static_cast<uint32_t>(room / sizeof(double)) & ~63u;
    if (!cached) cached = 1;  // no room: caching is off (see below)
  }
  *out = cached;
  return hipSuccess;
}

static hipError_t launch_pr_items(const PrPullArgs& a, bool renamed, const Tune& tn, uint32_t n, hipStream_t s) {
  if (!a.t.ni) return hipSuccess;
  uint32_t room = 0;
  hipError_t err = max_hot_entries(&room);
  if (err != hipSuccess) return err;
  uint32_t hot = renamed ? std::min(std::min(tn.pr_hot, n), room) : 0;
  if (hot < 64) hot = 0;
  if (hot) {
    constexpr int kW = 16;
    const uint32_t grid = std::min(a.t.ni, tn.pull_grid / 8 ? tn.pull_grid / 8 : 1u);
    hipLaunchKernelGGL(pr_items_kernel<kW>, dim3(grid), dim3(kW * kWave), hot * sizeof(double), s, a, hot);
  } else {
    hipLaunchKernelGGL(pr_items_kernel<kWavesPerBlock>, dim3(std::min(a.t.ni, tn.pull_grid)), dim3(kBlock), 0, s, a,
                       0u);
  }
  return hipGetLastError();
}

// What PageRank's pull form runs on: the hot-first store when the graph
// has one (every per-vertex array of the pull supersteps is then indexed by
// the new names, and the ranks are mapped back after the last update), else
// the caller's CSC.
struct PrPullStore {
  PullTiling t;
  const uint32_t* outdeg;
  const uint32_t* perm;  // null: no renaming
  double* value;         // ranks as the supersteps store them
  const BlockedTables* blk;  // blocked in-edges of the same CSC, or null
};
static PrPullStore pr_store_of(const ipg_graph* g, const RunWs& w) {
  PrPullStore p;
  if (g->t.perm) {
    p.t = make_tiling(g->t.off_hot, g->t.src_hot, g->t.pull_hot);
    p.outdeg = g->t.outdeg_hot;
    p.perm = g->t.perm;
    p.value = w.value_hot;
  } else {
    p.t = pull_tiling(g);
    p.outdeg = g->t.outdeg;
    p.perm = nullptr;
    p.value = w.value_f64;
  }
  p.blk = g->t.blk.edges ? &g->t.blk : nullptr;
  return p;
}

// One pull superstep: the blocked launches when the store has blocked
// in-edges and the tuning allows them, else the row items and the long-row
// sums.
static hipError_t launch_pr_pull(const PrPullArgs& a, const PrPullStore& ps, const Tune& tn, uint32_t n,
                                 hipStream_t s) {
  if (ps.blk && tn.blocked) {
    PrBlkArgs b;
    b.v = blk_view(*ps.blk);
    b.slots = ps.blk->hot ? ps.blk->slots : nullptr;
    b.n = n;
    if (ps.blk->hot && ps.blk->bin_nunits) {
      hipLaunchKernelGGL(pr_bin_kernel, dim3(ps.blk->bin_nunits), dim3(kBlkThreads), 0, s, a.contrib_in, n,
                         bin_tables(*ps.blk), ps.blk->slots);
      const hipError_t e0 = hipGetLastError();
      if (e0 != hipSuccess) return e0;
    }
    // the first launch folds the previous superstep's counts, the second
    // only adds (when the first has no workgroups, the second folds)
    PrPullArgs a2 = a;
    hipError_t err = hipSuccess;
    if (ps.blk->nslices) {  // none when the graph has no edges
      hipLaunchKernelGGL(pr_blocked_kernel, dim3(ps.blk->nslices), dim3(kBlkThreads), 0, s, a, b);
      err = hipGetLastError();
      a2.tr.fold = nullptr;
    }
    if (err != hipSuccess) return err;
    if (b.v.ngroups) {
      const uint32_t grid = grid_for(b.v.ngroups, kWavesPerBlock, 4096);
      hipLaunchKernelGGL(pr_blocked_finish_kernel, dim3(grid), dim3(kBlock), 0, s, a2, b);
      err = hipGetLastError();
      a2.tr.fold = nullptr;
    }
    if (err != hipSuccess || !a2.tr.fold) return err;
    hipLaunchKernelGGL(pr_trace_last_kernel, dim3(1), dim3(kWave), 0, s, a2.tr);
    return hipGetLastError();
  }
  hipError_t err = launch_pr_items(a, ps.perm != nullptr, tn, n, s);
  if (err != hipSuccess) return err;
  PrPullArgs a2 = a;
  if (a.t.ni) a2.tr.fold = nullptr;
  if (ps.t.nl) {
    hipLaunchKernelGGL(pr_longrow_kernel, dim3((ps.t.nl + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0, s,
                       a2);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    a2.tr.fold = nullptr;
  }
  if (!a2.tr.fold) return hipSuccess;
  hipLaunchKernelGGL(pr_trace_last_kernel, dim3(1), dim3(kWave), 0, s, a2.tr);
  return hipGetLastError();
}

// The trace slots of superstep `step` (and those it folds).
static PrTrace pr_trace_at(const RunWs& w, uint32_t step) {
  PrTrace t;
  t.add = w.pr_cnt + (step & 1) * kCtrSlots;
  t.fold = step ? w.pr_cnt + ((step - 1) & 1) * kCtrSlots : nullptr;
  t.rec = w.pr_rec;
  t.fold_step = step ? step - 1 : 0;
  return t;
}

// Clears both trace slot sets before superstep 0 adds into them.
static hipError_t pr_trace_begin(const RunWs& w, hipStream_t s) {
  return fill_u32(reinterpret_cast<uint32_t*>(w.pr_cnt), 2 * kCtrSlots * sizeof(PrCntSlot) / 4, 0, s);
}

// Folds the last superstep's counts into its record.
static hipError_t pr_trace_end(const RunWs& w, uint32_t last_step, hipStream_t s) {
  PrTrace t = pr_trace_at(w, last_step + 1);
  hipLaunchKernelGGL(pr_trace_last_kernel, dim3(1), dim3(kWave), 0, s, t);
  return hipGetLastError();
}

// Every launch of one PageRank run, in order, on stream s (also used to
// capture the run as a graph, with tm == nullptr).
static hipError_t enqueue_pagerank(ipg_graph* g, uint32_t T, double d, bool push, const RunWs& w,
                                   const uint32_t* part_off, uint32_t parts, const Tune& tn, hipStream_t s,
                                   StepTimer* tm) {
  hipError_t err;
  const uint32_t n = g->n;
  const double ratio = (1.0 - d) / static_cast<double>(n);
  const double init = 1.0 / static_cast<double>(n);
  const uint32_t gv = grid_for(n, kBlock, 16384);
  const PrPullStore ps = pr_store_of(g, w);
  const uint32_t* part_n = nullptr;
  if (part_off) {
    hipLaunchKernelGGL(pr_part_n_kernel, dim3(gv), dim3(kBlock), 0, s, part_off, parts, n, push ? nullptr : ps.perm,
                       w.part_n);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    part_n = w.part_n;
  }
  if ((err = pr_trace_begin(w, s)) != hipSuccess) return err;
  if (!push) {
    if (tm && (err = tm->start(s)) != hipSuccess) return err;
    hipLaunchKernelGGL(pr_pull_init_kernel, dim3(gv), dim3(kBlock), 0, s, n, ps.outdeg, init, part_n, w.f64_a, ps.value,
                       T == 0, 0, pr_trace_at(w, 0));
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (tm && (err = tm->step(s, 0)) != hipSuccess) return err;
    PrPullArgs a;
    a.t = ps.t;
    a.outdeg = ps.outdeg;
    a.value = ps.value;
    a.partial = w.partial;
    a.ratio = ratio;
    a.damp = d;
    a.teleport = 1.0 - d;
    a.part_n = part_n;
    a.l1 = nullptr;
    for (uint32_t step = 1; step <= T; ++step) {
      a.contrib_in = (step & 1) ? w.f64_a : w.f64_b;
      a.contrib_out = (step & 1) ? w.f64_b : w.f64_a;
      a.last = step == T;
      a.tr = pr_trace_at(w, step);
      if ((err = launch_pr_pull(a, ps, tn, n, s)) != hipSuccess) return err;
      if (tm && (err = tm->step(s, step)) != hipSuccess) return err;
    }
    if ((err = pr_trace_end(w, T, s)) != hipSuccess) return err;
    if (ps.perm) {
      hipLaunchKernelGGL(pr_unrename_kernel, dim3(gv), dim3(kBlock), 0, s, ps.value, ps.perm, n, w.value_f64);
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
  } else {
    if ((err = fill_f64(w.f64_a, n, 0.0, s)) != hipSuccess) return err;
    if ((err = fill_f64(w.f64_b, n, 0.0, s)) != hipSuccess) return err;
    if ((err = fill_u32(reinterpret_cast<uint32_t*>(w.ctr), 2 * kCtrSlots * sizeof(CtrSlot) / 4, 0, s)) != hipSuccess)
      return err;
    if (tm && (err = tm->start(s)) != hipSuccess) return err;
    PrPushArgs a;
    a.n = n;
    a.off = g->csr_off;
    a.dst = g->csr_dst;
    a.value = w.value_f64;
    a.ratio = ratio;
    a.init = init;
    a.damp = d;
    a.teleport = 1.0 - d;
    a.part_n = part_n;
    a.l1 = nullptr;
    const uint32_t grid = grid_for(n, kBlock, 0xFFFFFFFFu);
    for (uint32_t step = 0; step <= T; ++step) {
      a.mail_in = (step & 1) ? w.f64_b : w.f64_a;
      a.mail_out = (step & 1) ? w.f64_a : w.f64_b;
      a.first = step == 0;
      a.last = step == T;
      a.tr = pr_trace_at(w, step);
      if ((err = launch_pr_push(a, w, g->e, grid, step, s)) != hipSuccess) return err;
      if (tm && (err = tm->step(s, step)) != hipSuccess) return err;
    }
    if ((err = pr_trace_end(w, T, s)) != hipSuccess) return err;
  }
  return hipSuccess;
}

// The captured graph of the run described by the arguments, capturing it
// (again) when the handle holds none or one for another run.
static ipg_status pagerank_graph(ipg_graph* g, uint32_t T, double d, bool push, const RunWs& w, const void* ws,
                                 const uint32_t* part_off, uint32_t parts, const Tune& tn, hipGraphExec_t* out) {
  auto& k = g->pr_key;
  if (g->pr_exec && k.T == T && k.damp == d && k.push == (push ? 1 : 0) && k.ws == ws && k.parts == part_off &&
      k.num_parts == parts && k.hot == tn.pr_hot && k.grid == tn.pull_grid && k.blocked == tn.blocked) {
    *out = g->pr_exec;
    return IPG_OK;
  }
  if (g->pr_exec) {
    IPG_HIP(hipGraphExecDestroy(g->pr_exec));
    g->pr_exec = nullptr;
  }
  if (g->pr_graph) {
    IPG_HIP(hipGraphDestroy(g->pr_graph));
    g->pr_graph = nullptr;
  }
  if (!g->cap_stream) IPG_HIP(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
  IPG_HIP(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
  const hipError_t qe = enqueue_pagerank(g, T, d, push, w, part_off, parts, tn, g->cap_stream, nullptr);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(g->cap_stream, &graph);
  if (qe != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(qe, "capture of the PageRank supersteps");
  }
  IPG_HIP(ce);
  g->pr_graph = graph;
  IPG_HIP(hipGraphInstantiate(&g->pr_exec, graph, nullptr, nullptr, 0));
  k.T = T;
  k.damp = d;
  k.push = push ? 1 : 0;
  k.ws = ws;
  k.parts = part_off;
  k.num_parts = parts;
  k.hot = tn.pr_hot;
  k.grid = tn.pull_grid;
  k.blocked = tn.blocked;
  *out = g->pr_exec;
  return IPG_OK;
}

// PageRank to convergence: the same supersteps with every update's L1
// change reduced on the device and read back; the run stops after the
// first update whose change is below `tol`, or after Tmax updates.
// Returns the number of updates run in *T_out.
static ipg_status run_pagerank_converge(ipg_graph* g, uint32_t Tmax, double d, bool push, double tol,
                                        const RunWs& w, const uint32_t* part_off, uint32_t parts, const Tune& tn,
                                        hipStream_t s, StepTimer& tm, ipg_run_stats* st, uint32_t* T_out,
                                        bool* converged) {
  const uint32_t n = g->n;
  const double ratio = (1.0 - d) / static_cast<double>(n);
  const double init = 1.0 / static_cast<double>(n);
  const uint32_t gv = grid_for(n, kBlock, 16384);
  const PrPullStore ps = pr_store_of(g, w);
  const uint32_t* part_n = nullptr;
  if (part_off) {
    hipLaunchKernelGGL(pr_part_n_kernel, dim3(gv), dim3(kBlock), 0, s, part_off, parts, n, push ? nullptr : ps.perm,
                       w.part_n);
    IPG_HIP(hipGetLastError());
    part_n = w.part_n;
  }
  constexpr uint32_t kSlotDoubles = kCtrSlots * 16;
  double h[kSlotDoubles];
  // L1 change of the update just enqueued (read back, slots summed in order)
  auto change = [&](uint32_t step, double* out) -> ipg_status {
    IPG_HIP(hipMemcpyAsync(h, w.l1, sizeof(h), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    double d = 0.0;
    for (int b = 0; b < kCtrSlots; ++b) d += h[b * 16];
    if (st && st->residual && step < st->trace_cap) st->residual[step] = d;
    *out = d;
    return IPG_OK;
  };
  *converged = false;
  uint32_t T = Tmax;
  if (st && st->residual && st->trace_cap) st->residual[0] = 0.0;
  IPG_HIP(pr_trace_begin(w, s));
  if (!push) {
    IPG_HIP(tm.start(s));
    hipLaunchKernelGGL(pr_pull_init_kernel, dim3(gv), dim3(kBlock), 0, s, n, ps.outdeg, init, part_n, w.f64_a, ps.value,
                       0, 1, pr_trace_at(w, 0));
    IPG_HIP(hipGetLastError());
    IPG_HIP(tm.step(s, 0));
    PrPullArgs a;
    a.t = ps.t;
    a.outdeg = ps.outdeg;
    a.value = ps.value;
    a.partial = w.partial;
    a.ratio = ratio;
    a.damp = d;
    a.teleport = 1.0 - d;
    a.part_n = part_n;
    a.l1 = w.l1;
    a.last = 0;
    for (uint32_t step = 1; step <= Tmax; ++step) {
      IPG_HIP(fill_f64(w.l1, kSlotDoubles, 0.0, s));
      a.contrib_in = (step & 1) ? w.f64_a : w.f64_b;
      a.contrib_out = (step & 1) ? w.f64_b : w.f64_a;
      a.tr = pr_trace_at(w, step);
      IPG_HIP(launch_pr_pull(a, ps, tn, n, s));
      IPG_HIP(tm.step(s, step));
      double d = 0.0;
      const ipg_status rc = change(step, &d);
      if (rc != IPG_OK) return rc;
      if (d < tol) {
        T = step;
        *converged = true;
        break;
      }
    }
    if (ps.perm) {
      hipLaunchKernelGGL(pr_unrename_kernel, dim3(gv), dim3(kBlock), 0, s, ps.value, ps.perm, n, w.value_f64);
      IPG_HIP(hipGetLastError());
    }
  } else {
    IPG_HIP(fill_f64(w.f64_a, n, 0.0, s));
    IPG_HIP(fill_f64(w.f64_b, n, 0.0, s));
    IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.ctr), 2 * kCtrSlots * sizeof(CtrSlot) / 4, 0, s));
    IPG_HIP(tm.start(s));
    PrPushArgs a;
    a.n = n;
    a.off = g->csr_off;
    a.dst = g->csr_dst;
    a.value = w.value_f64;
    a.ratio = ratio;
    a.init = init;
    a.damp = d;
    a.teleport = 1.0 - d;
    a.part_n = part_n;
    a.l1 = w.l1;
    const uint32_t grid = grid_for(n, kBlock, 0xFFFFFFFFu);
    for (uint32_t step = 0; step <= Tmax; ++step) {
      IPG_HIP(fill_f64(w.l1, kSlotDoubles, 0.0, s));
      a.mail_in = (step & 1) ? w.f64_b : w.f64_a;
      a.mail_out = (step & 1) ? w.f64_a : w.f64_b;
      a.first = step == 0;
      a.last = step == Tmax;
      a.tr = pr_trace_at(w, step);
      IPG_HIP(launch_pr_push(a, w, g->e, grid, step, s));
      IPG_HIP(tm.step(s, step));
      if (step == 0) continue;
      double d = 0.0;
      const ipg_status rc = change(step, &d);
      if (rc != IPG_OK) return rc;
      if (d < tol) {
        T = step;
        *converged = true;
        break;
      }
    }
  }
  IPG_HIP(pr_trace_end(w, T, s));
  IPG_HIP(tm.finish(s));
  *T_out = T;
  return IPG_OK;
}

ipg_status run_pagerank(ipg_graph* g, uint32_t T, const ipg_run_opts& o, const RunWs& w, const void* ws,
                        hipStream_t s, StepTimer& tm, ipg_run_stats* st) {
  const uint32_t n = g->n;
  const bool push = (o.mode == IPG_MODE_PUSH);
  const Tune tn = resolve_tuning(o.tuning);
  const double d = o.damping == 0.0 ? 0.85 : o.damping;
  if (!(d > 0.0 && d <= 1.0)) return fail(IPG_EINVAL, "ipg_run: damping must be in (0, 1] (0 = 0.85)");
  uint32_t room = 0;
  IPG_HIP(max_hot_entries(&room));  // queried here, never during a stream capture
  const uint32_t* part_off = nullptr;
  uint32_t parts = 0;
  if (o.flags & IPG_RUN_ENQUEUE) {  // no host synchronisation: the offsets are the caller's to get right
    IPG_HIP(enqueue_pagerank(g, T, d, push, w, o.num_parts ? o.part_offsets : nullptr, o.num_parts, tn, s, nullptr));
    return IPG_OK;
  }
  if (o.part_offsets && o.num_parts) {
    std::vector<uint32_t> h(o.num_parts + 1);
    IPG_HIP(hipMemcpyAsync(h.data(), o.part_offsets, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    if (h[0] != 0 || h[o.num_parts] != n) return fail(IPG_EINVAL, "ipg_run: part_offsets must run from 0 to N");
    for (uint32_t p = 0; p < o.num_parts; ++p)
      if (h[p + 1] <= h[p]) return fail(IPG_EINVAL, "ipg_run: part_offsets must be strictly increasing");
    part_off = o.part_offsets;
    parts = o.num_parts;
  }
  bool converged = true;
  if (o.tolerance > 0.0) {
    uint32_t Tdone = T;
    const ipg_status rc = run_pagerank_converge(g, T, d, push, o.tolerance, w, part_off, parts, tn, s, tm, st, &Tdone,
                                                &converged);
    if (rc != IPG_OK) return rc;
    T = Tdone;
  } else if (o.flags & IPG_RUN_GRAPH) {
    hipGraphExec_t exec = nullptr;
    const ipg_status rc = pagerank_graph(g, T, d, push, w, ws, part_off, parts, tn, &exec);
    if (rc != IPG_OK) return rc;
    IPG_HIP(tm.start(s));
    IPG_HIP(hipGraphLaunch(exec, s));
    IPG_HIP(tm.finish(s));
  } else {
    IPG_HIP(enqueue_pagerank(g, T, d, push, w, part_off, parts, tn, s, &tm));
    IPG_HIP(tm.finish(s));
  }
  if (st) {
    // The trace as the kernels counted it: per superstep, the vertices that
    // ran compute, those that broadcast and their out-degree sum.  The
    // stream has been synchronised (tm.finish).
    const uint32_t steps = T + 1;
    const uint32_t nrec = std::min(steps, kPrTraceCap);
    std::vector<unsigned long long> rec(3 * static_cast<size_t>(nrec));
    IPG_HIP(hipMemcpy(rec.data(), w.pr_rec, 3 * sizeof(unsigned long long) * nrec, hipMemcpyDeviceToHost));
    if (o.tolerance > 0.0 && nrec == steps) {
      // a convergence run stops after update T: the outboxes its kernels
      // wrote in that superstep are never read (the run with a fixed T
      // broadcasts nothing there)
      rec[3 * (steps - 1) + 1] = 0;
      rec[3 * (steps - 1) + 2] = 0;
    }
    uint64_t traversed = 0;
    for (uint32_t k = 0; k < nrec; ++k) traversed += rec[3 * k + 2];
    st->supersteps = steps;
    st->halted = converged ? 1 : 0;
    // supersteps past the last record (nrec .. T - 1) each broadcast E messages
    st->edges_traversed = traversed + (steps > nrec ? static_cast<uint64_t>(T - nrec) * g->e : 0);
    st->edges_examined = static_cast<uint64_t>(T) * g->e;
    for (uint32_t k = 0; k < nrec && k < st->trace_cap; ++k) {
      if (st->active) st->active[k] = rec[3 * k + 0];
      if (st->senders) st->senders[k] = rec[3 * k + 1];
      if (st->messages) st->messages[k] = rec[3 * k + 2];
      if (st->examined) st->examined[k] = k < T ? g->e : 0;
      if (st->mode) st->mode[k] = push ? IPG_MODE_PUSH : IPG_MODE_PULL;
      if (st->frontier_deg) st->frontier_deg[k] = g->e;
      if ((o.flags & IPG_RUN_GRAPH) && st->usec) st->usec[k] = 0.f;
    }
  }
  return converged ? IPG_OK : IPG_NOT_CONVERGED;
}

}  // namespace ipg
