// blocked.h -- streaming the destination-blocked, source-sorted in-edges
// (IPG_GRAPH_BLOCKED; layout in common.h) through one workgroup per slice.
// Shared by the PageRank pull (FP64 sums) and the CC/SSSP pull (u32 minima).
#pragma once

#include "common.h"

namespace ipg {

constexpr uint32_t kBlkThreads = 1024;  // one workgroup per slice, one per CU (its LDS holds the block's values)
constexpr int kBlkGroup = 4;            // chunks a wavefront takes per step

// Device view of one set of blocked tables.
struct BlkView {
  const uint32_t* edges;
  const BlkChunk* chunks;
  const BlkSlice* slices;
  const BlkGroup* groups;
  void* partial;
  uint32_t ngroups;
};
inline BlkView blk_view(const BlockedTables& t) {
  BlkView v;
  v.edges = t.edges;
  v.chunks = t.chunks;
  v.slices = t.slices;
  v.groups = t.groups;
  v.partial = t.partial;
  v.ngroups = t.ngroups;
  return v;
}

// A chunk past the slice's end: no edges (its loads read the slice table).
__device__ __forceinline__ BlkChunk blk_chunk_at(const BlkView& b, uint64_t c, uint32_t c1) {
  if (c < c1) return b.chunks[c];
  BlkChunk z;
  z.e0 = 0;
  z.wbase = 0;
  z.n = 0;
  z.cold = 0;
  return z;
}

// The packed edges of a chunk, one per lane and register, the index clamped
// into the chunk so that every load is unconditional.
__device__ __forceinline__ void blk_load(const BlkView& b, const BlkChunk& ch, uint32_t (&p)[kBlkChunk / kWave]) {
  const uint32_t lane = lane_id();
  const uint32_t* base = ch.n ? b.edges + ch.e0 : reinterpret_cast<const uint32_t*>(b.slices);
  const uint32_t last = ch.n ? ch.n - 1 : 0;
#pragma unroll
  for (int k = 0; k < static_cast<int>(kBlkChunk / kWave); ++k) {
    const uint32_t i = lane + k * kWave;
    p[k] = __builtin_nontemporal_load(base + (i < last ? i : last));
  }
}

// The edge loop of one slice, run by every wavefront of the workgroup:
// chunk c of the slice goes to wavefront (c - c0) mod kWaves.  A wavefront
// takes kBlkGroup chunks per step: it gathers their sources' values
// (`value(wbase, packed, cold)`: the sources of a chunk are sorted and share
// one window, so neighbouring lanes mostly read the same cache lines; a cold
// chunk's values are slots, read in order), starts
// loading the next step's packed edges, and then combines each value into
// its destination's LDS slot (`combine(slot, v)`).  Lanes past a chunk's
// end combine `idle` into their own pad slot kBlkRows + lane, so that no
// combine is under a branch: a gather used only under a branch is issued
// late, inside it.  Two steps per iteration and no exit between them (past
// the slice's end the chunks are empty): an exit there would let the
// compiler move the first step's prefetch behind it, to just before use.
// The two register sets alternate, so no loaded value is copied (a copy
// would wait for its load).
template <class T, class Value, class Combine>
__device__ __forceinline__ void blk_stream(const BlkView& b, const BlkSlice& sl, T idle, Value value, Combine combine) {
  constexpr int kPer = kBlkChunk / kWave;
  constexpr uint32_t kWaves = kBlkThreads / kWave;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = lane_id();
  using Group = BlkChunk[kBlkGroup];
  using Edges = uint32_t[kBlkGroup][kPer];
  auto meta = [&](uint64_t c, Group& ch) {
#pragma unroll
    for (int g = 0; g < kBlkGroup; ++g) ch[g] = blk_chunk_at(b, c + g * kWaves, sl.c1);
  };
  auto load = [&](const Group& ch, Edges& p) {
#pragma unroll
    for (int g = 0; g < kBlkGroup; ++g) blk_load(b, ch[g], p[g]);
  };
  auto step = [&](const Group& ch, const Edges& p, const Group& next, Edges& pn) {
    T x[kBlkGroup][kPer];
#pragma unroll
    for (int g = 0; g < kBlkGroup; ++g)
#pragma unroll
      for (int k = 0; k < kPer; ++k) x[g][k] = value(ch[g].wbase, ch[g].n ? p[g][k] : 0u, ch[g].cold);
    load(next, pn);
#pragma unroll
    for (int g = 0; g < kBlkGroup; ++g)
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const bool in = lane + k * kWave < ch[g].n;
        combine(in ? p[g][k] & 0xFFFFu : kBlkRows + lane, in ? x[g][k] : idle);
      }
  };
  constexpr uint64_t kStride = static_cast<uint64_t>(kWaves) * kBlkGroup;
  uint64_t c = static_cast<uint64_t>(sl.c0) + wv;
  Group ca, cb, n1, n2;
  Edges pa, pb;
  meta(c, ca);
  meta(c + kStride, cb);
  load(ca, pa);
  while (c < sl.c1) {
    meta(c + 2 * kStride, n1);
    step(ca, pa, cb, pb);
    meta(c + 3 * kStride, n2);
    step(cb, pb, n1, pa);
    c += 2 * kStride;
#pragma unroll
    for (int g = 0; g < kBlkGroup; ++g) {
      ca[g] = n1[g];
      cb[g] = n2[g];
    }
  }
}

// Tables of the bin launch of a binned layout (IPG_GRAPH_BINNED).
struct BinTables {
  const uint16_t* src;
  const BinRun* runs;
  const uint64_t* wflat;
  const uint32_t* wrun;
  const uint64_t* wgroup;
  const uint32_t* group;
  const BinUnit* units;
  uint32_t w0;
};
inline BinTables bin_tables(const BlockedTables& t) {
  BinTables b;
  b.src = t.bin_src;
  b.runs = t.bin_runs;
  b.wflat = t.bin_wflat;
  b.wrun = t.bin_wrun;
  b.wgroup = t.bin_wgroup;
  b.group = t.bin_group;
  b.units = t.bin_units;
  b.w0 = t.hot >> kBinWinBits;
  return b;
}
constexpr uint32_t kBinWin = 1u << kBinWinBits;
constexpr int kBinBatch = 8;  // groups of kBinGroup list entries a wavefront handles per iteration
// Runs a group of kBinGroup list entries can meet: runs hold whole kBinPad
// lines, so a group meets at most kBinGroup / kBinPad of them after its first.
constexpr int kBinCand = kBinGroup / kBinPad + 1;
static_assert(kBinCand <= kWave && kBinGroup == kWave, "one group entry per lane, one candidate run per lane");

// The bin launch's work for one workgroup (one work unit: at most
// kBinUnitGroups groups of one cold window of kBinWin sources; kBlkThreads
// threads).  The window's values -- value(u) for source u < n -- are staged
// in LDS, then every entry of the unit's part of the window's list (its
// slots, in the window's run order) copies its source's value into its slot.
// Lane j of a group takes list entry j; the group's first run and the runs
// after it are loaded by the first kBinCand lanes, and each lane picks the
// last of them that starts at or before its entry.  Consecutive entries of a
// run go to consecutive slots, so a wavefront's stores are runs of whole
// lines.
template <class T, class Value>
__device__ __forceinline__ void bin_unit(const BinTables& bv, T* slots, uint32_t n, Value value) {
  __shared__ T win[kBinWin];
  const BinUnit unit = bv.units[blockIdx.x];
  const uint32_t k = unit.win;
  const uint64_t base = static_cast<uint64_t>(bv.w0 + k) << kBinWinBits;
  {
    constexpr int kPer = kBinWin / kBlkThreads;
    T x[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const uint64_t u = base + threadIdx.x + i * kBlkThreads;
      x[i] = value(static_cast<uint32_t>(u < n ? u : n - 1));  // sources past N have no slots
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) win[threadIdx.x + i * kBlkThreads] = x[i];
  }
  __syncthreads();
  const uint64_t f0 = bv.wflat[k];
  const uint32_t len = static_cast<uint32_t>(bv.wflat[k + 1] - f0);
  const uint32_t r0 = bv.wrun[k], nr = bv.wrun[k + 1] - r0;
  const uint64_t g0 = bv.wgroup[k];
  const uint32_t ng = unit.g1;  // groups [unit.g0, unit.g1) of the window, g1 <= ceil(len / kBinGroup)
  const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
  constexpr uint32_t kWaves = kBlkThreads / kWave;
  for (uint32_t g = unit.g0 + wv * kBinBatch; g < ng; g += kWaves * kBinBatch) {  // wave-uniform
    uint32_t fr[kBinBatch], so[kBinBatch];
    BinRun cand[kBinBatch];
#pragma unroll
    for (int b = 0; b < kBinBatch; ++b) {
      const uint32_t gi = g + b < ng ? g + b : ng - 1;
      fr[b] = bv.group[g0 + gi];
      const uint32_t j = gi * kBinGroup + lane;
      so[b] = bv.src[f0 + (j < len ? j : len - 1)];
    }
#pragma unroll
    for (int b = 0; b < kBinBatch; ++b) {
      const uint32_t r = fr[b] + (lane < kBinCand ? lane : 0);
      cand[b] = bv.runs[r0 + (r < nr ? r : nr - 1)];
      if (lane >= kBinCand || r >= nr) cand[b].flat = 0xFFFFFFFFu;  // not a run of this group
    }
#pragma unroll
    for (int b = 0; b < kBinBatch; ++b) {
      const uint32_t j = (g + b) * kBinGroup + lane;
      int t = 0;
#pragma unroll
      for (int c = 1; c < kBinCand; ++c)
        if (static_cast<uint32_t>(__shfl(static_cast<int>(cand[b].flat), c)) <= j) t = c;
      const uint32_t flat = static_cast<uint32_t>(__shfl(static_cast<int>(cand[b].flat), t));
      const uint32_t dst = static_cast<uint32_t>(__shfl(static_cast<int>(cand[b].dst), t));
      // non-temporal: the slots are read once, by the next launch, long after
      // the lines would have left L2
      if (g + b < ng && j < len) __builtin_nontemporal_store(win[so[b]], slots + static_cast<uint64_t>(dst) + (j - flat));
    }
  }
}

}  // namespace ipg
