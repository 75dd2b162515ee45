// blocked_layout.h -- the destination-blocked, source-sorted in-edges of a
// CSC (IPG_GRAPH_BLOCKED): layout, size bounds and the host build.  Plain
// C++ (no HIP): the library builds the layout on the host and copies it to
// the device; the CPU tests build it from the same code and check it.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <utility>
#include <vector>

namespace ipg {

// Destination-blocked, source-sorted copy of the in-edges for PageRank's
// blocked pull (IPG_GRAPH_BLOCKED).  The destinations are cut into blocks:
// runs of consecutive rows, at most kBlkRows of them (one workgroup's LDS
// of FP64 partial sums), closed early once they hold kBlkEdgeFactor / S of
// the edges, so that the rows with many in-edges form narrow blocks.  Each
// block's in-edges are stored sorted by source (ties by destination), one
// 32-bit word per edge: the source's offset within its window of
// 2^kBlkWinBits sources in the high half, the destination's row within the
// block in the low half.  The edges are cut into chunks of at most kBlkChunk
// edges that never straddle a window (so a wavefront's window base is
// uniform), and each block's chunks into slices, about one per CU.  A block
// with one slice is finished by that slice's workgroup; the slices of a
// larger block store partial sums that a second launch adds in slice order.
//
// Binned cold sources (optional, `hot` > 0): the sources from `hot` on,
// whose outboxes are too many to stay in any cache, are not gathered edge by
// edge.  Each block's edges from them ("cold" edges) follow its hot edges,
// still sorted by source, and every distinct (block, cold source) pair owns
// one slot of a slot array, numbered block by block in the order of the
// edges.  Before each pull a bin launch copies every cold source's outbox
// value into all of its slots, one workgroup per scatter window of
// 2^kBinWinBits sources or part of one (the window's outboxes staged in LDS): a block's
// slots from one window form a run of consecutive slots, padded to
// kBinPad slots so that runs start on 64-byte lines.  A cold edge's word
// holds its slot's offset from its chunk's first slot instead of a source
// offset, and a cold chunk (flag `cold`) reads slots instead of outboxes:
// the pull streams them in order.  For the bin launch every window lists
// its slots (source offsets, in the window's run order) and its runs (first
// slot in the window's list, first slot in the slot array), and a table
// gives the first run of every 64 slots of the list.
constexpr uint32_t kBlkRows = 20224;
constexpr uint32_t kBlkWinBits = 16;
constexpr uint32_t kBlkChunk = 256;
constexpr uint32_t kBlkSlices = 256;
constexpr uint64_t kBlkMinSliceEdges = 65536;
constexpr uint64_t kBlkEdgeFactor = 8;
// Slice balancing: a 128-byte outbox line a chunk touches costs about as
// much as this many edges (fitted to measured slice times on MI355X).
constexpr uint64_t kBlkLineCost = 6;
// XCDs of the chip: workgroup i of a launch runs on XCD i mod kBlkXcds.
constexpr size_t kBlkXcds = 8;
static_assert(kBlkRows <= (1u << 16), "row within a block fits 16 bits");
// Binned cold sources: scatter windows of 2^kBinWinBits sources (their FP64
// outboxes fill 64 KB of LDS, so two bin workgroups share a CU), runs padded
// to kBinPad slots (64 bytes).
constexpr uint32_t kBinWinBits = 13;
constexpr uint32_t kBinPad = 8;
constexpr uint32_t kBinGroup = 64;  // slots of a window's list per entry of its group table
// Hot-source count when binning is asked for without one (8 MB of outboxes).
constexpr uint32_t kBinHotDefault = 1u << 20;
// Work unit of the bin launch: at most this many groups of one window, so
// that the windows of many-slot sources are shared by several workgroups
// (each stages the window's outboxes itself).
constexpr uint32_t kBinUnitGroups = 4096;

struct BlkChunk {
  uint64_t e0;     // first edge
  uint32_t wbase;  // first source of the chunk's window; for a cold chunk, its first slot
  uint16_t n;      // edges (1 .. kBlkChunk)
  uint16_t cold;   // 1: the edges' high halves are slot offsets from wbase
};
static_assert(sizeof(BlkChunk) == 16, "16-byte chunk record");
// A run of one window's list: its first slot in the list (relative to the
// window's first) and in the slot array; it ends where the next run of the
// window starts.
struct BinRun {
  uint32_t flat;
  uint32_t dst;
};
// One workgroup of the bin launch: groups [g0, g1) of cold window `win`
// (counted from the first cold window).
struct BinUnit {
  uint32_t win;
  uint32_t g0, g1;
};
struct BlkSlice {
  uint32_t row0, rows;  // the block's rows [row0, row0 + rows)
  uint32_t c0, c1;      // chunks [c0, c1)
  uint64_t poff;        // partial sums at partial + poff (rows doubles), ~0 when the slice is the block's only one
};
// 64 rows of a block with more than one slice, for the finish launch.
struct BlkGroup {
  uint32_t row0;    // first row of the group
  uint32_t nrows;   // rows in the group (1 .. 64)
  uint32_t k;       // the block's slices
  uint32_t stride;  // the block's rows: slice j's partial of row row0 + i is at partial[poff + j * stride + i]
  uint64_t poff;
};
constexpr uint64_t kNoPartial = ~0ull;

// Target number of slices: about one per CU, none under kBlkMinSliceEdges edges.
inline uint32_t blk_target_slices(uint64_t e) {
  const uint64_t s = (e + kBlkMinSliceEdges - 1) / kBlkMinSliceEdges;
  return static_cast<uint32_t>(s < 1 ? 1 : (s > kBlkSlices ? kBlkSlices : s));
}
// Edges at which a block closes: kBlkEdgeFactor / S of the edges; on a
// graph whose row-capped blocks alone outnumber the S slices (blocks then
// run in several rounds, most as one slice), twice the mean edges of a
// row-capped block instead, so that dense rows form narrow blocks rather
// than a few blocks of E / 32 edges that one workgroup each would stream.
inline uint64_t blk_edge_target(uint32_t n, uint64_t e) {
  const uint64_t s = blk_target_slices(e), row_blocks = n / kBlkRows + 1;
  const uint64_t t = row_blocks >= s ? 2 * e / row_blocks : kBlkEdgeFactor * e / s;
  return t < 1 ? 1 : t;
}
inline uint64_t blk_windows(uint32_t n) { return (static_cast<uint64_t>(n) + (1u << kBlkWinBits) - 1) >> kBlkWinBits; }
// Blocks: one closed by the row cap takes kBlkRows rows; two consecutive
// blocks closed by the edge target hold more than the target together.
inline uint64_t blk_blocks_cap(uint32_t n, uint64_t e) {
  const uint64_t by_rows = n / kBlkRows + 1, by_edges = 2 * e / blk_edge_target(n, e) + 2;
  return by_rows + by_edges;
}
// Chunks: at most one partial chunk per non-empty (block, window) segment.
inline uint64_t blk_chunks_cap(uint32_t n, uint64_t e) {
  const uint64_t segs = blk_blocks_cap(n, e) * blk_windows(n);
  return e / kBlkChunk + (segs < e ? segs : e) + 1;
}
// Partial sums: the blocks with several slices hold at most S slices of at
// most kBlkRows rows.
inline uint64_t blk_partial_cap(uint64_t e) { return static_cast<uint64_t>(blk_target_slices(e)) * kBlkRows; }

// Finish groups: a multi-slice block of R rows has ceil(R / 64) of them.
inline uint64_t blk_groups_cap(uint32_t n, uint64_t e) { return n / 64 + blk_blocks_cap(n, e) + 1; }

// Binned cold sources: scatter windows, runs (at most one per (block,
// window) pair with edges), slots (one per pair plus padding), group table.
inline uint64_t bin_windows(uint32_t n) { return (static_cast<uint64_t>(n) + (1u << kBinWinBits) - 1) >> kBinWinBits; }
inline uint64_t bin_runs_cap(uint32_t n, uint64_t e) {
  const uint64_t pairs = blk_blocks_cap(n, e) * bin_windows(n);
  return e < pairs ? e : pairs;
}
inline uint64_t bin_slots_cap(uint32_t n, uint64_t e) { return e + (kBinPad - 1) * bin_runs_cap(n, e); }
inline uint64_t bin_groups_cap(uint32_t n, uint64_t e) { return bin_slots_cap(n, e) / kBinGroup + bin_windows(n) + 1; }
inline uint64_t bin_units_cap(uint32_t n, uint64_t e) { return bin_groups_cap(n, e) / kBinUnitGroups + bin_windows(n) + 1; }
// Chunks of a binned layout: the hot ones as before, plus at most one partial
// cold chunk per block.
inline uint64_t bin_chunks_cap(uint32_t n, uint64_t e) { return blk_chunks_cap(n, e) + blk_blocks_cap(n, e); }

// The host-side layout: packed edges (in block order), chunks, slices in
// launch order, finish groups; plus the block starts and each block's first
// chunk (used by the checks).
struct BlockedLayout {
  std::vector<uint32_t> packed;
  std::vector<BlkChunk> chunks;
  std::vector<BlkSlice> slices;
  std::vector<BlkGroup> groups;
  std::vector<uint32_t> row0;    // [blocks + 1] first row of each block
  std::vector<uint64_t> cfirst;  // [blocks + 1] first chunk of each block
  // binned cold sources (hot == 0: none)
  uint32_t hot = 0;               // sources below are gathered, the others binned (a multiple of the windows)
  uint64_t nslots = 0;            // entries of the slot array
  uint32_t bin_w0 = 0;            // first scatter window holding cold sources
  std::vector<uint16_t> bin_src;  // window lists: source offset within the window of every slot
  std::vector<BinRun> bin_runs;   // runs of every window, window by window, each window's in block order
  std::vector<uint64_t> bin_wflat;  // [cold windows + 1] first list entry of each window
  std::vector<uint32_t> bin_wrun;   // [cold windows + 1] first run of each window
  std::vector<uint64_t> bin_wgroup; // [cold windows + 1] first group of each window
  std::vector<uint32_t> bin_group;  // first run (window-relative) of every kBinGroup list entries of a window
  std::vector<BinUnit> bin_units;   // the bin launch's workgroups, window by window
};

// Build the layout of a CSC given in host memory (offsets [n+1], sources
// [e]): two stable counting sorts -- the edges by source (each source's
// edges in destination order), then by destination block -- so that every
// block holds its edges sorted by source; then the chunks, the slices and
// the finish groups.  Returns null, or a message when the CSC is malformed
// (it is read with these indices even when the graph was not validated) or
// a table would exceed its bound.
inline const char* blocked_layout(uint32_t n, uint64_t e, const uint64_t* off, const int32_t* src,
                                  BlockedLayout* out, uint32_t hot = 0) {
  // the host loops below index with these: check them here even without IPG_GRAPH_VALIDATE
  if (off[0] != 0 || off[n] != e) return "offsets: off[0] != 0 or off[N] != E";
  for (uint32_t v = 0; v < n; ++v)
    if (off[v] > off[(size_t)v + 1]) return "offsets decreasing";
  for (uint64_t i = 0; i < e; ++i)
    if (src[i] < 0 || static_cast<uint32_t>(src[i]) >= n) return "CSC source id outside [0, N)";
  // blocks: runs of consecutive rows, closed before the row that would take
  // them past the edge target (a row above it alone forms a block) or at
  // kBlkRows rows
  const uint64_t target = blk_edge_target(n, e);
  std::vector<uint32_t> row0{0};
  std::vector<uint32_t> blk_of(n);
  {
    uint64_t acc = 0;
    for (uint32_t v = 0; v < n; ++v) {
      const uint64_t d = off[(size_t)v + 1] - off[v];
      if (v > row0.back() && (acc + d > target || v - row0.back() == kBlkRows)) {
        row0.push_back(v);
        acc = 0;
      }
      acc += d;
      blk_of[v] = static_cast<uint32_t>(row0.size() - 1);
    }
    row0.push_back(n);
  }
  const uint64_t nblk = row0.size() - 1, nwin = blk_windows(n);
  if (nblk > blk_blocks_cap(n, e)) return "blocked block table overflow";
  // binning: the hot count rounded up to whole windows (of both sizes); none
  // when every source is hot
  if (hot) {
    const uint64_t unit = 1u << kBlkWinBits;
    const uint64_t h = (static_cast<uint64_t>(hot) + unit - 1) / unit * unit;
    hot = h >= n ? 0u : static_cast<uint32_t>(h);
  }
  // by source: dst_of[k] is the destination of the k-th edge in source order
  std::vector<uint64_t> sstart((size_t)n + 1, 0);
  for (uint64_t i = 0; i < e; ++i) ++sstart[(size_t)src[i] + 1];
  for (uint32_t u = 0; u < n; ++u) sstart[(size_t)u + 1] += sstart[u];
  std::vector<uint32_t> dst_of(e);
  {
    std::vector<uint64_t> cur(sstart.begin(), sstart.end() - 1);
    for (uint32_t v = 0; v < n; ++v)
      for (uint64_t i = off[v]; i < off[(size_t)v + 1]; ++i) dst_of[cur[src[i]]++] = v;
  }
  // by block, counting the edges of every (block, window) segment; with
  // binning a block's cold edges (sources >= hot) follow its hot ones
  std::vector<uint64_t> bstart(nblk + 1, 0);
  for (uint32_t v = 0; v < n; ++v) bstart[(size_t)blk_of[v] + 1] += off[(size_t)v + 1] - off[v];
  for (uint64_t k = 0; k < nblk; ++k) bstart[k + 1] += bstart[k];
  std::vector<uint64_t> hot_n(nblk, 0);  // hot edges of each block
  if (hot)
    for (uint32_t u = 0; u < hot; ++u)
      for (uint64_t k = sstart[u]; k < sstart[(size_t)u + 1]; ++k) ++hot_n[blk_of[dst_of[k]]];
  std::vector<uint64_t> seg(nblk * nwin, 0);
  std::vector<uint32_t> packed(e);
  std::vector<uint32_t> cold_src;  // source of every edge from the first cold edge of block 0 on (binning)
  if (hot) cold_src.assign(e, 0);
  {
    std::vector<uint64_t> cur(bstart.begin(), bstart.end() - 1), ccur(nblk);
    for (uint64_t b = 0; b < nblk; ++b) ccur[b] = bstart[b] + hot_n[b];
    for (uint32_t u = 0; u < n; ++u) {
      const uint64_t w = u >> kBlkWinBits;
      const uint32_t hi = (u & ((1u << kBlkWinBits) - 1)) << 16;
      const bool cold = hot && u >= hot;
      for (uint64_t k = sstart[u]; k < sstart[(size_t)u + 1]; ++k) {
        const uint32_t v = dst_of[k];
        const uint64_t blk = blk_of[v];
        if (cold) {
          const uint64_t at = ccur[blk]++;
          packed[at] = v - row0[blk];  // the slot offset comes with the cold chunks
          cold_src[at] = u;
        } else {
          packed[cur[blk]++] = hi | (v - row0[blk]);
          ++seg[blk * nwin + w];
        }
      }
    }
  }
  std::vector<uint32_t>().swap(dst_of);
  // slots: a new one at every change of source within a block's cold edges,
  // runs by (block, scatter window) padded to kBinPad slots; cold_src then
  // holds the edge's slot
  std::vector<uint32_t> slot_src;  // source of every slot (padding: its run's first source)
  struct RunRec {
    uint32_t w;    // scatter window
    uint64_t dst;  // first slot
    uint64_t len;  // slots, padding included
  };
  std::vector<RunRec> runs;
  if (hot) {
    uint64_t next = 0;
    for (uint64_t blk = 0; blk < nblk; ++blk) {
      uint32_t prev = 0xFFFFFFFFu;
      for (uint64_t i = bstart[blk] + hot_n[blk]; i < bstart[blk + 1]; ++i) {
        const uint32_t u = cold_src[i];
        if (u != prev) {
          const uint32_t w = u >> kBinWinBits;
          if (prev == 0xFFFFFFFFu || w != (prev >> kBinWinBits)) {
            if (!runs.empty() && runs.back().len % kBinPad) {  // pad the run this one follows
              const uint64_t pad = kBinPad - runs.back().len % kBinPad;
              const uint32_t fill = slot_src[runs.back().dst];
              slot_src.insert(slot_src.end(), pad, fill);
              runs.back().len += pad;
              next += pad;
            }
            runs.push_back(RunRec{w, next, 0});
          }
          slot_src.push_back(u);
          ++runs.back().len;
          ++next;
          prev = u;
        }
        cold_src[i] = static_cast<uint32_t>(next - 1);
        if (next - 1 > 0xFFFFFFFFull) return "binned slot index overflow";
      }
    }
    if (!runs.empty() && runs.back().len % kBinPad) {
      const uint64_t pad = kBinPad - runs.back().len % kBinPad;
      const uint32_t fill = slot_src[runs.back().dst];
      slot_src.insert(slot_src.end(), pad, fill);
      runs.back().len += pad;
      next += pad;
    }
    if (next > bin_slots_cap(n, e) || runs.size() > bin_runs_cap(n, e) || next >= 0xFFFFFFFFull)
      return "binned slot table overflow";
  }
  // chunks: every segment cut into pieces of at most kBlkChunk edges; the
  // cost of a chunk is its edges plus kBlkLineCost per outbox cache line its
  // sources touch (runs of equal source >> 4: 16 FP64 outboxes per 128-byte
  // line; the sources are sorted)
  std::vector<BlkChunk> chunks;
  std::vector<uint64_t> cost;
  std::vector<uint64_t> cfirst(nblk + 1, 0);
  for (uint64_t blk = 0; blk < nblk; ++blk) {
    cfirst[blk] = chunks.size();
    uint64_t at = bstart[blk];
    for (uint64_t w = 0; w < nwin; ++w) {
      for (uint64_t left = seg[blk * nwin + w]; left > 0;) {
        const uint32_t m = static_cast<uint32_t>(left < kBlkChunk ? left : kBlkChunk);
        chunks.push_back(BlkChunk{at, static_cast<uint32_t>(w << kBlkWinBits), static_cast<uint16_t>(m), 0});
        uint64_t lines = 1;
        for (uint64_t i = at + 1; i < at + m; ++i) lines += (packed[i] >> 20) != (packed[i - 1] >> 20);
        cost.push_back(m + kBlkLineCost * lines);
        at += m;
        left -= m;
      }
    }
    // cold chunks: up to kBlkChunk consecutive cold edges, their slots as
    // offsets from the first edge's slot (a line holds 16 slots)
    for (const uint64_t end = bstart[blk + 1]; at < end;) {
      const uint32_t m = static_cast<uint32_t>(end - at < kBlkChunk ? end - at : kBlkChunk);
      const uint32_t base = cold_src[at];
      uint64_t lines = 1;
      for (uint64_t i = at; i < at + m; ++i) {
        const uint32_t d = cold_src[i] - base;
        if (d >= (1u << 16)) return "binned chunk slot span exceeds 16 bits";
        packed[i] |= d << 16;
        if (i > at) lines += (packed[i] >> 20) != (packed[i - 1] >> 20);
      }
      chunks.push_back(BlkChunk{at, base, static_cast<uint16_t>(m), 1});
      cost.push_back(m + kBlkLineCost * lines);
      at += m;
    }
  }
  cfirst[nblk] = chunks.size();
  if (chunks.size() > (hot ? bin_chunks_cap(n, e) : blk_chunks_cap(n, e))) return "blocked chunk table overflow";
  // slices.  With fewer blocks than S (about one slice per CU, and only one
  // workgroup fits a CU's LDS): at most S slices in one even wave -- block
  // b gets K_b = ceil(C_b / L) slices (at least one, at most one per
  // chunk), C_b its chunks' cost, for the smallest limit L with
  // sum K_b <= S, which minimises the largest slice.  With more: the blocks
  // run in several rounds, one slice each, except those costlier than L,
  // cut into K_b slices, for the smallest L whose cut blocks' partial sums
  // (K_b x rows each) fit the partial buffer and add at most S slices.  A
  // block's slices hold about equal costs.
  std::vector<uint64_t> cb(nblk, 0);
  uint64_t ctotal = 0;
  for (uint64_t blk = 0; blk < nblk; ++blk) {
    for (uint64_t c = cfirst[blk]; c < cfirst[blk + 1]; ++c) cb[blk] += cost[c];
    ctotal += cb[blk];
  }
  const uint64_t S = blk_target_slices(e);
  std::vector<uint64_t> kb(nblk, 1);
  uint64_t nonempty = 0;
  for (uint64_t blk = 0; blk < nblk; ++blk) nonempty += cfirst[blk + 1] != cfirst[blk];
  if (e) {
    const bool one_wave = nonempty < S;
    // slices (of the blocks with edges) and partial rows under limit L
    auto cut = [&](uint64_t L, std::vector<uint64_t>* out, uint64_t* prow) {
      uint64_t total = 0, rows_cut = 0;
      for (uint64_t blk = 0; blk < nblk; ++blk) {
        const uint64_t nc = cfirst[blk + 1] - cfirst[blk];
        const uint64_t k = std::max<uint64_t>(1, std::min((cb[blk] + L - 1) / L, std::max<uint64_t>(nc, 1)));
        if (out) (*out)[blk] = k;
        if (nc) total += k;  // a block without edges only writes 0.15/N: not counted
        if (k > 1) rows_cut += k * (row0[blk + 1] - row0[blk]);
      }
      *prow = rows_cut;
      return total;
    };
    auto fits = [&](uint64_t L) {
      uint64_t prow = 0;
      const uint64_t total = cut(L, nullptr, &prow);
      return one_wave ? total <= S : (prow <= blk_partial_cap(e) && total <= nonempty + S);
    };
    uint64_t lo = 1, hi = ctotal;  // cut(ctotal): one slice per block, which fits either way
    while (lo < hi) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (fits(mid)) hi = mid;
      else lo = mid + 1;
    }
    uint64_t prow = 0;
    cut(lo, &kb, &prow);
  }
  std::vector<BlkSlice> slices;
  std::vector<BlkGroup> groups;
  uint64_t poff = 0;
  for (uint64_t blk = 0; blk < nblk; ++blk) {
    const uint64_t K = kb[blk];
    const uint32_t r0 = row0[blk], rows = row0[blk + 1] - row0[blk];
    if (cfirst[blk + 1] == cfirst[blk]) {  // no in-edges: the finish launch writes its rows (0.15/N)
      for (uint32_t g = 0; g < rows; g += 64) groups.push_back(BlkGroup{r0 + g, std::min<uint32_t>(64, rows - g), 0, rows, 0});
      continue;
    }
    if (K == 1) {
      slices.push_back(BlkSlice{r0, rows, static_cast<uint32_t>(cfirst[blk]), static_cast<uint32_t>(cfirst[blk + 1]),
                                kNoPartial});
      continue;
    }
    for (uint32_t g = 0; g < rows; g += 64)
      groups.push_back(BlkGroup{r0 + g, std::min<uint32_t>(64, rows - g), static_cast<uint32_t>(K), rows, poff + g});
    uint64_t c = cfirst[blk], done = 0;
    for (uint64_t j = 0; j < K; ++j) {
      const uint64_t c0 = c, goal = cb[blk] * (j + 1) / K;
      const uint64_t cmax = cfirst[blk + 1] - (K - 1 - j);  // leave a chunk for every later slice
      do {
        done += cost[c];
        ++c;
      } while (c < cmax && done < goal);
      if (j == K - 1) c = cfirst[blk + 1];
      slices.push_back(BlkSlice{r0, rows, static_cast<uint32_t>(c0), static_cast<uint32_t>(c), poff});
      poff += rows;
    }
  }
  if (poff > blk_partial_cap(e) || slices.size() > blk_blocks_cap(n, e) + blk_target_slices(e) ||
      groups.size() > blk_groups_cap(n, e))
    return "blocked slice table overflow";
  // Launch order.  With more slices than one wave of CUs (several rounds of
  // workgroups), the costliest first: workgroups are dispatched in launch
  // order as CUs free up, so the long slices start early and the short ones
  // fill the gaps at the end (measured at R-MAT scale 26: 3.76 -> 2.00 ms per
  // pull, every block holding edges of the same hot sources).
  if (slices.size() > kBlkSlices) {
    std::vector<uint64_t> sc(slices.size(), 0);
    for (size_t i = 0; i < slices.size(); ++i)
      for (uint32_t c = slices[i].c0; c < slices[i].c1; ++c) sc[i] += cost[c];
    std::vector<size_t> idx(slices.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return sc[x] > sc[y]; });
    std::vector<BlkSlice> sorted(slices.size());
    for (size_t i = 0; i < idx.size(); ++i) sorted[i] = slices[idx[i]];
    slices.swap(sorted);
  } else {
    // Within one wave, XCD-aware: workgroup i of a launch runs on XCD i mod
    // 8, and a slice's sources are a contiguous range (its chunks are sorted
    // by source).  The slices are sorted by their first source and XCD x
    // takes the x-th eighth of them, so that each XCD's L2 caches about an
    // eighth of the outbox array instead of all of it.
    const size_t ns = slices.size();
    auto first_src = [&](const BlkSlice& sl) -> uint64_t {
      const BlkChunk& ch = chunks[sl.c0];
      const uint64_t at = static_cast<uint64_t>(ch.wbase) + (packed[ch.e0] >> 16);
      return ch.cold ? slot_src[at] : at;
    };
    std::vector<size_t> idx(ns);
    for (size_t i = 0; i < ns; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](size_t x, size_t y) { return first_src(slices[x]) < first_src(slices[y]); });
    // XCD x runs the launch positions x, x + 8, ...: it takes that many
    // consecutive slices of the sorted order
    std::vector<BlkSlice> dealt(ns);
    size_t at = 0;
    for (size_t x = 0; x < kBlkXcds && x < ns; ++x)
      for (size_t p = x; p < ns; p += kBlkXcds) dealt[p] = slices[idx[at++]];
    slices.swap(dealt);
  }
  // the bin launch's tables: every cold window's runs in block order (a
  // stable counting sort of the runs by window), its list of slot sources,
  // and the first run of every kBinGroup list entries
  if (hot) {
    std::vector<uint32_t>().swap(cold_src);
    const uint32_t w0 = hot >> kBinWinBits;
    const uint64_t nw = bin_windows(n) - w0;
    std::vector<uint64_t> rstart(nw + 1, 0), fstart(nw + 1, 0);
    for (const RunRec& r : runs) {
      ++rstart[r.w - w0 + 1];
      fstart[r.w - w0 + 1] += r.len;
    }
    for (uint64_t w = 0; w < nw; ++w) {
      rstart[w + 1] += rstart[w];
      fstart[w + 1] += fstart[w];
    }
    std::vector<BinRun> wruns(runs.size());
    std::vector<uint16_t> wsrc(fstart[nw]);
    {
      std::vector<uint64_t> rc(rstart.begin(), rstart.end() - 1), fc(fstart.begin(), fstart.end() - 1);
      for (const RunRec& r : runs) {
        const uint64_t w = r.w - w0;
        const uint64_t f = fc[w];
        wruns[rc[w]++] = BinRun{static_cast<uint32_t>(f - fstart[w]), static_cast<uint32_t>(r.dst)};
        for (uint64_t j = 0; j < r.len; ++j)
          wsrc[f + j] = static_cast<uint16_t>(slot_src[r.dst + j] & ((1u << kBinWinBits) - 1));
        fc[w] += r.len;
      }
    }
    std::vector<uint64_t> gstart(nw + 1, 0);
    std::vector<uint32_t> group;
    for (uint64_t w = 0; w < nw; ++w) {
      gstart[w] = group.size();
      const uint64_t len = fstart[w + 1] - fstart[w];
      uint64_t r = rstart[w];
      for (uint64_t j = 0; j < len; j += kBinGroup) {
        while (r + 1 < rstart[w + 1] && wruns[r + 1].flat <= j) ++r;
        group.push_back(static_cast<uint32_t>(r - rstart[w]));
      }
    }
    gstart[nw] = group.size();
    if (group.size() > bin_groups_cap(n, e)) return "binned group table overflow";
    std::vector<BinUnit> units;
    for (uint64_t w = 0; w < nw; ++w) {
      const uint32_t ng = static_cast<uint32_t>(gstart[w + 1] - gstart[w]);
      for (uint32_t g = 0; g < ng; g += kBinUnitGroups)
        units.push_back(BinUnit{static_cast<uint32_t>(w), g, std::min(ng, g + kBinUnitGroups)});
    }
    if (units.size() > bin_units_cap(n, e)) return "binned unit table overflow";
    out->hot = hot;
    out->nslots = slot_src.size();
    out->bin_w0 = w0;
    out->bin_src.swap(wsrc);
    out->bin_runs.swap(wruns);
    out->bin_wflat.swap(fstart);
    out->bin_wrun.assign(rstart.begin(), rstart.end());
    out->bin_wgroup.swap(gstart);
    out->bin_group.swap(group);
    out->bin_units.swap(units);
  }
  out->packed.swap(packed);
  out->chunks.swap(chunks);
  out->slices.swap(slices);
  out->groups.swap(groups);
  out->row0.swap(row0);
  out->cfirst.swap(cfirst);
  return nullptr;
}

}  // namespace ipg
