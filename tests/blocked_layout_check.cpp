// Host check of the blocked in-edge layout (blocked_layout.h) on a CSC read
// from a file.  It decodes the tables the kernels read -- packed edges,
// chunks, slices in launch order, finish groups -- and checks, without
// re-running the layout construction's own steps:
//   * the decoded (source, destination) pairs are the CSC's edges, as a multiset;
//   * blocks partition [0, N) in order, each at most kBlkRows rows, closed by
//     the stated rule (edge target or row cap), and hold their edges sorted
//     by source, ties by destination;
//   * chunks tile [0, E) in order, hold 1 .. kBlkChunk edges, never leave
//     their source window, never straddle two blocks;
//   * each block's chunks are cut into K contiguous, non-empty slices, at
//     most S in all when fewer than S blocks have edges, else adding at
//     most S slices to one per block;
//   * partial-sum offsets: none for a one-slice block, K disjoint runs of
//     the block's rows otherwise, within the stated bound;
//   * finish groups cover exactly the rows of the multi-slice and edge-less
//     blocks, 64 rows at a time, with the block's K, stride and offsets;
//   * launch position p runs on XCD p mod 8: each XCD holds the number of
//     positions that mapping gives it, and the XCDs take consecutive runs
//     of the slices sorted by first source;
//   * every table stays within its size bound;
//   * with binned cold sources (a hot count as second argument): the bin
//     launch's tables give every slot exactly one source, runs of whole
//     kBinPad-slot lines, each window's runs in slot order, group entries
//     naming the run that holds their first list entry; cold chunks decode
//     through them (and hold only cold sources, after the block's hot
//     chunks), so that the edge multiset check covers the binned edges too.
// Input file: uint32 N, uint64 E, uint64 off[N + 1], int32 src[E].
// Prints "OK blocks=.. chunks=.. slices=.. groups=.. partial=..", or
// "ERR <message>" when the build rejects the CSC, or "FAIL <what>".
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <tuple>

#include "blocked_layout.h"

using namespace ipg;

static int fail(const std::string& what) {
  std::printf("FAIL %s\n", what.c_str());
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 2 && argc != 3) return fail("usage: blocked_layout_check <csc file> [hot sources]");
  const uint32_t hot_arg = argc == 3 ? static_cast<uint32_t>(std::strtoul(argv[2], nullptr, 10)) : 0u;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return fail("cannot open input");
  uint32_t n = 0;
  uint64_t e = 0;
  if (std::fread(&n, 4, 1, f) != 1 || std::fread(&e, 8, 1, f) != 1) return fail("short header");
  std::vector<uint64_t> off((size_t)n + 1);
  std::vector<int32_t> src(e);
  if (std::fread(off.data(), 8, off.size(), f) != off.size()) return fail("short offsets");
  if (e && std::fread(src.data(), 4, e, f) != e) return fail("short sources");
  std::fclose(f);

  BlockedLayout L;
  if (const char* msg = blocked_layout(n, e, off.data(), src.data(), &L, hot_arg)) {
    std::printf("ERR %s\n", msg);
    return 0;
  }
  const auto& P = L.packed;
  const auto& C = L.chunks;
  const auto& SL = L.slices;
  const auto& G = L.groups;
  if (P.size() != e) return fail("packed size");
  if (C.size() > (L.hot ? bin_chunks_cap(n, e) : blk_chunks_cap(n, e))) return fail("chunk cap");
  if (hot_arg && L.hot && (L.hot < hot_arg || L.hot % (1u << kBlkWinBits))) return fail("hot count not rounded up to windows");

  // bin tables: the source of every slot
  const uint32_t kNone = 0xFFFFFFFFu;
  std::vector<uint32_t> slot_src(L.nslots, kNone);
  if (L.hot) {
    const uint64_t nw = bin_windows(n) - L.bin_w0;
    if (L.bin_w0 != (L.hot >> kBinWinBits)) return fail("first cold window");
    if (L.bin_wflat.size() != nw + 1 || L.bin_wrun.size() != nw + 1 || L.bin_wgroup.size() != nw + 1)
      return fail("window table sizes");
    if (L.nslots > bin_slots_cap(n, e) || L.bin_runs.size() > bin_runs_cap(n, e) ||
        L.bin_group.size() > bin_groups_cap(n, e) || L.bin_src.size() != L.nslots)
      return fail("bin table caps");
    for (uint64_t w = 0; w < nw; ++w) {
      const uint64_t f0 = L.bin_wflat[w], f1 = L.bin_wflat[w + 1];
      const uint32_t r0 = L.bin_wrun[w], r1 = L.bin_wrun[w + 1];
      if (f1 < f0 || r1 < r0) return fail("window tables not ascending");
      if ((r0 == r1) != (f0 == f1)) return fail("window with slots but no runs, or runs but no slots");
      const uint64_t len = f1 - f0;
      for (uint32_t r = r0; r < r1; ++r) {
        const BinRun& R = L.bin_runs[r];
        const uint64_t end = r + 1 < r1 ? L.bin_runs[r + 1].flat : len;
        if (r == r0 && R.flat != 0) return fail("window's first run does not start its list");
        if (end <= R.flat || (end - R.flat) % kBinPad || R.dst % kBinPad) return fail("run not whole lines");
        if (r > r0 && R.dst <= L.bin_runs[r - 1].dst) return fail("window's runs not in slot order");
        for (uint64_t j = R.flat; j < end; ++j) {
          const uint64_t slot = R.dst + (j - R.flat);
          if (slot >= L.nslots) return fail("run past the slot array");
          if (slot_src[slot] != kNone) return fail("slot in two runs");
          slot_src[slot] = static_cast<uint32_t>(((L.bin_w0 + w) << kBinWinBits) + L.bin_src[f0 + j]);
          if (slot_src[slot] >= n) return fail("slot source outside the graph");
        }
      }
      const uint64_t g0 = L.bin_wgroup[w], g1 = L.bin_wgroup[w + 1];
      if (g1 - g0 != (len + kBinGroup - 1) / kBinGroup) return fail("group count of a window");
      for (uint64_t g = g0; g < g1; ++g) {
        const uint64_t j = (g - g0) * kBinGroup;
        const uint32_t r = r0 + L.bin_group[g];
        if (r >= r1 || L.bin_runs[r].flat > j || (r + 1 < r1 && L.bin_runs[r + 1].flat <= j))
          return fail("group entry does not name the run of its first slot");
      }
    }
    for (uint64_t k = 0; k < L.nslots; ++k)
      if (slot_src[k] == kNone) return fail("slot without a run");
    // work units: each window's groups in order, once, at most kBinUnitGroups per unit
    if (L.bin_units.size() > bin_units_cap(n, e)) return fail("unit cap");
    {
      uint64_t w = 0, g = 0;
      for (const BinUnit& u : L.bin_units) {
        while (w < nw && g == L.bin_wgroup[w + 1] - L.bin_wgroup[w]) {
          ++w;
          g = 0;
        }
        if (u.win != w || u.g0 != g || u.g1 <= u.g0 || u.g1 - u.g0 > kBinUnitGroups ||
            u.g1 > L.bin_wgroup[w + 1] - L.bin_wgroup[w])
          return fail("bin units do not tile the windows' groups");
        g = u.g1;
      }
      while (w < nw && g == L.bin_wgroup[w + 1] - L.bin_wgroup[w]) {
        ++w;
        g = 0;
      }
      if (w != nw) return fail("bin units miss groups");
    }
  }
  if (G.size() > blk_groups_cap(n, e)) return fail("group cap");
  if (SL.size() > blk_blocks_cap(n, e) + blk_target_slices(e)) return fail("slice cap");

  // blocks: partition of [0, N), row cap, closing rule
  const auto& R0 = L.row0;
  const size_t nb = R0.size() - 1;
  if (R0.empty() || R0.front() != 0 || R0.back() != n) return fail("block starts");
  if (nb > blk_blocks_cap(n, e)) return fail("block cap");
  const uint64_t target = blk_edge_target(n, e);
  auto deg = [&](uint32_t v) { return off[(size_t)v + 1] - off[v]; };
  std::vector<uint64_t> bedges(nb, 0);
  for (size_t b = 0; b < nb; ++b) {
    if (R0[b + 1] <= R0[b] && n) return fail("empty block");
    if (R0[b + 1] - R0[b] > kBlkRows) return fail("block over kBlkRows rows");
    for (uint32_t v = R0[b]; v < R0[b + 1]; ++v) bedges[b] += deg(v);
    if (R0[b + 1] - R0[b] > 1 && bedges[b] > target) return fail("block past the edge target");
    if (b + 1 < nb && R0[b + 1] - R0[b] < kBlkRows && bedges[b] + deg(R0[b + 1]) <= target)
      return fail("block closed early");
  }
  std::vector<uint32_t> blk_of(n);
  for (size_t b = 0; b < nb; ++b)
    for (uint32_t v = R0[b]; v < R0[b + 1]; ++v) blk_of[v] = static_cast<uint32_t>(b);

  // chunks: tile [0, E); decode every edge; block and window fixed per chunk
  std::vector<uint32_t> chunk_blk(C.size());
  std::vector<std::pair<uint32_t, uint32_t>> dec(e);  // (source, destination) in packed order
  {
    uint64_t at = 0;
    size_t b = 0;
    uint64_t bend = nb ? bedges[0] : 0;
    for (size_t c = 0; c < C.size(); ++c) {
      const BlkChunk& ch = C[c];
      if (ch.e0 != at) return fail("chunks do not tile the edges");
      if (ch.n < 1 || ch.n > kBlkChunk || ch.cold > 1) return fail("chunk size or flag");
      if (ch.cold && !L.hot) return fail("cold chunk without binning");
      if (!ch.cold && (ch.wbase & ((1u << kBlkWinBits) - 1))) return fail("window base not aligned");
      while (b + 1 < nb && at >= bend) bend += bedges[++b];
      if (at >= bend || at + ch.n > bend) return fail("chunk straddles two blocks");
      chunk_blk[c] = static_cast<uint32_t>(b);
      if (c && chunk_blk[c - 1] == b && C[c - 1].cold && !ch.cold) return fail("hot chunk after a cold one");
      for (uint64_t i = at; i < at + ch.n; ++i) {
        uint64_t u = static_cast<uint64_t>(ch.wbase) + (P[i] >> 16);
        if (ch.cold) {
          if (u >= L.nslots) return fail("cold edge past the slot array");
          u = slot_src[u];
          if (u < L.hot) return fail("cold chunk holds a hot source");
        } else if (L.hot && u >= L.hot) {
          return fail("hot chunk holds a cold source");
        }
        const uint64_t v = static_cast<uint64_t>(R0[b]) + (P[i] & 0xFFFFu);
        if (u >= n || v >= R0[b + 1]) return fail("decoded edge outside the graph or the block");
        dec[i] = {static_cast<uint32_t>(u), static_cast<uint32_t>(v)};
      }
      at += ch.n;
    }
    if (at != e) return fail("chunks do not cover the edges");
  }
  // sorted by source within every block (ties by destination)
  for (uint64_t i = 1; i < e; ++i)
    if (blk_of[dec[i].second] == blk_of[dec[i - 1].second] && dec[i] < dec[i - 1])
      return fail("block not sorted by source");
  // the same edges as the CSC
  {
    std::vector<std::pair<uint32_t, uint32_t>> a(dec), ref;
    ref.reserve(e);
    for (uint32_t v = 0; v < n; ++v)
      for (uint64_t i = off[v]; i < off[(size_t)v + 1]; ++i) ref.push_back({static_cast<uint32_t>(src[i]), v});
    std::sort(a.begin(), a.end());
    std::sort(ref.begin(), ref.end());
    if (a != ref) return fail("edges differ from the CSC");
  }

  // slices: per block, K contiguous non-empty chunk ranges covering its chunks
  std::vector<std::vector<const BlkSlice*>> by_blk(nb);
  for (const BlkSlice& s : SL) {
    if (s.c0 >= s.c1 || s.c1 > C.size()) return fail("slice chunk range");
    const uint32_t b = chunk_blk[s.c0];
    if (chunk_blk[s.c1 - 1] != b) return fail("slice spans two blocks");
    if (s.row0 != R0[b] || s.rows != R0[b + 1] - R0[b]) return fail("slice rows are not its block's");
    by_blk[b].push_back(&s);
  }
  const uint64_t S = blk_target_slices(e);
  uint64_t nonempty = 0, ksum = 0, maxk = 0;
  std::vector<uint64_t> kb(nb, 0);
  std::vector<std::pair<uint64_t, uint64_t>> runs;  // partial-sum runs [poff, poff + rows)
  for (size_t b = 0; b < nb; ++b) {
    auto& v = by_blk[b];
    std::sort(v.begin(), v.end(), [](const BlkSlice* x, const BlkSlice* y) { return x->c0 < y->c0; });
    const bool has_edges = bedges[b] > 0;
    if (!has_edges) {
      if (!v.empty()) return fail("slice for an edge-less block");
      continue;
    }
    ++nonempty;
    if (v.empty()) return fail("block with edges has no slice");
    uint32_t c = v.front()->c0;
    if (c > 0 && chunk_blk[c - 1] == b) return fail("block's first chunk not in a slice");
    for (const BlkSlice* s : v) {
      if (s->c0 != c) return fail("slices of a block not contiguous");
      c = s->c1;
    }
    if (c < C.size() && chunk_blk[c] == b) return fail("block's last chunk not in a slice");
    const uint64_t K = v.size();
    kb[b] = K;
    ksum += K;
    maxk = std::max(maxk, K);
    const uint64_t rows = R0[b + 1] - R0[b];
    if (K == 1) {
      if (v[0]->poff != kNoPartial) return fail("one-slice block with a partial offset");
    } else {
      for (uint64_t j = 0; j < K; ++j) {
        if (v[j]->poff != v[0]->poff + j * rows) return fail("partial offsets not in slice order");
        runs.push_back({v[j]->poff, v[j]->poff + rows});
      }
    }
  }
  if (nonempty < S) {
    if (e && ksum > S) return fail("more slices than the target");
  } else if (ksum > nonempty + S) {
    return fail("cut blocks add more than S slices");
  }
  std::sort(runs.begin(), runs.end());
  for (size_t i = 0; i < runs.size(); ++i) {
    if (i && runs[i].first < runs[i - 1].second) return fail("partial runs overlap");
    if (runs[i].second > blk_partial_cap(e)) return fail("partial runs past their bound");
  }

  // finish groups: exactly the rows of the multi-slice and edge-less blocks
  std::vector<uint8_t> covered(n, 0);
  for (const BlkGroup& g : G) {
    if (g.nrows < 1 || g.nrows > 64 || g.row0 + static_cast<uint64_t>(g.nrows) > n) return fail("group rows");
    const uint32_t b = blk_of[g.row0];
    if (g.row0 + g.nrows > R0[b + 1]) return fail("group spans two blocks");
    if ((g.row0 - R0[b]) % 64) return fail("group not on a 64-row step of its block");
    if (g.nrows != std::min<uint32_t>(64, R0[b + 1] - g.row0)) return fail("group shorter than it could be");
    if (g.k != kb[b] || g.stride != R0[b + 1] - R0[b]) return fail("group k or stride");
    if (kb[b] == 1) return fail("group for a one-slice block");
    if (g.k && g.poff != by_blk[b][0]->poff + (g.row0 - R0[b])) return fail("group partial offset");
    for (uint32_t r = g.row0; r < g.row0 + g.nrows; ++r) {
      if (covered[r]) return fail("row in two groups");
      covered[r] = 1;
    }
  }
  for (size_t b = 0; b < nb; ++b)
    for (uint32_t r = R0[b]; r < R0[b + 1]; ++r)
      if (covered[r] != (kb[b] != 1)) return fail("row not finished exactly once");

  // launch order: with more slices than kBlkSlices, costliest first (cost =
  // edges + kBlkLineCost per 128-byte line of values the chunk reads: 16
  // outboxes, or 16 slots of a cold chunk); else the XCD deal
  if (SL.size() > kBlkSlices) {
    auto chunk_cost = [&](const BlkChunk& ch) {
      uint64_t lines = 1;
      for (uint64_t i = ch.e0 + 1; i < ch.e0 + ch.n; ++i) lines += (P[i] >> 20) != (P[i - 1] >> 20);
      return ch.n + kBlkLineCost * lines;
    };
    uint64_t prev = UINT64_MAX;
    for (const BlkSlice& s : SL) {
      uint64_t c = 0;
      for (uint32_t k = s.c0; k < s.c1; ++k) c += chunk_cost(C[k]);
      if (c > prev) return fail("slices not in descending cost order");
      prev = c;
    }
  } else {
    const size_t ns = SL.size();
    auto first_src = [&](const BlkSlice& s) { return dec[C[s.c0].e0].first; };
    std::vector<uint32_t> last_on(kBlkXcds, 0), first_on(kBlkXcds, UINT32_MAX);
    std::vector<size_t> count(kBlkXcds, 0);
    for (size_t p = 0; p < ns; ++p) {
      const size_t x = p % kBlkXcds;
      const uint32_t fs = first_src(SL[p]);
      if (count[x] && fs < last_on[x]) return fail("slices of an XCD not sorted by first source");
      if (!count[x]) first_on[x] = fs;
      last_on[x] = fs;
      ++count[x];
    }
    for (size_t x = 0; x < kBlkXcds; ++x) {
      if (count[x] != (ns > x ? (ns - x + kBlkXcds - 1) / kBlkXcds : 0)) return fail("XCD slice count");
      if (x + 1 < kBlkXcds && count[x + 1] && last_on[x] > first_on[x + 1]) return fail("XCD ranges out of order");
    }
  }
  uint64_t partial = 0;
  for (const auto& r : runs) partial = std::max(partial, r.second);
  std::printf("OK blocks=%zu chunks=%zu slices=%zu groups=%zu partial=%llu hot=%u slots=%llu runs=%zu\n", nb,
              C.size(), SL.size(), G.size(), static_cast<unsigned long long>(partial), L.hot,
              static_cast<unsigned long long>(L.nslots), L.bin_runs.size());
  return 0;
}
