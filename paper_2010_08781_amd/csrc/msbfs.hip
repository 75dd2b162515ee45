// msbfs.hip -- batched unweighted SSSP: up to 256 sources in one superstep
// loop over one graph.
//
// With unit weights every message sent in superstep s carries s + 1 (Fig.
// 10), so all messages that reach a mailbox in one superstep are equal, the
// min combiner keeps the first of them, and a vertex's distance is the first
// superstep in which it receives a message.  Q <= 256 SSSP queries on one
// graph can therefore share one superstep loop in which the one-slot mailbox
// of each (query, vertex) pair shrinks to one bit:
//   vis(v)   queries whose distance at v is set,
//   F_s(v)   queries for which v broadcasts in superstep s,
//   R_s(v)   queries for which v has a message in superstep s: the OR of
//            F_{s-1} over v's in-neighbours (the exchange of superstep s-1),
// and compute in superstep s is F_s = R_s & ~vis, vis |= F_s,
// dist[q][v] = s for every bit q of F_s.  Superstep 0 sets F_0 = vis = the
// source bit of each query.  Per query this is exactly the single-source run:
// the same values, and a superstep trace whose sum over queries is
//   active(s)   = sum_v popcount(R_s(v))        (N per query at s = 0),
//   senders(s)  = sum_v popcount(F_s(v)),
//   messages(s) = sum_v popcount(F_s(v)) * outdeg(v).
// The loop halts after the first superstep with no message (every query has
// halted), so it runs max over queries of their superstep counts.
//
// Exchange (chosen per superstep on the union frontier {v : F_s(v) != 0}):
//  * pull: every vertex ORs the masks of its in-neighbours over the CSC, on
//    the store's pull items (row pieces and long-row chunks), with the
//    gathered 32-byte masks staged in a wavefront-owned LDS tile;
//  * push: every vertex of the union frontier ORs its mask into its
//    out-neighbours' receive rows with 64-bit atomics; the first sender to
//    reach a vertex appends it to a touched list (wave-ballot compaction) and
//    a settle pass runs compute over that list.
// Masks are [N][4] uint64 rows (query q is bit q % 64 of word q / 64);
// distances are written as [Q][N] uint32 (query-major, INF = unreached).
#include <algorithm>
#include <vector>

#include "common.h"
#include "engine.h"
#include "scatter.h"

namespace ipg {

constexpr int kMsWords = 4;
constexpr uint32_t kMsMaxQueries = 64 * kMsWords;
static_assert(kMsMaxQueries == IPG_BATCH_MAX_SOURCES, "mask width");
// Edges whose masks are staged in LDS at once by a row item (per wavefront).
constexpr uint32_t kMsPass = 256;

typedef unsigned long long u64;

struct MsRun {
  uint32_t n;
  uint32_t level;  // superstep being computed
  const uint32_t* outdeg;
  const u64* f_in;   // F_{level-1}
  u64* f_out;        // F_level
  u64* vis;
  uint32_t* dist;    // [Q][n]
  uint32_t* list_out;
  uint32_t* list_cnt;
  CtrSlot* ctr;
  CtrSlot* ctr_clear;
};

struct MsPullArgs {
  MsRun r;
  PullTiling t;
  u64* partial;  // [chunks][4]
};

struct MsPushArgs {
  MsRun r;
  const uint64_t* off;  // CSR
  const int32_t* dst;
  const uint32_t* list_in;  // union frontier of the previous superstep
  uint32_t list_in_count;
  u64* recv;          // [n][4], zero outside a push superstep
  uint32_t* tflag;    // [n], zero outside a push superstep
  uint32_t* touched;  // [n]
  uint32_t* touched_cnt;
};

__device__ __forceinline__ void load_mask(const u64* base, uint32_t v, u64 m[kMsWords]) {
  const ulonglong2* p = reinterpret_cast<const ulonglong2*>(base + (size_t)v * kMsWords);
  const ulonglong2 a = p[0], b = p[1];
  m[0] = a.x;
  m[1] = a.y;
  m[2] = b.x;
  m[3] = b.y;
}

__device__ __forceinline__ void store_mask(u64* base, uint32_t v, const u64 m[kMsWords]) {
  ulonglong2* p = reinterpret_cast<ulonglong2*>(base + (size_t)v * kMsWords);
  p[0] = make_ulonglong2(m[0], m[1]);
  p[1] = make_ulonglong2(m[2], m[3]);
}

__device__ __forceinline__ u64 shfl_xor_u64(u64 x, int o) {
  return static_cast<u64>(__shfl_xor(static_cast<unsigned long long>(x), o));
}

struct MsCount {
  uint64_t active = 0, senders = 0, messages = 0, next_count = 0, next_deg = 0;
};

// Compute of vertex v in superstep `level` given its received bits R: the
// new bits F, the visited update, and the trace counters.  Returns whether
// v broadcasts for some query.
__device__ __forceinline__ bool ms_compute(const MsRun& a, uint32_t v, const u64 R[kMsWords], u64 F[kMsWords],
                                           MsCount& c) {
  u64 old[kMsWords];
  load_mask(a.vis, v, old);
  uint32_t pr = 0, pn = 0;
#pragma unroll
  for (int k = 0; k < kMsWords; ++k) {
    F[k] = R[k] & ~old[k];
    pr += __popcll(R[k]);
    pn += __popcll(F[k]);
    old[k] |= F[k];
  }
  store_mask(a.f_out, v, F);
  const bool sends = pn != 0;
  if (sends) store_mask(a.vis, v, old);
  const uint32_t d = a.outdeg[v];
  c.active += pr;
  c.senders += pn;
  c.messages += static_cast<uint64_t>(pn) * d;
  if (sends) {
    c.next_count += 1;
    c.next_deg += d;
  }
  return sends;
}

// dist[q][v] = level for every bit q of F (one thread, scattered stores).
__device__ __forceinline__ void ms_write_dist(const MsRun& a, uint32_t v, const u64 F[kMsWords]) {
#pragma unroll
  for (int k = 0; k < kMsWords; ++k) {
    u64 m = F[k];
    while (m) {
      const uint32_t b = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(m)) - 1);
      m &= m - 1;
      a.dist[(size_t)(64 * k + b) * a.n + v] = a.level;
    }
  }
}

// Superstep 0: one thread per query sets its source's bit in vis and F_0,
// writes distance 0, and appends each distinct source to the union frontier.
__global__ __launch_bounds__(kBlock) void ms_init_kernel(const uint32_t* sources, uint32_t q, MsRun a,
                                                         uint32_t* tflag) {
  const uint32_t i = threadIdx.x;
  uint64_t senders = 0, messages = 0, next_count = 0, next_deg = 0;
  bool fresh = false;
  uint32_t v = 0;
  if (i < q) {
    v = sources[i];
    const u64 bit = 1ull << (i & 63);
    atomicOr(a.vis + (size_t)v * kMsWords + (i >> 6), bit);
    atomicOr(a.f_out + (size_t)v * kMsWords + (i >> 6), bit);
    a.dist[(size_t)i * a.n + v] = 0;
    const uint32_t d = a.outdeg[v];
    senders = 1;
    messages = d;
    fresh = atomicOr(tflag + v, 1u) == 0u;
    if (fresh) {
      next_count = 1;
      next_deg = d;
    }
  }
  wave_append(fresh, v, a.list_out, a.list_cnt);
  flush_counters(a.ctr, senders, messages, next_count, next_deg, 0);
}

// Zero tflag for the listed vertices.
__global__ void ms_unflag_kernel(const uint32_t* list, const uint32_t* cnt, uint32_t* tflag) {
  const uint32_t c = *cnt;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c; i += gridDim.x * blockDim.x) tflag[list[i]] = 0;
}

// Zero the mask rows of the listed vertices (the non-zero rows of a level
// buffer about to be reused by a push superstep).
__global__ void ms_clear_rows_kernel(const uint32_t* list, const uint32_t* cnt, u64* f) {
  const uint32_t c = *cnt;
  const u64 z[kMsWords] = {0, 0, 0, 0};
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c; i += gridDim.x * blockDim.x)
    store_mask(f, list[i], z);
}

// Pull exchange of superstep level-1 and compute of superstep `level`, over
// the pull items (one wavefront per item, grid-stride over wavefronts).
//  * row item: in passes of kMsPass edges, every lane gathers the masks of
//    its edges' sources into the wavefront's LDS tile; a group of G lanes
//    per row ORs the row's entries (G from the item's row count); the
//    group's first lane computes the row; distances are then written per
//    query bit, with lanes over the item's rows (coalesced along v);
//  * long-row chunk: the OR of its edges' masks is stored as the chunk's
//    partial (combined by ms_longrow_kernel).
__global__ __launch_bounds__(kBlock) void ms_pull_kernel(MsPullArgs a) {
  constexpr int kPer = kMsPass / kWave;
  constexpr int kChunkPer = kWaveTile / kWave;
  constexpr int kRowPer = (kItemRows + kWave) / kWave;
  static_assert(kItemRows * kMsWords <= kMsPass * kMsWords, "new masks reuse the tile");
  __shared__ u64 s_tile[kWavesPerBlock][kMsPass][kMsWords];
  __shared__ uint32_t s_off[kWavesPerBlock][kItemRows + 1];
  clear_slots(a.r.ctr_clear);
  const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
  u64(*tile)[kMsWords] = s_tile[wv];
  uint32_t* soff = s_off[wv];
  const int32_t* src = a.t.src;
  const uint64_t* off = a.t.off;
  const uint32_t n = a.r.n;
  MsCount c;
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  for (uint32_t item = blockIdx.x * kWavesPerBlock + wv; item < a.t.ni; item += nw) {
    const PullItem it = a.t.items[item];
    const uint32_t ne = it.ne < kWaveTile ? it.ne : kWaveTile;
    if (it.slot != kNoSlot) {
      u64 acc[kMsWords] = {0, 0, 0, 0};
      int32_t u[kChunkPer];
#pragma unroll
      for (int k = 0; k < kChunkPer; ++k) {
        const uint32_t i = lane + k * kWave;
        u[k] = i < ne ? src[it.e0 + i] : -1;
      }
#pragma unroll
      for (int k = 0; k < kChunkPer; ++k) {
        if (u[k] >= 0) {
          u64 m[kMsWords];
          load_mask(a.r.f_in, static_cast<uint32_t>(u[k]), m);
#pragma unroll
          for (int w = 0; w < kMsWords; ++w) acc[w] |= m[w];
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int w = 0; w < kMsWords; ++w) acc[w] |= shfl_xor_u64(acc[w], o);
      if (lane == 0) store_mask(a.partial, it.slot, acc);
      continue;
    }
    const uint32_t nrows = it.r1 - it.r0;
#pragma unroll
    for (int k = 0; k < kRowPer; ++k) {
      const uint32_t r = lane + k * kWave;
      if (r <= nrows) soff[r] = static_cast<uint32_t>(off[it.r0 + r] - it.e0);
    }
    uint32_t G = kWave;
    while (G > 1 && G * nrows > kWave) G >>= 1;
    const uint32_t gi = lane / G, li = lane % G;  // group gi owns row gi (G * nrows <= 64)
    wave_lds_sync();
    uint32_t lo = 0, hi = 0;
    if (gi < nrows) {
      lo = soff[gi];
      hi = soff[gi + 1];
      if (hi > ne) hi = ne;
    }
    u64 acc[kMsWords] = {0, 0, 0, 0};
    for (uint32_t p0 = 0; p0 < ne; p0 += kMsPass) {
      int32_t u[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const uint32_t i = p0 + lane + k * kWave;
        u[k] = i < ne ? src[it.e0 + i] : -1;
      }
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        if (u[k] >= 0) {
          u64 m[kMsWords];
          load_mask(a.r.f_in, static_cast<uint32_t>(u[k]), m);
#pragma unroll
          for (int w = 0; w < kMsWords; ++w) tile[lane + k * kWave][w] = m[w];
        }
      }
      wave_lds_sync();
      const uint32_t b = lo > p0 ? lo : p0;
      const uint32_t e = hi < p0 + kMsPass ? hi : p0 + kMsPass;
      for (uint32_t j = b + li; j < e; j += G) {
#pragma unroll
        for (int w = 0; w < kMsWords; ++w) acc[w] |= tile[j - p0][w];
      }
      wave_lds_sync();  // the tile is rewritten by the next pass
    }
    for (uint32_t o = G >> 1; o >= 1; o >>= 1)
#pragma unroll
      for (int w = 0; w < kMsWords; ++w) acc[w] |= shfl_xor_u64(acc[w], static_cast<int>(o));
    const bool owner = li == 0 && gi < nrows;
    const uint32_t v = it.r0 + gi;
    bool sends = false;
    if (owner) {
      u64 F[kMsWords];
      sends = ms_compute(a.r, v, acc, F, c);
#pragma unroll
      for (int w = 0; w < kMsWords; ++w) tile[gi][w] = F[w];
    }
    wave_append(sends, v, a.r.list_out, a.r.list_cnt);
    wave_lds_sync();
    // distances: lane r holds the new bits of row r; one coalesced store
    // per query bit present in the item
    u64 mine[kMsWords] = {0, 0, 0, 0};
    if (lane < nrows) {
#pragma unroll
      for (int w = 0; w < kMsWords; ++w) mine[w] = tile[lane][w];
    }
#pragma unroll
    for (int w = 0; w < kMsWords; ++w) {
      u64 any = mine[w];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) any |= shfl_xor_u64(any, o);
      while (any) {
        const uint32_t bit = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(any)) - 1);
        any &= any - 1;
        if ((mine[w] >> bit) & 1ull) a.r.dist[(size_t)(64 * w + bit) * n + it.r0 + lane] = a.r.level;
      }
    }
    wave_lds_sync();  // the tile and offsets are rewritten by the next item
  }
  flush_counters(a.r.ctr, c.senders, c.messages, c.next_count, c.next_deg, 0, c.active);
}

// Second launch of a pull superstep: one wavefront per long row ORs the
// partials of its chunks and computes the row.
__global__ __launch_bounds__(kBlock) void ms_longrow_kernel(MsPullArgs a) {
  const uint32_t l = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  const uint32_t lane = lane_id();
  MsCount c;
  if (l < a.t.nl) {  // wave-uniform
    const uint32_t f = a.t.lr_first[l], nch = a.t.lr_first[l + 1] - f;
    u64 acc[kMsWords] = {0, 0, 0, 0};
    for (uint32_t i = lane; i < nch; i += kWave) {
      u64 m[kMsWords];
      load_mask(a.partial, f + i, m);
#pragma unroll
      for (int w = 0; w < kMsWords; ++w) acc[w] |= m[w];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
      for (int w = 0; w < kMsWords; ++w) acc[w] |= shfl_xor_u64(acc[w], o);
    const uint32_t v = a.t.long_rows[l];
    u64 F[kMsWords] = {0, 0, 0, 0};
    bool sends = false;
    if (lane == 0) sends = ms_compute(a.r, v, acc, F, c);
    wave_append(sends, v, a.r.list_out, a.r.list_cnt);
#pragma unroll
    for (int w = 0; w < kMsWords; ++w) {
      const u64 fw = static_cast<u64>(__shfl(static_cast<unsigned long long>(F[w]), 0));
      if ((fw >> lane) & 1ull) a.r.dist[(size_t)(64 * w + lane) * a.r.n + v] = a.r.level;
    }
  }
  flush_counters(a.r.ctr, c.senders, c.messages, c.next_count, c.next_deg, 0, c.active);
}

// Push exchange of superstep level-1: one thread per union-frontier vertex,
// out-edges expanded by twc_scatter; each edge ORs the sender's mask into the
// recipient's receive row.  The first sender to flag a recipient appends it
// to the touched list.
__global__ __launch_bounds__(kBlock) void ms_push_kernel(MsPushArgs a) {
  clear_slots(a.r.ctr_clear);
  const uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
  bool has = false;
  uint64_t beg = 0, end = 0;
  uint32_t u = 0;
  if (i < a.list_in_count) {
    u = a.list_in[i];
    beg = a.off[u];
    end = a.off[u + 1];
    has = end > beg;
  }
  twc_scatter(has, beg, end, u, [&](uint64_t e, uint32_t p) {
    const uint32_t x = static_cast<uint32_t>(a.dst[e]);
    u64 m[kMsWords];
    load_mask(a.r.f_in, p, m);
#pragma unroll
    for (int w = 0; w < kMsWords; ++w)
      if (m[w]) atomicOr(a.recv + (size_t)x * kMsWords + w, m[w]);
    const bool fresh = atomicOr(a.tflag + x, 1u) == 0u;
    wave_append(fresh, x, a.touched, a.touched_cnt);
  });
}

// Compute of a push superstep over the touched list: consume (and zero) the
// receive rows.
__global__ __launch_bounds__(kBlock) void ms_settle_kernel(MsPushArgs a) {
  MsCount c;
  const uint32_t cnt = *a.touched_cnt;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const uint32_t v = a.touched[i];
    u64 R[kMsWords], F[kMsWords];
    load_mask(a.recv, v, R);
    const u64 z[kMsWords] = {0, 0, 0, 0};
    store_mask(a.recv, v, z);
    a.tflag[v] = 0;
    const bool sends = ms_compute(a.r, v, R, F, c);
    wave_append(sends, v, a.r.list_out, a.r.list_cnt);
    if (sends) ms_write_dist(a.r, v, F);
  }
  flush_counters(a.r.ctr, c.senders, c.messages, c.next_count, c.next_deg, 0, c.active);
}

// ------------------------------------------------------------------ host --

struct MsWs {
  u64* vis;
  u64* f[2];
  u64* recv;
  u64* partial;
  uint32_t* tflag;
  uint32_t* list[2];
  uint32_t* touched;
  uint32_t* cnt;  // [4]: list[0] length, list[1] length, touched length, spare
  CtrSlot* ctr;   // [2][kCtrSlots]
  Decision* decision;
};

static size_t carve_ms(Carver& c, uint32_t n, uint64_t e, MsWs* out) {
  MsWs w{};
  const size_t nn = n ? n : 1;
  w.vis = c.take<u64>(nn * kMsWords);
  w.f[0] = c.take<u64>(nn * kMsWords);
  w.f[1] = c.take<u64>(nn * kMsWords);
  w.recv = c.take<u64>(nn * kMsWords);
  w.partial = c.take<u64>(chunks_cap(e) * kMsWords);
  w.tflag = c.take<uint32_t>(nn);
  w.list[0] = c.take<uint32_t>(nn);
  w.list[1] = c.take<uint32_t>(nn);
  w.touched = c.take<uint32_t>(nn);
  w.cnt = c.take<uint32_t>(4);
  w.ctr = c.take<CtrSlot>(2 * kCtrSlots);
  w.decision = c.take<Decision>(1);
  if (out) *out = w;
  return align_up(c.used, 256);
}

// Superstep-level exchange choice on the union frontier: the library's
// fixed rule, pull when the frontier and its out-edges exceed E / div.
static ipg_mode ms_mode(ipg_mode forced, uint64_t e, uint64_t frontier, uint64_t frontier_deg, uint32_t div) {
  if (forced == IPG_MODE_PUSH || forced == IPG_MODE_PULL) return forced;
  if (e == 0) return IPG_MODE_PUSH;
  return frontier + frontier_deg > e / (div ? div : 20) ? IPG_MODE_PULL : IPG_MODE_PUSH;
}

static ipg_status run_msbfs(ipg_graph* g, const uint32_t* sources, uint32_t q, uint32_t cap, const ipg_run_opts& o,
                            uint32_t* dist, const MsWs& w, hipStream_t s, StepTimer& tm, ipg_run_stats* st) {
  const uint32_t n = g->n;
  const uint64_t e = g->e;
  IPG_HIP(fill_u32(dist, (uint64_t)q * n, kInf, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.vis), (uint64_t)n * 2 * kMsWords, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.f[0]), (uint64_t)n * 2 * kMsWords, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.f[1]), (uint64_t)n * 2 * kMsWords, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.recv), (uint64_t)n * 2 * kMsWords, 0, s));
  IPG_HIP(fill_u32(w.tflag, n, 0, s));
  IPG_HIP(fill_u32(w.cnt, 4, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.ctr), 2 * kCtrSlots * sizeof(CtrSlot) / 4, 0, s));

  MsRun r{};
  r.n = n;
  r.outdeg = g->t.outdeg;
  r.vis = w.vis;
  r.dist = dist;
  const PullTiling t = pull_tiling(g);
  uint64_t tot_msgs = 0, tot_exam = 0;
  uint64_t frontier = 0, frontier_deg = 0;
  uint64_t list_len[2] = {0, 0};  // union-frontier list lengths held in list[0] / list[1]
  uint32_t step = 0;
  ipg_status status = IPG_OK;
  IPG_HIP(tm.start(s));
  for (;;) {
    const int cur = step & 1, prev = cur ^ 1;
    CtrSlot* c = w.ctr + cur * kCtrSlots;
    CtrSlot* cc = w.ctr + prev * kCtrSlots;
    r.level = step;
    r.f_out = w.f[cur];
    r.f_in = w.f[prev];
    r.list_out = w.list[cur];
    r.list_cnt = w.cnt + cur;
    r.ctr = c;
    r.ctr_clear = cc;
    ipg_mode mode = IPG_MODE_PUSH;
    uint64_t examined = 0;
    if (step == 0) {
      hipLaunchKernelGGL(ms_init_kernel, dim3(1), dim3(kBlock), 0, s, sources, q, r, w.tflag);
      IPG_HIP(hipGetLastError());
      hipLaunchKernelGGL(ms_unflag_kernel, dim3(1), dim3(kBlock), 0, s, w.list[cur], w.cnt + cur, w.tflag);
      IPG_HIP(hipGetLastError());
    } else {
      mode = ms_mode(o.mode, e, frontier, frontier_deg, 20);
      if (mode == IPG_MODE_PUSH) {
        const uint32_t gc = grid_for(std::min<uint64_t>(frontier_deg + 1, n), kBlock, kExchangeGrid);
        if (list_len[cur]) {
          hipLaunchKernelGGL(ms_clear_rows_kernel, dim3(grid_for(list_len[cur], kBlock, kExchangeGrid)), dim3(kBlock),
                             0, s, w.list[cur], w.cnt + cur, w.f[cur]);
          IPG_HIP(hipGetLastError());
        }
        IPG_HIP(fill_u32(w.cnt + cur, 1, 0, s));
        IPG_HIP(fill_u32(w.cnt + 2, 1, 0, s));
        MsPushArgs a;
        a.r = r;
        a.off = g->csr_off;
        a.dst = g->csr_dst;
        a.list_in = w.list[prev];
        a.list_in_count = static_cast<uint32_t>(frontier);
        a.recv = w.recv;
        a.tflag = w.tflag;
        a.touched = w.touched;
        a.touched_cnt = w.cnt + 2;
        hipLaunchKernelGGL(ms_push_kernel, dim3(grid_for(frontier, kBlock, 0xFFFFFFFFu)), dim3(kBlock), 0, s, a);
        IPG_HIP(hipGetLastError());
        a.r.ctr_clear = nullptr;
        hipLaunchKernelGGL(ms_settle_kernel, dim3(gc), dim3(kBlock), 0, s, a);
        IPG_HIP(hipGetLastError());
        examined = frontier_deg;
      } else {
        IPG_HIP(fill_u32(w.cnt + cur, 1, 0, s));
        MsPullArgs a;
        a.r = r;
        a.t = t;
        a.partial = w.partial;
        if (g->ni) {
          hipLaunchKernelGGL(ms_pull_kernel, dim3(std::min(g->ni, kPullGrid)), dim3(kBlock), 0, s, a);
          IPG_HIP(hipGetLastError());
        }
        a.r.ctr_clear = nullptr;
        if (g->nl) {
          hipLaunchKernelGGL(ms_longrow_kernel, dim3((g->nl + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0,
                             s, a);
          IPG_HIP(hipGetLastError());
        }
        examined = e;
      }
    }
    IPG_HIP(tm.step(s, step));
    IPG_HIP(launch_decide(c, step + 1, e, nullptr, w.decision, s));
    Decision h;
    IPG_HIP(hipMemcpyAsync(&h, w.decision, sizeof(h), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    const uint64_t active = step == 0 ? (uint64_t)q * n : h.active;
    if (st && step < st->trace_cap) {
      if (st->active) st->active[step] = active;
      if (st->senders) st->senders[step] = h.senders;
      if (st->messages) st->messages[step] = h.messages;
      if (st->examined) st->examined[step] = examined;
      if (st->mode) st->mode[step] = static_cast<uint8_t>(step == 0 ? IPG_MODE_PUSH : mode);
      if (st->frontier_deg) st->frontier_deg[step] = frontier_deg;
    }
    tot_msgs += h.messages;
    tot_exam += examined;
    list_len[cur] = h.next_count;
    ++step;
    if (h.messages == 0) break;  // no message pending for any query: all halted
    if (cap && step >= cap) {
      status = IPG_NOT_CONVERGED;
      break;
    }
    frontier = h.next_count;
    frontier_deg = h.next_deg;
  }
  IPG_HIP(tm.finish(s));
  if (st) {
    st->supersteps = step;
    st->halted = status == IPG_OK;
    st->edges_traversed = tot_msgs;
    st->edges_examined = tot_exam;
  }
  return status;
}

}  // namespace ipg

using namespace ipg;

extern "C" size_t ipg_multi_sssp_workspace_bytes(uint32_t num_vertices, uint64_t num_edges) {
  Carver c(nullptr);
  return carve_ms(c, num_vertices, num_edges, nullptr);
}

extern "C" ipg_status ipg_run_multi_sssp(ipg_graph* g, const uint32_t* sources, uint32_t num_sources,
                                         uint32_t max_supersteps, const ipg_run_opts* opts, uint32_t* dist,
                                         size_t dist_bytes, void* ws, size_t ws_bytes, void* hip_stream,
                                         ipg_run_stats* st) {
  if (!g || !sources || !dist) return fail(IPG_EINVAL, "ipg_run_multi_sssp: NULL argument");
  if (num_sources == 0 || num_sources > kMsMaxQueries)
    return fail(IPG_EINVAL, "ipg_run_multi_sssp: num_sources must be in [1, 256]");
  if (g->csr_w) return fail(IPG_EUNSUPPORTED, "ipg_run_multi_sssp: the graph has edge weights (unit weights only)");
  ipg_run_opts o{0, IPG_MODE_AUTO, 0, nullptr};
  if (opts) o = *opts;
  if (o.mode != IPG_MODE_AUTO && o.mode != IPG_MODE_PUSH && o.mode != IPG_MODE_PULL)
    return fail(IPG_EINVAL, "ipg_run_multi_sssp: unknown mode");
  const size_t need_dist = (size_t)num_sources * g->n * sizeof(uint32_t);
  if (dist_bytes < need_dist)
    return fail(IPG_EINVAL, "ipg_run_multi_sssp: dist needs " + std::to_string(need_dist) + " bytes");
  const size_t need = ipg_multi_sssp_workspace_bytes(g->n, g->e);
  if (!ws || ws_bytes < need)
    return fail(IPG_EWORKSPACE, "ipg_run_multi_sssp: workspace needs " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(IPG_EWORKSPACE, "ipg_run_multi_sssp: workspace must be 256-byte aligned");
  int dev = -1;
  IPG_HIP(hipGetDevice(&dev));
  if (dev != g->device) return fail(IPG_EINVAL, "ipg_run_multi_sssp: current device differs from the graph's device");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // The sources are checked on the host before any kernel indexes with them.
  std::vector<uint32_t> hsrc(num_sources);
  IPG_HIP(hipMemcpyAsync(hsrc.data(), sources, num_sources * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipStreamSynchronize(s));
  for (uint32_t i = 0; i < num_sources; ++i)
    if (hsrc[i] >= g->n) return fail(IPG_EINVAL, "ipg_run_multi_sssp: source " + std::to_string(i) + " >= N");
  Carver c(ws);
  MsWs w;
  carve_ms(c, g->n, g->e, &w);
  StepTimer tm(st ? st->usec : nullptr, st ? st->trace_cap : 0);
  const ipg_status rc = run_msbfs(g, sources, num_sources, max_supersteps, o, dist, w, s, tm, st);
  if (st) st->seconds = tm.seconds();
  if (rc == IPG_OK) set_error("");
  return rc;
}
