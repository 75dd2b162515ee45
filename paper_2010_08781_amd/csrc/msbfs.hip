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
//    out-neighbours' receive rows with 64-bit atomics and sets their bits in
//    a touched bitmap; a settle pass runs compute on the touched vertices.
// The union frontier of each superstep is kept as a bitmap of the non-empty
// rows of F_s (set by wave-reduced atomic ORs spread over N/32 words: a
// list with one shared counter costs one same-address atomic per
// wavefront, and those serialize device-wide).
// Masks are [N][4] uint64 rows (query q is bit q % 64 of word q / 64).  The
// masks F_s of the last kMsHist supersteps are kept (a ring of level
// buffers); distances are not written per superstep but expanded from that
// history into [Q][N] uint32 (query-major, INF = unreached) by one
// coalesced pass when the ring is full and at the end of the run.  A sparse
// pull superstep reads a bitmap of the non-empty rows of F_{s-1} first and
// gathers only those rows.
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
// Supersteps of level masks kept before they are expanded into distances.
constexpr uint32_t kMsHist = 16;
constexpr int kMsHistBits = 4;
static_assert((1u << kMsHistBits) == kMsHist, "level index bits");

typedef unsigned long long u64;

// Control block of the device-driven form (the host loop's state, in device
// memory): advanced by ms_dd_decide_kernel at the end of every superstep and
// read by every kernel of the next one.
struct MsCtl {
  uint32_t step;       // superstep about to run
  uint32_t halted;
  int32_t status;      // IPG_OK or IPG_NOT_CONVERGED once halted
  int32_t mode;        // exchange of the superstep about to run
  int32_t forced;      // 0 = the fixed rule, else the forced exchange
  uint32_t cap;        // superstep cap, 0 = none
  uint32_t expanded;   // levels [0, expanded) are written to dist
  uint32_t sparse;     // the coming pull gathers only the non-empty rows
  uint32_t push_div;
  uint32_t bad_source; // a source id >= N was given (it is skipped)
  unsigned long long frontier, frontier_deg;  // union frontier after the last superstep
  unsigned long long t_last;                  // wall clock at the end of the last superstep
  unsigned long long tot_msgs, tot_exam;
  unsigned long long pad;
};
static_assert(sizeof(MsCtl) == 88, "control block layout");
constexpr uint32_t kMsRec = 1024;  // trace records kept on the device (enqueue-only runs)

struct MsRun {
  uint32_t n;
  uint32_t level;  // superstep being computed
  const uint32_t* outdeg;
  const u64* f_in;   // F_{level-1}
  u64* f_out;        // F_level
  u64* vis;
  uint32_t* nz_out;  // bitmap of the non-empty rows of f_out
  CtrSlot* ctr;
  CtrSlot* ctr_clear;
};

struct MsPullArgs {
  MsRun r;
  PullTiling t;
  u64* partial;        // [chunks][4]
  const uint32_t* nz;  // bitmap of the non-empty rows of f_in, or null (gather every row)
  const MsCtl* ctl;    // device-driven form: run only when it chose pull; nz used when it says sparse
};

struct MsPushArgs {
  MsRun r;
  const uint64_t* off;     // CSR
  const int32_t* dst;
  const uint32_t* nz_in;   // union frontier of the previous superstep (bitmap)
  u64* recv;               // [n][4], zero outside a push superstep
  uint32_t* touched;       // bitmap, zero outside a push superstep
  const MsCtl* ctl;        // device-driven form: run only when it chose push
};

__device__ __forceinline__ bool ms_skip(const MsCtl* ctl, int mode) {
  return ctl && (ctl->halted || ctl->mode != mode);
}

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

// Superstep 0: one thread per query sets its source's bit in vis and F_0 and
// marks the source in the union frontier (a repeated source counts once).
__global__ __launch_bounds__(kBlock) void ms_init_kernel(const uint32_t* sources, uint32_t q, MsRun a,
                                                         uint32_t* bad) {
  const uint32_t i = threadIdx.x;
  uint64_t senders = 0, messages = 0, next_count = 0, next_deg = 0;
  const uint32_t v = i < q ? sources[i] : 0;
  if (i < q && v >= a.n) atomicOr(bad, 1u);  // checked on the host unless the run is enqueue-only
  if (i < q && v < a.n) {
    const u64 bit = 1ull << (i & 63);
    atomicOr(a.vis + (size_t)v * kMsWords + (i >> 6), bit);
    atomicOr(a.f_out + (size_t)v * kMsWords + (i >> 6), bit);
    const uint32_t d = a.outdeg[v];
    senders = 1;
    messages = d;
    const uint32_t vb = 1u << (v & 31);
    if ((atomicOr(a.nz_out + (v >> 5), vb) & vb) == 0u) {
      next_count = 1;
      next_deg = d;
    }
  }
  flush_counters(a.ctr, senders, messages, next_count, next_deg, 0);
}

// Zero the mask rows whose bits are set in `bm` (the non-empty rows of a
// level buffer about to be reused by a push superstep); one thread per
// bitmap word.
__global__ void ms_clear_rows_kernel(const uint32_t* bm, uint32_t words, u64* f) {
  const u64 z[kMsWords] = {0, 0, 0, 0};
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) {
    uint32_t m = bm[i];
    while (m) {
      const uint32_t b = static_cast<uint32_t>(__ffs(m) - 1);
      m &= m - 1;
      store_mask(f, 32 * i + b, z);
    }
  }
}

// Pull exchange of superstep level-1 and compute of superstep `level`, over
// the pull items (one wavefront per item, grid-stride over wavefronts).
//  * row item: in passes of kMsPass edges, every lane gathers the masks of
//    its edges' sources into the wavefront's LDS tile; a group of G lanes
//    per row ORs the row's entries (G from the item's row count) and the
//    group's first lane computes the row;
//  * long-row chunk: the OR of its edges' masks is stored as the chunk's
//    partial (combined by ms_longrow_kernel).
__global__ __launch_bounds__(kBlock) void ms_pull_kernel(MsPullArgs a) {
  constexpr int kPer = kMsPass / kWave;
  constexpr int kChunkPer = kWaveTile / kWave;
  constexpr int kRowPer = (kItemRows + kWave) / kWave;
  __shared__ u64 s_tile[kWavesPerBlock][kMsPass][kMsWords];
  __shared__ uint32_t s_off[kWavesPerBlock][kItemRows + 1];
  if (ms_skip(a.ctl, IPG_MODE_PULL)) return;  // uniform over the grid
  const uint32_t* nz = a.ctl ? (a.ctl->sparse ? a.nz : nullptr) : a.nz;
  clear_slots(a.r.ctr_clear);
  const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
  u64(*tile)[kMsWords] = s_tile[wv];
  uint32_t* soff = s_off[wv];
  const int32_t* src = a.t.src;
  const uint64_t* off = a.t.off;
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
        if (u[k] >= 0 && row_live(nz, u[k])) {
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
          u64 m[kMsWords] = {0, 0, 0, 0};
          if (row_live(nz, u[k])) load_mask(a.r.f_in, static_cast<uint32_t>(u[k]), m);
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
    }
    wave_set_bits(sends, v, a.r.nz_out);
    wave_lds_sync();  // the offsets are rewritten by the next item
  }
  flush_counters(a.r.ctr, c.senders, c.messages, c.next_count, c.next_deg, 0, c.active);
}

// Second launch of a pull superstep: one wavefront per long row ORs the
// partials of its chunks and computes the row.
__global__ __launch_bounds__(kBlock) void ms_longrow_kernel(MsPullArgs a) {
  if (ms_skip(a.ctl, IPG_MODE_PULL)) return;
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
    if (sends) atomicOr(a.r.nz_out + (v >> 5), 1u << (v & 31));
  }
  flush_counters(a.r.ctr, c.senders, c.messages, c.next_count, c.next_deg, 0, c.active);
}

// Push exchange of superstep level-1: one thread per vertex, the vertices of
// the union frontier send, with out-edges expanded by twc_scatter; each edge
// ORs the sender's mask into the recipient's receive row and marks the
// recipient touched.
__global__ __launch_bounds__(kBlock) void ms_push_kernel(MsPushArgs a) {
  if (ms_skip(a.ctl, IPG_MODE_PUSH)) return;
  clear_slots(a.r.ctr_clear);
  const uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
  bool has = false;
  uint64_t beg = 0, end = 0;
  const uint32_t u = static_cast<uint32_t>(i);
  if (i < a.r.n && bit_of(a.nz_in, u)) {
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
    const uint32_t xb = 1u << (x & 31);
    if (!(a.touched[x >> 5] & xb)) atomicOr(a.touched + (x >> 5), xb);
  });
}

// Compute of a push superstep: every wavefront takes 64 consecutive vertices
// (two bitmap words it owns), consumes and zeroes the receive rows of the
// touched ones, and writes both words of the union-frontier bitmap and of
// the (cleared) touched bitmap with plain stores.
__global__ __launch_bounds__(kBlock) void ms_settle_kernel(MsPushArgs a) {
  if (ms_skip(a.ctl, IPG_MODE_PUSH)) return;
  MsCount c;
  const uint32_t lane = lane_id();
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * blockDim.x / kWave;
  for (uint64_t base = wave * kWave; base < a.r.n; base += nwaves * kWave) {  // wave-uniform
    const uint32_t v = static_cast<uint32_t>(base) + lane;
    const uint32_t word = static_cast<uint32_t>(base >> 5) + (lane >> 5);
    const bool touched = v < a.r.n && ((a.touched[word] >> (v & 31)) & 1u);
    bool sends = false;
    if (touched) {
      u64 R[kMsWords], F[kMsWords];
      load_mask(a.recv, v, R);
      const u64 z[kMsWords] = {0, 0, 0, 0};
      store_mask(a.recv, v, z);
      sends = ms_compute(a.r, v, R, F, c);
    }
    const uint64_t sm = __ballot(sends);
    if (lane == 0) {
      const uint32_t w0 = static_cast<uint32_t>(base >> 5);
      a.r.nz_out[w0] = static_cast<uint32_t>(sm);
      a.r.nz_out[w0 + 1] = static_cast<uint32_t>(sm >> 32);
      a.touched[w0] = 0;
      a.touched[w0 + 1] = 0;
    }
  }
  flush_counters(a.r.ctr, c.senders, c.messages, c.next_count, c.next_deg, 0, c.active);
}

// Distances from the level masks of supersteps lvl0 .. lvl0+nlev-1 (ring
// slot (lvl0 + j) % kMsHist): dist[q][v] = the superstep whose mask holds
// bit q at v.  One thread per vertex; the level index of each bit is read
// from bit planes built over the window, and the stores for one query are
// coalesced along v.  The first window also writes INF where no bit is set;
// later windows write only the distances they hold.
__device__ __forceinline__ void ms_expand_body(const u64* hist, uint32_t n, uint32_t q, uint32_t lvl0, uint32_t nlev,
                                               bool first, uint32_t* dist) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    u64 found[kMsWords] = {0, 0, 0, 0};
    u64 plane[kMsHistBits][kMsWords] = {};
    for (uint32_t j = 0; j < nlev; ++j) {
      const uint32_t slot = (lvl0 + j) % kMsHist;
      u64 m[kMsWords];
      load_mask(hist + (size_t)slot * n * kMsWords, static_cast<uint32_t>(v), m);
#pragma unroll
      for (int w = 0; w < kMsWords; ++w) {
        found[w] |= m[w];
#pragma unroll
        for (int b = 0; b < kMsHistBits; ++b)
          if ((j >> b) & 1u) plane[b][w] |= m[w];
      }
    }
#pragma unroll
    for (int w = 0; w < kMsWords; ++w) {
      const uint32_t qe = q > 64u * w ? (q - 64u * w < 64u ? q - 64u * w : 64u) : 0u;
      for (uint32_t bit = 0; bit < qe; ++bit) {
        uint32_t* out = dist + (size_t)(64u * w + bit) * n + v;
        if ((found[w] >> bit) & 1ull) {
          uint32_t lvl = 0;
#pragma unroll
          for (int b = 0; b < kMsHistBits; ++b) lvl |= static_cast<uint32_t>((plane[b][w] >> bit) & 1ull) << b;
          *out = lvl0 + lvl;
        } else if (first) {
          *out = kInf;
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void ms_expand_kernel(const u64* hist, uint32_t n, uint32_t q, uint32_t lvl0,
                                                           uint32_t nlev, int first, uint32_t* dist) {
  ms_expand_body(hist, n, q, lvl0, nlev, first != 0, dist);
}

// Superstep-level exchange choice on the union frontier: the library's
// fixed rule, pull when the frontier and its out-edges exceed E / div.
__host__ __device__ inline ipg_mode ms_mode(ipg_mode forced, uint64_t e, uint64_t frontier, uint64_t frontier_deg,
                                            uint32_t div) {
  if (forced == IPG_MODE_PUSH || forced == IPG_MODE_PULL) return forced;
  if (e == 0) return IPG_MODE_PUSH;
  return frontier + frontier_deg > e / (div ? div : 20) ? IPG_MODE_PULL : IPG_MODE_PUSH;
}

// ------------------------------------------------------- device-driven --

__global__ void ms_dd_start_kernel(MsCtl* ctl, int forced, uint32_t cap, uint32_t push_div) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    MsCtl c{};
    c.mode = IPG_MODE_PUSH;  // superstep 0 is the sources' broadcast
    c.forced = forced;
    c.cap = cap;
    c.push_div = push_div;
    c.t_last = static_cast<unsigned long long>(wall_clock64());
    *ctl = c;
  }
}

// First launch of a device-driven superstep: prepare its level buffer.  A
// push writes only the rows it reaches, so the rows left by the slot's
// previous level are zeroed (the whole slot if it was never used); a pull
// writes every row but builds its union-frontier bitmap with ORs, so the
// slot's bitmap is zeroed.
__global__ void ms_dd_prep_kernel(const MsCtl* ctl, u64* f_out, uint32_t* nz_out, uint32_t n, uint32_t words) {
  const MsCtl c = *ctl;
  if (c.halted) return;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (c.mode == IPG_MODE_PUSH) {
    if (c.step < kMsHist) {
      for (uint64_t i = tid; i < (uint64_t)n * kMsWords; i += stride) f_out[i] = 0;
    } else {
      const u64 z[kMsWords] = {0, 0, 0, 0};
      for (uint64_t i = tid; i < words; i += stride) {
        uint32_t m = nz_out[i];
        while (m) {
          const uint32_t b = static_cast<uint32_t>(__ffs(m) - 1);
          m &= m - 1;
          store_mask(f_out, static_cast<uint32_t>(32 * i + b), z);
        }
      }
    }
  } else {
    for (uint64_t i = tid; i < words; i += stride) nz_out[i] = 0;
  }
}

// End of a device-driven superstep: sum the counters, record the
// superstep, and take the host loop's decisions (halt when no query has a
// message pending or at the cap; the next exchange by the fixed rule on the
// union frontier, or forced; a sparse pull when that frontier is small).
__global__ __launch_bounds__(kWave) void ms_dd_decide_kernel(const CtrSlot* c, uint32_t n, uint64_t e, uint32_t q,
                                                             MsCtl* ctl, DevRec* rec) {
  static_assert(kCtrSlots == kWave, "one slot per lane");
  const unsigned long long now = static_cast<unsigned long long>(wall_clock64());
  const MsCtl k = *ctl;
  if (k.halted) return;
  const CtrSlot& x = c[threadIdx.x];
  const uint64_t nc = wave_sum_u64(x.next_count);
  const uint64_t se = wave_sum_u64(x.senders);
  const uint64_t me = wave_sum_u64(x.messages);
  const uint64_t nd = wave_sum_u64(x.next_deg);
  const uint64_t ac = wave_sum_u64(x.active);
  if (threadIdx.x != 0) return;
  const uint32_t s = k.step;
  const uint64_t examined = s == 0 ? 0 : (k.mode == IPG_MODE_PUSH ? k.frontier_deg : e);
  DevRec r;
  r.active = s == 0 ? (unsigned long long)q * n : ac;
  r.senders = se;
  r.messages = me;
  r.examined = examined;
  r.frontier_deg = k.frontier_deg;
  r.ticks = now - k.t_last;
  r.mode = static_cast<uint32_t>(k.mode);
  r.pad = 0;
  rec[s % kMsRec] = r;
  MsCtl nk = k;
  nk.step = s + 1;
  nk.t_last = now;
  nk.tot_msgs += me;
  nk.tot_exam += examined;
  if (me == 0) {
    nk.halted = 1;
    nk.status = IPG_OK;
  } else if (k.cap && s + 1 >= k.cap) {
    nk.halted = 1;
    nk.status = IPG_NOT_CONVERGED;
  } else {
    nk.frontier = nc;
    nk.frontier_deg = nd;
    nk.mode = k.forced ? k.forced : ms_mode(IPG_MODE_AUTO, e, nc, nd, k.push_div);
    nk.sparse = nc < n / 8 ? 1u : 0u;
  }
  *ctl = nk;
}

// After every chunk of 16 device-driven supersteps (16c .. 16c+15): expand
// the levels not yet in dist -- at most the 16 of the ring, which the next
// chunk overwrites; the first expansion also writes INF.
__global__ __launch_bounds__(kBlock) void ms_dd_expand_kernel(const MsCtl* ctl, const u64* hist, uint32_t n,
                                                              uint32_t q, uint32_t* dist) {
  const uint32_t lvl0 = ctl->expanded, nlev = ctl->step - lvl0;
  if (nlev == 0) return;
  ms_expand_body(hist, n, q, lvl0, nlev, lvl0 == 0, dist);
}

__global__ void ms_dd_mark_kernel(MsCtl* ctl) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->expanded = ctl->step;
}

// ------------------------------------------------------------------ host --

struct MsWs {
  u64* vis;
  u64* hist;        // [kMsHist][n][4] level masks, slot = superstep % kMsHist
  u64* recv;
  u64* partial;
  uint32_t* nzb;      // [kMsHist][words] union-frontier bitmap of each level slot
  uint32_t* touched;  // [words] push: recipients of the superstep
  CtrSlot* ctr;       // [2][kCtrSlots]
  MsCtl* ctl;         // device-driven form
  DevRec* rec;        // [kMsRec] its trace records
};

// Bitmap words per vertex set: whole 64-vertex wavefront tiles (the settle
// pass writes two words per wavefront).
static size_t ms_words(uint32_t n) { return ((size_t)n + 63) / 64 * 2 + 2; }

static size_t carve_ms(Carver& c, uint32_t n, uint64_t e, MsWs* out) {
  MsWs w{};
  const size_t nn = n ? n : 1;
  w.vis = c.take<u64>(nn * kMsWords);
  w.hist = c.take<u64>(kMsHist * nn * kMsWords);
  w.recv = c.take<u64>(nn * kMsWords);
  w.partial = c.take<u64>(chunks_cap(e) * kMsWords);
  w.nzb = c.take<uint32_t>(kMsHist * ms_words(n));
  w.touched = c.take<uint32_t>(ms_words(n));
  w.ctl = c.take<MsCtl>(1);
  w.rec = c.take<DevRec>(kMsRec);
  w.ctr = c.take<CtrSlot>(2 * kCtrSlots);
  if (out) *out = w;
  return align_up(c.used, 256);
}

static ipg_status run_msbfs(ipg_graph* g, const uint32_t* sources, uint32_t q, uint32_t cap, const ipg_run_opts& o,
                            uint32_t* dist, const MsWs& w, hipStream_t s, StepTimer& tm, ipg_run_stats* st) {
  const uint32_t n = g->n;
  const uint64_t e = g->e;
  const Tune tn = resolve_tuning(o.tuning);
  HostMirror *hm = nullptr, *hm_dev = nullptr;
  IPG_HIP(host_mirror(g, &hm, &hm_dev));
  const size_t rowset = (size_t)n * kMsWords;  // u64 per level buffer
  const size_t words = ms_words(n);
  auto slot_buf = [&](uint32_t level) { return w.hist + (size_t)(level % kMsHist) * rowset; };
  auto slot_bits = [&](uint32_t level) { return w.nzb + (size_t)(level % kMsHist) * words; };
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.vis), rowset * 2, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.hist), rowset * 2, 0, s));  // slot 0
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.recv), rowset * 2, 0, s));
  IPG_HIP(fill_u32(w.nzb, words, 0, s));  // slot 0
  IPG_HIP(fill_u32(w.touched, words, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.ctr), 2 * kCtrSlots * sizeof(CtrSlot) / 4, 0, s));

  // Expansion of the levels [lvl0, lvl0 + nlev) of the ring into dist.
  bool first_window = true;
  auto expand = [&](uint32_t lvl0, uint32_t nlev) -> hipError_t {
    hipLaunchKernelGGL(ms_expand_kernel, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, w.hist, n, q, lvl0, nlev,
                       first_window ? 1 : 0, dist);
    first_window = false;
    return hipGetLastError();
  };

  MsRun r{};
  r.n = n;
  r.outdeg = g->t.outdeg;
  r.vis = w.vis;
  const PullTiling t = pull_tiling(g);
  uint64_t tot_msgs = 0, tot_exam = 0;
  uint64_t frontier = 0, frontier_deg = 0;
  bool used[kMsHist] = {};  // slot written since the run started (slot 0 is zeroed above)
  uint32_t base = 0;        // first level not yet expanded into dist
  uint32_t step = 0;
  ipg_status status = IPG_OK;
  IPG_HIP(tm.start(s));
  for (;;) {
    const uint32_t slot = step % kMsHist;
    if (step - base == kMsHist) {  // the ring is full: expand it before reusing slot `slot`
      IPG_HIP(expand(base, kMsHist));
      base += kMsHist;
    }
    CtrSlot* c = w.ctr + (step & 1) * kCtrSlots;
    CtrSlot* cc = w.ctr + ((step + 1) & 1) * kCtrSlots;
    r.level = step;
    r.f_out = slot_buf(step);
    r.f_in = step ? slot_buf(step - 1) : nullptr;
    r.nz_out = slot_bits(step);
    r.ctr = c;
    r.ctr_clear = cc;
    ipg_mode mode = IPG_MODE_PUSH;
    uint64_t examined = 0;
    if (step == 0) {
      hipLaunchKernelGGL(ms_init_kernel, dim3(1), dim3(kBlock), 0, s, sources, q, r, &w.ctl->bad_source);
      IPG_HIP(hipGetLastError());
    } else {
      mode = ms_mode(o.mode, e, frontier, frontier_deg, tn.push_div);
      if (mode == IPG_MODE_PUSH) {
        // F_out must be zero outside the rows this superstep writes: zero the
        // rows left by the slot's previous level (its bitmap, still intact)
        if (!used[slot]) {
          IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(r.f_out), rowset * 2, 0, s));
        } else {
          hipLaunchKernelGGL(ms_clear_rows_kernel, dim3(grid_for(words, kBlock, kExchangeGrid)), dim3(kBlock), 0, s,
                             r.nz_out, static_cast<uint32_t>(words), r.f_out);
          IPG_HIP(hipGetLastError());
        }
        MsPushArgs a;
        a.r = r;
        a.off = g->csr_off;
        a.dst = g->csr_dst;
        a.nz_in = slot_bits(step - 1);
        a.recv = w.recv;
        a.touched = w.touched;
        a.ctl = nullptr;
        hipLaunchKernelGGL(ms_push_kernel, dim3(grid_for(n, kBlock, 0xFFFFFFFFu)), dim3(kBlock), 0, s, a);
        IPG_HIP(hipGetLastError());
        a.r.ctr_clear = nullptr;
        hipLaunchKernelGGL(ms_settle_kernel, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, a);
        IPG_HIP(hipGetLastError());
        examined = frontier_deg;
      } else {
        IPG_HIP(fill_u32(r.nz_out, words, 0, s));
        MsPullArgs a;
        a.r = r;
        a.t = t;
        a.partial = w.partial;
        // sparse superstep: gather only the non-empty rows of F_{s-1}
        a.nz = frontier < n / 8 ? slot_bits(step - 1) : nullptr;
        a.ctl = nullptr;
        if (t.ni) {
          hipLaunchKernelGGL(ms_pull_kernel, dim3(std::min(t.ni, tn.pull_grid)), dim3(kBlock), 0, s, a);
          IPG_HIP(hipGetLastError());
        }
        a.r.ctr_clear = nullptr;
        if (t.nl) {
          hipLaunchKernelGGL(ms_longrow_kernel, dim3((t.nl + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0,
                             s, a);
          IPG_HIP(hipGetLastError());
        }
        examined = e;
      }
    }
    used[slot] = true;
    IPG_HIP(tm.step(s, step));
    IPG_HIP(launch_decide(c, step + 1, e, nullptr, &hm_dev->decision, 0, nullptr, s));
    IPG_HIP(hipStreamSynchronize(s));
    const Decision h = hm->decision;
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
    ++step;
    if (h.messages == 0) break;  // no message pending for any query: all halted
    if (cap && step >= cap) {
      status = IPG_NOT_CONVERGED;
      break;
    }
    frontier = h.next_count;
    frontier_deg = h.next_deg;
  }
  IPG_HIP(expand(base, step - base));
  IPG_HIP(tm.finish(s));
  if (st) {
    st->supersteps = step;
    st->halted = status == IPG_OK;
    st->edges_traversed = tot_msgs;
    st->edges_examined = tot_exam;
  }
  return status;
}

// Device-driven form (IPG_RUN_PERSISTENT, IPG_RUN_ENQUEUE): superstep 0,
// then chunks of 16 supersteps whose kernels read the control block, each
// chunk followed by the expansion of its levels.  With `enqueue_only` the
// chunks needed to reach the cap are enqueued without any host
// synchronisation (the run can be captured into a graph);
// ipg_multi_sssp_result reads the outcome afterwards.  Otherwise the control
// block and the chunk's records are read back after every chunk.
static ipg_status run_msbfs_device(ipg_graph* g, const uint32_t* sources, uint32_t q, uint32_t cap,
                                   const ipg_run_opts& o, uint32_t* dist, const MsWs& w, hipStream_t s,
                                   bool enqueue_only) {
  const uint32_t n = g->n;
  const uint64_t e = g->e;
  const Tune tn = resolve_tuning(o.tuning);
  const size_t rowset = (size_t)n * kMsWords;
  const size_t words = ms_words(n);
  const int forced = o.mode == IPG_MODE_AUTO ? 0 : static_cast<int>(o.mode);
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.vis), rowset * 2, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.hist), rowset * 2, 0, s));  // slot 0
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.recv), rowset * 2, 0, s));
  IPG_HIP(fill_u32(w.nzb, words, 0, s));  // slot 0
  IPG_HIP(fill_u32(w.touched, words, 0, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.ctr), 2 * kCtrSlots * sizeof(CtrSlot) / 4, 0, s));
  hipLaunchKernelGGL(ms_dd_start_kernel, dim3(1), dim3(1), 0, s, w.ctl, forced, cap, tn.push_div);
  IPG_HIP(hipGetLastError());
  MsRun r{};
  r.n = n;
  r.outdeg = g->t.outdeg;
  r.vis = w.vis;
  r.level = 0;
  r.f_out = w.hist;
  r.f_in = nullptr;
  r.nz_out = w.nzb;
  r.ctr = w.ctr;
  r.ctr_clear = w.ctr + kCtrSlots;
  hipLaunchKernelGGL(ms_init_kernel, dim3(1), dim3(kBlock), 0, s, sources, q, r, &w.ctl->bad_source);
  IPG_HIP(hipGetLastError());
  hipLaunchKernelGGL(ms_dd_decide_kernel, dim3(1), dim3(kWave), 0, s, w.ctr, n, e, q, w.ctl, w.rec);
  IPG_HIP(hipGetLastError());
  const PullTiling t = pull_tiling(g);
  // Chunk c holds supersteps 16c .. 16c+15 (superstep 0, the sources'
  // broadcast, is enqueued above): superstep 16c+p uses ring slot p, and the
  // chunk's levels are expanded before the next chunk reuses the ring.
  const uint32_t chunks = enqueue_only ? (cap + kMsHist - 1) / kMsHist : 0xFFFFFFFFu;
  MsCtl h{};
  for (uint32_t chunk = 0; chunk < chunks; ++chunk) {
    for (uint32_t p = chunk == 0 ? 1 : 0; p < kMsHist; ++p) {
      const uint32_t slot = p, prev = (p + kMsHist - 1) % kMsHist;
      u64* f_out = w.hist + (size_t)slot * rowset;
      uint32_t* nz_out = w.nzb + (size_t)slot * words;
      hipLaunchKernelGGL(ms_dd_prep_kernel, dim3(grid_for(words, kBlock, 2048)), dim3(kBlock), 0, s, w.ctl, f_out,
                         nz_out, n, static_cast<uint32_t>(words));
      IPG_HIP(hipGetLastError());
      MsRun rr = r;
      rr.f_in = w.hist + (size_t)prev * rowset;
      rr.f_out = f_out;
      rr.nz_out = nz_out;
      rr.ctr = w.ctr + (p & 1) * kCtrSlots;
      rr.ctr_clear = w.ctr + ((p + 1) & 1) * kCtrSlots;
      MsPushArgs a;
      a.r = rr;
      a.off = g->csr_off;
      a.dst = g->csr_dst;
      a.nz_in = w.nzb + (size_t)prev * words;
      a.recv = w.recv;
      a.touched = w.touched;
      a.ctl = w.ctl;
      hipLaunchKernelGGL(ms_push_kernel, dim3(grid_for(n, kBlock, 0xFFFFFFFFu)), dim3(kBlock), 0, s, a);
      IPG_HIP(hipGetLastError());
      a.r.ctr_clear = nullptr;
      hipLaunchKernelGGL(ms_settle_kernel, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, a);
      IPG_HIP(hipGetLastError());
      MsPullArgs pa;
      pa.r = rr;
      pa.t = t;
      pa.partial = w.partial;
      pa.nz = w.nzb + (size_t)prev * words;
      pa.ctl = w.ctl;
      if (t.ni) {
        hipLaunchKernelGGL(ms_pull_kernel, dim3(std::min(t.ni, tn.pull_grid)), dim3(kBlock), 0, s, pa);
        IPG_HIP(hipGetLastError());
      }
      pa.r.ctr_clear = nullptr;
      if (t.nl) {
        hipLaunchKernelGGL(ms_longrow_kernel, dim3((t.nl + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0, s,
                           pa);
        IPG_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(ms_dd_decide_kernel, dim3(1), dim3(kWave), 0, s, rr.ctr, n, e, q, w.ctl, w.rec);
      IPG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(ms_dd_expand_kernel, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, w.ctl, w.hist, n, q,
                       dist);
    IPG_HIP(hipGetLastError());
    hipLaunchKernelGGL(ms_dd_mark_kernel, dim3(1), dim3(1), 0, s, w.ctl);
    IPG_HIP(hipGetLastError());
    if (enqueue_only) continue;
    IPG_HIP(hipMemcpyAsync(&h, w.ctl, sizeof(h), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    if (h.halted) break;
  }
  if (enqueue_only) return IPG_OK;
  return static_cast<ipg_status>(h.status);
}

// Statistics of a device-driven run from its control block and records.
static ipg_status ms_fill_stats(const MsCtl& h, const DevRec* recs, uint32_t first, int dev, ipg_run_stats* st) {
  if (!st) return IPG_OK;
  int khz = 0;
  IPG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  const double us_per_tick = khz > 0 ? 1e3 / khz : 0.0;
  double secs = 0.0;
  for (uint32_t k = first; k < h.step; ++k) {
    const DevRec& x = recs[k % kMsRec];
    secs += x.ticks * us_per_tick * 1e-6;
    if (k >= st->trace_cap) continue;
    if (st->active) st->active[k] = x.active;
    if (st->senders) st->senders[k] = x.senders;
    if (st->messages) st->messages[k] = x.messages;
    if (st->examined) st->examined[k] = x.examined;
    if (st->mode) st->mode[k] = static_cast<uint8_t>(x.mode);
    if (st->frontier_deg) st->frontier_deg[k] = x.frontier_deg;
    if (st->usec) st->usec[k] = static_cast<float>(x.ticks * us_per_tick);
  }
  st->supersteps = h.step;
  st->halted = h.halted && h.status == IPG_OK;
  st->edges_traversed = h.tot_msgs;
  st->edges_examined = h.tot_exam;
  st->seconds = secs;
  return IPG_OK;
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
  ipg_run_opts o{0, 0.0, IPG_MODE_AUTO, 0, nullptr, nullptr, 0, 0.0, nullptr};
  if (opts) o = *opts;
  if (o.mode != IPG_MODE_AUTO && o.mode != IPG_MODE_PUSH && o.mode != IPG_MODE_PULL)
    return fail(IPG_EINVAL, "ipg_run_multi_sssp: unknown mode");
  const bool enqueue = o.flags & IPG_RUN_ENQUEUE;
  const bool device = enqueue || (o.flags & IPG_RUN_PERSISTENT);
  if (enqueue && (max_supersteps == 0 || max_supersteps > kMsRec))
    return fail(IPG_EINVAL, "ipg_run_multi_sssp: an enqueue-only run needs 1 <= max_supersteps <= 1024");
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
  if (!enqueue) {
    // The sources are checked on the host before any kernel indexes with
    // them (an enqueue-only run checks them on the device: the result call
    // reports an out-of-range source).
    std::vector<uint32_t> hsrc(num_sources);
    IPG_HIP(hipMemcpyAsync(hsrc.data(), sources, num_sources * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < num_sources; ++i)
      if (hsrc[i] >= g->n) return fail(IPG_EINVAL, "ipg_run_multi_sssp: source " + std::to_string(i) + " >= N");
  }
  Carver c(ws);
  MsWs w;
  carve_ms(c, g->n, g->e, &w);
  ipg_status rc;
  if (device) {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (!enqueue && st) {
      IPG_HIP(pool_event(&g->events, 0, &t0));
      IPG_HIP(pool_event(&g->events, 1, &t1));
      IPG_HIP(hipEventRecord(t0, s));
    }
    rc = run_msbfs_device(g, sources, num_sources, max_supersteps, o, dist, w, s, enqueue);
    if (!enqueue && st && (rc == IPG_OK || rc == IPG_NOT_CONVERGED)) {
      // per-superstep times from the device's wall-clock stamps; the run's
      // time from events around it
      MsCtl h{};
      std::vector<DevRec> recs(kMsRec);
      IPG_HIP(hipEventRecord(t1, s));
      IPG_HIP(hipMemcpyAsync(&h, w.ctl, sizeof(h), hipMemcpyDeviceToHost, s));
      IPG_HIP(hipMemcpyAsync(recs.data(), w.rec, kMsRec * sizeof(DevRec), hipMemcpyDeviceToHost, s));
      IPG_HIP(hipStreamSynchronize(s));
      const uint32_t first = h.step > kMsRec ? h.step - kMsRec : 0;
      const ipg_status r2 = ms_fill_stats(h, recs.data(), first, dev, st);
      if (r2 != IPG_OK) return r2;
      float ms = 0.f;
      IPG_HIP(hipEventElapsedTime(&ms, t0, t1));
      st->seconds = ms * 1e-3;
    }
  } else {
    StepTimer tm(&g->events, st ? st->usec : nullptr, st ? st->trace_cap : 0);
    rc = run_msbfs(g, sources, num_sources, max_supersteps, o, dist, w, s, tm, st);
    if (st) st->seconds = tm.seconds();
  }
  if (rc == IPG_OK) set_error("");
  return rc;
}

extern "C" ipg_status ipg_multi_sssp_result(const ipg_graph* g, const void* ws, size_t ws_bytes, void* hip_stream,
                                            ipg_run_stats* st) {
  if (!g || !ws) return fail(IPG_EINVAL, "ipg_multi_sssp_result: NULL argument");
  if (ws_bytes < ipg_multi_sssp_workspace_bytes(g->n, g->e))
    return fail(IPG_EWORKSPACE, "ipg_multi_sssp_result: workspace too small");
  Carver c(const_cast<void*>(ws));
  MsWs w;
  carve_ms(c, g->n, g->e, &w);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  MsCtl h{};
  std::vector<DevRec> recs(kMsRec);
  IPG_HIP(hipMemcpyAsync(&h, w.ctl, sizeof(h), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipMemcpyAsync(recs.data(), w.rec, kMsRec * sizeof(DevRec), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipStreamSynchronize(s));
  if (h.bad_source) return fail(IPG_EINVAL, "ipg_multi_sssp_result: a source was >= N (skipped)");
  const ipg_status r2 = ms_fill_stats(h, recs.data(), 0, g->device, st);
  if (r2 != IPG_OK) return r2;
  if (!h.halted) return fail(IPG_EINVAL, "ipg_multi_sssp_result: no device-driven run has ended in this workspace");
  return static_cast<ipg_status>(h.status);
}
