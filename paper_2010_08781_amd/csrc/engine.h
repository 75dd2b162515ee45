// engine.h -- host-side superstep driver shared by the application sources.
#pragma once

#include <vector>

#include "common.h"

namespace ipg {

inline PullTiling make_tiling(const uint64_t* off, const int32_t* src, const TilingTables& tt) {
  PullTiling t;
  t.off = off;
  t.src = src;
  t.rb = tt.pull_rb;
  t.long_rows = tt.long_rows;
  t.lr_first = tt.lr_first;
  t.ch_row = tt.ch_row;
  t.items = tt.items;
  t.nl = tt.nl;
  t.nc = tt.nc;
  t.nb = tt.nb;
  t.ni = tt.ni;
  return t;
}

// The caller's CSC and its tiling.
inline PullTiling pull_tiling(const ipg_graph* g) { return make_tiling(g->csc_off, g->csc_src, g->t.pull); }

// End-of-superstep summary written by the decide kernel: the counter slots
// summed, and the selector's choice for the next superstep.
struct Decision {
  unsigned long long next_count, senders, messages, next_deg;
  uint16_t overflow;
  uint8_t late;   // the superstep was chosen as pull and exchanged by push (pick_kernel)
  uint8_t list;   // the selector's push for the next superstep visits the frontier list
  int32_t mode;   // IPG_MODE_PUSH / IPG_MODE_PULL from the selector, 0 if none ran
  double margin;  // predicted log2 time of push minus pull
  unsigned long long active;  // summed `active` counters (batched SSSP)
  unsigned long long list_len;  // next-frontier list length left by a push (when the decide was given it)
};
static_assert(sizeof(Decision) == 64, "one 64-byte record");

// Control block of the device-driven superstep loop (IPG_RUN_PERSISTENT):
// the state the host loop keeps between supersteps, kept in device memory
// and advanced by the decide kernel at the end of every superstep.  The
// exchange kernels of a superstep read it and return at once when the run
// has halted or the superstep uses the other exchange.
struct DevCtl {
  uint32_t step;      // superstep about to run
  uint32_t halted;    // 1 once the run has ended
  int32_t status;     // IPG_OK, IPG_NOT_CONVERGED, IPG_EOVERFLOW or IPG_EDEVICE once halted
  int32_t mode;       // exchange of the superstep about to run
  uint32_t list_ok;   // its active set is the frontier list (else: the non-empty mailboxes)
  uint32_t cap;       // superstep cap, 0 = none
  unsigned long long count;   // active vertices of the superstep about to run
  unsigned long long degsum;  // their out-degree sum
  unsigned long long t_last;  // device wall clock at the end of the previous superstep
  unsigned long long pad[2];
};
static_assert(sizeof(DevCtl) == 64, "one 64-byte block");

// One superstep's trace record, written by the decide kernel.
struct DevRec {
  unsigned long long active, senders, messages, examined, frontier_deg, ticks;
  uint32_t mode, pad;
};
constexpr uint32_t kDevRec = 256;  // ring of records; a chunk of supersteps never exceeds it

// Pinned host memory that the decide kernels write directly, so that a
// readback is one stream synchronisation and no copy: the device-driven
// loop's control block as its last decide left it and its trace ring, and
// the host-driven loops' end-of-superstep summary.  One per graph handle,
// created on first use and freed with the handle (runs on one handle are
// serial: each synchronises its stream before returning).
struct HostMirror {
  DevCtl ctl;
  Decision decision;
  DevRec rec[kDevRec];
};
// The block as the host reads it (*host) and as kernels address it (*dev).
hipError_t host_mirror(ipg_graph* g, HostMirror** host, HostMirror** dev);

// Sum the counter slots `c` of a superstep into *out (one wavefront) and,
// with a selector, choose the exchange of the next superstep.
// It also reports the length of the next-frontier list a push superstep
// left in the slots' segments (~0 when a segment overflowed: the list is
// then incomplete) and, with `lpre_out`, writes the prefix of the
// segments' lengths that the next superstep's list consumers read.
hipError_t launch_decide(const CtrSlot* c, uint32_t next_superstep, uint64_t e, const double* sel, Decision* out,
                         uint32_t lseg, uint32_t* lpre_out, hipStream_t s, const uint32_t* late = nullptr,
                         int mode = 0);

// Push exchange: a sender with at least kPieceMin out-edges is not expanded
// by its own workgroup.  Its out-edges are cut into pieces of at most kPiece
// edges and queued, and a second launch deals the pieces over the whole
// grid.  (R-MAT's high-degree vertices have low ids: expanded in place, a
// few workgroups would hold most of a dense superstep's edges.)  The queue,
// like the next-frontier list, is cut into kCtrSlots segments, one per
// counter slot, so that a workgroup's appends (one atomic per wavefront)
// go to its own slot's counter instead of one device-wide address.
constexpr uint32_t kPieceMin = 128;
constexpr uint32_t kPiece = 1024;
struct Piece {
  unsigned long long beg;  // first CSR edge
  uint32_t n;              // edges (0 = an unused entry, 1 .. kPiece)
  uint32_t msg;            // the value the sender broadcasts
};
// Segment of the piece queue: a sender with d >= kPieceMin out-edges queues
// ceil(d / kPiece) <= d / kPiece + d / kPieceMin pieces, so a superstep
// queues at most E / kPiece + E / kPieceMin; each segment holds its share
// of that plus slack.  A wavefront that finds its segment full expands its
// senders in place.
inline uint64_t piece_seg(uint64_t e) { return (e / kPiece + e / kPieceMin) / kCtrSlots + 64; }
// Segment of the next-frontier list: its share of N plus slack.  A full
// segment drops the list for that superstep (the next one sweeps the
// mailboxes instead).
inline uint32_t list_seg(uint32_t n) { return n / kCtrSlots + 64; }
// A piece of a PageRank push superstep: the sender's contribution instead
// of a u32 message.
struct PrPiece {
  unsigned long long beg;  // first CSR edge
  uint32_t n;              // edges (0 = an unused entry, 1 .. kPiece)
  uint32_t pad;
  double c;                // the sender's rank / out-degree
};

// Per-superstep counts of a PageRank run (vertices that ran compute, that
// broadcast, and their out-degree sum), added by the workgroups into one of
// kCtrSlots slots each.
struct alignas(64) PrCntSlot {
  unsigned long long active, senders, messages, pad[5];
};
static_assert(sizeof(PrCntSlot) == 64, "one slot per 64-byte line");
constexpr uint32_t kPrTraceCap = 4096;  // PageRank supersteps with a trace record (later ones are not recorded)

// Run workspace, carved from the caller's device buffer.
struct RunWs {
  // PageRank
  double* value_f64;  // [n] ranks after the last update
  double* f64_a;      // [n] outbox (pull) or mailbox (push), ping
  double* f64_b;      // [n] pong
  double* partial;    // [chunks] partial sums of long-row chunks (pull)
  uint32_t* part_n;   // [n] vertex count of each vertex's part (disjoint unions)
  double* l1;         // [kCtrSlots] L1 change of an update, spread over slots (convergence runs)
  double* value_hot;  // [n] ranks under the hot-first names (renamed store), mapped back at the end
  PrPiece* pr_pieces; // [kCtrSlots * piece_seg(e)] piece queue of a push superstep
  PrCntSlot* pr_cnt;  // [2][kCtrSlots] per-superstep counts (set s & 1)
  unsigned long long* pr_rec;  // [kPrTraceCap][3] trace records: active, senders, messages
  // CC / SSSP
  uint32_t* value_u32;  // [n] labels or distances
  uint32_t* value_u32_hot;  // [n] the same under the hot-first names, when the run works under them (min_space)
  uint32_t* mail_a;     // [n] one-slot min mailboxes, ping (INF = empty)
  uint32_t* mail_b;     // [n] pong
  uint32_t* fr_a;       // [kCtrSlots * list_seg(n)] frontier list in segments, ping
  uint32_t* fr_b;       // pong
  uint32_t* outbox;     // [n] one-slot outbox of the pull form: the broadcast value, INF if none
  uint32_t* sent;       // [n/64*2 + 2] bitmap of the vertices that broadcast in a pull superstep
  uint32_t* gate;       // [1] 1 when that superstep's senders are few enough to gate the gathers
  uint32_t* lpre;       // [2][kCtrSlots + 1] prefix of the list segments' lengths, by superstep parity
  uint32_t* late;       // [1] 1 when the pull superstep under way is exchanged by push (few messages)
  Piece* pieces;        // [kCtrSlots * piece_seg(e)] piece queue of a push superstep
  DevCtl* ctl;          // device-driven loop state
  // both
  CtrSlot* ctr;         // [2][kCtrSlots] per-superstep counters (set s & 1)
};

size_t carve_run(Carver& c, uint32_t n, uint64_t e, ipg_app app, RunWs* w);

// HIP-event timing of the superstep loop (first launch -> halt decision) and,
// when the caller asked for it, of every superstep.
// Entry i of a graph handle's event pool, created on first use.
hipError_t pool_event(std::vector<hipEvent_t>* pool, size_t i, hipEvent_t* out);

// The events come from the graph handle's pool (created on first use, kept
// until the handle is destroyed): creating and destroying a dozen events per
// run cost more host time than a short run's launches.
class StepTimer {
 public:
  StepTimer(std::vector<hipEvent_t>* pool, float* usec, uint32_t cap)
      : pool_(pool), usec_(usec), cap_(usec ? cap : 0) {}
  hipError_t start(hipStream_t s);
  hipError_t step(hipStream_t s, uint32_t k);  // end of superstep k
  // Record the end event now without waiting; finish() then waits for the
  // last such record instead of recording one after the host has seen the
  // halt (a loop that synchronises anyway saves a round trip to the device).
  hipError_t mark(hipStream_t s);
  hipError_t finish(hipStream_t s);            // synchronises
  double seconds() const { return seconds_; }

 private:
  hipError_t event(size_t i, hipEvent_t* out) { return pool_event(pool_, i, out); }  // 0 start, 1 end, 2 + k superstep k
  std::vector<hipEvent_t>* pool_;
  float* usec_;
  uint32_t cap_;
  bool started_ = false;
  bool marked_ = false;
  uint32_t nsteps_ = 0;  // supersteps recorded (k < nsteps_)
  double seconds_ = 0.0;
};

// Push/pull choice for one superstep of CC/SSSP (Section 4.3.2: the paper
// fixes it at compile time; Ligra switches at run time on a user threshold).
struct ModeQuery {
  uint32_t n;
  uint64_t e;
  uint64_t frontier;     // vertices active in this superstep
  uint64_t frontier_deg; // sum of their out-degrees
  uint32_t superstep;
  ipg_app app;
};
// Fixed heuristic used when no selector is given (the default of Ligra's
// direction switch, Shun and Blelloch 2013): pull when the frontier plus its
// out-edges exceed E/20.
__host__ __device__ inline int heuristic_pick(uint64_t e, uint64_t frontier, uint64_t frontier_deg,
                                              uint32_t div = 20) {
  if (e == 0) return IPG_MODE_PUSH;
  return (frontier + frontier_deg > e / (div ? div : 20)) ? IPG_MODE_PULL : IPG_MODE_PUSH;
}

// Launch parameters of a run, defaults filled in (see ipg_tuning).
struct Tune {
  uint32_t pr_hot;     // 0 = no LDS outbox cache
  uint32_t pull_grid;
  uint32_t push_div;
  uint32_t list_div;
  uint32_t gate_div;  // pull gathers only senders' outboxes when senders < N / gate_div (0 = never)
  uint32_t blocked;  // pull exchanges use the blocked in-edges when the store has them
  uint32_t late_div;  // AUTO: a pull superstep with messages <= E / late_div is exchanged by push instead (0 = never)
};
constexpr uint32_t kHotDefault = 8192;  // 64 KB of LDS; the launch also caps it to the LDS left by the tiles
inline Tune resolve_tuning(const ipg_tuning* t) {
  Tune r{kHotDefault, kPullGrid, 20, 16, 8, 1, 20};
  if (t) {
    if (t->blocked) r.blocked = t->blocked == 0xFFFFFFFFu ? 0 : 1;
    if (t->gate_div) r.gate_div = t->gate_div == 0xFFFFFFFFu ? 0 : t->gate_div;
    if (t->pr_hot) r.pr_hot = t->pr_hot == 0xFFFFFFFFu ? 0 : t->pr_hot;
    if (t->pull_grid) r.pull_grid = t->pull_grid;
    if (t->push_div) r.push_div = t->push_div;
    if (t->list_div) r.list_div = t->list_div;
    if (t->late_div) r.late_div = t->late_div == 0xFFFFFFFFu ? 0 : t->late_div;
  }
  return r;
}
ipg_mode heuristic_mode(const ModeQuery& q, uint32_t div = 20);

ipg_status run_pagerank(ipg_graph* g, uint32_t T, const ipg_run_opts& o, const RunWs& w, const void* ws,
                        hipStream_t s, StepTimer& tm, ipg_run_stats* st);
ipg_status run_minprop(ipg_graph* g, ipg_app app, uint32_t cap, const ipg_run_opts& o, const RunWs& w,
                       hipStream_t s, StepTimer& tm, ipg_run_stats* st);

}  // namespace ipg
