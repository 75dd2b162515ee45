// minprop.hip -- hash-min connected components (Fig. 9) and SSSP (Fig. 10)
// on the superstep engine, uint32 values and messages combined by min (Fig. 5).
//
// Both applications vote to halt after every compute ("systematic halt",
// Section 4.3.1), so the vertices active in superstep s+1 are exactly the
// recipients of a message in superstep s: the vertices whose one-slot
// mailbox is not empty (INF).  The mailbox array therefore *is* the next
// frontier; no separate selection pass is needed (the selection bypass of
// Section 4.3.1).  When the exchange is a push, the recipients whose mailbox
// was empty (the atomic min returned INF -- exactly one sender per recipient
// sees that, so there are no duplicates) are also appended to a compact list,
// so that a small next frontier can be visited without sweeping all N
// mailboxes.
//
// Superstep s >= 1 for an active vertex v: consume its mailbox (reset it to
// INF); if the message is below value(v), lower value(v) and broadcast --
// value(v) for CC, value(v) + 1 (or + w(v, x) per out-edge when weighted)
// for SSSP.  Superstep 0: CC sets value = id and every vertex broadcasts;
// SSSP sets value = 0 at the source (which broadcasts) and INF elsewhere.
//
// Mailboxes are double-buffered (consume from `mail_in`, deliver into
// `mail_out`) so that a superstep never sees a message sent in the same
// superstep (Section 4.2).
#include <algorithm>
#include <vector>

#include "common.h"
#include "blocked.h"
#include "engine.h"
#include "scatter.h"
#include "select.h"
#include "selector.h"

namespace ipg {

static_assert(kListSegs == static_cast<uint32_t>(kCtrSlots), "one list segment per counter slot");

// value = id (CC: `ids[v]` when the run works under other names than the
// caller's) or 0 at the source / INF elsewhere (SSSP).  With `pull_s0`
// superstep 0 is exchanged by pull: the senders' broadcast values are written
// to the outbox (INF for the others) and the senders are counted.  With a
// control block (device-driven loop) its exchange decides instead.  Given
// `mail_a` and `mail_b`, both mailboxes are emptied too (the device-driven
// loop's start; the host-driven loop clears them before).
__global__ __launch_bounds__(kBlock) void minprop_init_kernel(uint32_t n, int app, uint32_t source, uint32_t* value,
                                                              const uint32_t* outdeg, int pull_s0, uint32_t* outbox,
                                                              CtrSlot* ctr, const DevCtl* ctl, uint32_t* mail_a,
                                                              uint32_t* mail_b, const uint32_t* ids) {
  if (ctl) pull_s0 = ctl->mode == IPG_MODE_PULL;  // uniform over the grid
  uint64_t senders = 0, messages = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const bool sends = (app == IPG_APP_CC_HASHMIN) || v == source;
    const uint32_t x = app == IPG_APP_CC_HASHMIN ? (ids ? ids[v] : static_cast<uint32_t>(v)) : (v == source ? 0u : kInf);
    value[v] = x;
    if (mail_a) {
      mail_a[v] = kInf;
      mail_b[v] = kInf;
    }
    if (pull_s0) {
      outbox[v] = sends ? x : kInf;
      if (sends) {
        senders += 1;
        messages += outdeg[v];
      }
    }
  }
  if (pull_s0) flush_counters(ctr, senders, messages, 0, 0, 0);
}

// The list prefix of a launch in LDS (zeros when the phase has no list).
// Every thread calls it.
__device__ __forceinline__ void load_list_prefix(const Active& act, uint32_t* s_pre) {
  for (uint32_t t = threadIdx.x; t <= static_cast<uint32_t>(kCtrSlots); t += blockDim.x)
    s_pre[t] = act.phase == kStepList ? act.pre[t] : 0u;
  __syncthreads();
}

// Compute of vertex v in a launch: returns whether v broadcasts, and the
// value it broadcasts.
__device__ __forceinline__ bool compute_min(int phase, uint32_t v, uint32_t* value, uint32_t* mail_in, uint32_t& msg) {
  if (phase == kSendAll || phase == kSendSource) {
    msg = value[v];
    return true;
  }
  const uint32_t m = mail_in[v];
  if (m == kInf) return false;  // dense sweep: no message, not active
  mail_in[v] = kInf;
  if (m < value[v]) {
    value[v] = m;
    msg = m;
    return true;
  }
  return false;
}

struct MinPushArgs {
  Active act;
  const uint64_t* off;  // CSR
  const int32_t* dst;
  const uint32_t* w;    // CSR weights or null
  const uint32_t* outdeg;
  uint32_t* value;
  uint32_t* mail_in;
  uint32_t* mail_out;
  uint32_t* list_out;   // next frontier (recipients whose mailbox was empty), in segments
  uint32_t list_seg;
  CtrSlot* ctr;
  CtrSlot* ctr_clear;
  const DevCtl* ctl;    // device-driven loop: active set and exchange from here (else null)
  uint32_t n;
  Piece* pieces;        // piece queue (see kPieceMin), or null to expand every sender in place
  uint64_t piece_seg;
  const uint32_t* late;  // a pull superstep's late push: runs only when *late (else null)
};

// Append the lanes' items with `pred` to the workgroup's segment of the
// next-frontier list: one atomic per wavefront, on the slot's counter.
// Entries past the segment's end are dropped (the list is then not used).
__device__ __forceinline__ void seg_append(bool pred, uint32_t item, const MinPushArgs& a) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(mask)) - 1);
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(&my_slot(a.ctr)->list_len, static_cast<uint32_t>(__popcll(mask)));
  base = __shfl(base, static_cast<int>(leader));
  const uint32_t at = base + lanes_below(mask);
  if (pred && at < a.list_seg) a.list_out[static_cast<uint64_t>(blockIdx.x % kCtrSlots) * a.list_seg + at] = item;
}

// One message of a push exchange along CSR edge e: the combiner (atomic
// min into the recipient's next mailbox), the frontier append of a first
// message, and the counters.  The mailbox is read first and the atomic
// skipped when the message cannot lower it.  The read is a plain load that
// may hit this XCD's L2: writes of earlier launches are visible to it, and
// within the exchange only these atomics change a mailbox, and only
// downwards, so a stale copy holds a value at least the current one and the
// test never skips an atomic that would change anything -- nor the one that
// finds the mailbox empty (the value read is then already below INF).
// Device-scope atomics are performed past the XCDs' L2s; without the test,
// every message would pay for one.
template <int APP, bool W>
__device__ __forceinline__ void push_edge(const MinPushArgs& a, uint64_t e, uint32_t p, uint64_t& next_count,
                                          uint64_t& next_deg, uint32_t& overflow) {
  const uint32_t x = static_cast<uint32_t>(a.dst[e]);
  uint64_t m = p;
  if (APP == IPG_APP_SSSP) m += W ? a.w[e] : 1u;
  bool fresh = false;
  if (m >= kInf) {
    overflow = 1;
  } else {
    const uint32_t cur = a.mail_out[x];
    if (m < cur) fresh = atomicMin(a.mail_out + x, static_cast<uint32_t>(m)) == kInf;
  }
  seg_append(fresh, x, a);
  if (fresh) {
    next_count += 1;
    next_deg += a.outdeg[x];
  }
}

// Active set of a device-driven superstep s >= 1: the list left by a push
// superstep, or the non-empty mailboxes.  (Superstep 0 keeps the launch's
// own: every vertex for CC, the source for SSSP.)
__device__ __forceinline__ Active device_active(const DevCtl& c, const Active& own, const uint32_t* list, uint32_t n) {
  if (c.step == 0) return own;
  Active act = own;
  act.phase = c.list_ok ? kStepList : kStepDense;
  act.count = c.list_ok ? static_cast<uint32_t>(c.count) : n;
  act.list = list;
  act.source = 0;
  return act;
}

// Queue the out-edges of this wavefront's senders that have at least
// kPieceMin of them as pieces in the workgroup's segment of the queue (one
// atomic per wavefront, on the slot's counter); returns whether the lane
// still expands its sender itself.  A sender whose pieces do not fit in
// the segment is expanded in place and its entries marked unused.  All
// lanes of the wavefront call it together.
__device__ __forceinline__ bool queue_pieces(const MinPushArgs& a, bool has, uint64_t beg, uint64_t end, uint32_t msg) {
  const uint64_t d = has ? end - beg : 0;
  const uint32_t np = d >= kPieceMin ? static_cast<uint32_t>((d + kPiece - 1) / kPiece) : 0u;
  if (__ballot(np != 0) == 0) return has;  // uniform: no sender to queue
  const uint32_t lane = lane_id();
  uint32_t inc = np;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= static_cast<uint32_t>(o)) inc += t;
  }
  const uint32_t total = __shfl(inc, kWave - 1);
  if (total == 0) return has;  // uniform
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(&my_slot(a.ctr)->pieces, total);
  base = __shfl(base, 0);
  if (np == 0) return has;
  const uint64_t first = static_cast<uint64_t>(base) + (inc - np);
  const bool fits = first + np <= a.piece_seg;
  Piece* seg = a.pieces + static_cast<uint64_t>(blockIdx.x % kCtrSlots) * a.piece_seg;
  for (uint32_t k = 0; k < np && first + k < a.piece_seg; ++k) {
    const uint64_t b = beg + static_cast<uint64_t>(k) * kPiece;
    Piece p;
    p.beg = b;
    p.n = fits ? static_cast<uint32_t>(min(static_cast<uint64_t>(kPiece), end - b)) : 0u;
    p.msg = msg;
    seg[first + k] = p;
  }
  return !fits;
}

// Fused compute + push scatter of one superstep: one thread per active
// vertex (grid-stride in workgroup-uniform rounds); senders with many
// out-edges queue them as pieces, the others are expanded by twc_scatter.
// Recipients whose mailbox was empty are appended to the next-frontier list
// by wave-ballot compaction (one atomic per wave and ballot, on the slot's
// counter).
// The kernel's work for the active set `act` by the first `grid`
// workgroups of the launch.
template <int APP, bool W>
__device__ __forceinline__ void push_body(const MinPushArgs& a, const Active& act, uint32_t grid, uint32_t* s_lpre) {
  load_list_prefix(act, s_lpre);
  clear_slots(a.ctr_clear);
  uint64_t senders = 0, messages = 0, next_count = 0, next_deg = 0;
  uint32_t overflow = 0;
  const uint64_t stride = (uint64_t)grid * kBlock;
  for (uint64_t base = blockIdx.x * (uint64_t)kBlock; base < act.count; base += stride) {
    const uint64_t i = base + threadIdx.x;
    bool has = false;
    uint64_t beg = 0, end = 0;
    uint32_t msg = 0;
    if (i < act.count) {
      const uint32_t v = active_vertex(act, s_lpre, i);
      has = compute_min(act.phase, v, a.value, a.mail_in, msg);
      if (has) {
        beg = a.off[v];
        end = a.off[v + 1];
        senders += 1;
        messages += end - beg;
      }
    }
    if (a.pieces) has = queue_pieces(a, has, beg, end, msg);
    twc_scatter(has, beg, end, msg, [&](uint64_t e, uint32_t p) {
      push_edge<APP, W>(a, e, p, next_count, next_deg, overflow);
    });
  }
  flush_counters(a.ctr, senders, messages, next_count, next_deg, overflow);
}
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_push_kernel(MinPushArgs a) {
  __shared__ uint32_t s_lpre[kCtrSlots + 1];
  Active act = a.act;
  if (a.ctl) {
    const DevCtl c = *a.ctl;
    if (c.halted || c.mode != IPG_MODE_PUSH) return;  // uniform over the grid
    act = device_active(c, a.act, a.act.list, a.n);
  }
  push_body<APP, W>(a, act, gridDim.x, s_lpre);
}

// The messages of one piece: a workgroup, kPiece / kBlock edges per thread
// with their loads issued together.
template <int APP, bool W>
__device__ __forceinline__ void push_piece(const MinPushArgs& a, const Piece& pc, uint64_t& next_count,
                                           uint64_t& next_deg, uint32_t& overflow) {
  constexpr int kPer = kPiece / kBlock;
  uint32_t x[kPer], cur[kPer];
  uint64_t m[kPer];
  bool ok[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint32_t j = threadIdx.x + k * kBlock;
    ok[k] = j < pc.n;
    const uint64_t e = pc.beg + (ok[k] ? j : 0u);
    x[k] = ok[k] ? static_cast<uint32_t>(a.dst[e]) : 0u;
    m[k] = pc.msg;
    if (APP == IPG_APP_SSSP) m[k] += W ? (ok[k] ? a.w[e] : 0u) : 1u;
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) cur[k] = ok[k] && m[k] < kInf ? a.mail_out[x[k]] : 0u;  // see push_edge
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    bool fresh = false;
    if (ok[k]) {
      if (m[k] >= kInf) overflow = 1;
      else if (m[k] < cur[k]) fresh = atomicMin(a.mail_out + x[k], static_cast<uint32_t>(m[k])) == kInf;
    }
    seg_append(fresh, x[k], a);
    if (fresh) {
      next_count += 1;
      next_deg += a.outdeg[x[k]];
    }
  }
}

// Second launch of a push superstep: the queued pieces, dealt over the grid
// (piece g, counted over the segments in slot order, to workgroup
// g mod grid).
template <int APP, bool W>
__device__ __forceinline__ void piece_body(const MinPushArgs& a, uint32_t grid, uint32_t* s_pre) {
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
  if (blockIdx.x >= total) return;  // uniform: no piece, nothing to count
  uint64_t next_count = 0, next_deg = 0;
  uint32_t overflow = 0;
  for (uint32_t g = blockIdx.x; g < total; g += grid) {  // uniform over the workgroup
    uint32_t lo = 0, hi = kCtrSlots - 1;  // the last segment k with s_pre[k] <= g
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    const Piece pc = a.pieces[static_cast<uint64_t>(lo) * a.piece_seg + (g - s_pre[lo])];
    push_piece<APP, W>(a, pc, next_count, next_deg, overflow);
  }
  flush_counters(a.ctr, 0, 0, next_count, next_deg, overflow);
}
// With `late` set it belongs to the late push of a pull superstep (after
// minprop_late_kernel) and runs only when that push was chosen.
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_piece_kernel(MinPushArgs a) {
  __shared__ uint32_t s_pre[kCtrSlots + 1];
  if (a.ctl) {
    const DevCtl c = *a.ctl;
    if (c.halted || c.mode != (a.late ? IPG_MODE_PULL : IPG_MODE_PUSH)) return;
  }
  if (a.late && !*a.late) return;  // uniform over the grid
  piece_body<APP, W>(a, gridDim.x, s_pre);
}

struct MinApplyArgs {
  Active act;
  const uint32_t* outdeg;
  uint32_t* value;
  uint32_t* mail_in;
  uint32_t* outbox;  // all INF on entry (host-driven loop)
  CtrSlot* ctr;
  const DevCtl* ctl;  // device-driven loop: sweep all N and write every outbox slot (else null)
  uint32_t n;
  uint32_t* sent;     // bitmap of the senders (zero on entry), or null
};

// Compute phase of a pull superstep: consume the mailboxes of the active
// vertices; a vertex whose value drops broadcasts it through its one-slot
// outbox (Section 4.3.2: one broadcast value per vertex, read by the
// out-neighbours).
// The compute of a pull superstep over every vertex, four per thread with
// 16-byte accesses (the arrays are 256-byte aligned): consume the mailboxes
// (rewritten only when one of the four holds a message), lower the values,
// and write every outbox slot -- the new value for a vertex that
// broadcasts, INF otherwise.  The last N mod 4 vertices one per thread.
__device__ __forceinline__ void apply_dense4(const MinApplyArgs& a, uint32_t grid, uint64_t& senders,
                                             uint64_t& messages) {
  const uint64_t nq = a.n / 4;
  const uint64_t stride = (uint64_t)grid * blockDim.x;
  const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint4* mail = reinterpret_cast<uint4*>(a.mail_in);
  uint4* val = reinterpret_cast<uint4*>(a.value);
  uint4* out = reinterpret_cast<uint4*>(a.outbox);
  const uint4* deg = reinterpret_cast<const uint4*>(a.outdeg);
  for (uint64_t q = t0; q < nq; q += stride) {
    // The three loads are issued together -- one memory latency per thread
    // instead of three in a row -- and every loaded value is used outside
    // the branches (a value used only under a branch is loaded there).  A
    // quad without a message reads 8 bytes per vertex in vain.
    const uint4 m = mail[q];
    const uint4 x = val[q];
    const uint4 d = deg[q];
    const bool s0 = m.x < x.x, s1 = m.y < x.y, s2 = m.z < x.z, s3 = m.w < x.w;  // INF: no message, no send
    senders += static_cast<uint64_t>(s0) + s1 + s2 + s3;
    messages += static_cast<uint64_t>(s0 ? d.x : 0u) + (s1 ? d.y : 0u) + (s2 ? d.z : 0u) + (s3 ? d.w : 0u);
    if ((m.x & m.y & m.z & m.w) != kInf) mail[q] = make_uint4(kInf, kInf, kInf, kInf);  // consumed
    if (s0 || s1 || s2 || s3) val[q] = make_uint4(s0 ? m.x : x.x, s1 ? m.y : x.y, s2 ? m.z : x.z, s3 ? m.w : x.w);
    out[q] = make_uint4(s0 ? m.x : kInf, s1 ? m.y : kInf, s2 ? m.z : kInf, s3 ? m.w : kInf);
  }
  for (uint64_t v = 4 * nq + t0; v < a.n; v += stride) {
    uint32_t msg = kInf;
    const bool sends = compute_min(kStepDense, static_cast<uint32_t>(v), a.value, a.mail_in, msg);
    a.outbox[v] = sends ? msg : kInf;
    if (sends) {
      senders += 1;
      messages += a.outdeg[v];
    }
  }
}

// The compute for the active set `act` by the first `grid` workgroups of
// the launch.
__device__ __forceinline__ void apply_body(const MinApplyArgs& a, const Active& act, uint32_t grid, uint32_t* s_lpre) {
  uint64_t senders = 0, messages = 0;
  if (act.phase == kStepDense && !a.sent) {  // uniform over the grid
    apply_dense4(a, grid, senders, messages);
    flush_counters(a.ctr, senders, messages, 0, 0, 0);
    return;
  }
  load_list_prefix(act, s_lpre);
  // wavefront-uniform rounds (the sender bitmap is set a wavefront at a time)
  const uint64_t stride = (uint64_t)grid * blockDim.x;
  const uint64_t first = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~static_cast<uint32_t>(kWave - 1));
  for (uint64_t base = first; base < act.count; base += stride) {
    const uint64_t i = base + lane_id();
    bool sends = false;
    uint32_t v = 0;
    if (i < act.count) {
      v = active_vertex(act, s_lpre, i);
      uint32_t msg;
      sends = compute_min(act.phase, v, a.value, a.mail_in, msg);
      if (sends) {
        senders += 1;
        messages += a.outdeg[v];
        a.outbox[v] = msg;
      } else if (a.ctl) {
        a.outbox[v] = kInf;
      }
    }
    if (a.sent) wave_set_bits(sends, v, a.sent);
  }
  flush_counters(a.ctr, senders, messages, 0, 0, 0);
}
__global__ __launch_bounds__(kBlock) void minprop_apply_kernel(MinApplyArgs a) {
  __shared__ uint32_t s_lpre[kCtrSlots + 1];
  Active act = a.act;
  if (a.ctl) {
    const DevCtl c = *a.ctl;
    if (c.halted || c.mode != IPG_MODE_PULL) return;
    act.phase = kStepDense;
    act.count = a.n;
  }
  apply_body(a, act, gridDim.x, s_lpre);
}

// First launch of a device-driven superstep s >= 1: the push kernel's work
// when the control block chose push, the pull form's compute when it chose
// pull -- one launch where there were two, one of which returned at once.
// Each part runs on its own grid; the workgroups beyond it return.
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_front_kernel(MinPushArgs p, MinApplyArgs ap, uint32_t push_grid,
                                                               uint32_t apply_grid) {
  __shared__ uint32_t s_lpre[kCtrSlots + 1];
  const DevCtl c = *p.ctl;
  if (c.halted) return;  // uniform over the grid
  if (c.mode == IPG_MODE_PUSH) {
    if (blockIdx.x < push_grid) push_body<APP, W>(p, device_active(c, p.act, p.act.list, p.n), push_grid, s_lpre);
  } else if (c.mode == IPG_MODE_PULL) {
    Active act = ap.act;
    act.phase = kStepDense;
    act.count = ap.n;
    if (blockIdx.x < apply_grid) apply_body(ap, act, apply_grid, s_lpre);
  }
}

// Between the compute and the exchange of a pull superstep, once the
// broadcasts are counted (one wavefront sums the counter slots):
// - whether so few vertices broadcast that the gather should consult the
//   sender bitmap first (senders < N / gate_div; `gate`, when given);
// - whether their messages are so few (<= E / late_div) that the exchange is
//   done by push instead (`late`, when given): the push/pull choice of
//   Section 4.3.2 taken on the messages themselves rather than on the active
//   set before the compute, which overestimates them when most active
//   vertices do not improve.
__global__ __launch_bounds__(kWave) void pick_kernel(const CtrSlot* c, uint32_t n, uint64_t e, uint32_t gate_div,
                                                     uint32_t late_div, const DevCtl* ctl, uint32_t* gate,
                                                     uint32_t* late) {
  if (ctl && (ctl->halted || ctl->mode != IPG_MODE_PULL)) return;
  const uint64_t se = wave_sum_u64(c[threadIdx.x].senders);
  const uint64_t me = wave_sum_u64(c[threadIdx.x].messages);
  if (threadIdx.x == 0) {
    if (gate) *gate = (gate_div && se < n / gate_div) ? 1u : 0u;
    if (late) *late = (late_div && me <= e / late_div) ? 1u : 0u;
  }
}

struct MinPullArgs {
  PullTiling t;
  const uint32_t* w;       // CSC weights or null
  const uint32_t* outdeg;
  const uint32_t* outbox;  // broadcast values of this superstep, INF = no broadcast
  uint32_t* mail_out;
  CtrSlot* ctr;
  CtrSlot* ctr_clear;
  const DevCtl* ctl;       // device-driven loop: run only when it chose pull (else null)
  const uint32_t* sent;    // bitmap of the senders, read when *gate is set
  const uint32_t* gate;    // or null: gather every outbox
  const uint32_t* late;    // the superstep is exchanged by push instead when *late (or null)
};

// The message an in-edge carries: the source's broadcast value o (CC), plus
// 1 or the edge weight w (SSSP); INF when the source did not broadcast.
template <int APP, bool W>
__device__ __forceinline__ uint32_t edge_msg(uint32_t o, uint32_t w, uint32_t& overflow) {
  if (APP == IPG_APP_CC_HASHMIN) return o;
  const uint64_t m = static_cast<uint64_t>(o) + (W ? w : 1u);
  const bool live = o != kInf;
  overflow |= (live && m >= kInf) ? 1u : 0u;
  return (live && m < kInf) ? static_cast<uint32_t>(m) : kInf;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = min(x, static_cast<uint32_t>(__shfl_xor(x, o)));
  return x;
}

// Exchange of a pull superstep over the CSC: every wavefront works through
// its own pull items, as in the PageRank item kernel.  A long-row chunk
// folds the minimum of its in-edges into the row's mailbox with an atomic
// min, and the chunk that finds the mailbox empty counts the row as newly
// active; a row item min-reduces each row from its LDS tile.
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_pull_kernel(MinPullArgs a) {
  constexpr int kPer = kWaveTile / kWave;
  constexpr int kRowPer = (kItemRows + kWave) / kWave;
  __shared__ uint32_t s_tile[kWavesPerBlock][kWaveTile];
  __shared__ uint32_t s_off[kWavesPerBlock][kItemRows + 1];
  if (a.ctl && (a.ctl->halted || a.ctl->mode != IPG_MODE_PULL)) return;  // uniform over the grid
  if (a.late && *a.late) return;                                          // uniform as well
  const uint32_t* sent = (a.gate && *a.gate) ? a.sent : nullptr;
  clear_slots(a.ctr_clear);
  const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
  uint32_t* tile = s_tile[wv];
  uint32_t* soff = s_off[wv];
  const int32_t* src = a.t.src;
  const uint64_t* off = a.t.off;
  uint64_t next_count = 0, next_deg = 0;
  uint32_t overflow = 0;
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  for (uint32_t item = blockIdx.x * kWavesPerBlock + wv; item < a.t.ni; item += nw) {
    const PullItem it = a.t.items[item];
    const bool chunk = it.slot != kNoSlot;
    const uint32_t ne = it.ne < kWaveTile ? it.ne : kWaveTile;
    const uint32_t nrows = chunk ? 0 : it.r1 - it.r0;
    uint32_t ic[kPer];
    int32_t u[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = lane + k * kWave;
      ic[k] = i < ne ? i : (ne ? ne - 1 : 0);
      u[k] = ne ? __builtin_nontemporal_load(src + it.e0 + ic[k]) : 0;
    }
    if (!chunk) {
#pragma unroll
      for (int k = 0; k < kRowPer; ++k) {
        const uint32_t r = lane + k * kWave;
        if (r <= nrows) soff[r] = static_cast<uint32_t>(off[it.r0 + r] - it.e0);
      }
    }
    uint32_t o[kPer], w[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      o[k] = (ne && row_live(sent, u[k])) ? a.outbox[u[k]] : kInf;
      w[k] = (W && ne) ? a.w[it.e0 + ic[k]] : 1u;
    }
    if (chunk) {
      uint32_t m = kInf;
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (lane + k * kWave < ne) m = min(m, edge_msg<APP, W>(o[k], w[k], overflow));
      m = wave_min(m);
      if (lane == 0 && m < kInf && atomicMin(a.mail_out + it.r0, m) == kInf) {
        next_count += 1;
        next_deg += a.outdeg[it.r0];
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = lane + k * kWave;
      if (i < ne) tile[i] = edge_msg<APP, W>(o[k], w[k], overflow);
    }
    wave_lds_sync();
    uint32_t G = kWave;
    while (G > 1 && G * nrows > kWave) G >>= 1;
    const uint32_t groups = kWave / G, gi = lane / G, li = lane % G;
    for (uint32_t rb = 0; rb < nrows; rb += groups) {
      const uint32_t row = rb + gi;
      uint32_t m = kInf;
      if (row < nrows) {
        uint32_t lo = soff[row], hi = soff[row + 1];
        if (hi > ne) hi = ne;
        for (uint32_t j = lo + li; j < hi; j += G) m = min(m, tile[j]);
      }
      for (uint32_t x = G >> 1; x >= 1; x >>= 1) m = min(m, static_cast<uint32_t>(__shfl_xor(m, static_cast<int>(x))));
      if (li == 0 && row < nrows && m < kInf) {
        a.mail_out[it.r0 + row] = m;
        next_count += 1;
        next_deg += a.outdeg[it.r0 + row];
      }
    }
    wave_lds_sync();  // the tile is rewritten by the next item
  }
  flush_counters(a.ctr, 0, 0, next_count, next_deg, overflow);
}

// Late push of a pull superstep (pick_kernel set *late): the
// compute already ran over every vertex and left each broadcast value in the
// outbox (INF for a vertex that does not broadcast), so the senders are
// found by sweeping the outbox, and each one's message goes along its
// out-edges as in push_body (pieces for long rows, the other rows expanded
// by twc_scatter, recipients appended to the next-frontier list).  The
// senders and their messages were counted by the compute.
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_late_kernel(MinPushArgs a, const uint32_t* outbox) {
  if (a.ctl && (a.ctl->halted || a.ctl->mode != IPG_MODE_PULL)) return;  // uniform over the grid
  if (!*a.late) return;
  clear_slots(a.ctr_clear);
  uint64_t next_count = 0, next_deg = 0;
  uint32_t overflow = 0;
  // four outbox entries per thread (16-byte loads; the outbox is 256-byte
  // aligned); a round in which no vertex of the workgroup broadcasts skips
  // the expansion and its barriers
  const uint64_t nq = (static_cast<uint64_t>(a.n) + 3) / 4;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kBlock;
  for (uint64_t qb = blockIdx.x * static_cast<uint64_t>(kBlock); qb < nq; qb += stride) {  // uniform rounds
    const uint64_t q = qb + threadIdx.x;
    uint32_t m[4] = {kInf, kInf, kInf, kInf};
    if (4 * q + 3 < a.n) {
      const uint4 x = reinterpret_cast<const uint4*>(outbox)[q];
      m[0] = x.x;
      m[1] = x.y;
      m[2] = x.z;
      m[3] = x.w;
    } else {
      for (uint32_t k = 0; k < 4; ++k)
        if (4 * q + k < a.n) m[k] = outbox[4 * q + k];
    }
    if (!__syncthreads_or((m[0] & m[1] & m[2] & m[3]) != kInf)) continue;  // uniform
#pragma unroll 1
    for (uint32_t k = 0; k < 4; ++k) {
      const uint64_t v = 4 * q + k;
      bool has = m[k] != kInf;
      uint64_t beg = 0, end = 0;
      if (has) {
        beg = a.off[v];
        end = a.off[v + 1];
      }
      if (a.pieces) has = queue_pieces(a, has, beg, end, m[k]);
      twc_scatter(has, beg, end, m[k], [&](uint64_t e, uint32_t p) {
        push_edge<APP, W>(a, e, p, next_count, next_deg, overflow);
      });
    }
  }
  flush_counters(a.ctr, 0, 0, next_count, next_deg, overflow);
}

// Blocked pull (IPG_GRAPH_BLOCKED, CC and SSSP with unit weights): the
// blocked in-edges of the caller's CSC streamed through one workgroup per
// slice (blocked.h), each message min-combined into its destination's LDS
// slot.  The minima do not depend on the order, so results are exact.
struct MinBlkArgs {
  BlkView v;
  const uint32_t* outdeg;
  const uint32_t* outbox;
  uint32_t* mail_out;
  CtrSlot* ctr;
  CtrSlot* ctr_clear;
  const DevCtl* ctl;  // device-driven loop: run only when it chose pull (else null)
  const uint32_t* sent;  // bitmap of the senders, consulted when *gate is set (gate null: never)
  const uint32_t* gate;
  const uint32_t* slots;  // binned cold sources' outboxes (INF: did not broadcast), one per (block, source)
  const uint32_t* late;   // the superstep is exchanged by push instead when *late (or null)
};
// Whether the blocked pull's launches run in this superstep (uniform over the grid).
__device__ __forceinline__ bool blk_pulls(const MinBlkArgs& a) {
  if (a.ctl && (a.ctl->halted || a.ctl->mode != IPG_MODE_PULL)) return false;
  return !(a.late && *a.late);
}

// Bin launch of a binned layout (IPG_GRAPH_BINNED): every cold source's
// outbox (INF when it did not broadcast) copied into its slots (bin_unit).
// The window's outboxes are read as one coalesced block, so the senders'
// bitmap would only add a dependent load: the gate is not consulted.
__global__ __launch_bounds__(kBlkThreads) void min_bin_kernel(MinBlkArgs a, BinTables bv, uint32_t* slots, uint32_t n) {
  if (!blk_pulls(a)) return;
  const uint32_t* outbox = a.outbox;
  bin_unit<uint32_t>(bv, slots, n, [&](uint32_t u) { return outbox[u]; });
}

// Counters of a workgroup of any width: summed over its wavefronts in LDS,
// then at most one atomic per field into its slot.  Every thread calls it.
__device__ __forceinline__ void flush_next_counters(CtrSlot* base, uint64_t next_count, uint64_t next_deg,
                                                    uint32_t overflow) {
  __shared__ unsigned long long red[3][kBlkThreads / kWave];
  next_count = wave_sum_u64(next_count);
  next_deg = wave_sum_u64(next_deg);
  const bool ovf = __ballot(overflow != 0) != 0;
  const uint32_t w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    red[0][w] = next_count;
    red[1][w] = next_deg;
    red[2][w] = ovf ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long t = 0;
    for (uint32_t i = 0; i < blockDim.x / kWave; ++i) t += red[threadIdx.x][i];
    CtrSlot* c = my_slot(base);
    if (t && threadIdx.x == 0) atomicAdd(&c->next_count, static_cast<uint32_t>(t));
    if (t && threadIdx.x == 1) atomicAdd(&c->next_deg, t);
    if (t && threadIdx.x == 2) atomicOr(&c->overflow, 1u);
  }
}

// Blocked pull, first launch: workgroup = slice.  The block's minima start
// at INF in LDS; the workgroup streams the slice's chunks.  A block's only
// slice then writes its rows' mailboxes (rows with a message) and counts
// them; a slice of a larger block stores its minima as a partial.
template <int APP>
__global__ __launch_bounds__(kBlkThreads) void minprop_blocked_kernel(MinBlkArgs a) {
  __shared__ uint32_t part[kBlkRows + kWave];  // + one pad slot per lane (see blk_stream)
  if (!blk_pulls(a)) return;
  clear_slots(a.ctr_clear);
  const BlkSlice sl = a.v.slices[blockIdx.x];
  for (uint32_t r = threadIdx.x; r < sl.rows; r += kBlkThreads) part[r] = kInf;
  if (threadIdx.x < kWave) part[kBlkRows + threadIdx.x] = kInf;
  __syncthreads();
  uint32_t overflow = 0;
  const uint32_t* outbox = a.outbox;
  const uint32_t* sent = (a.gate && *a.gate) ? a.sent : nullptr;  // uniform over the grid
  auto combine = [&](uint32_t slot, uint32_t o) { atomicMin(&part[slot], edge_msg<APP, false>(o, 1u, overflow)); };
  // a cold chunk reads its slots, in which the bin launch already applied the gate
  const uint32_t* slots = a.slots;
  if (sent)  // few senders: a hot source's outbox is read only when its bit is set
    blk_stream<uint32_t>(
        a.v, sl, kInf,
        [&](uint32_t wbase, uint32_t q, uint32_t cold) {
          const uint64_t i = static_cast<uint64_t>(wbase) + (q >> 16);
          const uint32_t u = cold ? 0u : static_cast<uint32_t>(i);  // a bitmap index within [0, N)
          const uint32_t x = (cold ? slots : outbox)[i];
          return cold || row_live(sent, static_cast<int32_t>(u)) ? x : kInf;
        },
        combine);
  else
    blk_stream<uint32_t>(
        a.v, sl, kInf,
        [&](uint32_t wbase, uint32_t q, uint32_t cold) {
          return (cold ? slots : outbox)[static_cast<uint64_t>(wbase) + (q >> 16)];
        },
        combine);
  __syncthreads();
  const uint32_t r0 = sl.row0, rows = sl.rows;
  uint64_t next_count = 0, next_deg = 0;
  if (sl.poff == kNoPartial) {
    for (uint32_t r = threadIdx.x; r < rows; r += kBlkThreads) {
      const uint32_t m = part[r];
      if (m < kInf) {
        a.mail_out[r0 + r] = m;
        next_count += 1;
        next_deg += a.outdeg[r0 + r];
      }
    }
  } else {
    uint32_t* dst = static_cast<uint32_t*>(a.v.partial) + sl.poff;
    for (uint32_t r = threadIdx.x; r < rows; r += kBlkThreads) dst[r] = part[r];
  }
  flush_next_counters(a.ctr, next_count, next_deg, overflow);
}

// Blocked pull, second launch: the rows of every block with several slices
// take the minimum of the slices' partials (a wavefront per group of 64
// rows, every partial load in flight at once).
__device__ __forceinline__ void blocked_finish_body(const MinBlkArgs& a, uint32_t grid) {
  const uint32_t lane = lane_id();
  const uint32_t nw = grid * kWavesPerBlock;
  uint64_t next_count = 0, next_deg = 0;
  for (uint32_t w = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; w < a.v.ngroups; w += nw) {  // wave-uniform
    const BlkGroup gr = a.v.groups[w];
    const uint32_t rr = lane < gr.nrows ? lane : gr.nrows - 1;
    const uint32_t* p = static_cast<const uint32_t*>(a.v.partial) + gr.poff + rr;
    uint32_t m = kInf;
    for (uint32_t k = 0; k < gr.k; k += 8) {
      uint32_t x[8];
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) x[j] = p[static_cast<uint64_t>(k + j < gr.k ? k + j : gr.k - 1) * gr.stride];
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) m = min(m, x[j]);
    }
    if (lane < gr.nrows && m < kInf) {
      a.mail_out[gr.row0 + lane] = m;
      next_count += 1;
      next_deg += a.outdeg[gr.row0 + lane];
    }
  }
  flush_counters(a.ctr, 0, 0, next_count, next_deg, 0);
}
__global__ __launch_bounds__(kBlock) void minprop_blocked_finish_kernel(MinBlkArgs a) {
  if (!blk_pulls(a)) return;
  blocked_finish_body(a, gridDim.x);
}

// Last launch of a device-driven superstep s >= 1 over blocked in-edges:
// the piece launch's work when the control block chose push (or the pull
// superstep turned to a late push), the blocked pull's second launch when
// it pulls (one launch where there were two).  Each part runs on its own
// grid; the workgroups beyond it return.
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_back_kernel(MinPushArgs p, MinBlkArgs b, uint32_t piece_grid,
                                                              uint32_t finish_grid) {
  __shared__ uint32_t s_pre[kCtrSlots + 1];
  const DevCtl c = *p.ctl;
  if (c.halted) return;  // uniform over the grid
  const bool late = c.mode == IPG_MODE_PULL && b.late && *b.late;
  if (c.mode == IPG_MODE_PUSH || late) {
    if (blockIdx.x < piece_grid) piece_body<APP, W>(p, piece_grid, s_pre);
  } else if (c.mode == IPG_MODE_PULL) {
    if (blockIdx.x < finish_grid) blocked_finish_body(b, finish_grid);
  }
}

// End of a superstep: sum the counter slots (one wavefront, lane t reads
// slot t) and, when a selector is given and work is pending, choose the
// exchange of the next superstep with the network.
// The next-frontier list of a push superstep, from the slots (one
// wavefront, lane t reads slot t): its length (~0 if a segment overflowed)
// and, into `pre` when given, the prefix of the segments' lengths.
__device__ __forceinline__ uint64_t list_summary(const CtrSlot& x, uint32_t lseg, uint32_t* pre) {
  const uint32_t ll = x.list_len;
  const uint32_t lane = lane_id();
  uint32_t inc = min(ll, lseg);
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o);
    if (lane >= static_cast<uint32_t>(o)) inc += t;
  }
  if (pre) {
    pre[lane + 1] = inc;
    if (lane == 0) pre[0] = 0;
  }
  const bool lovf = __ballot(ll > lseg) != 0;
  const uint64_t sum = wave_sum_u64(ll);
  return lovf ? ~0ull : sum;
}

__global__ __launch_bounds__(kWave) void decide_kernel(const CtrSlot* c, uint32_t next_superstep, uint64_t e,
                                                       const double* sel, Decision* out, uint32_t lseg, uint32_t* lpre_out,
                                                       const uint32_t* late, int mode) {
  static_assert(kCtrSlots == kWave, "one slot per lane");
  const CtrSlot& x = c[threadIdx.x];
  const uint64_t nc = wave_sum_u64(x.next_count);
  const uint64_t se = wave_sum_u64(x.senders);
  const uint64_t me = wave_sum_u64(x.messages);
  const uint64_t nd = wave_sum_u64(x.next_deg);
  const uint64_t ac = wave_sum_u64(x.active);
  const bool ovf = __ballot(x.overflow != 0) != 0;
  const uint64_t ll = list_summary(x, lseg, lpre_out);
  const bool lt = late && *late;
  // the next superstep can visit a list when this one pushed (`mode`, or a
  // late push) and every list segment held its entries
  const bool list_avail = (mode == IPG_MODE_PUSH || lt) && ll != ~0ull;
  int m = 0;
  bool ul = false;
  double margin = 0.0;
  if (sel && nc) margin = sel_predict_mode_wave(sel, nc, nd, next_superstep, e, list_avail, &m, &ul);  // whole wavefront
  if (threadIdx.x == 0) {
    Decision d;
    d.next_count = nc;
    d.senders = se;
    d.messages = me;
    d.next_deg = nd;
    d.overflow = ovf ? 1u : 0u;
    d.late = lt ? 1u : 0u;
    d.list = ul ? 1u : 0u;
    d.mode = m;
    d.margin = margin;
    d.active = ac;
    d.list_len = ll;
    *out = d;
  }
}

// Start of a device-driven run: the state before superstep 0 -- its active
// set (every vertex for CC, the source for SSSP), their out-degree sum and
// its exchange (forced, the selector, or the fixed heuristic), decided here
// so that the host reads nothing before it enqueues -- and both sets of
// counter slots zeroed.  One wavefront.
__global__ __launch_bounds__(kWave) void dd_start_kernel(DevCtl* ctl, int app, uint32_t source, const uint64_t* off,
                                                         uint32_t n, uint64_t e, const double* sel, int forced,
                                                         uint32_t push_div, uint32_t cap, CtrSlot* ctr) {
  const unsigned long long now = static_cast<unsigned long long>(wall_clock64());
  uint4* cw = reinterpret_cast<uint4*>(ctr);  // 16-byte stores (the slots are 256-byte aligned)
  for (uint32_t i = threadIdx.x; i < 2 * kCtrSlots * sizeof(CtrSlot) / 16; i += kWave) cw[i] = make_uint4(0, 0, 0, 0);
  const bool cc = app == IPG_APP_CC_HASHMIN;
  const uint64_t count = cc ? n : 1;
  const uint64_t degsum = cc ? e : off[static_cast<uint64_t>(source) + 1] - off[source];
  int mode = forced;
  bool ul;
  if (!mode && sel) sel_predict_mode_wave(sel, count, degsum, 0, e, false, &mode, &ul);  // uniform: the whole wavefront infers
  if (!mode) mode = heuristic_pick(e, count, degsum, push_div);
  if (threadIdx.x == 0) {
    DevCtl c{};
    c.mode = mode;
    c.cap = cap;
    c.count = count;
    c.degsum = degsum;
    c.t_last = now;
    *ctl = c;
  }
}

// End of a device-driven superstep: sum the counter slots, record the
// superstep, and decide on the device what the host loop decides -- halt
// (no message pending, an overflow, the cap) and, otherwise, the active set
// and the exchange of the next superstep (forced, the selector, or the fixed
// heuristic).  Does nothing once the run has halted.
__global__ __launch_bounds__(kWave) void dd_decide_kernel(const CtrSlot* c, uint32_t lseg, uint32_t* lpre_out, uint64_t e,
                                                          uint32_t n, const double* sel, int forced,
                                                          uint64_t list_limit, uint32_t push_div, DevCtl* ctl,
                                                          HostMirror* hm, const uint32_t* late) {
  static_assert(kCtrSlots == kWave, "one slot per lane");
  const unsigned long long now = static_cast<unsigned long long>(wall_clock64());
  const DevCtl k = *ctl;
  // The slots are summed before the halted test (cross-lane sums are not
  // moved into a branch), so their loads are in flight with the control
  // block's instead of after it.
  const CtrSlot& x = c[threadIdx.x];
  const uint64_t nc = wave_sum_u64(x.next_count);
  const uint64_t se = wave_sum_u64(x.senders);
  const uint64_t me = wave_sum_u64(x.messages);
  const uint64_t nd = wave_sum_u64(x.next_deg);
  const bool ovf = __ballot(x.overflow != 0) != 0;
  if (k.halted) return;
  const uint64_t lcount = list_summary(x, lseg, lpre_out);  // ~0: a segment overflowed, no list
  const uint32_t s = k.step;
  // the exchange that ran: a pull superstep turned to a late push counts as a push
  const int ran = (k.mode == IPG_MODE_PULL && late && *late) ? IPG_MODE_PUSH : k.mode;
  // the next superstep can visit a list when this one pushed and every list segment held its entries
  const bool list_avail = ran == IPG_MODE_PUSH && lcount != ~0ull;
  int sel_mode = IPG_MODE_PUSH;
  bool sel_list = false;
  const bool use_sel = sel && !forced && nc && !ovf && !(k.cap && s + 1 >= k.cap);
  if (use_sel)  // uniform: the whole wavefront infers
    sel_predict_mode_wave(sel, nc, nd, s + 1, e, list_avail, &sel_mode, &sel_list);
  if (threadIdx.x != 0) return;
  DevRec r;
  r.active = s == 0 ? n : k.count;
  r.senders = se;
  r.messages = me;
  r.examined = ran == IPG_MODE_PUSH ? me : e;
  r.frontier_deg = k.degsum;
  r.ticks = now - k.t_last;
  r.mode = static_cast<uint32_t>(ran);
  r.pad = 0;
  hm->rec[s % kDevRec] = r;
  DevCtl nk = k;
  nk.step = s + 1;
  nk.t_last = now;
  nk.count = nc;
  nk.degsum = nd;
  // a push chosen by the selector visits the list when it predicted that
  // variant faster; otherwise the list is visited up to the size limit
  nk.list_ok = (list_avail && (use_sel && sel_mode == IPG_MODE_PUSH ? sel_list : nc <= list_limit)) ? 1u : 0u;
  if (ovf) {
    nk.halted = 1;
    nk.status = IPG_EOVERFLOW;
  } else if (nc == 0) {
    nk.halted = 1;
    nk.status = IPG_OK;
  } else if (k.cap && s + 1 >= k.cap) {
    nk.halted = 1;
    nk.status = IPG_NOT_CONVERGED;
  } else if (ran == IPG_MODE_PUSH && lcount != ~0ull && lcount != nc) {
    nk.halted = 1;
    nk.status = IPG_EDEVICE;
  } else if (forced) {
    nk.mode = forced;
  } else if (sel) {
    nk.mode = sel_mode;
  } else {
    nk.mode = heuristic_pick(e, nc, nd, push_div);
  }
  *ctl = nk;
  hm->ctl = nk;
}

// ------------------------------------------------------------------ host --

hipError_t launch_decide(const CtrSlot* c, uint32_t next_superstep, uint64_t e, const double* sel, Decision* out,
                         uint32_t lseg, uint32_t* lpre_out, hipStream_t s, const uint32_t* late, int mode) {
  hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(kWave), 0, s, c, next_superstep, e, sel, out, lseg, lpre_out, late,
                     mode);
  return hipGetLastError();
}

// Grid of the piece launch.
constexpr uint32_t kPieceGrid = 2048;

template <int APP, bool W>
static hipError_t launch_push(const MinPushArgs& a, uint32_t grid, bool pieces, hipStream_t s) {
  hipLaunchKernelGGL((minprop_push_kernel<APP, W>), dim3(grid), dim3(kBlock), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !a.pieces || !pieces) return err;
  hipLaunchKernelGGL((minprop_piece_kernel<APP, W>), dim3(kPieceGrid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
template <int APP, bool W>
static hipError_t launch_pull(const MinPullArgs& a, uint32_t max_grid, hipStream_t s) {
  const uint32_t grid = std::max(1u, std::min(a.t.ni, max_grid));
  hipLaunchKernelGGL((minprop_pull_kernel<APP, W>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// The front launch and, unless the back launch will run them, the pieces.
template <int APP, bool W>
static hipError_t launch_front(const MinPushArgs& a, const MinApplyArgs& ap, uint32_t push_grid, uint32_t apply_grid,
                               bool pieces, hipStream_t s) {
  hipLaunchKernelGGL((minprop_front_kernel<APP, W>), dim3(std::max(push_grid, apply_grid)), dim3(kBlock), 0, s, a, ap,
                     push_grid, apply_grid);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !a.pieces || !pieces) return err;
  hipLaunchKernelGGL((minprop_piece_kernel<APP, W>), dim3(kPieceGrid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
static hipError_t front_dispatch(ipg_app app, bool weighted, const MinPushArgs& a, const MinApplyArgs& ap,
                                 uint32_t push_grid, uint32_t apply_grid, bool pieces, hipStream_t s) {
  if (app == IPG_APP_CC_HASHMIN) return launch_front<IPG_APP_CC_HASHMIN, false>(a, ap, push_grid, apply_grid, pieces, s);
  return weighted ? launch_front<IPG_APP_SSSP, true>(a, ap, push_grid, apply_grid, pieces, s)
                  : launch_front<IPG_APP_SSSP, false>(a, ap, push_grid, apply_grid, pieces, s);
}
template <int APP, bool W>
static hipError_t launch_back(const MinPushArgs& a, const MinBlkArgs& b, uint32_t finish_grid, hipStream_t s) {
  hipLaunchKernelGGL((minprop_back_kernel<APP, W>), dim3(std::max(kPieceGrid, finish_grid)), dim3(kBlock), 0, s, a, b,
                     kPieceGrid, finish_grid);
  return hipGetLastError();
}
static hipError_t back_dispatch(ipg_app app, bool weighted, const MinPushArgs& a, const MinBlkArgs& b,
                                uint32_t finish_grid, hipStream_t s) {
  if (app == IPG_APP_CC_HASHMIN) return launch_back<IPG_APP_CC_HASHMIN, false>(a, b, finish_grid, s);
  return weighted ? launch_back<IPG_APP_SSSP, true>(a, b, finish_grid, s)
                  : launch_back<IPG_APP_SSSP, false>(a, b, finish_grid, s);
}
// The push launch and, unless the back launch will run them, the pieces.
static hipError_t push_dispatch(ipg_app app, bool weighted, const MinPushArgs& a, uint32_t grid, bool pieces,
                                hipStream_t s) {
  if (app == IPG_APP_CC_HASHMIN) return launch_push<IPG_APP_CC_HASHMIN, false>(a, grid, pieces, s);
  return weighted ? launch_push<IPG_APP_SSSP, true>(a, grid, pieces, s)
                  : launch_push<IPG_APP_SSSP, false>(a, grid, pieces, s);
}
// The late push of a device-driven pull superstep and, unless the back
// launch will run them, its pieces (both return at once unless *a.late).
template <int APP, bool W>
static hipError_t launch_late(const MinPushArgs& a, const uint32_t* outbox, bool pieces, hipStream_t s) {
  hipLaunchKernelGGL((minprop_late_kernel<APP, W>), dim3(kExchangeGrid), dim3(kBlock), 0, s, a, outbox);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !pieces) return err;
  hipLaunchKernelGGL((minprop_piece_kernel<APP, W>), dim3(kPieceGrid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
static hipError_t late_dispatch(ipg_app app, bool weighted, const MinPushArgs& a, const uint32_t* outbox, bool pieces,
                                hipStream_t s) {
  if (app == IPG_APP_CC_HASHMIN) return launch_late<IPG_APP_CC_HASHMIN, false>(a, outbox, pieces, s);
  return weighted ? launch_late<IPG_APP_SSSP, true>(a, outbox, pieces, s)
                  : launch_late<IPG_APP_SSSP, false>(a, outbox, pieces, s);
}
static hipError_t pull_dispatch(ipg_app app, bool weighted, const MinPullArgs& a, uint32_t grid, hipStream_t s) {
  if (app == IPG_APP_CC_HASHMIN) return launch_pull<IPG_APP_CC_HASHMIN, false>(a, grid, s);
  return weighted ? launch_pull<IPG_APP_SSSP, true>(a, grid, s) : launch_pull<IPG_APP_SSSP, false>(a, grid, s);
}

// Frontier lists up to this size are visited through the list; larger ones
// by sweeping the mailboxes (div = UINT32_MAX: never through the list).
static uint64_t list_limit(uint32_t n, uint32_t div) {
  if (div == 0xFFFFFFFFu) return 0;
  return std::max<uint64_t>(4096, n / (div ? div : 16));
}

// The names a CC/SSSP run works under.  The caller's, with the caller's CSR
// for the push and the blocked in-edges of the caller's CSC (blk_ids, or
// blk on a store without renaming) for the pull.  Or, on a symmetric store
// that is hot-first and blocked, the new names (Section 4.2's vertex arrays
// in another order): the push reads the renamed CSC as the CSR (the graph is
// symmetric), the pull PageRank's table, whose hot sources are the most-read
// ones; CC's labels start from the caller's ids (iperm), SSSP starts at the
// source's new name, and the values go back to the caller's order at the
// end (w.value_u32[v] = value under v's new name).  Hash-min labels are the
// caller's ids either way, and a vertex's distance does not depend on the
// names, so results and traces are the same.
struct MinSpace {
  bool renamed;
  const uint64_t* off;      // CSR offsets
  const int32_t* dst;       // CSR destinations
  const uint32_t* w;        // CSR weights or null
  const uint32_t* outdeg;
  uint32_t* value;
  const uint32_t* ids;      // CC's initial label of every vertex (null: its id)
  uint32_t source;
  const BlockedTables* bt;  // blocked in-edges for the pull, or null (row items)
};
static MinSpace min_space(const ipg_graph* g, ipg_app app, uint32_t source, const RunWs& w, const Tune& tn) {
  MinSpace sp;
  const bool weighted = app == IPG_APP_SSSP && g->csr_w != nullptr;
  const GraphTables& t = g->t;
  sp.renamed = (g->flags & IPG_GRAPH_SYMMETRIC) && t.perm && t.blk.edges && !weighted && tn.blocked &&
               g->perm_host.size() == g->n;
  if (sp.renamed) {
    sp.off = t.off_hot;
    sp.dst = t.src_hot;
    sp.w = nullptr;
    sp.outdeg = t.outdeg_hot;
    sp.value = w.value_u32_hot;
    sp.ids = t.iperm;
    sp.source = app == IPG_APP_SSSP ? g->perm_host[source] : 0u;
    sp.bt = &t.blk;
    return sp;
  }
  sp.off = g->csr_off;
  sp.dst = g->csr_dst;
  sp.w = weighted ? g->csr_w : nullptr;
  sp.outdeg = t.outdeg;
  sp.value = w.value_u32;
  sp.ids = nullptr;
  sp.source = source;
  // the blocked in-edges of the caller's CSC (CC, unit-weight SSSP), if the store has them
  sp.bt = nullptr;
  if (tn.blocked && !weighted) sp.bt = t.blk_ids.edges ? &t.blk_ids : (t.blk.edges && !t.perm ? &t.blk : nullptr);
  return sp;
}

// Values of a run under the new names back to the caller's order.
__global__ void min_unrename_kernel(const uint32_t* value_hot, const uint32_t* perm, uint32_t n, uint32_t* value) {
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
    value[v] = value_hot[perm[v]];
}
static ipg_status finish_space(const ipg_graph* g, const MinSpace& sp, const RunWs& w, hipStream_t s) {
  if (!sp.renamed) return IPG_OK;
  hipLaunchKernelGGL(min_unrename_kernel, dim3(grid_for(g->n, kBlock, 16384)), dim3(kBlock), 0, s, sp.value, g->t.perm,
                     g->n, w.value_u32);
  IPG_HIP(hipGetLastError());
  return IPG_OK;
}

// Ping-pong buffers of superstep `step`.
struct StepBufs {
  CtrSlot* c;    // this superstep's counters
  CtrSlot* cc;   // the next superstep's counters (cleared by this superstep's exchange)
  uint32_t* lpre_in;   // prefix of the list the previous superstep left (read by this one's list phase)
  uint32_t* lpre_out;  // prefix of the list this superstep leaves (written by its decide)
  uint32_t *fin, *fout, *mail_in, *mail_out;
};
static StepBufs bufs_for(const RunWs& w, uint32_t step) {
  const bool odd = step & 1;
  StepBufs b;
  b.c = w.ctr + (odd ? kCtrSlots : 0);
  b.cc = w.ctr + (odd ? 0 : kCtrSlots);
  b.lpre_out = w.lpre + (odd ? kCtrSlots + 1 : 0);
  b.lpre_in = w.lpre + (odd ? 0 : kCtrSlots + 1);
  b.fin = odd ? w.fr_b : w.fr_a;
  b.fout = odd ? w.fr_a : w.fr_b;
  b.mail_in = odd ? w.mail_b : w.mail_a;
  b.mail_out = odd ? w.mail_a : w.mail_b;
  return b;
}

// The launches of one superstep.  With ctl == null (host-driven loop) the
// exchange is `mode` and the active set `act`; with a control block
// (device-driven loop) both exchanges are launched on fixed grids, the
// control block picks one (and, from superstep 1, the active set), and work
// that only one exchange has shares a launch with the other's
// (minprop_front_kernel from superstep 1, minprop_back_kernel over blocked
// in-edges).
static ipg_status enqueue_step(ipg_graph* g, ipg_app app, const MinSpace& sp, uint32_t step, ipg_mode mode,
                               const Active& act, uint64_t degsum, const RunWs& w, const DevCtl* ctl, const Tune& tn,
                               hipStream_t s) {
  const uint32_t n = g->n;
  const bool weighted = sp.w != nullptr;
  const uint32_t gv = grid_for(n, kBlock, 16384);
  const StepBufs b = bufs_for(w, step);
  const bool device = ctl != nullptr;
  const BlockedTables* bt = sp.bt;
  // device-driven superstep s >= 1: the push and the pull form's compute
  // share one launch (minprop_front_kernel), made where the compute's was
  const bool front = device && step > 0;
  // device-driven loop over blocked in-edges: the pieces share the blocked
  // pull's second launch (minprop_back_kernel)
  const bool back = device && bt && bt->ngroups;
  MinPushArgs front_push{};
  uint32_t front_push_grid = 0;
  // pull superstep s >= 1 that may turn to a push once its messages are
  // counted (pick_kernel); the caller zeroes late_div when the exchange is
  // forced
  const bool late_on = step > 0 && tn.late_div != 0 && (device || mode == IPG_MODE_PULL);
  if (step == 0) {
    hipLaunchKernelGGL(minprop_init_kernel, dim3(gv), dim3(kBlock), 0, s, n, static_cast<int>(app), sp.source,
                       sp.value, sp.outdeg, mode == IPG_MODE_PULL ? 1 : 0, w.outbox, b.c, ctl,
                       device ? w.mail_a : nullptr, device ? w.mail_b : nullptr, sp.ids);
    IPG_HIP(hipGetLastError());
  }
  if (device || mode == IPG_MODE_PUSH || late_on) {
    MinPushArgs a;
    a.act = act;
    a.act.list = b.fin;
    a.act.pre = b.lpre_in;
    a.act.seg = list_seg(n);
    a.off = sp.off;
    a.dst = sp.dst;
    a.w = sp.w;
    a.outdeg = sp.outdeg;
    a.value = sp.value;
    a.mail_in = b.mail_in;
    a.mail_out = b.mail_out;
    a.list_out = b.fout;
    a.list_seg = list_seg(n);
    a.ctr = b.c;
    a.ctr_clear = b.cc;
    a.ctl = ctl;
    a.n = n;
    // piece queue and launch: always in the device-driven loop (the launch
    // returns at once without pieces), else when the frontier's out-degrees
    // could make one
    const bool pieces = device || late_on || degsum >= kPieceMin;
    a.pieces = pieces ? w.pieces : nullptr;
    a.piece_seg = piece_seg(g->e);
    a.late = nullptr;
    const uint32_t grid = device ? kExchangeGrid : grid_for(act.count, kBlock, 0xFFFFFFFFu);
    front_push = a;
    front_push_grid = grid;
    if (!front && (device || mode == IPG_MODE_PUSH)) IPG_HIP(push_dispatch(app, weighted, a, grid, !back, s));
  }
  if (device || mode == IPG_MODE_PULL) {
    const bool gating = step > 0 && tn.gate_div != 0;
    if (step > 0) {
      if (!device) IPG_HIP(fill_u32(w.outbox, n, kInf, s));
      if (gating) IPG_HIP(fill_u32(w.sent, (uint64_t)n / 64 * 2 + 2, 0, s));
      MinApplyArgs ap;
      ap.act = act;
      ap.act.list = b.fin;
      ap.act.pre = b.lpre_in;
      ap.act.seg = list_seg(n);
      ap.outdeg = sp.outdeg;
      ap.value = sp.value;
      ap.mail_in = b.mail_in;
      ap.outbox = w.outbox;
      ap.ctr = b.c;
      ap.ctl = ctl;
      ap.n = n;
      ap.sent = gating ? w.sent : nullptr;
      // the dense form without the sender bitmap takes four vertices per thread
      const bool dense4 = (device || act.phase == kStepDense) && !gating;
      const uint32_t grid = dense4 ? grid_for((static_cast<uint64_t>(n) + 3) / 4, kBlock, 16384)
                                   : (device ? gv : grid_for(act.count, kBlock, 8192));
      if (front) {
        // the compute is grid-stride: capped at the push grid, the launch is
        // no wider than the push needs (a wider one dispatched workgroups
        // that return at once in every push superstep of a large graph)
        IPG_HIP(front_dispatch(app, weighted, front_push, ap, front_push_grid, std::min(grid, front_push_grid), !back,
                               s));
      } else {
        hipLaunchKernelGGL(minprop_apply_kernel, dim3(grid), dim3(kBlock), 0, s, ap);
        IPG_HIP(hipGetLastError());
      }
      if (gating || late_on) {
        hipLaunchKernelGGL(pick_kernel, dim3(1), dim3(kWave), 0, s, b.c, n, g->e, gating ? tn.gate_div : 0u,
                           late_on ? tn.late_div : 0u, ctl, gating ? w.gate : nullptr, late_on ? w.late : nullptr);
        IPG_HIP(hipGetLastError());
      }
    }
    MinPushArgs late_push = front_push;
    late_push.late = w.late;
    if (bt) {
      MinBlkArgs ba;
      ba.v = blk_view(*bt);
      ba.outdeg = sp.outdeg;
      ba.outbox = w.outbox;
      ba.mail_out = b.mail_out;
      ba.ctr = b.c;
      ba.ctr_clear = b.cc;
      ba.ctl = ctl;
      ba.sent = w.sent;
      // over binned in-edges the gathers left are the hot sources' (a few MB
      // of outboxes): the senders' bitmap would only add a dependent load
      ba.gate = gating && !bt->hot ? w.gate : nullptr;
      ba.slots = bt->hot ? reinterpret_cast<const uint32_t*>(bt->slots) : nullptr;
      ba.late = late_on ? w.late : nullptr;
      if (bt->hot && bt->bin_nunits) {
        hipLaunchKernelGGL(min_bin_kernel, dim3(bt->bin_nunits), dim3(kBlkThreads), 0, s, ba, bin_tables(*bt),
                           reinterpret_cast<uint32_t*>(bt->slots), n);
        IPG_HIP(hipGetLastError());
      }
      if (bt->nslices) {
        if (app == IPG_APP_CC_HASHMIN)
          hipLaunchKernelGGL(minprop_blocked_kernel<IPG_APP_CC_HASHMIN>, dim3(bt->nslices), dim3(kBlkThreads), 0, s, ba);
        else
          hipLaunchKernelGGL(minprop_blocked_kernel<IPG_APP_SSSP>, dim3(bt->nslices), dim3(kBlkThreads), 0, s, ba);
        IPG_HIP(hipGetLastError());
      } else {  // no edges: nothing arrives, but the next superstep's counters are still cleared here
        IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(b.cc), kCtrSlots * sizeof(CtrSlot) / 4, 0, s));
      }
      if (late_on) IPG_HIP(late_dispatch(app, weighted, late_push, w.outbox, !back, s));
      if (back) {
        IPG_HIP(back_dispatch(app, weighted, front_push, ba, grid_for(bt->ngroups, kWavesPerBlock, 4096), s));
      } else if (bt->ngroups) {
        hipLaunchKernelGGL(minprop_blocked_finish_kernel, dim3(grid_for(bt->ngroups, kWavesPerBlock, 4096)),
                           dim3(kBlock), 0, s, ba);
        IPG_HIP(hipGetLastError());
      }
      return IPG_OK;
    }
    MinPullArgs pa;
    pa.t = pull_tiling(g);
    pa.w = weighted ? g->csc_w : nullptr;
    pa.outdeg = sp.outdeg;
    pa.outbox = w.outbox;
    pa.mail_out = b.mail_out;
    pa.ctr = b.c;
    pa.ctr_clear = b.cc;
    pa.ctl = ctl;
    pa.sent = w.sent;
    pa.gate = gating ? w.gate : nullptr;
    pa.late = late_on ? w.late : nullptr;
    IPG_HIP(pull_dispatch(app, weighted, pa, tn.pull_grid, s));
    if (late_on) IPG_HIP(late_dispatch(app, weighted, late_push, w.outbox, true, s));
  }
  return IPG_OK;
}

// State before superstep 0 shared by both loops: mailboxes empty, counters
// zero (one launch for the three arrays).
__global__ void minprop_clear_kernel(uint32_t* mail_a, uint32_t* mail_b, uint32_t n, uint32_t* ctr, uint32_t words) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  const uint64_t t = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  for (uint64_t i = t; i < n; i += stride) {
    mail_a[i] = kInf;
    mail_b[i] = kInf;
  }
  for (uint64_t i = t; i < words; i += stride) ctr[i] = 0;
}
static ipg_status clear_minprop(const ipg_graph* g, const RunWs& w, hipStream_t s) {
  const uint32_t n = g->n;
  const uint32_t words = 2 * kCtrSlots * sizeof(CtrSlot) / 4;
  hipLaunchKernelGGL(minprop_clear_kernel, dim3(grid_for(std::max(n, words), kBlock * 4, 8192)), dim3(kBlock), 0, s,
                     w.mail_a, w.mail_b, n, reinterpret_cast<uint32_t*>(w.ctr), words);
  IPG_HIP(hipGetLastError());
  return IPG_OK;
}

// The host loop's superstep 0: its active set (every vertex for CC, the
// source for SSSP), their out-degree sum and the selector's choice.
struct MinStart {
  uint64_t count, degsum;
  int sel_mode;  // the selector's choice for superstep 0, 0 if none
};
static ipg_status start_minprop(ipg_graph* g, ipg_app app, const ipg_run_opts& o, const RunWs& w, hipStream_t s,
                                MinStart* out) {
  const uint32_t n = g->n;
  const uint64_t e = g->e;
  uint64_t src_deg = 0;
  if (app == IPG_APP_SSSP) {
    uint64_t h[2];
    IPG_HIP(hipMemcpyAsync(h, g->csr_off + o.source, sizeof(h), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    src_deg = h[1] - h[0];
  }
  const ipg_status rc = clear_minprop(g, w, s);
  if (rc != IPG_OK) return rc;
  out->count = app == IPG_APP_CC_HASHMIN ? n : 1;
  out->degsum = app == IPG_APP_CC_HASHMIN ? e : src_deg;
  out->sel_mode = 0;
  if (o.mode == IPG_MODE_AUTO && o.selector) {
    double hp[kSelParams];
    IPG_HIP(hipMemcpyAsync(hp, o.selector, sizeof(hp), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    bool ul;
    sel_predict_mode(hp, out->count, out->degsum, 0, e, false, &out->sel_mode, &ul);
  }
  return IPG_OK;
}

static Active step0_active(ipg_app app, uint32_t n, uint32_t source) {
  Active act{};
  act.source = source;
  act.list = nullptr;
  act.phase = app == IPG_APP_CC_HASHMIN ? kSendAll : kSendSource;
  act.count = app == IPG_APP_CC_HASHMIN ? n : 1;
  return act;
}

// Device-driven loop (IPG_RUN_PERSISTENT): the host enqueues supersteps in
// chunks of growing length without reading anything back; the control
// block decides halt, active set and exchange on the device (superstep 0's
// too), the kernels of the supersteps after the halt return at once, and
// the decide kernels copy the control block and the trace records into
// pinned host memory, which the host reads after one synchronisation per
// chunk.
static ipg_status run_minprop_device(ipg_graph* g, ipg_app app, uint32_t cap, const ipg_run_opts& o, const RunWs& w,
                                     hipStream_t s, StepTimer& tm, ipg_run_stats* st) {
  const uint32_t n = g->n;
  const uint64_t e = g->e;
  Tune tn = resolve_tuning(o.tuning);
  HostMirror *hm = nullptr, *hm_dev = nullptr;
  IPG_HIP(host_mirror(g, &hm, &hm_dev));
  ipg_status rc = IPG_OK;
  if (!g->wall_khz) IPG_HIP(hipDeviceGetAttribute(&g->wall_khz, hipDeviceAttributeWallClockRate, g->device));
  const double us_per_tick = g->wall_khz > 0 ? 1e3 / g->wall_khz : 0.0;
  const double* sel = o.mode == IPG_MODE_AUTO ? o.selector : nullptr;
  const int forced = o.mode == IPG_MODE_AUTO ? 0 : static_cast<int>(o.mode);
  if (forced) tn.late_div = 0;  // a forced exchange stays as forced
  const MinSpace sp = min_space(g, app, o.source, w, tn);
  IPG_HIP(tm.start(s));
  // the counters are zeroed by dd_start_kernel and the mailboxes emptied by
  // superstep 0's init kernel, so the run starts with no clearing launch
  hipLaunchKernelGGL(dd_start_kernel, dim3(1), dim3(kWave), 0, s, w.ctl, static_cast<int>(app), sp.source, sp.off, n,
                     e, sel, forced, tn.push_div, cap, w.ctr);
  IPG_HIP(hipGetLastError());
  rc = enqueue_step(g, app, sp, 0, IPG_MODE_AUTO, step0_active(app, n, sp.source), 0, w, w.ctl, tn, s);
  if (rc != IPG_OK) return rc;
  uint32_t enqueued = 0;  // supersteps whose launches are in the stream, minus one
  uint32_t recorded = 0;  // supersteps whose records were read
  // supersteps enqueued per readback: first as many as the last device-driven
  // run of this application on the handle took (repeated runs mostly take
  // the same number, and then read back once; a longer guess costs only
  // launches that return at once), else 2; then doubling, up to 64
  const uint32_t last = g->dd_steps[static_cast<int>(app) & 3];
  uint32_t chunk = last ? std::min<uint32_t>(std::max<uint32_t>(last, 2), 64) : 2;
  DevCtl h{};
  uint64_t tot_msgs = 0, tot_exam = 0;
  for (;;) {
    for (uint32_t k = 0; k < chunk; ++k) {
      const uint32_t step = enqueued + k;
      if (step > 0) {
        Active unused{};
        rc = enqueue_step(g, app, sp, step, IPG_MODE_AUTO, unused, 0, w, w.ctl, tn, s);
        if (rc != IPG_OK) return rc;
      }
      const StepBufs b = bufs_for(w, step);
      hipLaunchKernelGGL(dd_decide_kernel, dim3(1), dim3(kWave), 0, s, b.c, list_seg(n), b.lpre_out, e, n, sel, forced,
                         list_limit(n, tn.list_div), tn.push_div, w.ctl, hm_dev,
                         step > 0 && tn.late_div ? static_cast<const uint32_t*>(w.late) : nullptr);
      IPG_HIP(hipGetLastError());
    }
    enqueued += chunk;
    IPG_HIP(tm.mark(s));  // the run's end if this chunk holds the halt
    IPG_HIP(hipStreamSynchronize(s));
    h = hm->ctl;  // as the chunk's last decide (before or at the halt) left it
    for (; recorded < h.step; ++recorded) {
      const DevRec r = hm->rec[recorded % kDevRec];
      if (st && recorded < st->trace_cap) {
        if (st->active) st->active[recorded] = r.active;
        if (st->senders) st->senders[recorded] = r.senders;
        if (st->messages) st->messages[recorded] = r.messages;
        if (st->examined) st->examined[recorded] = r.examined;
        if (st->mode) st->mode[recorded] = static_cast<uint8_t>(r.mode);
        if (st->frontier_deg) st->frontier_deg[recorded] = r.frontier_deg;
        // device time of the superstep, between the wall-clock stamps of two decide kernels
        if (st->usec) st->usec[recorded] = static_cast<float>(r.ticks * us_per_tick);
      }
      tot_msgs += r.messages;
      tot_exam += r.examined;
    }
    if (h.halted) break;
    chunk = std::min<uint32_t>(chunk * 2, 64);
  }
  rc = finish_space(g, sp, w, s);
  if (rc != IPG_OK) return rc;
  IPG_HIP(tm.finish(s));
  g->dd_steps[static_cast<int>(app) & 3] = h.step;
  if (st) {
    st->supersteps = h.step;
    st->halted = h.status == IPG_OK;
    st->edges_traversed = tot_msgs;
    st->edges_examined = tot_exam;
  }
  if (h.status == IPG_EOVERFLOW) return fail(IPG_EOVERFLOW, "SSSP distance would reach 0xFFFFFFFF (INF)");
  if (h.status == IPG_EDEVICE) return fail(IPG_EDEVICE, "frontier list length disagrees with the mailbox count");
  return static_cast<ipg_status>(h.status);
}

ipg_status run_minprop(ipg_graph* g, ipg_app app, uint32_t cap, const ipg_run_opts& o, const RunWs& w,
                       hipStream_t s, StepTimer& tm, ipg_run_stats* st) {
  if (o.flags & IPG_RUN_PERSISTENT) return run_minprop_device(g, app, cap, o, w, s, tm, st);
  const uint32_t n = g->n;
  const uint64_t e = g->e;
  Tune tn = resolve_tuning(o.tuning);
  if (o.mode != IPG_MODE_AUTO) tn.late_div = 0;  // a forced exchange stays as forced
  const MinSpace sp = min_space(g, app, o.source, w, tn);
  HostMirror *hm = nullptr, *hm_dev = nullptr;
  IPG_HIP(host_mirror(g, &hm, &hm_dev));
  MinStart m0;
  ipg_status status = start_minprop(g, app, o, w, s, &m0);
  if (status != IPG_OK) return status;
  uint64_t count = m0.count, degsum = m0.degsum;
  int next_sel_mode = m0.sel_mode;  // the selector's choice for the coming superstep
  bool list_ok = false;             // the superstep's active set is the list left by a push
  uint32_t step = 0;
  uint64_t tot_msgs = 0, tot_exam = 0;
  IPG_HIP(tm.start(s));
  for (;;) {
    ModeQuery q{n, e, count, degsum, step, app};
    ipg_mode mode = o.mode;
    if (mode == IPG_MODE_AUTO) mode = next_sel_mode ? static_cast<ipg_mode>(next_sel_mode) : heuristic_mode(q, tn.push_div);
    const StepBufs b = bufs_for(w, step);
    Active act{};
    if (step == 0) {
      act = step0_active(app, n, sp.source);
    } else {
      act.source = sp.source;
      act.list = b.fin;
      act.phase = list_ok ? kStepList : kStepDense;
      act.count = list_ok ? static_cast<uint32_t>(count) : n;
    }
    status = enqueue_step(g, app, sp, step, mode, act, degsum, w, nullptr, tn, s);
    if (status != IPG_OK) return status;
    IPG_HIP(tm.step(s, step));
    const double* sel = o.mode == IPG_MODE_AUTO ? o.selector : nullptr;
    const bool late_on = step > 0 && mode == IPG_MODE_PULL && tn.late_div != 0;
    IPG_HIP(launch_decide(b.c, step + 1, e, sel, &hm_dev->decision, list_seg(n), b.lpre_out, s,
                          late_on ? w.late : nullptr, static_cast<int>(mode)));
    IPG_HIP(hipStreamSynchronize(s));
    const Decision h = hm->decision;
    const uint64_t lcount = h.list_len;  // ~0: a segment overflowed, no list
    const ipg_mode ran = h.late ? IPG_MODE_PUSH : mode;  // a late push counts as a push
    const uint64_t examined = ran == IPG_MODE_PUSH ? h.messages : e;
    if (st && step < st->trace_cap) {
      if (st->active) st->active[step] = step == 0 ? n : count;
      if (st->senders) st->senders[step] = h.senders;
      if (st->messages) st->messages[step] = h.messages;
      if (st->examined) st->examined[step] = examined;
      if (st->mode) st->mode[step] = static_cast<uint8_t>(ran);
      if (st->frontier_deg) st->frontier_deg[step] = degsum;
    }
    tot_msgs += h.messages;
    tot_exam += examined;
    ++step;
    if (h.overflow) {
      status = fail(IPG_EOVERFLOW, "SSSP distance would reach 0xFFFFFFFF (INF)");
      break;
    }
    if (h.next_count == 0) break;  // every vertex halted and no message is pending
    if (cap && step >= cap) {
      status = IPG_NOT_CONVERGED;
      break;
    }
    if (ran == IPG_MODE_PUSH && lcount != ~0ull && lcount != h.next_count) {
      status = fail(IPG_EDEVICE, "frontier list length disagrees with the mailbox count");
      break;
    }
    count = h.next_count;
    degsum = h.next_deg;
    next_sel_mode = h.mode;
    // as the device-driven loop decides it: a push chosen by the selector
    // visits the list when it predicted that variant faster
    const bool list_avail = ran == IPG_MODE_PUSH && lcount != ~0ull;
    list_ok = list_avail && (h.mode == IPG_MODE_PUSH ? h.list != 0 : count <= list_limit(n, tn.list_div));
  }
  const ipg_status fs = finish_space(g, sp, w, s);
  if (fs != IPG_OK) return fs;
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
