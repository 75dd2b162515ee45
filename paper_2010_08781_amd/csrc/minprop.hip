// minprop.hip -- hash-min connected components (Fig. 9) and SSSP (Fig. 10)
// on the superstep engine, uint32 values and messages combined by min (Fig. 5).
//
// Both applications vote to halt after every compute ("systematic halt",
// Section 4.3.1), so the vertices active in superstep s+1 are exactly the
// recipients of a message in superstep s.  The next frontier is therefore
// built while messages are delivered: a recipient is appended when its
// mailbox was empty (the atomic min returns the identity INF), which also
// removes duplicates -- the selection bypass of Section 4.3.1, with the
// per-thread lists replaced by wavefront-ballot compaction.
//
// Superstep s >= 1 for a frontier vertex v: consume its one-slot mailbox
// (reset it to INF); if the message is below value(v), lower value(v) and
// broadcast -- value(v) for CC, value(v) + 1 (or + w(v, x) per out-edge when
// weighted) for SSSP.  Superstep 0: CC sets value = id and every vertex
// broadcasts; SSSP sets value = 0 at the source (which broadcasts) and INF
// elsewhere.
//
// Mailboxes are double-buffered (consume from `mail_in`, deliver into
// `mail_out`) so that a superstep never sees a message sent in the same
// superstep (Section 4.2).
#include "common.h"
#include "engine.h"
#include "scatter.h"

namespace ipg {

enum : int { kPhaseSendAll = 0, kPhaseSendSource = 1, kPhaseStep = 2 };

__device__ __forceinline__ void clear_counters(StepCounters* c) {
  if (c && blockIdx.x == 0 && threadIdx.x < sizeof(StepCounters) / 4) reinterpret_cast<uint32_t*>(c)[threadIdx.x] = 0;
}

// value = id (CC) or 0 at the source / INF elsewhere (SSSP).  With `pull_s0`
// the superstep-0 senders are also recorded in the sent bitmap (which must be
// zero) and counted.
__global__ __launch_bounds__(kBlock) void minprop_init_kernel(uint32_t n, int app, uint32_t source, uint32_t* value,
                                                              const uint32_t* outdeg, int pull_s0, uint32_t* sent,
                                                              StepCounters* ctr) {
  uint64_t senders = 0, messages = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const bool sends = (app == IPG_APP_CC_HASHMIN) || v == source;
    value[v] = app == IPG_APP_CC_HASHMIN ? static_cast<uint32_t>(v) : (v == source ? 0u : kInf);
    if (pull_s0 && sends) {
      atomicOr(sent + (v >> 5), 1u << (v & 31));
      senders += 1;
      messages += outdeg[v];
    }
  }
  if (pull_s0) {
    block_add_u64(senders, &ctr->senders);
    block_add_u64(messages, &ctr->messages);
  }
}

struct MinPushArgs {
  int phase;
  uint32_t source;
  uint32_t count;             // frontier entries (or N for kPhaseSendAll)
  const uint32_t* frontier_in;
  const uint64_t* off;        // CSR
  const int32_t* dst;
  const uint32_t* w;          // CSR weights or null
  const uint32_t* outdeg;
  uint32_t* value;
  uint32_t* mail_in;
  uint32_t* mail_out;
  uint32_t* frontier_out;
  StepCounters* ctr;
  StepCounters* ctr_clear;
};

// Fused compute + push scatter of one superstep (one thread per frontier
// entry, out-edges expanded by twc_scatter).
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_push_kernel(MinPushArgs a) {
  clear_counters(a.ctr_clear);
  const uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
  bool has = false;
  uint64_t beg = 0, end = 0;
  uint32_t msg = 0;
  if (i < a.count) {
    uint32_t v;
    if (a.phase == kPhaseSendAll) {
      v = static_cast<uint32_t>(i);
      has = true;
      msg = a.value[v];
    } else if (a.phase == kPhaseSendSource) {
      v = a.source;
      has = true;
      msg = a.value[v];
    } else {
      v = a.frontier_in[i];
      const uint32_t m = a.mail_in[v];
      a.mail_in[v] = kInf;
      if (m < a.value[v]) {
        a.value[v] = m;
        has = true;
        msg = m;
      }
    }
    if (has) {
      beg = a.off[v];
      end = a.off[v + 1];
    }
  }
  const uint64_t senders = has ? 1 : 0, messages = end - beg;
  uint64_t next_deg = 0;
  uint32_t overflow = 0;
  uint32_t* mail = a.mail_out;
  twc_scatter(has, beg, end, msg, [&](uint64_t e, uint32_t p) {
    const uint32_t x = static_cast<uint32_t>(a.dst[e]);
    uint64_t m = p;
    if (APP == IPG_APP_SSSP) m += W ? a.w[e] : 1u;
    bool fresh = false;
    if (m >= kInf) overflow = 1;
    else fresh = atomicMin(mail + x, static_cast<uint32_t>(m)) == kInf;
    wave_append(fresh, x, a.frontier_out, &a.ctr->next_count);
    if (fresh) next_deg += a.outdeg[x];
  });
  block_add_u64(senders, &a.ctr->senders);
  block_add_u64(messages, &a.ctr->messages);
  block_add_u64(messages, &a.ctr->examined);
  block_add_u64(next_deg, &a.ctr->next_deg);
  if (__ballot(overflow) && lane_id() == 0) atomicOr(&a.ctr->overflow, 1u);
}

struct MinApplyArgs {
  uint32_t count;
  const uint32_t* frontier_in;
  const uint32_t* outdeg;
  uint32_t* value;
  uint32_t* mail_in;
  uint32_t* sent;             // bitmap, zero on entry
  StepCounters* ctr;
  StepCounters* ctr_clear;
};

// Compute phase of a pull superstep: consume mailboxes of the frontier,
// record the senders in the bitmap (their value is the one-slot outbox).
__global__ __launch_bounds__(kBlock) void minprop_apply_kernel(MinApplyArgs a) {
  clear_counters(a.ctr_clear);
  uint64_t senders = 0, messages = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < a.count; i += stride) {
    const uint32_t v = a.frontier_in[i];
    const uint32_t m = a.mail_in[v];
    a.mail_in[v] = kInf;
    if (m < a.value[v]) {
      a.value[v] = m;
      atomicOr(a.sent + (v >> 5), 1u << (v & 31));
      senders += 1;
      messages += a.outdeg[v];
    }
  }
  block_add_u64(senders, &a.ctr->senders);
  block_add_u64(messages, &a.ctr->messages);
}

struct MinPullArgs {
  const uint64_t* off;   // CSC
  const int32_t* src;
  const uint32_t* w;     // CSC weights or null
  const uint32_t* outdeg;
  const uint32_t* rb;
  const uint32_t* long_rows;
  uint32_t nl;
  const uint32_t* sent;
  const uint32_t* value;
  uint32_t* mail_out;
  uint32_t* frontier_out;
  StepCounters* ctr;
  StepCounters* ctr_clear;
};

// Message a sender u offers over in-edge e (INF when u did not broadcast).
template <int APP, bool W>
__device__ __forceinline__ uint32_t pull_msg(const MinPullArgs& a, uint64_t e, uint32_t& overflow) {
  const uint32_t u = static_cast<uint32_t>(a.src[e]);
  if (!((a.sent[u >> 5] >> (u & 31)) & 1u)) return kInf;
  uint64_t m = a.value[u];
  if (APP == IPG_APP_SSSP) m += W ? a.w[e] : 1u;
  if (m >= kInf) {
    overflow = 1;
    return kInf;
  }
  return static_cast<uint32_t>(m);
}

__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = min(x, static_cast<uint32_t>(__shfl_xor(x, o)));
  return x;
}

// Exchange of a pull superstep over the CSC, same tiling as the PageRank
// pull: long rows first (a workgroup each), then LDS-staged row-groups.
template <int APP, bool W>
__global__ __launch_bounds__(kBlock) void minprop_pull_kernel(MinPullArgs a) {
  __shared__ uint32_t tile[2 * kPullTile];
  __shared__ uint32_t red[kWavesPerBlock];
  clear_counters(a.ctr_clear);
  const uint32_t b = blockIdx.x, tid = threadIdx.x;
  uint64_t examined = 0, next_deg = 0;
  uint32_t overflow = 0;
  if (b < a.nl) {
    const uint32_t v = a.long_rows[b];
    const uint64_t beg = a.off[v], end = a.off[v + 1];
    uint32_t m = kInf;
    for (uint64_t e = beg + tid; e < end; e += kBlock) m = min(m, pull_msg<APP, W>(a, e, overflow));
    m = wave_min(m);
    if (lane_id() == 0) red[tid / kWave] = m;
    __syncthreads();
    if (tid == 0) {
      m = min(min(red[0], red[1]), min(red[2], red[3]));
      examined = end - beg;
      if (m < kInf) {
        a.mail_out[v] = m;
        a.frontier_out[atomicAdd(&a.ctr->next_count, 1u)] = v;
        next_deg = a.outdeg[v];
      }
    }
  } else {
    const uint32_t k = b - a.nl;
    const uint32_t r0 = a.rb[k];
    uint32_t r1 = a.rb[k + 1];
    if (r1 > r0 && a.off[r1] - a.off[r1 - 1] > kPullTile) --r1;
    if (r0 < r1) {  // block-uniform
      const uint64_t e0 = a.off[r0];
      uint32_t span = static_cast<uint32_t>(a.off[r1] - e0);
      if (span > 2 * kPullTile) span = 2 * kPullTile;
      for (uint32_t i = tid; i < span; i += kBlock) tile[i] = pull_msg<APP, W>(a, e0 + i, overflow);
      if (tid == 0) examined = span;
      __syncthreads();
      const uint32_t nrows = r1 - r0;
      uint32_t G = kWave;
      while (G > 1 && G * nrows > kBlock) G >>= 1;
      const uint32_t groups = kBlock / G, gi = tid / G, li = tid % G;
      for (uint32_t base = 0; base < nrows; base += groups) {
        const uint32_t row = base + gi;
        uint32_t m = kInf;
        if (row < nrows) {
          const uint32_t v = r0 + row;
          uint32_t lo = static_cast<uint32_t>(a.off[v] - e0), hi = static_cast<uint32_t>(a.off[v + 1] - e0);
          if (hi > span) hi = span;
          for (uint32_t j = lo + li; j < hi; j += G) m = min(m, tile[j]);
        }
        for (uint32_t o = G >> 1; o >= 1; o >>= 1) m = min(m, static_cast<uint32_t>(__shfl_xor(m, static_cast<int>(o))));
        const bool got = li == 0 && row < nrows && m < kInf;
        if (got) {
          a.mail_out[r0 + row] = m;
          next_deg += a.outdeg[r0 + row];
        }
        wave_append(got, r0 + row, a.frontier_out, &a.ctr->next_count);
      }
    }
  }
  block_add_u64(examined, &a.ctr->examined);
  block_add_u64(next_deg, &a.ctr->next_deg);
  if (__ballot(overflow) && lane_id() == 0) atomicOr(&a.ctr->overflow, 1u);
}

// ------------------------------------------------------------------ host --

template <int APP, bool W>
static hipError_t launch_push(const MinPushArgs& a, uint32_t items, hipStream_t s) {
  hipLaunchKernelGGL((minprop_push_kernel<APP, W>), dim3(grid_for(items, kBlock, 0xFFFFFFFFu)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
template <int APP, bool W>
static hipError_t launch_pull(const MinPullArgs& a, uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((minprop_pull_kernel<APP, W>), dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

static hipError_t push_dispatch(ipg_app app, bool weighted, const MinPushArgs& a, uint32_t items, hipStream_t s) {
  if (app == IPG_APP_CC_HASHMIN) return launch_push<IPG_APP_CC_HASHMIN, false>(a, items, s);
  return weighted ? launch_push<IPG_APP_SSSP, true>(a, items, s) : launch_push<IPG_APP_SSSP, false>(a, items, s);
}
static hipError_t pull_dispatch(ipg_app app, bool weighted, const MinPullArgs& a, uint32_t blocks, hipStream_t s) {
  if (app == IPG_APP_CC_HASHMIN) return launch_pull<IPG_APP_CC_HASHMIN, false>(a, blocks, s);
  return weighted ? launch_pull<IPG_APP_SSSP, true>(a, blocks, s) : launch_pull<IPG_APP_SSSP, false>(a, blocks, s);
}

ipg_status run_minprop(ipg_graph* g, ipg_app app, uint32_t cap, const ipg_run_opts& o, const RunWs& w,
                       hipStream_t s, StepTimer& tm, ipg_run_stats* st) {
  const uint32_t n = g->n;
  const uint64_t e = g->e;
  const bool weighted = app == IPG_APP_SSSP && g->csr_w != nullptr;
  const uint32_t words = n / 32 + 1;
  const uint32_t gv = grid_for(n, kBlock, 16384);

  // Out-degree of the SSSP source, for the superstep-0 exchange choice.
  uint64_t src_deg = 0;
  if (app == IPG_APP_SSSP) {
    uint64_t h[2];
    IPG_HIP(hipMemcpyAsync(h, g->csr_off + o.source, sizeof(h), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    src_deg = h[1] - h[0];
  }
  IPG_HIP(fill_u32(w.mail_a, n, kInf, s));
  IPG_HIP(fill_u32(w.mail_b, n, kInf, s));
  IPG_HIP(fill_u32(reinterpret_cast<uint32_t*>(w.ctr), 2 * sizeof(StepCounters) / 4, 0, s));

  uint32_t *fin = w.fr_a, *fout = w.fr_b, *min_ = w.mail_a, *mout = w.mail_b;
  uint64_t count = app == IPG_APP_CC_HASHMIN ? n : 1;
  uint64_t degsum = app == IPG_APP_CC_HASHMIN ? e : src_deg;
  uint32_t step = 0;
  ipg_status status = IPG_OK;
  uint64_t tot_msgs = 0, tot_exam = 0;
  IPG_HIP(tm.start(s));
  for (;;) {
    ModeQuery q{n, e, count, degsum, step, app};
    const ipg_mode mode = choose_mode(o.mode, q);
    StepCounters* c = w.ctr + (step & 1);
    StepCounters* cc = w.ctr + ((step + 1) & 1);
    if (mode == IPG_MODE_PUSH) {
      if (step == 0) {
        hipLaunchKernelGGL(minprop_init_kernel, dim3(gv), dim3(kBlock), 0, s, n, static_cast<int>(app), o.source,
                           w.value_u32, g->t.outdeg, 0, w.sent, c);
        IPG_HIP(hipGetLastError());
      }
      MinPushArgs a;
      a.phase = step > 0 ? kPhaseStep : (app == IPG_APP_CC_HASHMIN ? kPhaseSendAll : kPhaseSendSource);
      a.source = o.source;
      a.count = static_cast<uint32_t>(count);
      a.frontier_in = fin;
      a.off = g->csr_off;
      a.dst = g->csr_dst;
      a.w = weighted ? g->csr_w : nullptr;
      a.outdeg = g->t.outdeg;
      a.value = w.value_u32;
      a.mail_in = min_;
      a.mail_out = mout;
      a.frontier_out = fout;
      a.ctr = c;
      a.ctr_clear = cc;
      IPG_HIP(push_dispatch(app, weighted, a, a.count, s));
    } else {
      IPG_HIP(fill_u32(w.sent, words, 0u, s));
      if (step == 0) {
        hipLaunchKernelGGL(minprop_init_kernel, dim3(gv), dim3(kBlock), 0, s, n, static_cast<int>(app), o.source,
                           w.value_u32, g->t.outdeg, 1, w.sent, c);
        IPG_HIP(hipGetLastError());
      } else {
        MinApplyArgs ap;
        ap.count = static_cast<uint32_t>(count);
        ap.frontier_in = fin;
        ap.outdeg = g->t.outdeg;
        ap.value = w.value_u32;
        ap.mail_in = min_;
        ap.sent = w.sent;
        ap.ctr = c;
        ap.ctr_clear = nullptr;
        hipLaunchKernelGGL(minprop_apply_kernel, dim3(grid_for(count, kBlock, 16384)), dim3(kBlock), 0, s, ap);
        IPG_HIP(hipGetLastError());
      }
      MinPullArgs pa;
      pa.off = g->csc_off;
      pa.src = g->csc_src;
      pa.w = weighted ? g->csc_w : nullptr;
      pa.outdeg = g->t.outdeg;
      pa.rb = g->t.pull_rb;
      pa.long_rows = g->t.long_rows;
      pa.nl = g->nl;
      pa.sent = w.sent;
      pa.value = w.value_u32;
      pa.mail_out = mout;
      pa.frontier_out = fout;
      pa.ctr = c;
      pa.ctr_clear = cc;
      IPG_HIP(pull_dispatch(app, weighted, pa, g->nl + g->nb, s));
    }
    IPG_HIP(tm.step(s, step));
    StepCounters h;
    IPG_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    if (st && step < st->trace_cap) {
      if (st->active) st->active[step] = step == 0 ? n : count;
      if (st->senders) st->senders[step] = h.senders;
      if (st->messages) st->messages[step] = h.messages;
      if (st->examined) st->examined[step] = h.examined;
      if (st->mode) st->mode[step] = static_cast<uint8_t>(mode);
    }
    tot_msgs += h.messages;
    tot_exam += h.examined;
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
    count = h.next_count;
    degsum = h.next_deg;
    std::swap(fin, fout);
    std::swap(min_, mout);
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
