// pagerank.hip -- PageRank (Fig. 8) on the superstep engine, FP64.
//
// Superstep 0 sets every rank to 1/N; superstep s >= 1 sets
//   rank(v) = 0.15/N + 0.85 * (sum of the messages v received),
// and while s < T every vertex broadcasts rank / out-degree (a vertex
// without out-edges reaches nobody).  At s = T all vertices halt.  Messages
// are combined by '+=' (the sum combiner of Fig. 8).
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

#include "common.h"
#include "engine.h"
#include "scatter.h"

namespace ipg {

struct PrPullArgs {
  PullTiling t;
  const uint32_t* outdeg;
  const double* contrib_in;
  double* contrib_out;
  double* value;
  double* partial;        // per long-row chunk
  double ratio;           // 0.15 / N
  int last;               // superstep == T: store the rank, no broadcast
};

__device__ __forceinline__ void pr_finish(const PrPullArgs& a, uint32_t v, double sum) {
  const double rank = a.ratio + 0.85 * sum;
  if (a.last) {
    a.value[v] = rank;
  } else {
    const uint32_t d = a.outdeg[v];
    a.contrib_out[v] = d ? rank / static_cast<double>(d) : 0.0;
  }
}

// Sum over the workgroup in a fixed order; every thread gets the result.
__device__ __forceinline__ double block_sum(double s, double* red) {
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// Pull superstep, first launch.  Every wavefront works through its own pull
// items (grid-stride over wavefronts), with its own LDS tile and no
// workgroup barrier, so 32 items per CU are in flight.  An item needs one
// metadata load; then all of its independent loads are issued together --
// the CSC sources (non-temporal; indices clamped into the item so no lane
// branches), the row offsets and out-degrees -- and the outbox gathers
// follow in one more round trip.
//  * row item: the gathered outboxes are staged in LDS and each row is
//    summed by G lanes (G from the item's row count), then finished here;
//  * long-row chunk: a fixed-order wavefront sum stored as the chunk's
//    partial (added up by the second launch).
__global__ __launch_bounds__(kBlock) void pr_items_kernel(PrPullArgs a) {
  constexpr int kPer = kWaveTile / kWave;
  constexpr int kRowPer = (kItemRows + kWave) / kWave;
  __shared__ double s_tile[kWavesPerBlock][kWaveTile];
  __shared__ uint32_t s_off[kWavesPerBlock][kItemRows + 1];
  __shared__ uint32_t s_deg[kWavesPerBlock][kItemRows];
  const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
  double* tile = s_tile[wv];
  uint32_t* soff = s_off[wv];
  uint32_t* sdeg = s_deg[wv];
  const int32_t* src = a.t.src;
  const uint64_t* off = a.t.off;
  const uint32_t nw = gridDim.x * kWavesPerBlock;
  for (uint32_t item = blockIdx.x * kWavesPerBlock + wv; item < a.t.ni; item += nw) {
    const PullItem it = a.t.items[item];
    const bool chunk = it.slot != kNoSlot;
    const uint32_t ne = it.ne < kWaveTile ? it.ne : kWaveTile;  // ne > kWaveTile only with bad offsets
    const uint32_t nrows = chunk ? 0 : it.r1 - it.r0;
    int32_t u[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = lane + k * kWave;
      u[k] = ne ? __builtin_nontemporal_load(src + it.e0 + (i < ne ? i : ne - 1)) : 0;
    }
    if (!chunk) {
#pragma unroll
      for (int k = 0; k < kRowPer; ++k) {
        const uint32_t r = lane + k * kWave;
        if (r <= nrows) soff[r] = static_cast<uint32_t>(off[it.r0 + r] - it.e0);
        if (r < nrows) sdeg[r] = a.outdeg[it.r0 + r];
      }
    }
    double x[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) x[k] = ne ? a.contrib_in[u[k]] : 0.0;
    if (chunk) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kPer; ++k)
        if (lane + k * kWave < ne) s += x[k];
      s = wave_sum(s);
      if (lane == 0) a.partial[it.slot] = s;
      continue;
    }
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
        const double rank = a.ratio + 0.85 * s;
        const uint32_t v = it.r0 + row;
        if (a.last) {
          a.value[v] = rank;
        } else {
          const uint32_t d = sdeg[row];
          a.contrib_out[v] = d ? rank / static_cast<double>(d) : 0.0;
        }
      }
    }
    wave_lds_sync();  // the tile is rewritten by the next item
  }
}

// Pull superstep, second launch: each long row adds its chunk partials in
// chunk order (one wavefront per row; a fixed order, so results are
// bitwise reproducible).
__global__ __launch_bounds__(kBlock) void pr_longrow_kernel(PrPullArgs a) {
  const uint32_t l = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (l >= a.t.nl) return;  // wave-uniform
  const uint32_t f = a.t.lr_first[l], nch = a.t.lr_first[l + 1] - f;
  double s = 0.0;
  for (uint32_t i = lane_id(); i < nch; i += kWave) s += a.partial[f + i];
  s = wave_sum(s);
  if (lane_id() == 0) pr_finish(a, a.t.long_rows[l], s);
}

// Superstep 0 of the pull form: rank 1/N, outbox 1/N/outdeg.
__global__ void pr_pull_init_kernel(uint32_t n, const uint32_t* outdeg, double init, double* contrib, double* value,
                                    int last) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    if (last) {
      value[v] = init;
    } else {
      const uint32_t d = outdeg[v];
      contrib[v] = d ? init / static_cast<double>(d) : 0.0;
    }
  }
}

struct PrPushArgs {
  uint32_t n;
  const uint64_t* off;   // CSR offsets
  const int32_t* dst;    // CSR destinations
  double* mail_in;       // consumed and reset to 0.0
  double* mail_out;      // atomically accumulated
  double* value;
  double ratio, init;
  int first, last;
};

// Fused compute + push for one superstep: every vertex consumes its mailbox,
// updates its rank and (unless last) adds rank/outdeg into each
// out-neighbour's next mailbox.
__global__ __launch_bounds__(kBlock) void pr_push_kernel(PrPushArgs a) {
  const uint64_t v = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
  bool has = false;
  uint64_t beg = 0, end = 0;
  double c = 0.0;
  if (v < a.n) {
    double rank;
    if (a.first) {
      rank = a.init;
    } else {
      const double m = a.mail_in[v];
      a.mail_in[v] = 0.0;
      rank = a.ratio + 0.85 * m;
    }
    if (a.last) {
      a.value[v] = rank;
    } else {
      beg = a.off[v];
      end = a.off[v + 1];
      has = end > beg;
      if (has) c = rank / static_cast<double>(end - beg);
    }
  }
  double* mail = a.mail_out;
  const int32_t* dst = a.dst;
  twc_scatter(has, beg, end, c, [&](uint64_t e, double p) { unsafeAtomicAdd(mail + dst[e], p); });
}

// ------------------------------------------------------------------ host --

ipg_status run_pagerank(ipg_graph* g, uint32_t T, ipg_mode mode, const RunWs& w, hipStream_t s, StepTimer& tm,
                        ipg_run_stats* st) {
  const uint32_t n = g->n;
  const double ratio = 0.15 / static_cast<double>(n);
  const double init = 1.0 / static_cast<double>(n);
  const bool push = (mode == IPG_MODE_PUSH);
  const uint32_t gv = grid_for(n, kBlock, 16384);
  if (!push) {
    IPG_HIP(tm.start(s));
    hipLaunchKernelGGL(pr_pull_init_kernel, dim3(gv), dim3(kBlock), 0, s, n, g->t.outdeg, init, w.f64_a,
                       w.value_f64, T == 0);
    IPG_HIP(hipGetLastError());
    IPG_HIP(tm.step(s, 0));
    PrPullArgs a;
    a.t = pull_tiling(g);
    a.outdeg = g->t.outdeg;
    a.value = w.value_f64;
    a.partial = w.partial;
    a.ratio = ratio;
    for (uint32_t step = 1; step <= T; ++step) {
      a.contrib_in = (step & 1) ? w.f64_a : w.f64_b;
      a.contrib_out = (step & 1) ? w.f64_b : w.f64_a;
      a.last = step == T;
      if (g->ni) {
        hipLaunchKernelGGL(pr_items_kernel, dim3(std::min(g->ni, kPullGrid)), dim3(kBlock), 0, s, a);
        IPG_HIP(hipGetLastError());
      }
      if (g->nl) {
        hipLaunchKernelGGL(pr_longrow_kernel, dim3((g->nl + kWavesPerBlock - 1) / kWavesPerBlock), dim3(kBlock), 0, s,
                           a);
        IPG_HIP(hipGetLastError());
      }
      IPG_HIP(tm.step(s, step));
    }
  } else {
    IPG_HIP(fill_f64(w.f64_a, n, 0.0, s));
    IPG_HIP(fill_f64(w.f64_b, n, 0.0, s));
    IPG_HIP(tm.start(s));
    PrPushArgs a;
    a.n = n;
    a.off = g->csr_off;
    a.dst = g->csr_dst;
    a.value = w.value_f64;
    a.ratio = ratio;
    a.init = init;
    const uint32_t grid = grid_for(n, kBlock, 0xFFFFFFFFu);
    for (uint32_t step = 0; step <= T; ++step) {
      a.mail_in = (step & 1) ? w.f64_b : w.f64_a;
      a.mail_out = (step & 1) ? w.f64_a : w.f64_b;
      a.first = step == 0;
      a.last = step == T;
      hipLaunchKernelGGL(pr_push_kernel, dim3(grid), dim3(kBlock), 0, s, a);
      IPG_HIP(hipGetLastError());
      IPG_HIP(tm.step(s, step));
    }
  }
  IPG_HIP(tm.finish(s));
  // The PageRank trace is fixed by Fig. 8: every vertex runs in every
  // superstep and broadcasts while s < T.
  if (st) {
    const uint32_t steps = T + 1;
    st->supersteps = steps;
    st->halted = 1;
    st->edges_traversed = static_cast<uint64_t>(T) * g->e;
    st->edges_examined = static_cast<uint64_t>(T) * g->e;
    for (uint32_t k = 0; k < steps && k < st->trace_cap; ++k) {
      if (st->active) st->active[k] = n;
      if (st->senders) st->senders[k] = k < T ? n : 0;
      if (st->messages) st->messages[k] = k < T ? g->e : 0;
      if (st->examined) st->examined[k] = k < T ? g->e : 0;
      if (st->mode) st->mode[k] = push ? IPG_MODE_PUSH : IPG_MODE_PULL;
      if (st->frontier_deg) st->frontier_deg[k] = g->e;
    }
  }
  return IPG_OK;
}

}  // namespace ipg
