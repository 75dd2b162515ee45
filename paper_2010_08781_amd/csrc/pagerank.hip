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

// First launch of a pull superstep: the partial sum of every chunk of
// kPullTile in-edges of a long row (grid-stride over chunks).  Loads are
// unconditional (index clamped into the chunk) so that all of a thread's
// gathers are in flight together; out-of-range lanes are masked.
__global__ __launch_bounds__(kBlock) void pr_chunk_kernel(PrPullArgs a) {
  __shared__ double red[kWavesPerBlock];
  const uint32_t tid = threadIdx.x;
  const int32_t* src = a.t.src;
  for (uint32_t c = blockIdx.x; c < a.t.nc; c += gridDim.x) {
    const ChunkRef r = chunk_ref(a.t, c);
    constexpr int kPer = kPullTile / kBlock;
    int32_t u[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      uint64_t e = r.beg + tid + k * kBlock;
      e = e < r.end ? e : r.end - 1;
      u[k] = __builtin_nontemporal_load(src + e);
    }
    double x[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) x[k] = a.contrib_in[u[k]];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (r.beg + tid + k * kBlock < r.end) s += x[k];
    s = block_sum(s, red);
    if (tid == 0) a.partial[c] = s;
  }
}

// Second launch of a pull superstep (grid-stride over nl + nb work items):
//  * item l < nl: finish long row l -- add its chunk partials in chunk order
//    (a fixed order, so results are bitwise reproducible);
//  * item nl + k: row-group k.  Its in-edges (fewer than 2*kPullTile) are
//    streamed from the CSC with coalesced loads, their sources' outboxes
//    gathered into LDS, then each row is reduced from LDS by G lanes (G from
//    the group's row count so that the 256 lanes stay busy).
__global__ __launch_bounds__(kBlock) void pr_pull_kernel(PrPullArgs a) {
  __shared__ double tile[2 * kPullTile];
  __shared__ double red[kWavesPerBlock];
  const uint32_t tid = threadIdx.x;
  const int32_t* src = a.t.src;
  const uint64_t* off = a.t.off;
  const uint32_t items = a.t.nl + a.t.nb;
  for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
    if (item < a.t.nl) {
      const uint32_t f = a.t.lr_first[item], nch = a.t.lr_first[item + 1] - f;
      double x = 0.0;
      for (uint32_t i = tid; i < nch; i += kBlock) x += a.partial[f + i];
      x = block_sum(x, red);
      if (tid == 0) pr_finish(a, a.t.long_rows[item], x);
      continue;
    }
    uint32_t r0, r1;
    group_rows(a.t, item - a.t.nl, r0, r1);
    if (r0 >= r1) continue;  // block-uniform
    const uint64_t e0 = off[r0];
    uint32_t span = static_cast<uint32_t>(off[r1] - e0);
    if (span > 2 * kPullTile) span = 2 * kPullTile;  // only reachable with inconsistent offsets
    for (uint32_t base = 0; base < span; base += 4 * kBlock) {  // block-uniform, at most 2 passes
      int32_t u[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t i = base + tid + k * kBlock;
        u[k] = __builtin_nontemporal_load(src + e0 + (i < span ? i : span - 1));
      }
      double x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = a.contrib_in[u[k]];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t i = base + tid + k * kBlock;
        if (i < span) tile[i] = x[k];
      }
    }
    __syncthreads();
    const uint32_t nrows = r1 - r0;
    uint32_t G = kWave;
    while (G > 1 && G * nrows > kBlock) G >>= 1;
    const uint32_t groups = kBlock / G, gi = tid / G, li = tid % G;
    for (uint32_t rb = 0; rb < nrows; rb += groups) {
      const uint32_t row = rb + gi;
      double s = 0.0;
      if (row < nrows) {
        const uint32_t v = r0 + row;
        uint32_t lo = static_cast<uint32_t>(off[v] - e0), hi = static_cast<uint32_t>(off[v + 1] - e0);
        if (hi > span) hi = span;
        for (uint32_t j = lo + li; j < hi; j += G) s += tile[j];
      }
      for (uint32_t o = G >> 1; o >= 1; o >>= 1) s += __shfl_xor(s, static_cast<int>(o));
      if (li == 0 && row < nrows) pr_finish(a, r0 + row, s);
    }
    __syncthreads();  // the tile is reused by the next item
  }
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
      if (g->nc) {
        hipLaunchKernelGGL(pr_chunk_kernel, dim3(std::min(g->nc, kExchangeGrid)), dim3(kBlock), 0, s, a);
        IPG_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(pr_pull_kernel, dim3(std::min(g->nl + g->nb, kExchangeGrid)), dim3(kBlock), 0, s, a);
      IPG_HIP(hipGetLastError());
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
    }
  }
  return IPG_OK;
}

}  // namespace ipg
