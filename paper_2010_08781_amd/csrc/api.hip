// api.hip -- the ipg_run / ipg_read_values entry points, run workspace
// layout, superstep timing and the per-superstep exchange choice.
#include <cstring>

#include "common.h"
#include "engine.h"

namespace ipg {

size_t carve_run(Carver& c, uint32_t n, uint64_t e, ipg_app app, RunWs* w) {
  RunWs r{};
  const size_t nn = n ? n : 1;
  if (app == IPG_APP_PAGERANK) {
    r.value_f64 = c.take<double>(nn);
    r.f64_a = c.take<double>(nn);
    r.f64_b = c.take<double>(nn);
    r.partial = c.take<double>(chunks_cap(e));
    r.part_n = c.take<uint32_t>(nn);
    r.l1 = c.take<double>(kCtrSlots * 16);  // one 128-byte line per slot
    r.value_hot = c.take<double>(nn);
    r.pr_pieces = c.take<PrPiece>(kCtrSlots * piece_seg(e));
    r.pr_cnt = c.take<PrCntSlot>(2 * kCtrSlots);
    r.pr_rec = c.take<unsigned long long>(3 * static_cast<size_t>(kPrTraceCap));
  } else {
    r.value_u32 = c.take<uint32_t>(nn);
    r.value_u32_hot = c.take<uint32_t>(nn);
    r.mail_a = c.take<uint32_t>(nn);
    r.mail_b = c.take<uint32_t>(nn);
    r.fr_a = c.take<uint32_t>(static_cast<size_t>(kCtrSlots) * list_seg(static_cast<uint32_t>(nn)));
    r.fr_b = c.take<uint32_t>(static_cast<size_t>(kCtrSlots) * list_seg(static_cast<uint32_t>(nn)));
    r.outbox = c.take<uint32_t>(nn);
    r.sent = c.take<uint32_t>(nn / 64 * 2 + 2);
    r.gate = c.take<uint32_t>(1);
    r.lpre = c.take<uint32_t>(2 * (kCtrSlots + 1));
    r.late = c.take<uint32_t>(1);
    r.pieces = c.take<Piece>(kCtrSlots * piece_seg(e));
    r.ctl = c.take<DevCtl>(1);
  }
  r.ctr = c.take<CtrSlot>(2 * kCtrSlots);
  if (w) *w = r;
  return align_up(c.used, 256);
}

hipError_t pool_event(std::vector<hipEvent_t>* pool, size_t i, hipEvent_t* out) {
  while (pool->size() <= i) {
    hipEvent_t ev;
    // Entry 1 ends a run and is the one waited on: it keeps the system-scope
    // fence.  The others only take timestamps between launches, so they
    // skip the fence and the cache write-back and invalidation it brings
    // between two supersteps (about 1 us per PageRank superstep).
    const hipError_t e =
        hipEventCreateWithFlags(&ev, pool->size() == 1 ? hipEventDefault : hipEventDisableSystemFence);
    if (e != hipSuccess) return e;
    pool->push_back(ev);
  }
  *out = (*pool)[i];
  return hipSuccess;
}

hipError_t host_mirror(ipg_graph* g, HostMirror** host, HostMirror** dev) {
  if (!g->mirror) {
    void* p = nullptr;
    void* d = nullptr;
    hipError_t e = hipHostMalloc(&p, sizeof(HostMirror), hipHostMallocMapped);
    if (e != hipSuccess) return e;
    e = hipHostGetDevicePointer(&d, p, 0);
    if (e != hipSuccess) {
      (void)hipHostFree(p);
      return e;
    }
    std::memset(p, 0, sizeof(HostMirror));
    g->mirror = p;
    g->mirror_dev = d;
  }
  *host = static_cast<HostMirror*>(g->mirror);
  *dev = static_cast<HostMirror*>(g->mirror_dev);
  return hipSuccess;
}

hipError_t StepTimer::start(hipStream_t s) {
  hipEvent_t ev;
  hipError_t e = event(0, &ev);
  if (e != hipSuccess) return e;
  started_ = true;
  return hipEventRecord(ev, s);
}

hipError_t StepTimer::step(hipStream_t s, uint32_t k) {
  if (k >= cap_) return hipSuccess;
  hipEvent_t ev;
  hipError_t e = event(2 + k, &ev);
  if (e != hipSuccess) return e;
  if (k + 1 > nsteps_) nsteps_ = k + 1;
  return hipEventRecord(ev, s);
}

hipError_t StepTimer::mark(hipStream_t s) {
  hipEvent_t end;
  hipError_t e = event(1, &end);
  if (e != hipSuccess) return e;
  marked_ = true;
  return hipEventRecord(end, s);
}

hipError_t StepTimer::finish(hipStream_t s) {
  hipEvent_t end;
  hipError_t e = event(1, &end);
  if (e != hipSuccess) return e;
  if (!marked_ && (e = hipEventRecord(end, s)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(end)) != hipSuccess) return e;
  float ms = 0.f;
  if (started_ && (e = hipEventElapsedTime(&ms, (*pool_)[0], end)) != hipSuccess) return e;
  seconds_ = ms * 1e-3;
  hipEvent_t prev = (*pool_)[0];
  for (uint32_t k = 0; k < nsteps_ && k < cap_; ++k) {
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, prev, (*pool_)[2 + k])) != hipSuccess) return e;
    usec_[k] = t * 1e3f;
    prev = (*pool_)[2 + k];
  }
  // keep the events of up to kKeep supersteps for later runs
  constexpr size_t kKeep = 2 + 1024;
  while (pool_->size() > kKeep) {
    (void)hipEventDestroy(pool_->back());
    pool_->pop_back();
  }
  return hipSuccess;
}

ipg_mode heuristic_mode(const ModeQuery& q, uint32_t div) {
  return static_cast<ipg_mode>(heuristic_pick(q.e, q.frontier, q.frontier_deg, div));
}

}  // namespace ipg

using namespace ipg;

extern "C" size_t ipg_run_workspace_bytes(uint32_t num_vertices, uint64_t num_edges, ipg_app app) {
  Carver c(nullptr);
  return carve_run(c, num_vertices, num_edges, app, nullptr);
}

extern "C" ipg_status ipg_run(ipg_graph* g, ipg_app app, ipg_combiner combiner, uint32_t max_supersteps,
                              const ipg_run_opts* opts, void* ws, size_t ws_bytes, void* hip_stream,
                              ipg_run_stats* st) {
  if (!g) return fail(IPG_EINVAL, "ipg_run: graph is NULL");
  const bool ok_pair = (app == IPG_APP_PAGERANK && combiner == IPG_COMBINE_SUM) ||
                       (app == IPG_APP_CC_HASHMIN && combiner == IPG_COMBINE_MIN) ||
                       (app == IPG_APP_SSSP && combiner == IPG_COMBINE_MIN);
  if (!ok_pair) return fail(IPG_EUNSUPPORTED, "ipg_run: (app, combiner) must be (PAGERANK, SUM), (CC, MIN) or (SSSP, MIN)");
  ipg_run_opts o{0, 0.0, IPG_MODE_AUTO, 0, nullptr, nullptr, 0, 0.0, nullptr};
  if (opts) o = *opts;
  if (o.mode != IPG_MODE_AUTO && o.mode != IPG_MODE_PUSH && o.mode != IPG_MODE_PULL)
    return fail(IPG_EINVAL, "ipg_run: unknown mode");
  if (app == IPG_APP_SSSP && o.source >= g->n) return fail(IPG_EINVAL, "ipg_run: SSSP source >= N");
  if ((o.flags & IPG_RUN_GRAPH) && app != IPG_APP_PAGERANK)
    return fail(IPG_EUNSUPPORTED, "ipg_run: IPG_RUN_GRAPH applies to PageRank only");
  if (o.num_parts && app != IPG_APP_PAGERANK)
    return fail(IPG_EUNSUPPORTED, "ipg_run: part_offsets apply to PageRank only");
  if (o.num_parts && !o.part_offsets) return fail(IPG_EINVAL, "ipg_run: num_parts without part_offsets");
  if ((o.flags & IPG_RUN_ENQUEUE) && (app != IPG_APP_PAGERANK || o.tolerance != 0.0 || (o.flags & IPG_RUN_GRAPH)))
    return fail(IPG_EUNSUPPORTED, "ipg_run: IPG_RUN_ENQUEUE applies to fixed-length PageRank without IPG_RUN_GRAPH");
  if (o.tolerance != 0.0) {
    if (app != IPG_APP_PAGERANK) return fail(IPG_EUNSUPPORTED, "ipg_run: a tolerance applies to PageRank only");
    if (!(o.tolerance > 0.0)) return fail(IPG_EINVAL, "ipg_run: tolerance must be > 0");
    if (max_supersteps == 0) return fail(IPG_EINVAL, "ipg_run: a tolerance needs max_supersteps >= 1 (cap on updates)");
    if (o.flags & IPG_RUN_GRAPH) return fail(IPG_EUNSUPPORTED, "ipg_run: a tolerance cannot be combined with IPG_RUN_GRAPH");
  }
  const size_t need = ipg_run_workspace_bytes(g->n, g->e, app);
  if (!ws || ws_bytes < need)
    return fail(IPG_EWORKSPACE, "ipg_run: run workspace needs " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(IPG_EWORKSPACE, "ipg_run: workspace must be 256-byte aligned");
  int dev = -1;
  IPG_HIP(hipGetDevice(&dev));
  if (dev != g->device) return fail(IPG_EINVAL, "ipg_run: current device differs from the graph's device");

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Carver c(ws);
  RunWs w;
  carve_run(c, g->n, g->e, app, &w);
  g->has_values = 0;
  const bool enqueue = o.flags & IPG_RUN_ENQUEUE;
  StepTimer tm(&g->events, st && !enqueue ? st->usec : nullptr, st && !enqueue ? st->trace_cap : 0);
  ipg_status rc;
  if (app == IPG_APP_PAGERANK) rc = run_pagerank(g, max_supersteps, o, w, ws, s, tm, st);
  else rc = run_minprop(g, app, max_supersteps, o, w, s, tm, st);
  if (st && !enqueue) st->seconds = tm.seconds();
  if (rc == IPG_OK || rc == IPG_NOT_CONVERGED) {
    g->has_values = 1;
    g->last_app = app;
    g->last_values = app == IPG_APP_PAGERANK ? static_cast<const void*>(w.value_f64) : static_cast<const void*>(w.value_u32);
    if (rc == IPG_OK) set_error("");
  }
  return rc;
}

extern "C" ipg_status ipg_read_values(const ipg_graph* g, void* dst, size_t dst_bytes, int dst_is_device,
                                      void* hip_stream) {
  if (!g || !dst) return fail(IPG_EINVAL, "ipg_read_values: NULL argument");
  if (!g->has_values) return fail(IPG_EINVAL, "ipg_read_values: no completed run on this graph");
  const size_t elt = g->last_app == IPG_APP_PAGERANK ? sizeof(double) : sizeof(uint32_t);
  const size_t bytes = elt * g->n;
  if (dst_bytes < bytes) return fail(IPG_EINVAL, "ipg_read_values: destination needs " + std::to_string(bytes) + " bytes");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  IPG_HIP(hipMemcpyAsync(dst, g->last_values, bytes, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  if (!dst_is_device) IPG_HIP(hipStreamSynchronize(s));  // a device copy is ordered on the stream
  return IPG_OK;
}
