// engine.h -- host-side superstep driver shared by the application sources.
#pragma once

#include <vector>

#include "common.h"

namespace ipg {

// Run workspace, carved from the caller's device buffer.
struct RunWs {
  // PageRank
  double* value_f64;  // [n] ranks after the last update
  double* f64_a;      // [n] outbox (pull) or mailbox (push), ping
  double* f64_b;      // [n] pong
  // CC / SSSP
  uint32_t* value_u32;  // [n] labels or distances
  uint32_t* mail_a;     // [n] one-slot min mailboxes, ping (INF = empty)
  uint32_t* mail_b;     // [n] pong
  uint32_t* fr_a;       // [n] frontier list, ping
  uint32_t* fr_b;       // [n] pong
  uint32_t* sent;       // [n/32+1] senders of the current superstep (pull form)
  // both
  StepCounters* ctr;    // [2] per-superstep counters (slot s & 1)
};

size_t carve_run(Carver& c, uint32_t n, uint64_t e, ipg_app app, RunWs* w);

// HIP-event timing of the superstep loop (first launch -> halt decision) and,
// when the caller asked for it, of every superstep.
class StepTimer {
 public:
  StepTimer(float* usec, uint32_t cap) : usec_(usec), cap_(usec ? cap : 0) {}
  ~StepTimer();
  hipError_t start(hipStream_t s);
  hipError_t step(hipStream_t s, uint32_t k);  // end of superstep k
  hipError_t finish(hipStream_t s);            // synchronises
  double seconds() const { return seconds_; }

 private:
  float* usec_;
  uint32_t cap_;
  hipEvent_t start_ = nullptr, end_ = nullptr;
  std::vector<hipEvent_t> steps_;
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
ipg_mode choose_mode(ipg_mode requested, const ModeQuery& q);

ipg_status run_pagerank(ipg_graph* g, uint32_t T, ipg_mode mode, const RunWs& w, hipStream_t s, StepTimer& tm,
                        ipg_run_stats* st);
ipg_status run_minprop(ipg_graph* g, ipg_app app, uint32_t cap, const ipg_run_opts& o, const RunWs& w,
                       hipStream_t s, StepTimer& tm, ipg_run_stats* st);

}  // namespace ipg
