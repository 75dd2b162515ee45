/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, obviously-correct bulk-synchronous Pregel that the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg use to
 * check and time the GPU library.  Nothing in the product path may load it,
 * and it shares no code with the GPU path.
 *
 * What it executes (iPregel, Capelli et al., Parallel Computing 2019):
 *   - Supersteps made of local computation, communication and a global
 *     synchronisation; a message sent in superstep s is visible only in
 *     superstep s+1 (Section 4.2, Fig. 3).
 *   - Naive vertex selection (Section 4.3.1): in every superstep every vertex
 *     is examined and runs compute if (1) it is the first superstep, or
 *     (2) it has not voted to halt, or (3) it received a message.  A halted
 *     vertex that receives a message runs again.
 *   - One-slot mailboxes combined on arrival with the application's combiner
 *     (Section 4.3.3): '+=' for PageRank (Fig. 8), 'min' (Fig. 5) for
 *     connected components (Fig. 9) and SSSP (Fig. 10).
 *   - Push delivery: vertices run in ascending id order and a broadcast visits
 *     the out-edges in CSR order (a broadcast reaches every out-neighbour,
 *     Section 3).
 *   - Termination when every vertex has voted to halt and no message is
 *     pending (the Pregel rule the paper quotes in Section 8.3).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - PageRank: initial value 1/N, ratio 0.15/N (Pregel's form, Fig. 12),
 *     damping 0.85 as printed in Fig. 8; `threshold` is the superstep number at
 *     which vertices stop broadcasting and halt (10 in Fig. 8), so the result
 *     is the rank after `threshold` updates and `threshold`+1 supersteps run.
 *     A vertex without out-edges broadcasts to nobody: its mass is not
 *     redistributed.
 *   - SSSP: INF = 0xFFFFFFFF; on a weighted graph the sender's message to
 *     out-neighbour x is value + w(v, x) (Pregel's Bellman-Ford, cited in
 *     Section 6.3); unweighted uses + 1 as printed in Fig. 10.  A message
 *     that would reach INF is reported as an overflow error.
 *   - CC: labels start at the vertex id (Fig. 9).  On a directed graph the
 *     label is the minimum id among vertices with a path *to* the vertex.
 *   - Self-loops and duplicate edges are ordinary edges: a duplicate delivers
 *     two messages, a self-loop delivers to the sender itself.
 *
 * Per-superstep trace: trace[3*s+0] = vertices that ran compute,
 * trace[3*s+1] = vertices that broadcast, trace[3*s+2] = messages delivered
 * (sum of the senders' out-degrees).
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math; IEEE round-to-nearest).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_APP_PAGERANK 0
#define ORC_APP_CC 1
#define ORC_APP_SSSP 2

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_EBADGRAPH (-2)
#define ORC_EOVERFLOW (-3)

#define ORC_INF 0xFFFFFFFFu

/* Check the CSR: off[0] == 0, off non-decreasing, every id in [0, n). */
static int orc_check_graph(uint32_t n, const uint64_t* off, const int32_t* adj) {
  if (off[0] != 0) return 0;
  for (uint32_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) return 0;
  for (uint64_t e = 0; e < off[n]; ++e)
    if (adj[e] < 0 || (uint32_t)adj[e] >= n) return 0;
  return 1;
}

/* ---------------------------------------------------------------------- */
/* PageRank, Fig. 8: messages are doubles combined with '+='.             */

typedef struct {
  double* box;
  uint8_t* has;
} orc_fbox;

static void orc_send_sum(orc_fbox* next, uint32_t w, double m) {
  if (next->has[w]) {
    next->box[w] += m; /* the sum combiner of Fig. 8 */
  } else {
    next->box[w] = m;
    next->has[w] = 1;
  }
}

static int orc_pagerank(uint32_t n, const uint64_t* off, const int32_t* adj, uint32_t threshold,
                        uint32_t max_supersteps, double* value, uint64_t* trace, uint32_t trace_cap,
                        uint32_t* supersteps_out, double* deltas) {
  const double initial_value = 1.0 / (double)n;
  const double ratio = 0.15 / (double)n;
  uint8_t* halted = calloc(n ? n : 1, 1);
  orc_fbox in = {calloc(n ? n : 1, sizeof(double)), calloc(n ? n : 1, 1)};
  orc_fbox next = {calloc(n ? n : 1, sizeof(double)), calloc(n ? n : 1, 1)};
  int status = ORC_OK;
  uint32_t s = 0;
  for (;; ++s) {
    uint64_t active = 0, senders = 0, messages = 0;
    double l1 = 0.0; /* L1 change of this update, summed in ascending vertex order */
    for (uint32_t v = 0; v < n; ++v) {
      if (!(s == 0 || !halted[v] || in.has[v])) continue;
      halted[v] = 0;
      ++active;
      /* compute(v), Fig. 8 */
      if (s == 0) {
        value[v] = initial_value;
      } else {
        double sum = 0.0;
        if (in.has[v]) sum += in.box[v]; /* at most one combined message */
        const double old = value[v];
        value[v] = ratio + 0.85 * sum;
        if (deltas) l1 += fabs(value[v] - old);
      }
      if (s < threshold) {
        /* broadcast(value / out_neighbour_count) */
        ++senders;
        uint64_t deg = off[v + 1] - off[v];
        if (deg > 0) {
          double m = value[v] / (double)deg;
          for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
            orc_send_sum(&next, (uint32_t)adj[e], m);
            ++messages;
          }
        }
      } else {
        halted[v] = 1; /* vote to halt */
      }
    }
    if (s < trace_cap) {
      trace[3 * (uint64_t)s + 0] = active;
      trace[3 * (uint64_t)s + 1] = senders;
      trace[3 * (uint64_t)s + 2] = messages;
    }
    if (deltas) deltas[s] = l1;
    /* global synchronisation: next becomes the inbox, next is emptied */
    orc_fbox t = in;
    in = next;
    next = t;
    memset(next.has, 0, n ? n : 1);
    int done = 1;
    for (uint32_t v = 0; v < n && done; ++v)
      if (!halted[v] || in.has[v]) done = 0;
    if (done) break;
    if (max_supersteps && s + 1 >= max_supersteps) {
      status = ORC_NOT_CONVERGED;
      break;
    }
  }
  *supersteps_out = s + 1;
  free(halted);
  free(in.box);
  free(in.has);
  free(next.box);
  free(next.has);
  return status;
}

/* ---------------------------------------------------------------------- */
/* CC (Fig. 9) and SSSP (Fig. 10): uint32 messages combined with min      */
/* (Fig. 5).                                                              */

typedef struct {
  uint32_t* box;
  uint8_t* has;
} orc_ubox;

static void orc_send_min(orc_ubox* next, uint32_t w, uint32_t m) {
  if (next->has[w]) {
    if (next->box[w] > m) next->box[w] = m; /* the min combiner of Fig. 5 */
  } else {
    next->box[w] = m;
    next->has[w] = 1;
  }
}

/* broadcast for the min applications: value (CC), value + 1 or value + w
 * (SSSP) to every out-neighbour.  Returns 0 on overflow. */
static int orc_broadcast_min(int app, uint32_t v, uint32_t val, const uint64_t* off, const int32_t* adj,
                             const uint32_t* w, orc_ubox* next, uint64_t* messages) {
  for (uint64_t e = off[v]; e < off[v + 1]; ++e) {
    uint64_t m = val;
    if (app == ORC_APP_SSSP) m += w ? (uint64_t)w[e] : 1u;
    if (m >= ORC_INF) return 0;
    orc_send_min(next, (uint32_t)adj[e], (uint32_t)m);
    ++*messages;
  }
  return 1;
}

static int orc_minprop(int app, uint32_t n, const uint64_t* off, const int32_t* adj, const uint32_t* w,
                       uint32_t source, uint32_t max_supersteps, uint32_t* value, uint64_t* trace,
                       uint32_t trace_cap, uint32_t* supersteps_out) {
  uint8_t* halted = calloc(n ? n : 1, 1);
  orc_ubox in = {calloc(n ? n : 1, sizeof(uint32_t)), calloc(n ? n : 1, 1)};
  orc_ubox next = {calloc(n ? n : 1, sizeof(uint32_t)), calloc(n ? n : 1, 1)};
  int status = ORC_OK;
  uint32_t s = 0;
  for (;; ++s) {
    uint64_t active = 0, senders = 0, messages = 0;
    for (uint32_t v = 0; v < n; ++v) {
      if (!(s == 0 || !halted[v] || in.has[v])) continue;
      halted[v] = 0;
      ++active;
      int send = 0;
      if (app == ORC_APP_CC) {
        /* Fig. 9 */
        if (s == 0) {
          value[v] = v;
          send = 1;
        } else {
          uint32_t old_value = value[v];
          if (in.has[v] && in.box[v] < value[v]) value[v] = in.box[v];
          if (value[v] < old_value) send = 1;
        }
      } else {
        /* Fig. 10 */
        if (s == 0) {
          if (v == source) {
            value[v] = 0;
            send = 1;
          } else {
            value[v] = ORC_INF;
          }
        } else {
          uint32_t mindist = ORC_INF;
          if (in.has[v] && in.box[v] < mindist) mindist = in.box[v];
          if (mindist < value[v]) {
            value[v] = mindist;
            send = 1;
          }
        }
      }
      if (send) {
        ++senders;
        if (!orc_broadcast_min(app, v, value[v], off, adj, w, &next, &messages)) {
          status = ORC_EOVERFLOW;
          goto out;
        }
      }
      halted[v] = 1; /* both applications vote to halt after every compute */
    }
    if (s < trace_cap) {
      trace[3 * (uint64_t)s + 0] = active;
      trace[3 * (uint64_t)s + 1] = senders;
      trace[3 * (uint64_t)s + 2] = messages;
    }
    orc_ubox t = in;
    in = next;
    next = t;
    memset(next.has, 0, n ? n : 1);
    int done = 1;
    for (uint32_t v = 0; v < n && done; ++v)
      if (!halted[v] || in.has[v]) done = 0;
    if (done) break;
    if (max_supersteps && s + 1 >= max_supersteps) {
      status = ORC_NOT_CONVERGED;
      break;
    }
  }
out:
  *supersteps_out = s + 1;
  free(halted);
  free(in.box);
  free(in.has);
  free(next.box);
  free(next.has);
  return status;
}

/*
 * Entry point.
 *   app: 0 PageRank, 1 hash-min CC, 2 SSSP.
 *   n, off[n+1], adj[off[n]]: CSR out-adjacency (host memory).
 *   w: per-edge weights aligned with adj, or NULL (unit weights; SSSP only).
 *   source: SSSP source vertex.
 *   param: PageRank -> the superstep at which broadcasting stops (number of
 *          rank updates); CC/SSSP -> cap on supersteps executed, 0 = none.
 *   values: n doubles (PageRank) or n uint32 (CC/SSSP).
 *   trace: trace_cap rows of 3 uint64 (may be NULL when trace_cap == 0).
 * Returns ORC_OK, ORC_NOT_CONVERGED (values valid) or a negative error.
 */
int orc_run(int app, uint32_t n, const uint64_t* off, const int32_t* adj, const uint32_t* w, uint32_t source,
            uint32_t param, void* values, uint64_t* trace, uint32_t trace_cap, uint32_t* supersteps) {
  *supersteps = 0;
  if (!off || (!adj && n && off[n]) || !values) return ORC_EINVAL;
  if (!orc_check_graph(n, off, adj)) return ORC_EBADGRAPH;
  if (app == ORC_APP_PAGERANK) {
    if (n == 0) return ORC_EINVAL;
    return orc_pagerank(n, off, adj, param, 0, (double*)values, trace, trace_cap, supersteps, NULL);
  }
  if (app == ORC_APP_CC) return orc_minprop(app, n, off, adj, NULL, 0, param, (uint32_t*)values, trace, trace_cap, supersteps);
  if (app == ORC_APP_SSSP) {
    if (source >= n) return ORC_EINVAL;
    return orc_minprop(app, n, off, adj, w, source, param, (uint32_t*)values, trace, trace_cap, supersteps);
  }
  return ORC_EINVAL;
}

/*
 * PageRank run to convergence (an extension the paper points to in Section
 * 6.1: real PageRank stops once the ranks settle rather than after a fixed
 * number of iterations).  Runs Fig. 8 for `threshold` updates and stores in
 * deltas[s] (s = 1..threshold) the L1 change of update s, the sum over all
 * vertices, in ascending id order, of |rank after s - rank after s-1|;
 * deltas[0] = 0.  The caller picks the first update whose change is below
 * its tolerance.
 */
int orc_pagerank_deltas(uint32_t n, const uint64_t* off, const int32_t* adj, uint32_t threshold, double* values,
                        double* deltas) {
  uint32_t steps = 0;
  if (!off || (!adj && n && off[n]) || !values || !deltas || n == 0) return ORC_EINVAL;
  if (!orc_check_graph(n, off, adj)) return ORC_EBADGRAPH;
  return orc_pagerank(n, off, adj, threshold, 0, values, NULL, 0, &steps, deltas);
}
