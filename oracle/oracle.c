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
 *   - PageRank: initial value 1/N, ratio (1 - d)/N with the damping d a run
 *     parameter (0.85 as printed in Fig. 8; the teleport term 0.15/N of
 *     Pregel's form, Fig. 12, is its d = 0.85 case: 1 - 0.85 is evaluated in
 *     double); `threshold` is the superstep number at
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
 * A second entry point, orc_run_pull, executes the same supersteps in the
 * pull form (Section 4.3.2): every vertex that broadcasts leaves one value in
 * its outbox, and every vertex combines the outboxes of its in-neighbours
 * (CSC) that broadcast.  Its vertex loop runs under an OpenMP static schedule
 * (the paper's parallelisation, Section 4.2: the vertices split evenly into
 * one contiguous block per thread, no work stealing; a chunk size may be
 * given instead, dealing fixed chunks round-robin); each vertex combines its
 * in-neighbours in CSC order whatever the thread count, so the output does
 * not depend on the number of threads, and with every CSC list sorted by
 * source it equals the push form's bit for bit (the same additions in the
 * same order).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math; IEEE
 * round-to-nearest).
 */
#include <math.h>
#include <omp.h>
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

static int orc_pagerank(uint32_t n, const uint64_t* off, const int32_t* adj, uint32_t threshold, double damping,
                        uint32_t max_supersteps, double* value, uint64_t* trace, uint32_t trace_cap,
                        uint32_t* supersteps_out, double* deltas) {
  const double initial_value = 1.0 / (double)n;
  const double ratio = (1.0 - damping) / (double)n;
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
        value[v] = ratio + damping * sum;
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
    return orc_pagerank(n, off, adj, param, 0.85, 0, (double*)values, trace, trace_cap, supersteps, NULL);
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
int orc_pagerank_deltas(uint32_t n, const uint64_t* off, const int32_t* adj, uint32_t threshold, double damping,
                        double* values, double* deltas) {
  uint32_t steps = 0;
  if (!off || (!adj && n && off[n]) || !values || !deltas || n == 0) return ORC_EINVAL;
  if (!(damping > 0.0 && damping <= 1.0)) return ORC_EINVAL;
  if (!orc_check_graph(n, off, adj)) return ORC_EBADGRAPH;
  return orc_pagerank(n, off, adj, threshold, damping, 0, values, NULL, 0, &steps, deltas);
}

/*
 * PageRank of Fig. 8 with damping d (0 < d <= 1): orc_run's PageRank with
 * ratio (1 - d)/N and the message sum weighted by d.
 */
int orc_pagerank_run(uint32_t n, const uint64_t* off, const int32_t* adj, uint32_t threshold, double damping,
                     double* values, uint64_t* trace, uint32_t trace_cap, uint32_t* supersteps) {
  *supersteps = 0;
  if (!off || (!adj && n && off[n]) || !values || n == 0) return ORC_EINVAL;
  if (!(damping > 0.0 && damping <= 1.0)) return ORC_EINVAL;
  if (!orc_check_graph(n, off, adj)) return ORC_EBADGRAPH;
  return orc_pagerank(n, off, adj, threshold, damping, 0, values, trace, trace_cap, supersteps, NULL);
}

/* ---------------------------------------------------------------------- */
/* Pull form under an OpenMP static schedule.                             */

/*
 * Supersteps of Figs. 8-10 in the pull form.  State per vertex: value,
 * halted, and the outbox of the previous superstep (the value it broadcast,
 * with a flag saying whether it broadcast at all).  Superstep s:
 *   1. every vertex v (static schedule) combines the outboxes of the
 *      in-neighbours that broadcast in s-1, in CSC order (its mailbox);
 *   2. v runs compute if s == 0, or it has not voted to halt, or its mailbox
 *      is non-empty (selection, Section 4.3.1), writing its own outbox for
 *      s+1 when it broadcasts;
 *   3. stop when every vertex has voted to halt and nobody sent a message.
 * The per-superstep trace counts are integer sums (thread-count independent).
 * An SSSP broadcast whose message to some out-neighbour would reach INF is an
 * overflow, detected when the vertex broadcasts (as in the push form).
 *   csr_off: out-degrees (and, with csr_w, the overflow check of weighted SSSP);
 *   csc_off/csc_src/csc_w: in-adjacency, weights aligned with csc_src.
 */
int orc_run_pull(int app, uint32_t n, const uint64_t* csr_off, const uint32_t* csr_w, const uint64_t* csc_off,
                 const int32_t* csc_src, const uint32_t* csc_w, uint32_t source, uint32_t param, double damping,
                 int threads, int chunk, void* values, uint64_t* trace, uint32_t trace_cap,
                 uint32_t* supersteps_out) {
  *supersteps_out = 0;
  if (!csr_off || !csc_off || (!csc_src && n && csc_off[n]) || !values) return ORC_EINVAL;
  if (app != ORC_APP_PAGERANK && app != ORC_APP_CC && app != ORC_APP_SSSP) return ORC_EINVAL;
  if (app == ORC_APP_PAGERANK && (n == 0 || !(damping > 0.0 && damping <= 1.0))) return ORC_EINVAL;
  if (app == ORC_APP_SSSP && source >= n) return ORC_EINVAL;
  if (!orc_check_graph(n, csc_off, csc_src) || csr_off[0] != 0 || csr_off[n] != csc_off[n]) return ORC_EBADGRAPH;
  for (uint32_t v = 0; v < n; ++v)
    if (csr_off[v + 1] < csr_off[v]) return ORC_EBADGRAPH;
  if (threads < 1) threads = 1;
  /* the default static schedule: one contiguous block of ceil(n / threads) vertices per thread */
  if (chunk < 1) chunk = (int)(((uint64_t)n + (uint64_t)threads - 1) / (uint64_t)threads);
  if (chunk < 1) chunk = 1;
  const size_t nn = n ? n : 1;
  const int pr = app == ORC_APP_PAGERANK;
  double* fval = pr ? (double*)values : NULL;
  uint32_t* uval = pr ? NULL : (uint32_t*)values;
  double* fout[2] = {pr ? malloc(nn * sizeof(double)) : NULL, pr ? malloc(nn * sizeof(double)) : NULL};
  uint32_t* uout[2] = {pr ? NULL : malloc(nn * sizeof(uint32_t)), pr ? NULL : malloc(nn * sizeof(uint32_t))};
  uint8_t* sent[2] = {calloc(nn, 1), calloc(nn, 1)};
  uint8_t* halted = calloc(nn, 1);
  const double initial_value = pr ? 1.0 / (double)n : 0.0;
  const double ratio = pr ? (1.0 - damping) / (double)n : 0.0;
  const uint32_t threshold = param, cap = pr ? 0 : param;
  int status = ORC_OK;
  uint32_t s = 0;
  for (;; ++s) {
    const uint8_t* sin = sent[(s + 1) & 1]; /* broadcasts of superstep s-1 */
    uint8_t* sout = sent[s & 1];
    const double* fin = pr ? fout[(s + 1) & 1] : NULL;
    double* fo = pr ? fout[s & 1] : NULL;
    const uint32_t* uin = pr ? NULL : uout[(s + 1) & 1];
    uint32_t* uo = pr ? NULL : uout[s & 1];
    unsigned long long active = 0, senders = 0, messages = 0, awake = 0, overflow = 0;
#pragma omp parallel for schedule(static, chunk) num_threads(threads) \
    reduction(+ : active, senders, messages, awake, overflow)
    for (int64_t iv = 0; iv < (int64_t)n; ++iv) {
      const uint32_t v = (uint32_t)iv;
      /* 1. the mailbox: the in-neighbours' broadcasts, combined in CSC order */
      int has = 0;
      double facc = 0.0;
      uint32_t umin = ORC_INF;
      if (s > 0) {
        for (uint64_t e = csc_off[v]; e < csc_off[v + 1]; ++e) {
          const uint32_t u = (uint32_t)csc_src[e];
          if (!sin[u]) continue;
          if (pr) {
            if (has) facc += fin[u]; /* the sum combiner of Fig. 8 */
            else facc = fin[u];
          } else {
            uint32_t m = uin[u];
            if (app == ORC_APP_SSSP) m += csc_w ? csc_w[e] : 1u; /* checked at the broadcast */
            if (!has || m < umin) umin = m; /* the min combiner of Fig. 5 */
          }
          has = 1;
        }
      }
      sout[v] = 0;
      /* 2. selection and compute */
      if (!(s == 0 || !halted[v] || has)) continue;
      halted[v] = 0;
      ++active;
      int send = 0;
      if (pr) {
        if (s == 0) {
          fval[v] = initial_value;
        } else {
          double sum = 0.0;
          if (has) sum += facc;
          fval[v] = ratio + damping * sum;
        }
        if (s < threshold) send = 1;
        else halted[v] = 1;
      } else if (app == ORC_APP_CC) {
        if (s == 0) {
          uval[v] = v;
          send = 1;
        } else {
          const uint32_t old_value = uval[v];
          if (has && umin < uval[v]) uval[v] = umin;
          if (uval[v] < old_value) send = 1;
        }
        halted[v] = 1;
      } else {
        if (s == 0) {
          uval[v] = v == source ? 0u : ORC_INF;
          send = v == source;
        } else {
          const uint32_t mindist = has ? umin : ORC_INF;
          if (mindist < uval[v]) {
            uval[v] = mindist;
            send = 1;
          }
        }
        halted[v] = 1;
      }
      if (!halted[v]) ++awake;
      if (!send) continue;
      /* broadcast: one outbox value read by every out-neighbour */
      const uint64_t deg = csr_off[v + 1] - csr_off[v];
      ++senders;
      messages += deg;
      sout[v] = 1;
      if (pr) {
        fo[v] = deg ? fval[v] / (double)deg : 0.0;
      } else {
        uo[v] = uval[v];
        if (app == ORC_APP_SSSP)
          for (uint64_t e = csr_off[v]; e < csr_off[v + 1]; ++e)
            if ((uint64_t)uval[v] + (csr_w ? (uint64_t)csr_w[e] : 1u) >= ORC_INF) ++overflow;
      }
    }
    if (s < trace_cap) {
      trace[3 * (uint64_t)s + 0] = active;
      trace[3 * (uint64_t)s + 1] = senders;
      trace[3 * (uint64_t)s + 2] = messages;
    }
    if (overflow) {
      status = ORC_EOVERFLOW;
      break;
    }
    /* 3. every vertex halted and no message pending */
    if (awake == 0 && messages == 0) break;
    if (cap && s + 1 >= cap) {
      status = ORC_NOT_CONVERGED;
      break;
    }
  }
  *supersteps_out = s + 1;
  free(fout[0]);
  free(fout[1]);
  free(uout[0]);
  free(uout[1]);
  free(sent[0]);
  free(sent[1]);
  free(halted);
  return status;
}

/* Threads the OpenMP runtime offers to orc_run_pull by default. */
int orc_max_threads(void) { return omp_get_max_threads(); }
