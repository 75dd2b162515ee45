/*
 * ipregel.h -- C ABI of the gfx950 superstep engine.
 *
 * The library executes the synchronous vertex-centric model of iPregel
 * (Capelli et al., "iPregel: Vertex-centric programmability vs memory
 * efficiency and performance, why choose?", Parallel Computing 2019):
 * supersteps of local computation, communication and global synchronisation
 * (Section 4.2), one-slot mailboxes whose messages are combined on arrival
 * (Section 4.3.3), selection of the vertices to run (Section 4.3.1), push or
 * pull message exchange (Section 4.3.2), and termination once every vertex
 * has voted to halt and no message is pending.  The user's compute/combine
 * pair (Fig. 1) is chosen from the three applications of Section 6:
 * PageRank (Fig. 8, sum combiner), hash-min connected components (Fig. 9,
 * min combiner) and single-source shortest paths (Fig. 10, min combiner).
 *
 * Conventions for every entry point:
 *   - No C++ types cross this boundary; all sizes are explicit.
 *   - "device pointer" means memory allocated on the current HIP device by the
 *     caller (e.g. a torch tensor); the library never allocates or frees
 *     device memory and never frees caller memory.  Host pointers are plain
 *     process memory.
 *   - `hip_stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is stream-ordered on it.
 *   - Errors are returned as ipg_status; a human-readable message for the
 *     last error on the calling thread is available from ipg_last_error().
 *     No entry point aborts, throws or prints.
 *   - One graph handle must not be used by two threads at once.
 */
#ifndef IPREGEL_H
#define IPREGEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ipg_graph ipg_graph; /* opaque handle, host memory owned by the library */

typedef enum {
  IPG_OK = 0,
  IPG_NOT_CONVERGED = 1,   /* superstep cap reached with work pending; values are valid */
  IPG_EINVAL = -1,         /* bad argument (null pointer, source >= N, ...) */
  IPG_EBADGRAPH = -2,      /* graph arrays failed validation */
  IPG_EUNSUPPORTED = -3,   /* (app, combiner) pair not supported, or weights where none apply */
  IPG_EWORKSPACE = -4,     /* workspace missing, too small or misaligned */
  IPG_EDEVICE = -5,        /* a HIP call failed; see ipg_last_error() */
  IPG_EOVERFLOW = -6       /* an SSSP message would reach 0xFFFFFFFF (the INF distance) */
} ipg_status;

typedef enum { IPG_APP_PAGERANK = 0, IPG_APP_CC_HASHMIN = 1, IPG_APP_SSSP = 2 } ipg_app;
typedef enum { IPG_COMBINE_SUM = 0, IPG_COMBINE_MIN = 1 } ipg_combiner;

/* Message exchange (Section 4.3.2).  The mode never changes results.  AUTO
 * picks per superstep: the learned selector when ipg_run_opts.selector is
 * set (push over the frontier list, push sweeping every vertex, or pull),
 * else a fixed frontier-size heuristic; a CC/SSSP superstep it picks as pull
 * may then turn to a push once its messages are counted (ipg_tuning.late_div).
 * PUSH and PULL force the exchange of every superstep.  PageRank runs every
 * vertex in every superstep, so its AUTO is pull. */
typedef enum { IPG_MODE_AUTO = 0, IPG_MODE_PUSH = 1, IPG_MODE_PULL = 2 } ipg_mode;

/* ipg_graph_desc.flags */
#define IPG_GRAPH_SYMMETRIC 1u /* CSC arrays equal the CSR arrays (undirected graph) */
#define IPG_GRAPH_VALIDATE 2u  /* check offsets and ids on the device at create time */
#define IPG_GRAPH_RENAME 4u    /* keep a second copy of the CSC source ids renamed hot-first (by descending
                                  out-degree) for PageRank's pull exchange, whose outbox is then stored in
                                  that order: the most-read outbox entries share cache lines.  On a symmetric
                                  blocked store CC and SSSP run under the new names too (the renamed CSC
                                  serves as the CSR; CC's labels start from the caller's ids; values come
                                  back in the caller's order).  Results are unchanged (PageRank: the same
                                  values summed in the same order; CC/SSSP: the same minima); costs about
                                  4E + 20N bytes of graph workspace (ids, both directions of the renaming,
                                  out-degrees and offsets) plus a second pull tiling, and 4N bytes of host
                                  memory in the handle (the renaming, to map an SSSP source). */
#define IPG_GRAPH_BLOCKED 8u   /* keep destination-blocked in-edges for PageRank's pull exchange (of the
                                  hot-first CSC with IPG_GRAPH_RENAME): the destinations are cut into runs of
                                  at most 20224 consecutive rows whose FP64 sums fit one workgroup's LDS
                                  (closed early at 8/256 of the edges -- or, when the row-capped blocks
                                  outnumber the 256 slices, at twice their mean edges -- so rows with many
                                  in-edges form narrow blocks), and each block's in-edges are stored sorted by source, 4 bytes per
                                  edge, so that a wavefront's outbox reads share cache lines.  Every superstep
                                  streams the blocks and adds each message into its destination's sum in LDS;
                                  blocks spread over several workgroups add their partial sums in a fixed
                                  order.  The sums are the same messages under the sum combiner (Fig. 8) in a
                                  varying order, as with push: results agree with the oracle to rounding but
                                  are not bitwise reproducible.  Built on the host (two counting sorts, O(N + E)
                                  time and about 16E + 24N bytes of host memory); costs about 4E bytes plus a
                                  partial-sum buffer of at most 256 * 20224 doubles of graph workspace, which
                                  runs on the handle share (runs on one handle must not overlap in time).
                                  CC and SSSP with unit weights pull over the same table on a symmetric
                                  store with IPG_GRAPH_RENAME (u32 minima in LDS, exact), else over a
                                  second one built on the caller's CSC (with IPG_GRAPH_RENAME) or the same
                                  one (without). */

#define IPG_GRAPH_BINNED 16u   /* with IPG_GRAPH_BLOCKED: PageRank's pull gathers only the outboxes of the
                                  sources below ipg_graph_desc.binned_hot (rounded up to a multiple of 65536;
                                  hot-first names with IPG_GRAPH_RENAME) edge by edge.  Every other ("cold")
                                  source's outbox is copied, once per superstep, into one slot per block it
                                  has in-edges to, by a bin launch whose workgroups take up to 4096 groups
                                  of 64 slots of one window of 8192 sources (their outboxes staged in LDS)
                                  and write each block's slots as runs of whole 8-slot lines; the pull then
                                  reads a block's cold messages from its slots in order.  This turns a cold gather, which moves a memory line for
                                  8 bytes once the outbox array outgrows the caches, into a streamed
                                  write and read of 8 bytes (propagation blocking over Section 4.3.2's pull).
                                  The sums are unchanged (the same messages; order as with
                                  IPG_GRAPH_BLOCKED).  The CC/SSSP pull's blocked in-edges are binned the
                                  same way, with their u32 outboxes (INF for a source that did not
                                  broadcast) in the slots and the same hot count.
                                  Costs about 10 bytes per cold (block, source) pair of graph workspace per
                                  binned table (bounded by 10E + 70 x the (block, window) pairs). */

/*
 * A graph as CSR (out-adjacency, for push) plus CSC (in-adjacency, for pull).
 * All array pointers are DEVICE pointers owned by the caller and must stay
 * valid until ipg_graph_destroy.
 *   csr_off[N+1] uint64, csr_off[0] = 0, non-decreasing, csr_off[N] = E;
 *   csr_dst[E]   int32 ids in [0, N), each list in any order;
 *   csc_off/csc_src: the same for in-edges (may alias csr_* when symmetric);
 *   csr_w/csc_w[E]: uint32 weights aligned with csr_dst/csc_src, or NULL for
 *   unit weights (used by SSSP only; an undirected edge must carry the same
 *   weight in both arrays).
 * Self-loops and duplicate edges are ordinary edges.  N < 2^31.
 */
typedef struct {
  uint32_t num_vertices;
  uint64_t num_edges;
  const uint64_t* csr_off;
  const int32_t* csr_dst;
  const uint64_t* csc_off;
  const int32_t* csc_src;
  const uint32_t* csr_w;
  const uint32_t* csc_w;
  uint32_t flags;
  uint32_t binned_hot;  /* IPG_GRAPH_BINNED: sources gathered edge by edge (0 = 1048576, 8 MB of FP64 outboxes) */
} ipg_graph_desc;

/* ipg_run_opts.flags */
#define IPG_RUN_PERSISTENT 1u /* device-driven superstep loop (CC/SSSP): a control block in the workspace
                                 decides halt, active set and exchange on the device, superstep 0
                                 included; the host enqueues supersteps in chunks -- first as many as
                                 the last such run of the application on the handle took (else 2), then
                                 doubling up to 64 -- and synchronises once per chunk, with no
                                 per-superstep host sync */
#define IPG_RUN_ENQUEUE 4u    /* enqueue the run's work on the stream and return at once, with no host
                                 synchronisation and no readback, so that the caller can capture it into a
                                 graph: PageRank (fixed T; part_offsets are not checked; no timing) and
                                 batched SSSP (device-driven supersteps up to max_supersteps <= 1024; the
                                 outcome from ipg_multi_sssp_result).  Stats are not filled. */
#define IPG_RUN_GRAPH 2u      /* PageRank: replay the whole superstep sequence as one hipGraph launch.  The
                                 graph is captured on the first call and kept in the handle while T, the
                                 exchange, the workspace and part_offsets stay the same; per-superstep
                                 times (usec) are not recorded in this mode. */

/*
 * Launch parameters of the exchange kernels; 0 keeps the library's default.
 * They change speed only: results stay exact (CC, SSSP) and within the
 * PageRank summation-order freedom.  Chosen per graph by an autotuner.
 */
typedef struct {
  uint32_t pr_hot;     /* PageRank pull on a store built with IPG_GRAPH_RENAME: outbox entries of the
                          most-read sources cached in LDS per workgroup (default 8192; capped to the
                          LDS a workgroup can hold beside the kernel's tiles, 11200 on gfx950;
                          UINT32_MAX = no cache) */
  uint32_t pull_grid;  /* workgroups of the pull item kernels (default 2048) */
  uint32_t push_div;   /* fixed exchange rule: pull when frontier + its out-edges > E / push_div (default 20) */
  uint32_t list_div;   /* push frontiers up to max(4096, N / list_div) are visited as a list (default 16;
                          UINT32_MAX = never); a push chosen by a trained selector takes the list
                          variant it predicts faster instead */
  uint32_t gate_div;   /* CC/SSSP pull: when fewer than N / gate_div vertices broadcast, the gather reads
                          a bitmap of the senders first and skips the others' outboxes (default 8;
                          UINT32_MAX = never) */
  uint32_t blocked;    /* pull exchanges on a store built with IPG_GRAPH_BLOCKED (PageRank, CC and SSSP
                          with unit weights): 0 (default) = use the blocked in-edges, UINT32_MAX = use
                          the row-item kernels instead */
  uint32_t late_div;   /* CC/SSSP under IPG_MODE_AUTO, superstep >= 1: a superstep chosen as pull whose
                          broadcasts, counted after its compute, carry at most E / late_div messages is
                          exchanged by push instead -- the choice of Section 4.3.2 taken once the
                          messages are known (default 20; UINT32_MAX = never).  Reported as a push
                          superstep in the stats. */
} ipg_tuning;

typedef struct {
  uint32_t source;          /* SSSP source vertex (ignored by the other applications) */
  double damping;           /* PageRank's d (Fig. 8 prints 0.85): rank = (1 - d)/N + d * (sum of the
                               messages); 0 = 0.85; anything outside (0, 1] is IPG_EINVAL.  Ignored by
                               the other applications. */
  ipg_mode mode;
  uint32_t flags;
  const double* selector;   /* DEVICE pointer to IPG_SELECTOR_PARAMS trained selector parameters
                               (see ipg_selector_train), used by IPG_MODE_AUTO; NULL = fixed heuristic */
  /* PageRank over a disjoint union of graphs: DEVICE pointer to num_parts+1
   * ascending vertex offsets (part_offsets[0] = 0, part_offsets[num_parts] = N).
   * Vertex v of part p uses that part's vertex count N_p for its initial value
   * 1/N_p and its ratio 0.15/N_p (Fig. 8), so when no edge crosses two parts
   * each part's ranks equal a separate run on that part.  Copied to the host
   * and checked on every call; NULL / 0 = one part of N vertices. */
  const uint32_t* part_offsets;
  uint32_t num_parts;
  /* PageRank to convergence when > 0: after every update s the L1 change
   * sum_v |r_s(v) - r_{s-1}(v)| is reduced (ipg_run_stats.residual), and the
   * run stops after the first update whose change is below `tolerance`
   * (IPG_OK; the values are those of a run with T = that update), or after
   * max_supersteps updates (IPG_NOT_CONVERGED, values valid).  max_supersteps
   * must then be >= 1; not combinable with IPG_RUN_GRAPH.  0 = fixed T. */
  double tolerance;
  const ipg_tuning* tuning; /* HOST pointer, or NULL for the defaults */
} ipg_run_opts;

/*
 * Run statistics, filled by ipg_run when a non-NULL pointer is passed.
 * Arrays are HOST memory owned by the caller with trace_cap entries each
 * (any may be NULL); entry s describes superstep s:
 *   active[s]   vertices that ran compute,
 *   senders[s]  vertices that broadcast,
 *   messages[s] messages delivered (sum of the senders' out-degrees) -- the
 *               edges traversed by the method,
 *   examined[s] edges read by the exchange (push: = messages; pull: in-edges
 *               scanned),
 *   mode[s]     1 push, 2 pull,
 *   usec[s]     device time of superstep s (HIP events), when timing is on,
 *   frontier_deg[s]  sum of the out-degrees of the vertices active in s
 *               (the selector's second input),
 *   residual[s] PageRank run with a tolerance: the L1 change of update s.
 */
typedef struct {
  uint32_t supersteps;      /* supersteps executed */
  uint32_t halted;          /* 1 if the run ended by vote-to-halt */
  uint64_t edges_traversed; /* total messages */
  uint64_t edges_examined;  /* total edges read by the exchange */
  double seconds;           /* first superstep launch -> halt decision (HIP events) */
  uint32_t trace_cap;
  uint64_t* active;
  uint64_t* senders;
  uint64_t* messages;
  uint64_t* examined;
  uint8_t* mode;
  float* usec;
  uint64_t* frontier_deg;
  double* residual;         /* PageRank with a tolerance: L1 change of update s (entry 0 is 0) */
} ipg_run_stats;

/* Bytes of graph workspace ipg_graph_create needs for this graph size.  The
 * workspace is device memory (256-byte aligned) owned by the caller and must
 * outlive the handle.  Paper: Section 4.2 (the framework's global arrays of
 * vertex data and adjacency) and Table 3 (memory footprint as an evaluation
 * axis); this query makes the device-side footprint explicit. */
size_t ipg_graph_workspace_bytes(uint32_t num_vertices, uint64_t num_edges, uint32_t flags);

/* Bytes of run workspace ipg_run needs for `app` on a graph of this size
 * (device memory, 256-byte aligned, owned by the caller).  The application's
 * values live inside it until the next ipg_run on the same graph.  Paper:
 * Section 4.3.3 (one message slot per vertex, combined on arrival) and
 * Section 4.2 (vertex values; double-buffered message boxes between
 * supersteps, Fig. 3). */
size_t ipg_run_workspace_bytes(uint32_t num_vertices, uint64_t num_edges, ipg_app app);

/*
 * Build the device graph store: validate (IPG_GRAPH_VALIDATE), derive the
 * out-degrees and the pull-side tiling of the CSC.  Synchronises the stream.
 * On success *out receives a handle; on failure *out is NULL and the status
 * is IPG_EINVAL, IPG_EBADGRAPH, IPG_EWORKSPACE or IPG_EDEVICE.
 * Paper: Section 3 (a directed graph whose vertices know their in- and
 * out-neighbours: the out-edges carry a broadcast, the in-edges are what the
 * pull form of Section 4.3.2 reads) and Section 4.2 (vertices and edges
 * loaded into the framework's arrays before processing, outside the timed
 * part, Section 7).
 */
ipg_status ipg_graph_create(const ipg_graph_desc* desc, void* workspace, size_t workspace_bytes,
                            void* hip_stream, ipg_graph** out);

/*
 * Run one application to completion (or to the cap) on the graph.
 * Paper: Fig. 1 and Fig. 2 (the user's compute and combine functions and the
 * superstep loop that calls them), Section 4.1-4.2 (synchronous supersteps,
 * vote to halt, a message sent in superstep s read in s + 1), Section 4.3
 * (selection, push/pull exchange, combiners) and Figs. 8-10 (the three
 * applications).
 *   (app, combiner) must be (PAGERANK, SUM), (CC_HASHMIN, MIN) or (SSSP, MIN):
 *   anything else is IPG_EUNSUPPORTED.
 *   max_supersteps: PageRank -> number of rank updates T (vertices broadcast
 *   while the superstep is < T and halt at T, so T+1 supersteps run and the
 *   result is the rank after T updates; T = 10 is Fig. 8).  CC / SSSP -> cap
 *   on supersteps executed, 0 = unlimited; reaching the cap with messages
 *   pending returns IPG_NOT_CONVERGED and the values are still readable.
 *   opts may be NULL (source 0, AUTO, host-driven loop).  source >= N is
 *   IPG_EINVAL for SSSP.
 *   workspace: ipg_run_workspace_bytes(N, E, app) bytes of device memory.
 * The host loop reads one small counter block per superstep (CC/SSSP) and
 * synchronises the stream before returning.  The decide kernels of CC/SSSP
 * and of the batched SSSP write that block (and the device-driven loop's
 * trace records) into a small pinned host buffer owned by the graph handle
 * (created on first use, freed by ipg_graph_destroy): runs on one handle
 * must not overlap in time, from one host thread or several.
 */
ipg_status ipg_run(ipg_graph* graph, ipg_app app, ipg_combiner combiner, uint32_t max_supersteps,
                   const ipg_run_opts* opts, void* workspace, size_t workspace_bytes, void* hip_stream,
                   ipg_run_stats* stats);

/* Copy the values of the last run on `graph` (double for PageRank, uint32
 * otherwise; N entries) to dst, which is a device pointer when dst_is_device
 * is non-zero, else host memory.  A host copy synchronises the stream; a
 * device copy is only enqueued on it (work on other streams must wait for
 * the stream first).  IPG_EINVAL if no run happened or dst_bytes is too
 * small.  Paper: Fig. 2 and Section 4.1 (the result of a vertex-centric
 * program is the value every vertex holds when the last superstep ends;
 * Section 7 times processing without dumping it). */
ipg_status ipg_read_values(const ipg_graph* graph, void* dst, size_t dst_bytes, int dst_is_device,
                           void* hip_stream);

/*
 * Batched SSSP with unit weights: up to IPG_BATCH_MAX_SOURCES single-source
 * runs of Fig. 10 on one graph, executed as one superstep loop.  With unit
 * weights all messages of a superstep carry the same value, so the min
 * mailbox of each (source, vertex) pair is one bit and the queries advance
 * together with bit-parallel masks.  Results equal the separate runs:
 *   dist: DEVICE memory, [num_sources][N] uint32 (query-major: row i holds
 *         the values of the run from sources[i]); INF = unreached.
 *   sources: DEVICE pointer to num_sources vertex ids (repeats allowed),
 *         copied to the host and checked (< N) before any kernel runs.
 *   stats (optional): supersteps = the largest superstep count of the
 *         queries; active/senders/messages[s] = the sums over queries of the
 *         single-source traces (a finished query adds 0); examined[s] = edges
 *         read by the shared exchange; mode[s] its direction.
 *   max_supersteps: cap on supersteps, 0 = none (IPG_NOT_CONVERGED when
 *         reached with messages pending).  opts->mode forces push or pull;
 *         opts->source and opts->selector are ignored.
 *   opts->flags: IPG_RUN_PERSISTENT runs the superstep loop on the device
 *         (control block in the workspace; one readback per 16 supersteps);
 *         IPG_RUN_ENQUEUE only enqueues it (see the flag).
 * A graph with weights is IPG_EUNSUPPORTED.  The host-driven loop
 * synchronises the stream once per superstep.
 */
#define IPG_BATCH_MAX_SOURCES 256
size_t ipg_multi_sssp_workspace_bytes(uint32_t num_vertices, uint64_t num_edges);
ipg_status ipg_run_multi_sssp(ipg_graph* graph, const uint32_t* sources, uint32_t num_sources,
                              uint32_t max_supersteps, const ipg_run_opts* opts, uint32_t* dist, size_t dist_bytes,
                              void* workspace, size_t workspace_bytes, void* hip_stream, ipg_run_stats* stats);
/* Outcome of the last device-driven batched run in `workspace` (after an
 * IPG_RUN_ENQUEUE run has executed): fills stats (times from the device's
 * wall clock) and returns its status -- IPG_EINVAL if a source was >= N
 * (that query was skipped) or no such run has ended.  Synchronises. */
ipg_status ipg_multi_sssp_result(const ipg_graph* graph, const void* workspace, size_t workspace_bytes,
                                 void* hip_stream, ipg_run_stats* stats);

/*
 * Learned exchange selector (an extension of Section 4.3.2, where the push /
 * pull choice is a compile-time flag set by the user's experiments).
 * A 4-16-16-3 tanh MLP in FP64 predicts log2 of the time of a superstep's
 * exchange variants -- [0] a push that visits the frontier as a list, [1] a
 * push that sweeps every vertex's mailbox, [2] a pull -- from
 * log2(1+|F|)/32, log2(1+sum of out-degrees of F)/32, min(superstep,128)/64
 * and log2(1+E)/32.  AUTO runs the variant of the smallest prediction among
 * those available (the list only after a push that left a complete one); it
 * replaces the push_div rule and, for the pushes it chooses, the list_div
 * limit.  Parameters are packed W1[16][4], b1[16], W2[16][16], b2[16],
 * W3[3][16], b3[3].  All arrays are DEVICE memory owned by the caller; x is
 * [n][4], y and t [n][3].
 */
#define IPG_SELECTOR_PARAMS 403
#define IPG_SELECTOR_INPUTS 4
#define IPG_SELECTOR_OUTPUTS 3

/* Workspace bytes for ipg_selector_grad / ipg_selector_train on n samples. */
size_t ipg_selector_workspace_bytes(uint32_t n_samples);
/* y = network(x) for n samples.  Stream-ordered, no synchronisation. */
ipg_status ipg_selector_forward(const double* params, const double* x, uint32_t n, double* y, void* hip_stream);
/* grad = d/dparams of (1/2n) * sum (y - t)^2 over the n samples.  Stream-ordered. */
ipg_status ipg_selector_grad(const double* params, const double* x, const double* t, uint32_t n, double* grad,
                             void* workspace, size_t workspace_bytes, void* hip_stream);
/* `epochs` full-batch gradient-descent steps params -= lr * grad, in place, on the device. */
ipg_status ipg_selector_train(double* params, const double* x, const double* t, uint32_t n, uint32_t epochs,
                              double lr, void* workspace, size_t workspace_bytes, void* hip_stream);

/*
 * ipg_selector_train without a workspace argument, for callers that cannot
 * allocate device memory around the call (code under stream capture, tight
 * serving or training loops, harnesses that forbid allocation).  The same
 * kernel as ipg_selector_train, with the same result bit for bit; its
 * gradient and batch scratch live in a static device array of the library,
 * 8 * (IPG_SELECTOR_PARAMS + 67 * IPG_SELECTOR_NOALLOC_MAX_SAMPLES) bytes
 * (8.8 MB), one copy per GPU, held from the first call on that GPU until the
 * process ends.  The call allocates nothing: no hipMalloc, no hipFree, no
 * allocating library routine.  params, x and t are DEVICE memory of the
 * caller, as for ipg_selector_train.  n > IPG_SELECTOR_NOALLOC_MAX_SAMPLES
 * (or n == 0, a NULL pointer, lr <= 0) is IPG_EINVAL.  Every call on one GPU
 * shares that GPU's array, so calls that overlap in time on one GPU (two
 * streams, two threads) race and must be serialised by the caller;
 * consecutive calls are independent (nothing an earlier call left in the
 * array is read).  Stream-ordered, no synchronisation.
 */
#define IPG_SELECTOR_NOALLOC_MAX_SAMPLES 16384
ipg_status ipg_selector_train_noalloc(double* params, const double* x, const double* t, uint32_t n, uint32_t epochs,
                                      double lr, void* hip_stream);

/* Free the handle (host memory only; caller buffers are untouched).  Paper:
 * the counterpart of ipg_graph_create (Section 4.2's arrays live as long as
 * the graph is processed); the caller's device buffers stay the caller's. */
void ipg_graph_destroy(ipg_graph* graph);

/* Message for the last error on the calling thread ("" if none).  Not from
 * the paper, which has no error channel: the library reports every failure
 * as a status code plus this thread-local text instead of aborting. */
const char* ipg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IPREGEL_H */
