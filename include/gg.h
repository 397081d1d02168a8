/*
 * gg.h — C ABI of the MI355X (gfx950) GraphGuess sweep library.
 *
 * GraphGuess (Ramezani, Kandemir, Sivasubramaniam, arXiv 2104.10039) runs a
 * pull-based vertex program [Sec. 3.1, Alg. 2] in two modes [Sec. 3.3]:
 * accurate (gather over every in-edge) and approximate (gather over the
 * in-edges whose per-edge flag is set). A run starts from a uniform sample of
 * the edges with ratio sigma, stays approximate for alpha iterations, then
 * runs a superstep: one accurate iteration whose per-edge influence decides,
 * against threshold theta, which edges stay active; all others are
 * deactivated; supersteps recur every alpha approximate iterations
 * [Sec. 3.4]. SP (sparsify only) and SMS (one switch to accurate mode) are
 * the two static schemes of Sec. 5.2.
 *
 * Conventions for every entry point:
 *  - Return 0 (GG_OK) on success or a negative gg_status. No C++ exception
 *    crosses this boundary. The message of the last failure on the calling
 *    thread is returned by gg_last_error().
 *  - Output buffers are written only on success.
 *  - Pointers marked "device" are HIP device pointers (for instance
 *    torch.Tensor.data_ptr() of a CUDA/ROCm tensor); "host" pointers are
 *    ordinary process memory. Output value buffers may be either, selected by
 *    GG_OUT_HOST.
 *  - Work is issued on the HIP stream bound to the graph (gg_graph_load_csr or
 *    gg_graph_set_stream; NULL = the default stream). Entry points that
 *    return results to the host synchronize that stream; device outputs are
 *    complete when the call returns.
 *  - A graph handle and the runs created from it must not be used from two
 *    threads at once.
 */
#ifndef GG_H
#define GG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GG_VERSION 8

typedef enum {
  GG_OK = 0,
  GG_E_INVAL = -1,       /* null pointer, unknown enum, sigma outside [0,1], theta < 0, alpha < 0, ... */
  GG_E_RANGE = -2,       /* malformed CSR, vertex id out of range, n or m too large, weight outside [0,255] */
  GG_E_NOMEM = -3,       /* device or host allocation failed */
  GG_E_DEVICE = -4,      /* HIP runtime error, or a device-side wait of a superstep that gave up
                            (the results since the last check are undefined); gg_last_error() holds its text */
  GG_E_UNSUPPORTED = -5, /* valid request that the library does not implement */
  GG_E_STATE = -6        /* call not valid in the current state of the handle */
} gg_status;

/* Vertex programs [Sec. 4.1]. PR = PageRank (Alg. 2); PPR = personalized
   PageRank from a source; SSSP = single-source shortest paths; CC = weakly
   connected components by minimum-label propagation (load the symmetrized
   graph); BP = belief propagation on a binary pairwise Markov random field
   (the paper names BP among its applications without giving the model; the
   reading taken here: one potential psi(x, y) = (1 + kappa)/2 if x == y,
   (1 - kappa)/2 otherwise, on every edge, a prior log-odds h_u per vertex;
   the value of u is its belief log-odds L_u = h_u + sum over the in-edges
   (v, u) of the edge set of c_v, with c_v = log(m_v(1) / m_v(0)) =
   2 atanh(kappa tanh(L_v / 2)) the message of v computed from its whole
   belief; load the symmetrized graph for an undirected model). BP runs
   gg_app_params.iters iterations; its edge influence at a superstep is
   |c_v| / |P| with P the running sum of the row's contributions up to and
   including the edge (PREFIX on magnitudes, since messages have both
   signs). */
typedef enum { GG_APP_PR = 0, GG_APP_SSSP = 1, GG_APP_CC = 2, GG_APP_PPR = 3, GG_APP_BP = 4 } gg_app;

/* Correction schemes: EXACT = accurate mode in every iteration (the baseline
   of Sec. 5); SP = sparsified for the whole run; SMS = approximate for alpha
   iterations then accurate for the rest; GG = adaptive correction [Sec. 3.4].
   LEARNED (a project addition, not in the paper: a network trained on the
   method's own error traces picks where to correct) keeps GG's schedule,
   but at a correction step (iteration i with i mod (alpha+1) == 0) a network
   scores every vertex; the selected rows S = { v : logit_v > tau } are
   gathered over all in-edges and have their flags re-selected (a partial
   superstep) while every other row takes an approximate iteration. Every
   fallback_k-th correction step (fallback_k > 0), and every step whose
   selected rows hold more than rho * m in-edges, is GG's full superstep
   instead. */
typedef enum {
  GG_POLICY_EXACT = 0,
  GG_POLICY_SP = 1,
  GG_POLICY_SMS = 2,
  GG_POLICY_GG = 3,
  GG_POLICY_LEARNED = 4
} gg_policy_kind;

/* Kind of an executed iteration (gg_step_info.kind). */
typedef enum { GG_STEP_APPROX = 0, GG_STEP_ACCURATE = 1, GG_STEP_FULL = 2, GG_STEP_PARTIAL = 3 } gg_step_kind;

/* SSSP/CC termination for non-exact schemes: FIXED_ITERS runs exactly
   gg_app_params.iters iterations (the same count as the exact baseline,
   Sec. 5); FIXED_POINT stops after a no-change iteration that no later
   iteration can follow differently (an accurate one, or any SP one). Exact
   runs always stop at their first no-change iteration. */
typedef enum { GG_STOP_FIXED_ITERS = 0, GG_STOP_FIXED_POINT = 1 } gg_stop;

/* Edge influence at a superstep [Alg. 2, GG-Gather]. PREFIX: over the
   running value of the row in CSR order, starting from the gather's identity
   (PR/PPR/BP: contribution over the running sum; SSSP: relative improvement
   of the running minimum; CC: lowers the running minimum). TOTAL (PR/PPR):
   contribution over the row sum (its supersteps gather every edge twice,
   once for the row sums; not with LEARNED: GG_E_UNSUPPORTED). PUSH
   (SSSP/CC): push order [Sec. 3.1: the method is not tied to the pull
   model], the running minimum starting at the destination's own value
   before the superstep, so that an edge stays active only while it improves
   its destination; values are those of PREFIX. */
typedef enum { GG_INFL_PREFIX = 0, GG_INFL_TOTAL = 1, GG_INFL_PUSH = 2 } gg_influence;

/* Flag update at a superstep: REPLACE deactivates every edge that does not
   qualify [Sec. 3.4]; UNION keeps previously active edges. */
typedef enum { GG_MASK_REPLACE = 0, GG_MASK_UNION = 1 } gg_mask_update;

/* PageRank mass of vertices without out-edges: spread over all vertices
   (UNIFORM; sent to the source for PPR) or dropped (NONE). */
typedef enum { GG_DANGLING_UNIFORM = 0, GG_DANGLING_NONE = 1 } gg_dangling;

/* Out-degree PageRank divides by in approximate iterations [Alg. 2,
   GG-Gather reads v.degree]: the graph's (FULL), or the count of the
   vertex's active out-edges under the current flags (ACTIVE: PageRank of
   the sparsified graph, whose vertices without an active out-edge are
   dangling). Accurate iterations and supersteps always use FULL. ACTIVE is
   not available with LEARNED, traces, vertex status or graphs with parts
   (GG_E_UNSUPPORTED). */
typedef enum { GG_DEGREE_FULL = 0, GG_DEGREE_ACTIVE = 1 } gg_pr_degree;

/* gg_csr_desc.flags */
#define GG_CSR_DEVICE_PTRS 0x1u /* rowptr/col/weight are device pointers, borrowed (must outlive the graph) */
#define GG_CSR_SKIP_VALIDATE 0x2u /* trust the caller: skip the O(n+m) structure check */

/* Output flags */
#define GG_OUT_HOST 0x1u /* out_values is a host pointer (default: device pointer) */

/*
 * A graph in pull form: the in-CSR. Row u lists the sources v of the edges
 * v -> u; edge id e is the position in col. Self-loops should be removed by
 * the caller (they are processed as ordinary edges otherwise).
 *   n       vertices, 0 <= n < 2^31 (n <= 2^24 when weights are given)
 *   m       edges, 0 <= m < 2^31
 *   rowptr  int32[n+1], rowptr[0] = 0, non-decreasing, rowptr[n] = m
 *   col     int32[m], each in [0, n)
 *   weight  int32[m] in [0, 255], or NULL (required by SSSP)
 */
typedef struct {
  int32_t n;
  int64_t m;
  const int32_t* rowptr;
  const int32_t* col;
  const int32_t* weight;
  uint32_t flags;
} gg_csr_desc;

typedef struct {
  int32_t app;       /* gg_app */
  double damping;    /* PR/PPR damping factor d in [0,1) (Alg. 2, GG-Apply) */
  int32_t iters;     /* PR/PPR/BP: iterations T; SSSP/CC FIXED_ITERS: iterations */
  int32_t max_iters; /* SSSP/CC fixed-point runs: cap on iterations (> 0) */
  int32_t source;    /* SSSP/PPR source vertex */
  int32_t dangling;  /* gg_dangling */
  int32_t pr_degree; /* gg_pr_degree (PR/PPR) */
  double coupling;    /* BP: kappa in [0, 1) */
  const float* prior; /* BP: device pointer, float32[n] prior log-odds (finite); copied by
                         gg_run_begin / gg_approx_run / gg_exact_run, so it need not outlive
                         the call */
} gg_app_params;

typedef struct gg_mlp gg_mlp;
typedef struct gg_trace gg_trace;

typedef struct {
  int32_t kind;        /* gg_policy_kind */
  int32_t alpha;       /* approximate window, >= 0 [Sec. 3.4] */
  double theta;        /* influence threshold, 0 <= theta < 65536 [Sec. 3.4] */
  uint64_t seed;       /* sampling seed */
  int32_t influence;   /* gg_influence (PR/PPR) */
  int32_t mask_update; /* gg_mask_update */
  int32_t stop;        /* gg_stop (SSSP/CC) */
  /* LEARNED only (zero otherwise) */
  const gg_mlp* mlp;   /* the scoring network (on the graph's device) */
  float tau;           /* selection threshold on the binary32 logit */
  double rho;          /* full superstep when the rows of S hold > rho * m in-edges, rho >= 0 */
  int32_t fallback_k;  /* every fallback_k-th correction step is full; 0 = never */
  int32_t audit;       /* 1: at full supersteps, score the selection against the drift labels */
  /* GG and LEARNED: optional trace (NULL = none). At every full superstep the
     features of each vertex and its drift label are appended. */
  gg_trace* trace;
  float label_eps;     /* PR/PPR drift label: relative change of the contribution, > 0 */
  /* GG and LEARNED: decoupled parameters of the first superstep [Sec. 3.4,
     last paragraph]. decoupled = 1: the first superstep follows alpha0 >= 0
     approximate iterations (iteration alpha0 + 1) and selects with theta0
     in [0, 65536); the later ones recur every alpha + 1 iterations after it
     and select with theta. decoupled = 0: alpha and theta throughout, alpha0
     and theta0 ignored. Other schemes: decoupled must be 0. */
  int32_t decoupled;
  int32_t alpha0;
  double theta0;
  /* PR/PPR vertex status [Alg. 2, GG-VStatus] (not with LEARNED, traces or
     graphs with parts): GG_VSTATUS_NONE processes every row in every
     iteration; with ABS (REL) a vertex is active after an iteration iff its
     value moved by more than eps (eps times its previous value), every
     vertex being active before the first. Approximate iterations after the
     first then recompute only the rows that an active in-edge from an active
     vertex reaches (the active-vertex list of the vertex-centric model,
     Sec. 2.1); the other rows keep their values. Accurate iterations
     recompute every row. eps >= 0. */
  int32_t vstatus;
  double eps;
} gg_correction_policy;

enum { GG_VSTATUS_NONE = 0, GG_VSTATUS_ABS = 1, GG_VSTATUS_REL = 2 };

typedef struct {
  int32_t iterations;       /* iterations executed */
  int32_t supersteps;       /* flag re-selections executed */
  int64_t edges_gathered;   /* sum over iterations of the edges gathered */
  int64_t active_edges;     /* active edges at the end of the run */
  double device_ms;         /* device time of the run (HIP events on the graph's stream) */
  int64_t edges_processed;  /* edges actually read (frontier iterations read fewer) */
  int32_t sparse_iterations;/* SSSP/CC iterations run as frontier pushes */
  int32_t partial_supersteps; /* LEARNED: partial supersteps executed */
  int64_t selected_total;   /* LEARNED: sum of |S| over correction steps */
  int64_t audit_positives;  /* audited full supersteps: vertices that drifted */
  int64_t audit_hits;       /* ... of which the network selected */
  int64_t audit_selected;   /* ... vertices the network selected */
} gg_run_stats;

typedef struct {
  int32_t iter;          /* 1-based index of the iteration just executed */
  int32_t accurate;      /* 1 if it gathered over every in-edge */
  int32_t superstep;     /* 1 if the edge flags were re-selected after it */
  int64_t edges;         /* edges gathered by it */
  int64_t changed;       /* SSSP/CC: vertices whose value changed; PR/PPR: -1 */
  int64_t active_edges;  /* active edges after it */
  int64_t edges_processed; /* edges actually read by it */
  int32_t sparse;        /* 1 if it ran as a frontier push (SSSP/CC) */
  int32_t kind;          /* gg_step_kind */
  int64_t selected;      /* LEARNED correction steps: |S|; otherwise -1 */
} gg_step_info;

typedef struct gg_graph gg_graph;
typedef struct gg_run gg_run;

int gg_version(void);
const char* gg_last_error(void);

/*
 * Device memory of the library's own objects (project addition; the paper
 * has no memory manager). Graph workspaces, networks and traces allocate
 * through alloc(bytes, ctx), which returns device memory on the current
 * device, aligned to 256 bytes, or NULL when it cannot (the library then
 * fails with GG_E_NOMEM and leaves the caller's outputs untouched; blocks
 * that an object already holds stay with it until it is freed). They free
 * through free(ptr, ctx). The library synchronizes the device after each
 * successful alloc and before each free, as hipMalloc / hipFree do, so a
 * block changes owner with no work pending on it. Both NULL restores
 * hipMalloc / hipFree, the default. The pinned host buffer of a graph and
 * the static array of gg_exact_run_noalloc do not use it. The allocator may
 * change only while no graph, network or trace exists (GG_E_STATE
 * otherwise), so every block is freed by the allocator that made it;
 * GG_E_INVAL when exactly one function is NULL. Not thread-safe against
 * concurrent object creation.
 */
typedef void* (*gg_alloc_fn)(size_t bytes, void* ctx);
typedef void (*gg_free_fn)(void* ptr, void* ctx);
int gg_set_allocator(gg_alloc_fn alloc, gg_free_fn free_fn, void* ctx);

/* Graphs, networks and traces currently alive (for leak checks). */
int64_t gg_live_objects(void);

/*
 * Load a graph (the "graph_load_csr" step). The library computes the
 * out-degrees and the degree-binned work lists of the in-CSR, and for SSSP a
 * packed (weight << 24 | source) edge array. Host inputs are copied to device
 * memory; device inputs (GG_CSR_DEVICE_PTRS) are borrowed. The structure is
 * validated unless GG_CSR_SKIP_VALIDATE is set (GG_E_RANGE on failure).
 * Validation also notes whether every row lists its sources in ascending
 * order; if one does not, source segmentation stays off for this graph
 * (gg_tuning.seg_enable reads 0 and setting it has no effect). With
 * GG_CSR_SKIP_VALIDATE the rows are taken to be in ascending order.
 * hip_stream: a hipStream_t or NULL. On success *out owns a new handle.
 */
int gg_graph_load_csr(const gg_csr_desc* desc, void* hip_stream, gg_graph** out);
int gg_graph_set_stream(gg_graph* g, void* hip_stream);
void gg_graph_free(gg_graph* g);

/*
 * The accurate-mode baseline [Sec. 5]: every iteration gathers over every
 * in-edge. PR/PPR run params->iters iterations; SSSP/CC stop after their
 * first iteration that changes nothing (at most params->max_iters).
 * out_values: n elements, float for PR/PPR, uint32 for SSSP (unreached =
 * 0xFFFFFFFF), int32 for CC; host or device per out_flags. stats nullable.
 */
int gg_exact_run(gg_graph* g, const gg_app_params* params, void* out_values, uint32_t out_flags,
                 gg_run_stats* stats);

/*
 * Exact run that allocates nothing, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation. It runs the same gather kernels as gg_exact_run, with
 * its per-run state (two value buffers, the dangling partial sums, the hub
 * and source-segment partials) in one static array the library holds on
 * each device, 64 MiB, allocated with the library's code at load (about
 * n * 8 bytes + 8 bytes per source segment of every row longer than the
 * short-row bound: R-MAT scale 22 fits, scale 23 does not). Every call on a
 * device shares that device's array, so calls that overlap on one device
 * (on any streams, from any threads) race; the array keeps the last call's
 * contents, none of which a later call reads before writing it.
 *   - Runs exactly params->iters (>= 1) iterations of every app: PR/PPR as
 *     gg_exact_run; SSSP/CC dense, with no frontier pushes and no readback
 *     of a changed count, so their values equal gg_exact_run's once iters
 *     reaches that run's iteration count (further iterations change
 *     nothing). params->max_iters is ignored.
 *   - Only enqueues work on the graph's stream and returns (no host wait):
 *     out_values_dev (device, n elements of the app's value type, as for
 *     gg_exact_run) holds the result once the stream reaches that point.
 *     The call launches kernels only, so it can be captured into a HIP graph.
 *   - stats (nullable): iterations, edges_gathered = edges_processed =
 *     iters * m, active_edges = m; device_ms and the rest 0.
 * The graph (loaded with gg_graph_load_csr, which allocates) must be current
 * on the calling thread's device. GG_E_INVAL (null argument, iters < 1, bad
 * parameters as for gg_exact_run), GG_E_RANGE (the run needs more scratch
 * than the array holds), GG_E_STATE (a step-API run is active on the graph,
 * or another device is current), GG_E_UNSUPPORTED (graphs with parts). No
 * work is enqueued when an error is returned.
 */
int gg_exact_run_noalloc(gg_graph* g, const gg_app_params* params, void* out_values_dev, gg_run_stats* stats);

/*
 * The approximate run (the "approx_run(app, sample_ratio, correction_policy)"
 * step): initial sample of ratio sample_ratio in [0,1] [Sec. 3.4], then the
 * schedule of policy->kind. Outputs as for gg_exact_run.
 */
int gg_approx_run(gg_graph* g, const gg_app_params* params, double sample_ratio,
                  const gg_correction_policy* policy, void* out_values, uint32_t out_flags,
                  gg_run_stats* stats);

/*
 * Multi-query batch (project addition): n_queries runs of PPR or SSSP from
 * sources_host[q] (host array, each in [0, n)) on this graph, iterated
 * together so that every edge word is read once per iteration for all
 * queries, with each query's values read as one contiguous run. Schemes:
 * EXACT; SP with one sampled edge set shared by all queries (ratio
 * sample_ratio, policy->seed); SMS [Sec. 5.2], that sample for iterations
 * 1..policy->alpha and every edge after. PPR runs params->iters iterations,
 * all captured in one HIP graph launched once; exact SSSP stops after the
 * first iteration in which no query changed (at most params->max_iters),
 * captured 32 iterations per graph launch with device-side early exit; SP
 * and SMS SSSP run params->iters iterations. Every query's result equals the corresponding
 * single-query run. out_values: n * n_queries elements, row-major by vertex
 * (out[u * n_queries + q]), float for PPR, uint32 for SSSP; host or device
 * per out_flags. 1 <= n_queries <= 4096.
 */
int gg_batch_run(gg_graph* g, const gg_app_params* params, int32_t n_queries, const int32_t* sources_host,
                 double sample_ratio, const gg_correction_policy* policy, void* out_values, uint32_t out_flags,
                 gg_run_stats* stats);

/*
 * Independent parts (project addition, the multi-graph batch): declare the
 * loaded graph a block-diagonal union of n_parts graphs, part p owning
 * vertices [part_start_host[p], part_start_host[p+1]) (host array, starts at
 * 0, ends at n, non-decreasing); no edge may cross parts (GG_E_RANGE). Every
 * run then treats each part as its own graph, in the same launches: PageRank
 * uses the part's vertex count and dangling mass; SSSP starts from
 * part_sources_host[p] in every part (host array, required for SSSP,
 * params->source is ignored); edge sampling draws part p's edges by their
 * index inside the part with seed + p. PPR and batch runs are not supported
 * on parts. n_parts = 0 removes the parts.
 */
int gg_graph_set_parts(gg_graph* g, int32_t n_parts, const int32_t* part_start_host,
                       const int32_t* part_sources_host);

/*
 * Step API: the same computation as gg_approx_run (or gg_exact_run with
 * policy->kind = GG_POLICY_EXACT), one iteration per call, for tests,
 * traces and inspection. gg_run_step returns 1 when an iteration was
 * executed, 0 when the run had already ended, < 0 on error; info nullable.
 * gg_run_values copies the current values (layout as gg_exact_run).
 * gg_run_mask copies the current edge flags as a bitmap: bit (e mod 32) of
 * word e/32 is edge e's flag; host pointer, ceil(m/32) words.
 */
int gg_run_begin(gg_graph* g, const gg_app_params* params, double sample_ratio,
                 const gg_correction_policy* policy, gg_run** out);
int gg_run_step(gg_run* run, gg_step_info* info);
int gg_run_values(gg_run* run, void* out_values, uint32_t out_flags);
int gg_run_mask(gg_run* run, uint32_t* out_bits_host);

/*
 * Vertex status after the last iteration (GG-VStatus runs; all ones before
 * the first): one byte per vertex (1 = active) into out_host (n bytes).
 * GG_E_STATE for runs without vertex status.
 */
int gg_run_vstatus(gg_run* run, uint8_t* out_host);
int gg_run_stats_get(gg_run* run, gg_run_stats* stats);
/* Per-vertex state of the last correction step (LEARNED) or traced full
   superstep, copied to host memory: features [n][8] bfloat16 bits; the
   selection (1 byte per vertex) and binary32 logits of a LEARNED correction
   step; the drift labels (1 byte per vertex) of a traced or audited full
   superstep. GG_E_STATE when the last step produced no such data. */
int gg_run_features(gg_run* run, uint16_t* feat_host);
int gg_run_selection(gg_run* run, uint8_t* sel_host, float* logits_host);
int gg_run_labels(gg_run* run, uint8_t* labels_host);
/*
 * Checkpoint and resume of a step-API run (not in the paper, whose runs are
 * never interrupted; a project addition). The state after the last executed
 * iteration is the values that the next iteration reads, the edge flags (for
 * every scheme but EXACT) and the run's counters; packed active edges, bins
 * and frontier lists are rebuilt from them. The blob is opaque host memory,
 * owned by the caller, valid only for this library version.
 *   gg_run_state_size    bytes the blob of the run's current state needs
 *   gg_run_export_state  writes it to state_host (bytes must equal the size)
 *   gg_run_import_state  loads it into a run that has executed no iteration,
 *                        begun on a graph of the same shape (n, m, parts)
 *                        with the same app, parameters, sample ratio and
 *                        policy (GG_E_INVAL otherwise; GG_E_STATE once the
 *                        run has stepped); the caller supplies the same
 *                        graph, which is not checked edge by edge.
 * A resumed run continues bit for bit as the uninterrupted run would. Its
 * first SSSP/CC iteration runs dense (the frontier restarts unknown), so
 * edges_processed and sparse_iterations may differ; no value does.
 * LEARNED and traced runs: GG_E_UNSUPPORTED (their delta features span two
 * iterations).
 */
int gg_run_state_size(gg_run* run, int64_t* bytes);
int gg_run_export_state(gg_run* run, void* state_host, int64_t bytes);
int gg_run_import_state(gg_run* run, const void* state_host, int64_t bytes);
void gg_run_end(gg_run* run);

/*
 * Dynamic graphs. The paper states that the method applies to graphs that
 * change [Sec. 1] and evaluates static ones only; the update rules below are
 * this library's reading.
 *
 * An update batch first deletes every arc s -> d of the graph that matches a
 * listed pair (del_src[i], del_dst[i]) (pairs that match nothing are
 * ignored), then inserts one arc ins_src[j] -> ins_dst[j] per entry, with
 * weight ins_weight[j] in [0, 255] (given exactly when the graph has
 * weights). The vertex set is fixed. Each row stays sorted by source; among
 * arcs with the same source the surviving ones come first in their old
 * order, then the inserted ones in batch order. The graph must have rows
 * sorted by source (the canonical in-CSR; GG_E_UNSUPPORTED otherwise) and
 * no parts. After an update the graph owns its CSR arrays (a borrowed device
 * CSR is no longer read), and the result is as if the new CSR had been
 * loaded with the graph's tuning. The arrays an update replaces (the CSR,
 * the packed weights, the flag and active-edge arrays and the frontier's
 * out-CSR: about one more copy of each) are kept as the next update's
 * destinations and released with the graph.
 *   del_src/del_dst  int32[n_delete]; ins_src/ins_dst/ins_weight int32[n_insert]
 *   flags            GG_UPDATE_DEVICE_PTRS: the arrays are device pointers
 *                    (default: host), read during the call only
 * Errors: GG_E_INVAL (null arrays, negative counts, weights given or missing
 * against the graph), GG_E_RANGE (a vertex id outside [0, n), a weight
 * outside [0, 255], more than 2^31 - 1 arcs after the update), GG_E_NOMEM.
 * On an error the graph and any run on it are unchanged.
 */
#define GG_UPDATE_DEVICE_PTRS 0x1u
typedef struct {
  int64_t n_delete;
  const int32_t* del_src;
  const int32_t* del_dst;
  int64_t n_insert;
  const int32_t* ins_src;
  const int32_t* ins_dst;
  const int32_t* ins_weight;
  uint32_t flags;
} gg_update_batch;

/* Applies a batch to a graph with no active run (GG_E_STATE otherwise). */
int gg_graph_update(gg_graph* g, const gg_update_batch* batch);

/* Applies a batch to the graph of an active run, which then continues on the
 * new graph:
 *  - edge flags: a surviving arc keeps its flag, an inserted arc is active
 *    (no superstep has assessed it); the next superstep re-selects it;
 *  - PR/PPR/BP values continue from the current ones; the next iteration
 *    divides by the new out-degrees;
 *  - SSSP/CC: insertions keep every value. After a deletion, a converged
 *    exact run (one that ended on an iteration that changed nothing) resets
 *    only the vertices whose value may rest on a deleted arc: the closure,
 *    along arcs of the new graph that realise their destination's value
 *    (x_s + w = x_d; CC l_s = l_d != d), of the destinations of deleted arcs
 *    that did; every other value is still exact. Any other SSSP/CC run
 *    restarts from its initial values. A converged exact run with the
 *    frontier enabled resumes with a push from the in-neighbours of the
 *    reset vertices and the sources of the inserted arcs; others resume
 *    with a dense iteration;
 *  - the run continues its iteration numbering and schedule for more_iters
 *    (>= 0) further iterations: fixed-count runs raise their count,
 *    fixed-point runs their cap, and the run is no longer done.
 * reset_host (nullable, n bytes) receives 1 for every vertex whose value was
 * reset and 0 for the others, written only on success. LEARNED, traced,
 * vertex-status and ACTIVE-degree runs:
 * GG_E_UNSUPPORTED. */
int gg_run_update(gg_run* run, const gg_update_batch* batch, int32_t more_iters, uint8_t* reset_host);

/* Host copies of the graph's in-CSR: rowptr_host int32[n+1] (required),
 * col_host int32[m] (nullable), weight_host int32[m] (nullable; GG_E_INVAL
 * when requested from a graph without weights). */
int gg_graph_get_csr(gg_graph* g, int32_t* rowptr_host, int32_t* col_host, int32_t* weight_host);

/* Arc count m of the graph's current in-CSR (it changes with updates);
 * -1 for a null graph. Host-side, no device work. */
int64_t gg_graph_num_arcs(const gg_graph* g);

/*
 * Tuning knobs of the degree-binned sweep (set directly or by gg_graph_autotune):
 * rows of degree <= small_max are processed by teams of small_team lanes
 * (4, 8, 16 or 32); rows of degree <= wave_max by one 64-lane wavefront;
 * longer rows by 256-thread workgroups, split into chunks of hub_chunk edges
 * (a multiple of 256).
 * With seg_enable, plain gathers over rows longer than small_max are split by
 * source segment (seg_vertices consecutive source ids per segment; 0 = about
 * 2 MiB of vertex values): each (row, segment) piece is reduced by blocks
 * scheduled so that one GPU die works on one segment at a time, and the pieces
 * are combined in segment order.
 * With frontier_enable, an SSSP/CC iteration whose edge set is contained in
 * the previous iteration's runs as a push from the vertices that changed in
 * the previous iteration (the active-vertex list of the vertex-centric model,
 * Sec. 2.1) when their out-degree sum times frontier_div is at most m;
 * otherwise it runs as a dense pull. Both give identical results.
 * Results do not depend on these knobs except for the rounding order of
 * PageRank sums.
 */
typedef struct {
  int32_t small_max;
  int32_t small_team;
  int32_t wave_max;
  int32_t hub_chunk;
  int32_t seg_enable;
  int32_t seg_vertices;
  int32_t frontier_enable;
  int32_t frontier_div;
} gg_tuning;

int gg_graph_get_tuning(const gg_graph* g, gg_tuning* out);
int gg_graph_set_tuning(gg_graph* g, const gg_tuning* t);

/*
 * Bounded waits of the superstep (project addition, no counterpart in the
 * paper). The workgroups that share one long row take their row prefix and
 * write offset from the row's earlier chunks, polling words those chunks
 * publish; every such wait ends by construction. A wait that still reaches
 * `polls` polls gives up: the chunk writes no active edge and no active
 * count, and the step that ran the superstep returns GG_E_DEVICE with its
 * results undefined (the next run on the graph starts clean). The default is
 * 2^20 polls; polls <= 0 makes every such wait give up at once, so that
 * callers can test their handling of that failure. GG_E_STATE while a run is
 * active on the graph.
 */
int gg_graph_set_wait_limit(gg_graph* g, int32_t polls);

/*
 * Captured schedules (project addition). A whole run (gg_exact_run,
 * gg_approx_run) of PR, PPR or BP under EXACT, SP or SMS has a static
 * iteration schedule: once the run has begun, no host decision depends on
 * device data. Its iterations are captured into a HIP graph on the graph's
 * private stream the first time and replayed by later runs with the same
 * parameters, scheme, sample ratio, seed and tuning, as long as the graph's
 * buffers and binning are unchanged (an update, a new tuning or a grown
 * workspace captures again). Results are identical either way; the launch
 * is ordered after the work already on the graph's stream and before what
 * follows (a union of parts included: one launch for the whole union). Not
 * while profiling, nor with vertex status, the ACTIVE degree or traces. enable = 1 turns capture on; it is off by default,
 * because on gfx950 a replayed schedule was measured no faster than the
 * same kernels launched one by one (the gaps between dependent kernels are
 * the device's, and the graph launch adds its own). GG_E_STATE while a run
 * is active on the graph.
 */
int gg_graph_set_capture(gg_graph* g, int enable);

/*
 * Autotuner (project addition): picks the tuning knobs for one workload on
 * this graph by timing that workload. With n_queries = 0 the workload is a
 * single run (gg_exact_run when policy is NULL or EXACT, else gg_approx_run
 * with sample_ratio and policy); with n_queries > 0 it is gg_batch_run over
 * sources_host. Coordinate descent over small_max, small_team, wave_max,
 * hub_chunk, seg_vertices and frontier_div (only the knobs the workload
 * reads), two passes at most; each candidate is timed as the median device
 * time of reps runs after one warm-up run (1 <= reps <= 64), and replaces
 * the best one only when at least 1% faster. The best tuning is left set on
 * the graph and returned in *out_best (*out_ms: its time, nullable). Keep
 * params->iters small: every candidate runs the workload reps + 1 times.
 * Results do not depend on the tuning except for the rounding order of
 * PageRank sums. On error the graph keeps its previous tuning.
 */
int gg_graph_autotune(gg_graph* g, const gg_app_params* params, double sample_ratio,
                      const gg_correction_policy* policy, int32_t n_queries, const int32_t* sources_host,
                      int32_t reps, gg_tuning* out_best, double* out_ms);

/*
 * Kernel profiling. When enabled, every launch of the sweep's main kernels is
 * bracketed by HIP events on the graph's stream, and its algorithmic bytes
 * are counted: per gathered edge, the 4-byte edge word plus the 4-byte
 * source value; per processed row, its list entry, row offset, (active count
 * in approximate mode,) out-degree or own value, and the value written.
 * kind: 0 = accurate gather, 1 = approximate gather, 2 = superstep,
 * 3 = frontier push (SSSP/CC; per pushed edge: edge id, destination, weight
 * and flag words and the atomic on the target), 4 = partial superstep of the
 * learned policy (approximate gather of the unselected rows plus the
 * superstep of the selected ones).
 * gg_graph_set_profiling(g, 1) clears the counters. gg_graph_get_profile
 * synchronizes the stream and reports the totals for (kind, app).
 */
typedef struct {
  int64_t launches;
  double total_ms;     /* sum of the event-measured launch durations */
  double alg_bytes;    /* sum of the algorithmic bytes of those launches */
  int64_t edges;       /* edges gathered by those launches */
} gg_kernel_profile;

int gg_graph_set_profiling(gg_graph* g, int enable);
int gg_graph_get_profile(gg_graph* g, int kind, int app, gg_kernel_profile* out);

/*
 * Learned correction network (GG_POLICY_LEARNED). An 8-64-64-1 ReLU MLP over
 * per-vertex features, all computed in binary32 and rounded to bfloat16
 * (round to nearest even):
 *   f0 = lg(1 + out-degree), f1 = lg(1 + in-degree), where lg(y) = L +
 *        (y - 2^L) / 2^L with L = floor(log2 y);
 *   f2 = active in-edges / in-degree (0 without in-edges);
 *   f3 = delta of the vertex state between iterations i-1 and i-2, f4 the
 *        same between i-2 and i-3 (0 before iteration 0); the state is the
 *        binary32 contribution x_v / outdeg_v for PR/PPR (x_v without
 *        out-edges; delta = relative change capped at 1), the distance for
 *        SSSP (relative decrease; 1 when it becomes finite, 0 while
 *        infinite), the label for CC (1 iff it changed);
 *   f5..f7 = 0.
 * Layers: h1 = bf16(relu(x W1 + b1)), h2 = bf16(relu(h1 W2 + b2)),
 * logit = h2 w3 + b3, with bfloat16 W1, W2, w3 and binary32 biases and
 * accumulation (matrix cores). Parameters in host order (GG_MLP_PARAMS
 * binary32): W1 [8][64], b1 [64], W2 [64][64], b2 [64], w3 [64], b3.
 *
 * The drift label of a vertex at a full superstep is 1 when its accurate
 * update differs from the approximate update its current flags would give:
 * PR/PPR binary32 contributions differing by more than label_eps relative,
 * SSSP a shorter distance, CC a smaller label.
 *
 * Training minimises the mean weighted binary cross-entropy on the logit
 * (weight pos_weight on label-1 samples) with Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) on the binary32 master parameters; the bfloat16 copies are
 * refreshed after every step.
 *
 * All MLP calls run on the network's stream (set at creation); pointers
 * marked _dev are device pointers on that device. A gg_mlp may be used by a
 * run on any graph of the same device; the run reads it on the graph's
 * stream, so the caller orders the two streams (or uses one stream).
 */
#define GG_MLP_IN 8
#define GG_MLP_HIDDEN 64
#define GG_MLP_PARAMS 4801

/* He-uniform initial weights from a SplitMix64 stream seeded by seed, zero
   biases. */
int gg_mlp_create(void* hip_stream, uint64_t seed, gg_mlp** out);
void gg_mlp_free(gg_mlp* mlp);
/* Host arrays of GG_MLP_PARAMS binary32 values; set resets Adam's state. */
int gg_mlp_set_weights(gg_mlp* mlp, const float* params_host);
int gg_mlp_get_weights(gg_mlp* mlp, float* params_host);
/* Logits of n samples: feat_dev [n][8] bfloat16 bits (8-byte aligned, else
   GG_E_INVAL), logits_dev float[n]. */
int gg_mlp_forward(gg_mlp* mlp, const uint16_t* feat_dev, int64_t n, float* logits_dev);
/* Gradient of the mean loss over n samples (labels 0/1 as float) into
   grad_dev[0..GG_MLP_PARAMS), and the loss sum into grad_dev[GG_MLP_PARAMS]. */
int gg_mlp_loss_grad(gg_mlp* mlp, const uint16_t* feat_dev, const float* label_dev, int64_t n, float pos_weight,
                     float* grad_dev);
/* One Adam step with the gradient in grad_dev (GG_MLP_PARAMS floats). */
int gg_mlp_adam_step(gg_mlp* mlp, const float* grad_dev, float lr);
/* epochs passes over the trace in mini-batches of `batch` consecutive
   samples, batch order shuffled per epoch (SplitMix64 Fisher-Yates on seed);
   epoch_loss_host (nullable) receives each epoch's mean loss. */
int gg_mlp_train(gg_mlp* mlp, const gg_trace* trace, int32_t epochs, int32_t batch, float lr, float pos_weight,
                 uint64_t seed, float* epoch_loss_host);

/* A device-resident trace of (features, drift label) samples, on the current
   device. Appends stop at capacity; the samples that did not fit are
   counted as dropped. */
int gg_trace_create(int64_t capacity, gg_trace** out);
void gg_trace_free(gg_trace* trace);
int gg_trace_clear(gg_trace* trace);
int gg_trace_info(gg_trace* trace, int64_t* size, int64_t* positives, int64_t* dropped);
/* Copies samples [first, first + count) to host: feat [count][8] bfloat16
   bits, labels float [count] (either nullable). */
int gg_trace_export(gg_trace* trace, int64_t first, int64_t count, uint16_t* feat_host, float* label_host);

#ifdef __cplusplus
}
#endif

#endif /* GG_H */
