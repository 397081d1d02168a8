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

#define GG_VERSION 1

typedef enum {
  GG_OK = 0,
  GG_E_INVAL = -1,       /* null pointer, unknown enum, sigma outside [0,1], theta < 0, alpha < 0, ... */
  GG_E_RANGE = -2,       /* malformed CSR, vertex id out of range, n or m too large, weight outside [0,255] */
  GG_E_NOMEM = -3,       /* device or host allocation failed */
  GG_E_DEVICE = -4,      /* HIP runtime error; gg_last_error() holds its text */
  GG_E_UNSUPPORTED = -5, /* valid request that this build does not implement */
  GG_E_STATE = -6        /* call not valid in the current state of the handle */
} gg_status;

/* Vertex programs [Sec. 4.1]. PR = PageRank (Alg. 2); PPR = personalized
   PageRank from a source; SSSP = single-source shortest paths; CC = weakly
   connected components by minimum-label propagation (load the symmetrized
   graph). */
typedef enum { GG_APP_PR = 0, GG_APP_SSSP = 1, GG_APP_CC = 2, GG_APP_PPR = 3 } gg_app;

/* Correction schemes: EXACT = accurate mode in every iteration (the baseline
   of Sec. 5); SP = sparsified for the whole run; SMS = approximate for alpha
   iterations then accurate for the rest; GG = adaptive correction [Sec. 3.4]. */
typedef enum { GG_POLICY_EXACT = 0, GG_POLICY_SP = 1, GG_POLICY_SMS = 2, GG_POLICY_GG = 3 } gg_policy_kind;

/* SSSP/CC termination for non-exact schemes: FIXED_ITERS runs exactly
   gg_app_params.iters iterations (the same count as the exact baseline,
   Sec. 5); FIXED_POINT stops after a no-change iteration that no later
   iteration can follow differently (an accurate one, or any SP one). Exact
   runs always stop at their first no-change iteration. */
typedef enum { GG_STOP_FIXED_ITERS = 0, GG_STOP_FIXED_POINT = 1 } gg_stop;

/* PageRank edge influence [Alg. 2, GG-Gather]: PREFIX = contribution over the
   running sum of the row in CSR order; TOTAL = contribution over the row sum. */
typedef enum { GG_INFL_PREFIX = 0, GG_INFL_TOTAL = 1 } gg_influence;

/* Flag update at a superstep: REPLACE deactivates every edge that does not
   qualify [Sec. 3.4]; UNION keeps previously active edges. */
typedef enum { GG_MASK_REPLACE = 0, GG_MASK_UNION = 1 } gg_mask_update;

/* PageRank mass of vertices without out-edges: spread over all vertices
   (UNIFORM; sent to the source for PPR) or dropped (NONE). */
typedef enum { GG_DANGLING_UNIFORM = 0, GG_DANGLING_NONE = 1 } gg_dangling;

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
  int32_t iters;     /* PR/PPR: iterations T; SSSP/CC FIXED_ITERS: iterations */
  int32_t max_iters; /* SSSP/CC fixed-point runs: cap on iterations (> 0) */
  int32_t source;    /* SSSP/PPR source vertex */
  int32_t dangling;  /* gg_dangling */
} gg_app_params;

typedef struct {
  int32_t kind;        /* gg_policy_kind */
  int32_t alpha;       /* approximate window, >= 0 [Sec. 3.4] */
  double theta;        /* influence threshold, 0 <= theta < 65536 [Sec. 3.4] */
  uint64_t seed;       /* sampling seed */
  int32_t influence;   /* gg_influence (PR/PPR) */
  int32_t mask_update; /* gg_mask_update */
  int32_t stop;        /* gg_stop (SSSP/CC) */
} gg_correction_policy;

typedef struct {
  int32_t iterations;       /* iterations executed */
  int32_t supersteps;       /* flag re-selections executed */
  int64_t edges_gathered;   /* sum over iterations of the edges gathered */
  int64_t active_edges;     /* active edges at the end of the run */
  double device_ms;         /* device time of the run (HIP events on the graph's stream) */
  int64_t edges_processed;  /* edges actually read (frontier iterations read fewer) */
  int32_t sparse_iterations;/* SSSP/CC iterations run as frontier pushes */
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
} gg_step_info;

typedef struct gg_graph gg_graph;
typedef struct gg_run gg_run;

int gg_version(void);
const char* gg_last_error(void);

/*
 * Load a graph (the "graph_load_csr" step). The library computes the
 * out-degrees and the degree-binned work lists of the in-CSR, and for SSSP a
 * packed (weight << 24 | source) edge array. Host inputs are copied to device
 * memory; device inputs (GG_CSR_DEVICE_PTRS) are borrowed. The structure is
 * validated unless GG_CSR_SKIP_VALIDATE is set (GG_E_RANGE on failure).
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
 * EXACT, and SP with one sampled edge set shared by all queries (ratio
 * sample_ratio, policy->seed). PPR runs params->iters iterations, all
 * captured in one HIP graph launched once; exact SSSP stops after the first
 * iteration in which no query changed (at most params->max_iters), captured
 * 32 iterations per graph launch with device-side early exit; SP SSSP runs
 * params->iters iterations. Every query's result equals the corresponding
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
int gg_run_stats_get(gg_run* run, gg_run_stats* stats);
void gg_run_end(gg_run* run);

/*
 * Tuning knobs of the degree-binned sweep (the autotuner sets them):
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
 * Kernel profiling. When enabled, every launch of the sweep's main kernels is
 * bracketed by HIP events on the graph's stream, and its algorithmic bytes
 * are counted: per gathered edge, the 4-byte edge word plus the 4-byte
 * source value; per processed row, its list entry, row offset, (active count
 * in approximate mode,) out-degree or own value, and the value written.
 * kind: 0 = accurate gather, 1 = approximate gather, 2 = superstep,
 * 3 = frontier push (SSSP/CC; per pushed edge: edge id, destination, weight
 * and flag words and the atomic on the target).
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

#ifdef __cplusplus
}
#endif

#endif /* GG_H */
