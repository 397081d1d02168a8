/*
 * CPU oracle for GraphGuess (Ramezani, Kandemir, Sivasubramaniam,
 * "GraphGuess: Approximate Graph Processing System with Adaptive Correction",
 * arXiv 2104.10039).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, single-threaded
 * implementation of the exact and the sampled-plus-corrected vertex-centric
 * iterations, used to check the GPU library. Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it. The GPU library never
 * links, includes or calls anything here, and nothing here comes from it.
 *
 * Graph: canonical in-CSR (pull model, Sec. 3.1). Row u holds the in-edges
 * v -> u; edge id e is the position in the CSR.
 *
 * Values: PageRank in binary64; SSSP distances uint32 with INF = 0xFFFFFFFF;
 * CC labels int32.
 */
#ifndef GG_ORACLE_H
#define GG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GGO_PR = 0, GGO_SSSP = 1, GGO_CC = 2, GGO_PPR = 3, GGO_BP = 4 };
/* BP (belief propagation, Sec. 4.1, whose model the paper does not give):
   a pairwise binary Markov random field on the graph. Vertex u has prior
   log-odds prior[u]; every edge v -> u couples the two endpoints with the
   potential psi(x, y) = (1 + coupling) / 2 if x == y, (1 - coupling) / 2
   otherwise, 0 <= coupling < 1. Each iteration, in the vertex-centric pull
   model, v sends u the message m(x) = sum_y psi(x, y) b_v(y) built from its
   current belief b_v (no exclusion of u's own message), and u's new belief
   is its prior times the product of its incoming messages. The value of a
   vertex is the log-odds of its belief; the gather sums the log-ratios
   log(m(1) / m(0)) over the row's edge set. */
/* Correction schemes: EXACT = accurate mode every iteration (the baseline of
   Sec. 5); SP = sparsified only; SMS = static mode switch; GG = adaptive
   correction with periodic supersteps (Sec. 3.4, Sec. 5.2). */
enum { GGO_EXACT = 0, GGO_SP = 1, GGO_SMS = 2, GGO_GG = 3, GGO_LEARNED = 4 };
/* LEARNED (not in the paper): GG's schedule, but at a correction step an MLP
   over per-vertex features selects the rows S that are corrected (gathered
   over all in-edges, flags re-selected); the other rows take an approximate
   iteration. A full superstep replaces it every fallback_k-th correction
   step (fallback_k > 0) and whenever the rows of S hold more than rho * m
   in-edges (a partial superstep would then cost more than a full one). */
/* Kind of an executed iteration. */
enum { GGO_KIND_APPROX = 0, GGO_KIND_ACCURATE = 1, GGO_KIND_FULL = 2, GGO_KIND_PARTIAL = 3 };
#define GGO_MLP_IN 8
#define GGO_MLP_HIDDEN 64
/* Parameter vector: W1 [8][64], b1 [64], W2 [64][64], b2 [64], w3 [64], b3. */
#define GGO_MLP_PARAMS \
  (GGO_MLP_IN * GGO_MLP_HIDDEN + GGO_MLP_HIDDEN + GGO_MLP_HIDDEN * GGO_MLP_HIDDEN + GGO_MLP_HIDDEN + GGO_MLP_HIDDEN + 1)
enum { GGO_STOP_FIXED_ITERS = 0, GGO_STOP_FIXED_POINT = 1 };
/* PUSH (SSSP/CC): influence in push order, the destination's running value
   starting at its own value before the superstep instead of at INF. */
enum { GGO_INFL_PREFIX = 0, GGO_INFL_TOTAL = 1, GGO_INFL_PUSH = 2 };
enum { GGO_MASK_REPLACE = 0, GGO_MASK_UNION = 1 };
enum { GGO_DANGLING_UNIFORM = 0, GGO_DANGLING_NONE = 1 };
/* PR/PPR out-degree in approximate iterations: the full graph's (FULL) or
   the count of active out-edges (ACTIVE: PageRank of the sparsified graph,
   whose vertices without active out-edges are dangling). */
enum { GGO_DEGREE_FULL = 0, GGO_DEGREE_ACTIVE = 1 };
/* Vertex status (GG-VStatus, Alg. 2) for PR/PPR: NONE = every vertex is
   processed in every iteration; ABS = a vertex is active after an iteration
   iff its value moved by more than eps; REL = by more than eps times its
   previous value. Approximate iterations after the first recompute only
   the rows with an active in-edge from an active vertex (the active-vertex
   list of the vertex-centric model, Sec. 2.1, which starts with every
   vertex); the others keep their value. Accurate iterations recompute
   every row. */
enum { GGO_VSTATUS_NONE = 0, GGO_VSTATUS_ABS = 1, GGO_VSTATUS_REL = 2 };

#define GGO_INF_U32 0xFFFFFFFFu

typedef struct {
  int32_t n;
  int64_t m;
  const int32_t* rowptr; /* n+1 */
  const int32_t* col;    /* m: source of each in-edge */
  const int32_t* weight; /* m or NULL; SSSP requires it, values in [0, 255] */
} ggo_csr;

typedef struct {
  int32_t app;        /* GGO_PR / GGO_SSSP / GGO_CC / GGO_PPR */
  double damping;     /* PR/PPR d */
  int32_t iters;      /* T: iterations for PR/PPR and for FIXED_ITERS runs */
  int32_t max_iters;  /* cap for fixed-point runs */
  int32_t source;     /* SSSP/PPR source */
  int32_t dangling;   /* GGO_DANGLING_* */
  int32_t pr_degree;  /* GGO_DEGREE_* (PR/PPR) */
  double coupling;    /* BP: edge coupling in [0, 1) */
  const double* prior;/* BP: n prior log-odds */
} ggo_app_params;

typedef struct {
  int32_t kind;        /* GGO_EXACT / GGO_SP / GGO_SMS / GGO_GG / GGO_LEARNED */
  int32_t alpha;       /* approximate window */
  double theta;        /* influence threshold */
  double sigma;        /* sparsification parameter (sampling ratio) */
  uint64_t seed;       /* sampling seed */
  int32_t influence;   /* GGO_INFL_* */
  int32_t mask_update; /* GGO_MASK_* */
  int32_t stop;        /* GGO_STOP_* (SSSP/CC) */
  const double* mlp;   /* LEARNED: GGO_MLP_PARAMS binary32 master values */
  double tau;          /* LEARNED: select v iff binary32(logit_v) > binary32(tau) */
  double rho;          /* LEARNED: full superstep when the rows of S hold > rho * m in-edges */
  int32_t fallback_k;  /* LEARNED: every k-th correction step is full (0: never) */
  int32_t trace;       /* 1: features and drift labels at every full superstep */
  double label_eps;    /* PR/PPR drift label: relative contribution change */
  /* GG / LEARNED with decoupled = 1: the first superstep follows alpha0
     approximate iterations and uses threshold theta0; later ones recur
     every alpha+1 iterations after it with theta (Sec. 3.4, last
     paragraph). decoupled = 0: alpha and theta throughout. */
  int32_t decoupled;
  int32_t alpha0;
  double theta0;
  int32_t vstatus;     /* GGO_VSTATUS_* (PR/PPR) */
  double eps;          /* its epsilon, >= 0 */
} ggo_policy;

typedef struct {
  int32_t iter;        /* 1-based index of the iteration just executed */
  int32_t accurate;    /* 1 if accurate mode */
  int32_t superstep;   /* 1 if the edge flags were re-selected after it */
  int64_t edges;       /* edges gathered */
  int64_t changed;     /* vertices whose value changed */
  int64_t active_edges;/* active edges after the iteration */
  int32_t kind;        /* GGO_KIND_* */
  int64_t selected;    /* LEARNED correction steps: |S|; else -1 */
} ggo_step_info;

typedef struct ggo_run ggo_run;

/* Philox4x64-10 (Salmon et al., SC'11), exposed for tests. */
void ggo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* The 32-bit sampling draw for edge e at epoch t under seed s. */
uint32_t ggo_sample_draw(uint64_t seed, uint64_t epoch, int64_t e);
/* Keep threshold for ratio sigma in [0, 1]: floor(sigma * 2^32 + 1/2). */
uint64_t ggo_keep_threshold(double sigma);

/* Returns NULL on invalid arguments (message via ggo_last_error). */
ggo_run* ggo_begin(const ggo_csr* g, const ggo_app_params* app, const ggo_policy* pol);
/* Executes one iteration. Returns 1 if executed, 0 if the run had ended. */
int ggo_step(ggo_run* r, ggo_step_info* info);
int ggo_done(const ggo_run* r);
int32_t ggo_iterations(const ggo_run* r);
int64_t ggo_edges_total(const ggo_run* r);
/* PR/PPR: double[n]; BP: double[n] log-odds; SSSP: uint32[n]; CC: int32[n]. */
void ggo_get_values(const ggo_run* r, void* out);
/* One byte per edge: current active flag. */
void ggo_get_mask(const ggo_run* r, uint8_t* out);
/* BP message of a sender with belief log-odds L: log(m(1) / m(0)), from
   the definition m(x) = sum_y psi(x, y) b(y); exposed for the pins. */
double ggo_bp_message(double L, double coupling);
/* Per-edge influence computed at the last superstep (PR: the ratio; BP: the
   same on magnitudes, |message| / |running sum|; SSSP:
   relative improvement, 1 for the first finite candidate, -1 when not
   assessable; CC: 1/0). */
void ggo_get_influence(const ggo_run* r, double* out);
/* Replace the current edge flags (one byte per edge, nonzero = active), for
   the replay check: after a superstep whose floating-point decisions the
   GPU took differently within rounding, the oracle continues from the GPU's
   flags. */
void ggo_set_mask(ggo_run* r, const uint8_t* mask);
/* Vertex status after the last iteration (one byte per vertex; all 1 before
   the first), and its replacement for the replay check. */
void ggo_get_vactive(const ggo_run* r, uint8_t* out);
void ggo_set_vactive(ggo_run* r, const uint8_t* in);
/* Features [n][8] (bfloat16 bits) of the last correction or traced step. */
void ggo_get_features(const ggo_run* r, uint16_t* out);
/* Selection and logits of this step (LEARNED correction steps); 0 if none. */
int ggo_get_selection(const ggo_run* r, uint8_t* sel, double* logits);
/* Drift labels of this step (traced full supersteps); 0 if none. */
int ggo_get_labels(const ggo_run* r, uint8_t* out);
/* Dynamic graphs (the paper states GraphGuess applies to changing graphs
   and evaluates none; the reading is the oracle's): the run continues on
   g_new, the graph after an update batch, with the same vertex set.
   old_of_new[e] is the old edge that new edge e continues, or -1 for an
   inserted edge; deleted_old[e] is 1 for every old edge the batch removed.
   Surviving edges keep their flags and inserted edges are active.
   PR/PPR/BP values continue (the next iteration divides by the new
   out-degrees). SSSP/CC after a deletion: a converged exact run resets the
   vertices whose value may rest on a deleted edge (a taint closure over
   supporting edges), any other run restarts from the initial values.
   more_iters (>= 0) extends the run: fixed-count runs raise their
   iteration count, fixed-point runs their cap, and the run resumes.
   LEARNED, traced, vertex-status and ACTIVE-degree runs are refused.
   g_new's arrays must outlive the run. Returns 0, or -1 with a message. */
int ggo_run_update(ggo_run* r, const ggo_csr* g_new, const int64_t* old_of_new, const uint8_t* deleted_old,
                   int32_t more_iters);
/* Vertices reset by the last update (one byte per vertex). */
void ggo_get_reset(const ggo_run* r, uint8_t* out);
void ggo_end(ggo_run* r);

/* bfloat16: round to nearest even from binary32 (NaN -> 0x7FC0), and back. */
uint16_t ggo_bf16_bits(float f);
float ggo_bf16_value(uint16_t b);
void ggo_bf16_array(const float* in, uint16_t* out, int64_t n);
/* Feature helpers (binary32): piecewise-linear log2 of y >= 1, and the delta
   of two state words (PR/PPR: binary32 contribution bits; SSSP: distance;
   CC: label). */
float ggo_lg_feature(int64_t y);
float ggo_delta_feature(int32_t app, uint32_t now, uint32_t before);
/* MLP: logits of n samples (features [n][8] bfloat16 bits); rounding = 1
   follows the GPU's rounding points, 0 is plain binary64. */
void ggo_mlp_forward(const double* params, const uint16_t* feat, int64_t n, int rounding, double* logits);
/* Mean weighted BCE-with-logits loss and its gradient (GGO_MLP_PARAMS). */
void ggo_mlp_loss_grad(const double* params, const uint16_t* feat, const float* label, int64_t n,
                       double pos_weight, int rounding, double* grad, double* loss);
/* One Adam step at step number t >= 1 (beta1 0.9, beta2 0.999, eps 1e-8). */
void ggo_adam_step(double* p, double* m, double* v, const double* grad, int64_t count, double lr, int64_t t);
const char* ggo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
