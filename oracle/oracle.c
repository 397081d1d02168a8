/*
 * CPU oracle for GraphGuess (arXiv 2104.10039). TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the GPU library. Single-threaded and deliberately plain: every
 * vertex is processed in every iteration, edges are walked in CSR order, and
 * there is no blocking, fusion or reordering.
 *
 * What is computed (paper sections in brackets):
 *  - Pull-based vertex program: gather over in-edges, apply, vertex status
 *    [Sec. 2.1 Alg. 1; Sec. 3.1 Alg. 2]. Synchronous (Jacobi/BSP) updates:
 *    iteration i reads only the values and flags left by iteration i-1.
 *  - A flag per edge [Sec. 3.3]; accurate mode gathers over every in-edge,
 *    approximate mode only over active in-edges [Sec. 3.3].
 *  - Initial sparsification: each edge kept independently with probability
 *    sigma [Sec. 2.3 Fig. 1a; Sec. 3.4], decided by a counter-based draw.
 *  - Adaptive correction: alpha approximate iterations, then a superstep (an
 *    accurate iteration) whose edge influences re-select the active edges
 *    with threshold theta, deactivating all others; supersteps recur with the
 *    same alpha [Sec. 3.4].
 *  - SP and SMS schemes [Sec. 5.2].
 *  - Dynamic graphs: a run continues on the graph after an update batch
 *    (ggo_run_update; Sec. 1 states the method applies to changing graphs).
 *
 * Readings where the paper is silent (each is a flag where a variant exists):
 *  - Iteration i (1-based) is accurate for GG iff i mod (alpha+1) == 0; for
 *    SMS iff i >= alpha+1.
 *  - PR edge influence: running prefix in CSR order with the accumulator
 *    starting at zero; influence of the k-th edge = c_k / P_k where c is the
 *    contribution x_v / outdeg_v and P_k the running sum [Alg. 2, GG-Gather].
 *    The contribution entering this decision is rounded to binary32 and the
 *    running sum is binary64 (the precision in which the GPU library takes
 *    the same decision). TOTAL variant: c_k / (row sum).
 *  - EStatus is strict: active iff influence > theta [Alg. 2, GG-EStatus].
 *  - PR dangling mass D (vertices without out-edges) is spread uniformly
 *    (UNIFORM) or dropped (NONE); PPR sends it to the source.
 *  - SSSP influence: relative improvement of the running minimum,
 *    (r - new) / r > theta, compared in integers as (r-new)*2^16 > theta_q*r
 *    with theta_q = floor(theta*2^16 + 1/2); the first finite candidate of a
 *    row is always active; an edge whose source is unreached is not assessed
 *    and keeps its flag.
 *  - CC influence is binary: the edge is active iff it strictly lowers the
 *    running minimum label [Sec. 5.2, WCC].
 *  - SSSP/CC exact runs stop after the first iteration that changes nothing;
 *    approximate runs either run a fixed number of iterations or stop after a
 *    no-change iteration that no later iteration can follow differently.
 *
 * Belief propagation [Sec. 4.1 lists it; the paper defines neither its
 * potentials nor its messages]: the reading taken is a binary pairwise
 * Markov random field with a homophily coupling and per-vertex priors.
 * A vertex's value is the log-odds of its belief; each iteration every
 * in-neighbour v sends the message m(x) = sum_y psi(x, y) b_v(y), built from
 * v's current belief, and the new log-odds are the prior plus the sum of
 * the log-ratios log(m(1) / m(0)) over the row's edge set. Influence of an
 * edge at a superstep: the magnitude of its (binary32-rounded) log-ratio
 * over the magnitude of the row's running sum, in CSR order [Alg. 2 with
 * magnitudes, since log-ratios take both signs].
 *
 * Variants the paper mentions without fixing them (each a flag):
 *  - Decoupled parameters: the first superstep after alpha0 approximate
 *    iterations with threshold theta0, later ones every alpha+1 iterations
 *    with theta [Sec. 3.4, last paragraph].
 *  - ACTIVE out-degree: in approximate iterations PageRank divides by the
 *    count of active out-edges and treats vertices without one as dangling,
 *    i.e. it is PageRank of the sparsified graph [Alg. 2 reads v.degree].
 *  - GG-VStatus with epsilon > 0 [Alg. 2]: approximate PageRank iterations
 *    after the first recompute only rows with an active in-edge from a
 *    vertex whose value moved by more than epsilon (absolute, or relative to
 *    its old value) in the previous iteration; the active-vertex list of
 *    Sec. 2.1, which starts with every vertex.
 *
 * A project addition, not part of the paper: a LEARNED policy keeps GG's
 * correction schedule but lets a small MLP pick the rows corrected at each
 * correction step (a partial superstep), with GG's full superstep as
 * fallback every k-th correction step or when the selected rows hold more
 * than rho * m in-edges. Its features, the network, the loss and Adam are
 * plain definitions written out below; the drift label of a traced full
 * superstep compares the accurate update with the approximate one the flags
 * alone would have given.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static __thread char g_err[256];

static void set_err(const char* msg) {
  strncpy(g_err, msg, sizeof(g_err) - 1);
  g_err[sizeof(g_err) - 1] = 0;
}

const char* ggo_last_error(void) { return g_err; }

/* ---------------------------------------------------------------------------
 * Philox4x64-10, as defined by Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3" (SC'11): 10 rounds of two 64x64->128
 * multiplies with a Weyl-sequence key schedule.
 * ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void ggo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* Draw for edge e: the Philox block e/8 (counter (e/8, epoch, 0, 0), key
   (seed, 0)) yields 8 32-bit halves; edge e takes half e mod 8, low half of
   word 0 first. */
uint32_t ggo_sample_draw(uint64_t seed, uint64_t epoch, int64_t e) {
  uint64_t ctr[4] = {(uint64_t)e >> 3, epoch, 0, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t w[4];
  ggo_philox4x64_10(ctr, key, w);
  int j = (int)(e & 7);
  uint64_t word = w[j >> 1];
  return (j & 1) ? (uint32_t)(word >> 32) : (uint32_t)(word & 0xFFFFFFFFu);
}

uint64_t ggo_keep_threshold(double sigma) {
  return (uint64_t)floor(sigma * 4294967296.0 + 0.5);
}


/* ---------------------------------------------------------------------------
 * BF16 (bfloat16) rounding and the correction MLP. The MLP scores vertices
 * for drift; it is a project addition, not part of the paper's method, and
 * is written here as the plain definition of a 8-64-64-1 ReLU network.
 * ------------------------------------------------------------------------- */

/* Round-to-nearest-even from binary32 to bfloat16 bits (NaN -> 0x7FC0). */
uint16_t ggo_bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

void ggo_bf16_array(const float* in, uint16_t* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = ggo_bf16_bits(in[i]);
}

float ggo_bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

/* binary64 -> binary32 -> bfloat16, the two roundings the GPU performs. */
static double to_bf16(double v) { return (double)ggo_bf16_value(ggo_bf16_bits((float)v)); }
static double to_f32(double v) { return (double)(float)v; }

#define P_W1 0
#define P_B1 (P_W1 + GGO_MLP_IN * GGO_MLP_HIDDEN)
#define P_W2 (P_B1 + GGO_MLP_HIDDEN)
#define P_B2 (P_W2 + GGO_MLP_HIDDEN * GGO_MLP_HIDDEN)
#define P_W3 (P_B2 + GGO_MLP_HIDDEN)
#define P_B3 (P_W3 + GGO_MLP_HIDDEN)

/* Forward pass of one sample. rounding = 1 rounds where the GPU kernels do:
   weights W1, W2, w3 to bfloat16, each pre-activation to binary32 before its
   bias (binary32) is added, the hidden activations to bfloat16; rounding = 0
   is plain binary64 throughout. Keeps z1, z2, h1, h2 for the backward pass. */
typedef struct {
  double z1[GGO_MLP_HIDDEN], h1[GGO_MLP_HIDDEN];
  double z2[GGO_MLP_HIDDEN], h2[GGO_MLP_HIDDEN];
  double z;
} mlp_cache;

static double wt(const double* p, int i, int rounding) { return rounding ? to_bf16(p[i]) : p[i]; }
static double bs(const double* p, int i, int rounding) { return rounding ? to_f32(p[i]) : p[i]; }

static double mlp_forward(const double* p, const double* x, int rounding, mlp_cache* c) {
  for (int j = 0; j < GGO_MLP_HIDDEN; ++j) {
    double a = 0.0;
    for (int f = 0; f < GGO_MLP_IN; ++f) a += x[f] * wt(p, P_W1 + f * GGO_MLP_HIDDEN + j, rounding);
    double z = rounding ? to_f32(to_f32(a) + bs(p, P_B1 + j, 1)) : a + p[P_B1 + j];
    c->z1[j] = z;
    c->h1[j] = z > 0.0 ? (rounding ? to_bf16(z) : z) : 0.0;
  }
  for (int j = 0; j < GGO_MLP_HIDDEN; ++j) {
    double a = 0.0;
    for (int k = 0; k < GGO_MLP_HIDDEN; ++k) a += c->h1[k] * wt(p, P_W2 + k * GGO_MLP_HIDDEN + j, rounding);
    double z = rounding ? to_f32(to_f32(a) + bs(p, P_B2 + j, 1)) : a + p[P_B2 + j];
    c->z2[j] = z;
    c->h2[j] = z > 0.0 ? (rounding ? to_bf16(z) : z) : 0.0;
  }
  double a = 0.0;
  for (int j = 0; j < GGO_MLP_HIDDEN; ++j) a += c->h2[j] * wt(p, P_W3 + j, rounding);
  c->z = rounding ? to_f32(to_f32(a) + bs(p, P_B3, 1)) : a + p[P_B3];
  return c->z;
}

static void feat_to_double(const uint16_t* f8, double* x) {
  for (int f = 0; f < GGO_MLP_IN; ++f) x[f] = (double)ggo_bf16_value(f8[f]);
}

void ggo_mlp_forward(const double* params, const uint16_t* feat, int64_t n, int rounding, double* logits) {
  mlp_cache c;
  double x[GGO_MLP_IN];
  for (int64_t i = 0; i < n; ++i) {
    feat_to_double(feat + i * GGO_MLP_IN, x);
    logits[i] = mlp_forward(params, x, rounding, &c);
  }
}

/* Weighted binary cross-entropy on the logit, mean over the n samples:
   L = (1/n) sum_i w_i (softplus(z_i) - y_i z_i), w_i = pos_weight for y_i = 1.
   Gradient by the chain rule; with rounding = 1 the backward pass rounds the
   pre-activation gradients that enter the W2, W1 and hidden-layer products to
   bfloat16 (the GPU feeds them to matrix cores), and the ReLU gate reads the
   rounded activation. */
void ggo_mlp_loss_grad(const double* p, const uint16_t* feat, const float* label, int64_t n, double pos_weight,
                       int rounding, double* grad, double* loss_out) {
  memset(grad, 0, sizeof(double) * GGO_MLP_PARAMS);
  double loss = 0.0;
  mlp_cache c;
  double x[GGO_MLP_IN], g2[GGO_MLP_HIDDEN], g2r[GGO_MLP_HIDDEN], g1[GGO_MLP_HIDDEN];
  for (int64_t i = 0; i < n; ++i) {
    feat_to_double(feat + i * GGO_MLP_IN, x);
    const double z = mlp_forward(p, x, rounding, &c);
    const double y = label[i];
    const double w = y > 0.5 ? pos_weight : 1.0;
    loss += w * ((z > 0.0 ? z : 0.0) - z * y + log1p(exp(-fabs(z))));
    const double sig = 1.0 / (1.0 + exp(-z));
    const double dz = w * (sig - y) / (double)n;
    grad[P_B3] += dz;
    for (int j = 0; j < GGO_MLP_HIDDEN; ++j) {
      grad[P_W3 + j] += dz * c.h2[j];
      g2[j] = c.h2[j] > 0.0 ? dz * wt(p, P_W3 + j, rounding) : 0.0;
      g2r[j] = rounding ? to_bf16(g2[j]) : g2[j];
      grad[P_B2 + j] += g2[j];
    }
    for (int k = 0; k < GGO_MLP_HIDDEN; ++k) {
      double dh = 0.0;
      for (int j = 0; j < GGO_MLP_HIDDEN; ++j) {
        grad[P_W2 + k * GGO_MLP_HIDDEN + j] += c.h1[k] * g2r[j];
        dh += g2r[j] * wt(p, P_W2 + k * GGO_MLP_HIDDEN + j, rounding);
      }
      g1[k] = c.h1[k] > 0.0 ? dh : 0.0;
      grad[P_B1 + k] += g1[k];
    }
    for (int k = 0; k < GGO_MLP_HIDDEN; ++k) {
      const double g = rounding ? to_bf16(g1[k]) : g1[k];
      for (int f = 0; f < GGO_MLP_IN; ++f) grad[P_W1 + f * GGO_MLP_HIDDEN + k] += x[f] * g;
    }
  }
  if (loss_out) *loss_out = n > 0 ? loss / (double)n : 0.0;
}

/* One Adam step (Kingma and Ba, ICLR'15) with beta1 = 0.9, beta2 = 0.999,
   eps = 1e-8 and bias correction at step t >= 1. */
void ggo_adam_step(double* p, double* m, double* v, const double* grad, int64_t count, double lr, int64_t t) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < count; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
    v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}

/* ---------------------------------------------------------------------------
 * Per-vertex features of the learned policy, each computed in binary32 and
 * rounded to bfloat16:
 *   0: lg(1 + out-degree)   1: lg(1 + in-degree)
 *   2: active in-edges / in-degree (0 without in-edges)
 *   3: delta(x(i-1), x(i-2))   4: delta(x(i-2), x(i-3))   5-7: zero
 * lg(y) = L + (y - 2^L) / 2^L with L = floor(log2 y), the piecewise-linear
 * base-2 logarithm, exact at powers of two. delta compares a vertex's state
 * in two consecutive iterations: PR/PPR the relative change of its binary32
 * contribution, capped at 1; SSSP the relative decrease of the distance (1
 * when it becomes finite, 0 while infinite); CC 1 iff the label changed.
 * Deltas reaching before iteration 0 are 0.
 * ------------------------------------------------------------------------- */
float ggo_lg_feature(int64_t y) {
  int L = 63 - __builtin_clzll((unsigned long long)y);
  float t = (float)(y - ((int64_t)1 << L));
  t = t / ldexpf(1.0f, L);
  return (float)L + t;
}

static float word_float(uint32_t w) {
  float f;
  memcpy(&f, &w, 4);
  return f;
}

float ggo_delta_feature(int32_t app, uint32_t now, uint32_t before) {
  if (app == GGO_PR || app == GGO_PPR) {
    const float cn = word_float(now), co = word_float(before);
    if (!(cn > 0.0f)) return 0.0f;
    const float r = fabsf(cn - co) / cn;
    return r < 1.0f ? r : 1.0f;
  }
  if (app == GGO_SSSP) {
    if (now == GGO_INF_U32) return 0.0f;
    if (before == GGO_INF_U32) return 1.0f;
    if (before == 0) return 0.0f;
    return (float)(before - now) / (float)before;
  }
  return now != before ? 1.0f : 0.0f;
}

/* ------------------------------------------------------------------------- */

/* Row modes of one iteration: APPROX gathers over the row's active in-edges,
   ACCURATE over all of them, SUPER also re-selects their flags (GG-EStatus,
   Alg. 2) from the influences of this gather. */
enum { ROW_APPROX = 0, ROW_ACCURATE = 1, ROW_SUPER = 2 };

struct ggo_run {
  ggo_csr g;
  ggo_app_params app;
  ggo_policy pol;
  int32_t* outdeg;
  int32_t* indeg;
  uint8_t* active; /* edge flags */
  double* infl;    /* influence at the last superstep (diagnostics) */
  uint8_t* mode;   /* ROW_* of every row in this iteration */
  /* values: x (current, iteration i-1), xn (next), sh (approximate shadow
     pass of a traced superstep) */
  double* pr_x;
  double* pr_xn;
  double* pr_sh;
  uint32_t* d_x;
  uint32_t* d_xn;
  uint32_t* d_sh;
  int32_t* l_x;
  int32_t* l_xn;
  int32_t* l_sh;
  /* learned policy and traces */
  uint32_t* hist[2]; /* state words of iterations i-2 and i-3 */
  int32_t hist_n;    /* how many of them exist */
  uint16_t* feat;    /* [n][8] features of the last correction step */
  double* logit;
  uint8_t* sel;
  uint8_t* label;
  int32_t corrections;
  int32_t have_sel, have_label;
  int32_t iter;
  int32_t done;
  int64_t edges_total;
  /* variants */
  int32_t* odeg_act; /* ACTIVE: active out-degree of the current flags */
  uint8_t* vact;     /* vertex status after the last iteration (GG-VStatus) */
  uint8_t* skip;     /* rows not recomputed in this iteration (GG-VStatus) */
  double theta_now;  /* threshold of this iteration's superstep */
  /* dynamic graphs */
  int32_t converged; /* an exact SSSP/CC run that ended on a no-change iteration */
  uint8_t* reset;    /* vertices reset by the last update */
};

/* Superstep (correction step) of GG and LEARNED at iteration i, 1-based:
   every (alpha+1)-th iteration; with decoupled parameters the first comes
   after alpha0 approximate iterations and the later ones every alpha+1
   iterations after it [Sec. 3.4]. */
static int is_correction(const ggo_policy* p, int32_t i) {
  if (!p->decoupled) return i % (p->alpha + 1) == 0;
  const int32_t first = p->alpha0 + 1;
  return i == first || (i > first && (i - first) % (p->alpha + 1) == 0);
}

/* Influence threshold of the superstep at iteration i. */
static double theta_at(const ggo_policy* p, int32_t i) {
  return (p->decoupled && i == p->alpha0 + 1) ? p->theta0 : p->theta;
}

/* State word of vertex u for the delta features: PR/PPR the binary32
   contribution x_u / outdeg_u (x_u without out-edges), SSSP the distance,
   CC the label. */
static uint32_t state_word(const ggo_run* r, int32_t u) {
  switch (r->app.app) {
    case GGO_PR:
    case GGO_PPR: {
      const int32_t od = r->outdeg[u];
      const float c = od > 0 ? (float)(r->pr_x[u] / od) : (float)r->pr_x[u];
      uint32_t w;
      memcpy(&w, &c, 4);
      return w;
    }
    case GGO_BP: {
      const float c = (float)ggo_bp_message(r->pr_x[u], r->app.coupling);
      uint32_t w;
      memcpy(&w, &c, 4);
      return w;
    }
    case GGO_SSSP: return r->d_x[u];
    default: return (uint32_t)r->l_x[u];
  }
}

ggo_run* ggo_begin(const ggo_csr* g, const ggo_app_params* app, const ggo_policy* pol) {
  if (!g || !app || !pol) { set_err("null argument"); return NULL; }
  if (g->n < 0 || g->m < 0 || !g->rowptr || (g->m > 0 && !g->col)) { set_err("bad csr"); return NULL; }
  if (g->rowptr[0] != 0 || g->rowptr[g->n] != g->m) { set_err("rowptr ends"); return NULL; }
  for (int32_t u = 0; u < g->n; ++u)
    if (g->rowptr[u + 1] < g->rowptr[u]) { set_err("rowptr not monotone"); return NULL; }
  for (int64_t e = 0; e < g->m; ++e)
    if (g->col[e] < 0 || g->col[e] >= g->n) { set_err("col out of range"); return NULL; }
  if (app->app < GGO_PR || app->app > GGO_BP) { set_err("bad app"); return NULL; }
  if (app->app == GGO_BP) {
    if (!app->prior || !(app->coupling >= 0.0 && app->coupling < 1.0)) {
      set_err("BP needs priors and a coupling in [0, 1)");
      return NULL;
    }
    if (pol->kind == GGO_LEARNED || pol->trace || pol->vstatus != GGO_VSTATUS_NONE ||
        app->pr_degree != GGO_DEGREE_FULL) {
      set_err("BP runs EXACT, SP, SMS or GG without traces, vertex status or ACTIVE degree");
      return NULL;
    }
  }
  if (pol->kind < GGO_EXACT || pol->kind > GGO_LEARNED) { set_err("bad policy"); return NULL; }
  if (pol->alpha < 0 || !(pol->theta >= 0) || !(pol->sigma >= 0 && pol->sigma <= 1)) {
    set_err("bad alpha/theta/sigma");
    return NULL;
  }
  if (pol->kind == GGO_LEARNED && (!pol->mlp || pol->fallback_k < 0 || !(pol->rho >= 0))) {
    set_err("LEARNED needs mlp, fallback_k >= 0, rho >= 0");
    return NULL;
  }
  if ((app->app == GGO_SSSP || app->app == GGO_PPR) && (app->source < 0 || app->source >= g->n)) {
    set_err("bad source");
    return NULL;
  }
  if (app->app == GGO_SSSP) {
    if (!g->weight) { set_err("SSSP needs weights"); return NULL; }
    if (g->n > (1 << 24)) { set_err("SSSP needs n <= 2^24"); return NULL; }
    for (int64_t e = 0; e < g->m; ++e)
      if (g->weight[e] < 0 || g->weight[e] > 255) { set_err("weight out of [0,255]"); return NULL; }
  }
  if (pol->influence == GGO_INFL_TOTAL && app->app != GGO_PR && app->app != GGO_PPR) {
    set_err("TOTAL influence is defined for PR/PPR only");
    return NULL;
  }
  if (pol->influence == GGO_INFL_PUSH && app->app != GGO_SSSP && app->app != GGO_CC) {
    set_err("PUSH influence is defined for SSSP/CC only");
    return NULL;
  }
  if (pol->influence < GGO_INFL_PREFIX || pol->influence > GGO_INFL_PUSH) { set_err("bad influence"); return NULL; }
  const int pr_app = app->app == GGO_PR || app->app == GGO_PPR;
  if (app->pr_degree != GGO_DEGREE_FULL && app->pr_degree != GGO_DEGREE_ACTIVE) { set_err("bad pr_degree"); return NULL; }
  if (app->pr_degree == GGO_DEGREE_ACTIVE && (!pr_app || pol->kind == GGO_LEARNED || pol->trace)) {
    set_err("ACTIVE degree: PR/PPR under EXACT, SP, SMS or GG without traces");
    return NULL;
  }
  if (pol->decoupled && (pol->alpha0 < 0 || !(pol->theta0 >= 0))) { set_err("bad alpha0/theta0"); return NULL; }
  if (pol->vstatus < GGO_VSTATUS_NONE || pol->vstatus > GGO_VSTATUS_REL) { set_err("bad vstatus"); return NULL; }
  if (pol->vstatus != GGO_VSTATUS_NONE && (!pr_app || !(pol->eps >= 0) || pol->kind == GGO_LEARNED || pol->trace)) {
    set_err("VStatus: PR/PPR, eps >= 0, not LEARNED, no traces");
    return NULL;
  }

  ggo_run* r = (ggo_run*)calloc(1, sizeof(ggo_run));
  r->g = *g;
  r->app = *app;
  r->pol = *pol;
  int32_t n = g->n;
  int64_t m = g->m;
  r->outdeg = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  r->indeg = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  for (int64_t e = 0; e < m; ++e) r->outdeg[g->col[e]]++;
  for (int32_t u = 0; u < n; ++u) r->indeg[u] = g->rowptr[u + 1] - g->rowptr[u];
  r->active = (uint8_t*)calloc((size_t)m + 1, 1);
  r->infl = (double*)calloc((size_t)m + 1, sizeof(double));
  r->mode = (uint8_t*)calloc((size_t)n + 1, 1);
  for (int k = 0; k < 2; ++k) r->hist[k] = (uint32_t*)calloc((size_t)n + 1, sizeof(uint32_t));
  r->feat = (uint16_t*)calloc(((size_t)n + 1) * GGO_MLP_IN, sizeof(uint16_t));
  r->logit = (double*)calloc((size_t)n + 1, sizeof(double));
  r->sel = (uint8_t*)calloc((size_t)n + 1, 1);
  r->label = (uint8_t*)calloc((size_t)n + 1, 1);
  r->odeg_act = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  r->vact = (uint8_t*)malloc((size_t)n + 1);
  memset(r->vact, 1, (size_t)n + 1); /* every vertex starts active */
  r->skip = (uint8_t*)calloc((size_t)n + 1, 1);
  r->reset = (uint8_t*)calloc((size_t)n + 1, 1);
  r->theta_now = pol->theta;

  /* Initial sparsification [Sec. 3.4]: each edge kept iff its draw falls
     below floor(sigma * 2^32 + 1/2). The exact baseline ignores the flags. */
  uint64_t keep = ggo_keep_threshold(pol->sigma);
  for (int64_t e = 0; e < m; ++e)
    r->active[e] = pol->kind == GGO_EXACT ? 1 : ((uint64_t)ggo_sample_draw(pol->seed, 0, e) < keep);

  /* Initial values. */
  switch (app->app) {
    case GGO_PR:
    case GGO_PPR:
      r->pr_x = (double*)calloc((size_t)n + 1, sizeof(double));
      r->pr_xn = (double*)calloc((size_t)n + 1, sizeof(double));
      r->pr_sh = (double*)calloc((size_t)n + 1, sizeof(double));
      if (app->app == GGO_PR)
        for (int32_t u = 0; u < n; ++u) r->pr_x[u] = 1.0 / n;
      else
        r->pr_x[app->source] = 1.0;
      break;
    case GGO_BP:
      /* every belief starts at its prior */
      r->pr_x = (double*)calloc((size_t)n + 1, sizeof(double));
      r->pr_xn = (double*)calloc((size_t)n + 1, sizeof(double));
      r->pr_sh = (double*)calloc((size_t)n + 1, sizeof(double));
      for (int32_t u = 0; u < n; ++u) r->pr_x[u] = app->prior[u];
      break;
    case GGO_SSSP:
      r->d_x = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
      r->d_xn = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
      r->d_sh = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
      for (int32_t u = 0; u < n; ++u) r->d_x[u] = GGO_INF_U32;
      r->d_x[app->source] = 0;
      break;
    case GGO_CC:
      r->l_x = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
      r->l_xn = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
      r->l_sh = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
      for (int32_t u = 0; u < n; ++u) r->l_x[u] = u;
      break;
  }
  r->iter = 0;
  r->done = (app->app == GGO_PR || app->app == GGO_PPR || app->app == GGO_BP || pol->stop == GGO_STOP_FIXED_ITERS) &&
            app->iters <= 0;
  return r;
}

/* ---------------------------------------------------------------------------
 * One PageRank / personalized PageRank pass [Alg. 2] into out[]. Gather sums
 * the contributions x_v / outdeg_v over the row's edge set; Apply computes
 * (1-d)/N + d * (sum + D/N) (PPR: teleport and dangling mass go to the
 * source). For a SUPER row each edge's influence is computed from the
 * running sum of the row, all in-edges in CSR order.
 * ------------------------------------------------------------------------- */
static void pass_pr(ggo_run* r, const uint8_t* mode, const int32_t* deg, const uint8_t* skip, double* out,
                    int64_t* edges_out, int64_t* changed_out) {
  const ggo_csr* g = &r->g;
  const int32_t n = g->n;
  const double d = r->app.damping;
  const int ppr = r->app.app == GGO_PPR;
  const int32_t s = r->app.source;
  /* deg: the out-degree this iteration divides by; vertices with none are
     dangling */
  double D = 0.0;
  if (r->app.dangling == GGO_DANGLING_UNIFORM)
    for (int32_t v = 0; v < n; ++v)
      if (deg[v] == 0) D += r->pr_x[v];

  int64_t edges = 0, changed = 0;
  for (int32_t u = 0; u < n; ++u) {
    if (skip && skip[u]) {
      /* not recomputed: keeps its value (GG-VStatus) */
      out[u] = r->pr_x[u];
      continue;
    }
    double sum = 0.0; /* gather accumulator */
    double P = 0.0;   /* running sum of binary32 contributions (influence) */
    const int32_t b = g->rowptr[u], e_end = g->rowptr[u + 1];
    for (int32_t e = b; e < e_end; ++e) {
      if (mode[u] == ROW_APPROX && !r->active[e]) continue;
      const int32_t v = g->col[e];
      sum += r->pr_x[v] / deg[v];
      ++edges;
    }
    if (mode[u] == ROW_SUPER) {
      double rowsum32 = 0.0;
      if (r->pol.influence == GGO_INFL_TOTAL)
        for (int32_t e = b; e < e_end; ++e) {
          const int32_t v = g->col[e];
          rowsum32 += (double)(float)(r->pr_x[v] / r->outdeg[v]);
        }
      for (int32_t e = b; e < e_end; ++e) {
        const int32_t v = g->col[e];
        const double c = (double)(float)(r->pr_x[v] / r->outdeg[v]);
        P += c;
        double influence;
        if (r->pol.influence == GGO_INFL_TOTAL)
          influence = rowsum32 > 0.0 ? c / rowsum32 : 0.0;
        else
          influence = P > 0.0 ? c / P : 0.0;
        r->infl[e] = influence;
      }
    }
    double xn;
    if (ppr)
      xn = (u == s ? (1.0 - d) : 0.0) + d * (sum + (u == s ? D : 0.0));
    else
      xn = (1.0 - d) / n + d * (sum + D / n);
    if (xn != r->pr_x[u]) ++changed;
    out[u] = xn;
  }
  *edges_out = edges;
  *changed_out = changed;
}

/* BP message log-ratio of a sender with log-odds L: its belief is
   b(1) = 1 / (1 + e^-L), b(0) = 1 / (1 + e^L), and the message
   m(x) = psi(x, 1) b(1) + psi(x, 0) b(0). */
double ggo_bp_message(double L, double coupling) {
  const double b1 = 1.0 / (1.0 + exp(-L));
  const double b0 = 1.0 / (1.0 + exp(L));
  const double same = (1.0 + coupling) / 2.0, diff = (1.0 - coupling) / 2.0;
  const double m1 = same * b1 + diff * b0;
  const double m0 = diff * b1 + same * b0;
  return log(m1) - log(m0);
}

/* ---------------------------------------------------------------------------
 * One BP pass: new log-odds = prior + sum over the edge set of the senders'
 * message log-ratios. For a SUPER row the influence of each edge is the
 * magnitude of its binary32-rounded log-ratio over the magnitude of the
 * running sum (in CSR order, including the edge).
 * ------------------------------------------------------------------------- */
static void pass_bp(ggo_run* r, const uint8_t* mode, double* out, int64_t* edges_out, int64_t* changed_out) {
  const ggo_csr* g = &r->g;
  const int32_t n = g->n;
  const double kappa = r->app.coupling;
  int64_t edges = 0, changed = 0;
  for (int32_t u = 0; u < n; ++u) {
    double sum = 0.0;
    const int32_t b = g->rowptr[u], e_end = g->rowptr[u + 1];
    for (int32_t e = b; e < e_end; ++e) {
      if (mode[u] == ROW_APPROX && !r->active[e]) continue;
      sum += ggo_bp_message(r->pr_x[g->col[e]], kappa);
      ++edges;
    }
    if (mode[u] == ROW_SUPER) {
      double P = 0.0;
      for (int32_t e = b; e < e_end; ++e) {
        const double c = (double)(float)ggo_bp_message(r->pr_x[g->col[e]], kappa);
        P += c;
        r->infl[e] = fabs(P) > 0.0 ? fabs(c) / fabs(P) : 0.0;
      }
    }
    const double xn = r->app.prior[u] + sum;
    if (xn != r->pr_x[u]) ++changed;
    out[u] = xn;
  }
  *edges_out = edges;
  *changed_out = changed;
}

/* ---------------------------------------------------------------------------
 * One SSSP pass: x_u <- min(x_u, min over the edge set of x_v + w_e),
 * unreached sources (INF) contribute nothing. For a SUPER row the running
 * minimum r over the row (starting at INF) gives each assessable edge its
 * influence.
 * ------------------------------------------------------------------------- */
static void pass_sssp(ggo_run* r, const uint8_t* mode, uint32_t* out, int64_t* edges_out, int64_t* changed_out) {
  const ggo_csr* g = &r->g;
  const int32_t n = g->n;
  int64_t edges = 0, changed = 0;
  for (int32_t u = 0; u < n; ++u) {
    uint32_t best = r->d_x[u];
    const int32_t b = g->rowptr[u], e_end = g->rowptr[u + 1];
    for (int32_t e = b; e < e_end; ++e) {
      if (mode[u] == ROW_APPROX && !r->active[e]) continue;
      ++edges;
      const uint32_t xv = r->d_x[g->col[e]];
      if (xv == GGO_INF_U32) continue;
      const uint64_t cand = (uint64_t)xv + (uint64_t)g->weight[e];
      if (cand < best) best = (uint32_t)cand;
    }
    if (mode[u] == ROW_SUPER) {
      /* running minimum: starts at INF, or (push order) at the vertex's own
         value, which the pushes then lower in source order */
      uint64_t run = r->pol.influence == GGO_INFL_PUSH ? r->d_x[u] : GGO_INF_U32;
      for (int32_t e = b; e < e_end; ++e) {
        const uint32_t xv = r->d_x[g->col[e]];
        if (xv == GGO_INF_U32) { r->infl[e] = -1.0; continue; } /* not assessable */
        const uint64_t cand = (uint64_t)xv + (uint64_t)g->weight[e];
        const uint64_t nw = cand < run ? cand : run;
        if (run == GGO_INF_U32) {
          r->infl[e] = 1.0;
        } else {
          r->infl[e] = (double)(run - nw) / (double)run;
        }
        run = nw;
      }
    }
    if (best != r->d_x[u]) ++changed;
    out[u] = best;
  }
  *edges_out = edges;
  *changed_out = changed;
}

/* ---------------------------------------------------------------------------
 * One CC (label propagation) pass on the symmetrized graph:
 * x_u <- min(x_u, min over the edge set of x_v). For a SUPER row the
 * influence is binary: 1 iff x_v lowers the running minimum of the row.
 * ------------------------------------------------------------------------- */
static void pass_cc(ggo_run* r, const uint8_t* mode, int32_t* out, int64_t* edges_out, int64_t* changed_out) {
  const ggo_csr* g = &r->g;
  const int32_t n = g->n;
  int64_t edges = 0, changed = 0;
  for (int32_t u = 0; u < n; ++u) {
    int32_t best = r->l_x[u];
    const int32_t b = g->rowptr[u], e_end = g->rowptr[u + 1];
    for (int32_t e = b; e < e_end; ++e) {
      if (mode[u] == ROW_APPROX && !r->active[e]) continue;
      ++edges;
      const int32_t xv = r->l_x[g->col[e]];
      if (xv < best) best = xv;
    }
    if (mode[u] == ROW_SUPER) {
      int64_t run = r->pol.influence == GGO_INFL_PUSH ? (int64_t)r->l_x[u] : INT64_MAX;
      for (int32_t e = b; e < e_end; ++e) {
        const int32_t xv = r->l_x[g->col[e]];
        r->infl[e] = xv < run ? 1.0 : 0.0;
        if (xv < run) run = xv;
      }
    }
    if (best != r->l_x[u]) ++changed;
    out[u] = best;
  }
  *edges_out = edges;
  *changed_out = changed;
}

/* GG-EStatus [Alg. 2] for the SUPER rows after their pass: an assessed edge
   is active iff its influence exceeds theta; every other edge of the row is
   deactivated whether or not it was active before [Sec. 3.4] (the UNION
   variant keeps old flags). */
static void estatus(ggo_run* r) {
  const ggo_csr* g = &r->g;
  for (int32_t u = 0; u < g->n; ++u) {
    if (r->mode[u] != ROW_SUPER) continue;
    for (int32_t e = g->rowptr[u]; e < g->rowptr[u + 1]; ++e) {
      const int flag = r->infl[e] > r->theta_now;
      r->active[e] = r->pol.mask_update == GGO_MASK_UNION ? (uint8_t)(r->active[e] | flag) : (uint8_t)flag;
    }
  }
}

/* SSSP EStatus compares integers on the values the pass gathered from
   (iteration i-1): relative improvement (r - new) / r > theta as
   (r - new) * 2^16 > theta_q * r; the first finite candidate is active; an
   edge whose source is unreached is not assessed and keeps its flag. */
static void estatus_sssp(ggo_run* r) {
  const ggo_csr* g = &r->g;
  const uint64_t theta_q = (uint64_t)floor(r->theta_now * 65536.0 + 0.5);
  for (int32_t u = 0; u < g->n; ++u) {
    if (r->mode[u] != ROW_SUPER) continue;
    uint64_t run = r->pol.influence == GGO_INFL_PUSH ? r->d_x[u] : GGO_INF_U32;
    for (int32_t e = g->rowptr[u]; e < g->rowptr[u + 1]; ++e) {
      const uint32_t xv = r->d_x[g->col[e]];
      if (xv == GGO_INF_U32) continue; /* not assessable: keeps its flag */
      const uint64_t cand = (uint64_t)xv + (uint64_t)g->weight[e];
      const uint64_t nw = cand < run ? cand : run;
      int flag;
      if (run == GGO_INF_U32)
        flag = 1;
      else
        flag = ((run - nw) << 16) > theta_q * run;
      run = nw;
      r->active[e] = r->pol.mask_update == GGO_MASK_UNION ? (uint8_t)(r->active[e] | flag) : (uint8_t)flag;
    }
  }
}

/* Features of every vertex before iteration i (state of iteration i-1 and
   the two before it). */
static void compute_features(ggo_run* r) {
  const ggo_csr* g = &r->g;
  for (int32_t u = 0; u < g->n; ++u) {
    uint16_t* f = r->feat + (size_t)u * GGO_MLP_IN;
    int64_t act = 0;
    for (int32_t e = g->rowptr[u]; e < g->rowptr[u + 1]; ++e) act += r->active[e];
    const int32_t id = r->indeg[u];
    const uint32_t now = state_word(r, u);
    const float d1 = r->hist_n >= 1 ? ggo_delta_feature(r->app.app, now, r->hist[0][u]) : 0.0f;
    const float d2 = r->hist_n >= 2 ? ggo_delta_feature(r->app.app, r->hist[0][u], r->hist[1][u]) : 0.0f;
    f[0] = ggo_bf16_bits(ggo_lg_feature(1 + (int64_t)r->outdeg[u]));
    f[1] = ggo_bf16_bits(ggo_lg_feature(1 + (int64_t)id));
    f[2] = ggo_bf16_bits(id > 0 ? (float)act / (float)id : 0.0f);
    f[3] = ggo_bf16_bits(d1);
    f[4] = ggo_bf16_bits(d2);
    f[5] = f[6] = f[7] = 0;
  }
}

/* Logits of the learned policy (rounding as on the GPU) and the selected set
   S = { v : binary32(logit_v) > tau }. Returns |S|. */
/* S = { v : logit_v > tau } (binary32 comparison); returns |S| and, in
   *sel_edges, the number of in-edges of the rows in S. */
static int64_t select_rows(ggo_run* r, int64_t* sel_edges) {
  ggo_mlp_forward(r->pol.mlp, r->feat, r->g.n, 1, r->logit);
  int64_t cnt = 0, edges = 0;
  for (int32_t u = 0; u < r->g.n; ++u) {
    r->sel[u] = (float)r->logit[u] > (float)r->pol.tau;
    cnt += r->sel[u];
    if (r->sel[u]) edges += (int64_t)r->g.rowptr[u + 1] - r->g.rowptr[u];
  }
  r->have_sel = 1;
  *sel_edges = edges;
  return cnt;
}

static void run_pass(ggo_run* r, const uint8_t* mode, int shadow, int64_t* edges, int64_t* changed) {
  switch (r->app.app) {
    case GGO_PR:
    case GGO_PPR: pass_pr(r, mode, r->outdeg, NULL, shadow ? r->pr_sh : r->pr_xn, edges, changed); break;
    case GGO_BP: pass_bp(r, mode, shadow ? r->pr_sh : r->pr_xn, edges, changed); break;
    case GGO_SSSP: pass_sssp(r, mode, shadow ? r->d_sh : r->d_xn, edges, changed); break;
    case GGO_CC: pass_cc(r, mode, shadow ? r->l_sh : r->l_xn, edges, changed); break;
  }
}

/* Drift labels of a traced full superstep: 1 where the approximate update
   (shadow pass over the active edges) differs from the accurate one: PR/PPR
   binary32 contributions differing by more than label_eps relative, SSSP a
   shorter accurate distance, CC a smaller accurate label. */
static void compute_labels(ggo_run* r) {
  const int32_t n = r->g.n;
  for (int32_t u = 0; u < n; ++u) {
    int y;
    switch (r->app.app) {
      case GGO_PR:
      case GGO_PPR: {
        const int32_t od = r->outdeg[u];
        const float ca = od > 0 ? (float)(r->pr_xn[u] / od) : (float)r->pr_xn[u];
        const float cs = od > 0 ? (float)(r->pr_sh[u] / od) : (float)r->pr_sh[u];
        y = fabsf(ca - cs) > (float)r->pol.label_eps * ca;
        break;
      }
      case GGO_SSSP: y = r->d_xn[u] < r->d_sh[u]; break;
      default: y = r->l_xn[u] < r->l_sh[u]; break;
    }
    r->label[u] = (uint8_t)y;
  }
  r->have_label = 1;
}

int ggo_step(ggo_run* r, ggo_step_info* info) {
  ggo_step_info tmp;
  if (!info) info = &tmp;
  memset(info, 0, sizeof(*info));
  if (r->done) return 0;
  const int32_t i = r->iter + 1;
  const int32_t n = r->g.n;
  const ggo_policy* p = &r->pol;
  /* Kind of this iteration: every row alike, except the partial superstep
     of the learned policy. */
  int kind = GGO_KIND_APPROX;
  int64_t selected = -1;
  r->have_sel = 0;
  r->have_label = 0;
  switch (p->kind) {
    case GGO_EXACT: kind = GGO_KIND_ACCURATE; break;
    case GGO_SP: kind = GGO_KIND_APPROX; break;
    case GGO_SMS: kind = i >= p->alpha + 1 ? GGO_KIND_ACCURATE : GGO_KIND_APPROX; break;
    case GGO_GG: kind = is_correction(p, i) ? GGO_KIND_FULL : GGO_KIND_APPROX; break;
    case GGO_LEARNED:
      if (is_correction(p, i)) {
        const int32_t c = ++r->corrections;
        compute_features(r);
        int64_t sel_edges = 0;
        selected = select_rows(r, &sel_edges);
        /* fallback: every fallback_k-th correction, and any selection whose
           rows hold more than rho * m in-edges */
        if ((p->fallback_k > 0 && c % p->fallback_k == 0) || (double)sel_edges > p->rho * (double)r->g.m)
          kind = GGO_KIND_FULL;
        else
          kind = GGO_KIND_PARTIAL;
      }
      break;
  }
  for (int32_t u = 0; u < n; ++u) {
    switch (kind) {
      case GGO_KIND_APPROX: r->mode[u] = ROW_APPROX; break;
      case GGO_KIND_ACCURATE: r->mode[u] = ROW_ACCURATE; break;
      case GGO_KIND_FULL: r->mode[u] = ROW_SUPER; break;
      default: r->mode[u] = r->sel[u] ? ROW_SUPER : ROW_APPROX; break;
    }
  }
  r->theta_now = theta_at(p, i);
  const int traced = p->trace && kind == GGO_KIND_FULL;
  if (traced && p->kind != GGO_LEARNED) compute_features(r);
  int64_t edges = 0, changed = 0;
  if (traced) {
    /* approximate shadow pass: the update the flags alone would give */
    uint8_t* approx = (uint8_t*)calloc((size_t)n + 1, 1);
    int64_t e2, c2;
    run_pass(r, approx, 1, &e2, &c2);
    free(approx);
  }
  const int pr_app = r->app.app == GGO_PR || r->app.app == GGO_PPR;
  if (pr_app && kind == GGO_KIND_APPROX &&
      (r->app.pr_degree == GGO_DEGREE_ACTIVE || p->vstatus != GGO_VSTATUS_NONE)) {
    const int32_t* deg = r->outdeg;
    if (r->app.pr_degree == GGO_DEGREE_ACTIVE) {
      /* active out-degree of the current flags */
      memset(r->odeg_act, 0, sizeof(int32_t) * (size_t)n);
      for (int64_t e = 0; e < r->g.m; ++e)
        if (r->active[e]) r->odeg_act[r->g.col[e]]++;
      deg = r->odeg_act;
    }
    const uint8_t* skip = NULL;
    if (p->vstatus != GGO_VSTATUS_NONE && i > 1) {
      /* every vertex is on the active list of iteration 1; later a row is
         recomputed iff one of its active in-edges comes from a vertex that
         was active after the previous iteration */
      for (int32_t u = 0; u < n; ++u) {
        int any = 0;
        for (int32_t e = r->g.rowptr[u]; e < r->g.rowptr[u + 1] && !any; ++e)
          any = r->active[e] && r->vact[r->g.col[e]];
        r->skip[u] = (uint8_t)!any;
      }
      skip = r->skip;
    }
    pass_pr(r, r->mode, deg, skip, r->pr_xn, &edges, &changed);
  } else {
    run_pass(r, r->mode, 0, &edges, &changed);
  }
  if (pr_app && p->vstatus != GGO_VSTATUS_NONE) {
    /* GG-VStatus [Alg. 2]: active iff the value moved by more than eps */
    for (int32_t u = 0; u < n; ++u) {
      const double delta = fabs(r->pr_xn[u] - r->pr_x[u]);
      const double bound = p->vstatus == GGO_VSTATUS_ABS ? p->eps : p->eps * fabs(r->pr_x[u]);
      r->vact[u] = (uint8_t)(delta > bound);
    }
  }
  if (traced) compute_labels(r);
  if (kind == GGO_KIND_FULL || kind == GGO_KIND_PARTIAL) {
    if (r->app.app == GGO_SSSP)
      estatus_sssp(r); /* reads d_x, still iteration i-1 */
    else
      estatus(r);
  }
  /* history of state words for the delta features, then the swap */
  {
    uint32_t* t = r->hist[1];
    r->hist[1] = r->hist[0];
    r->hist[0] = t;
    for (int32_t u = 0; u < n; ++u) r->hist[0][u] = state_word(r, u);
    if (r->hist_n < 2) r->hist_n++;
  }
  switch (r->app.app) {
    case GGO_PR:
    case GGO_PPR:
    case GGO_BP: {
      double* t = r->pr_x;
      r->pr_x = r->pr_xn;
      r->pr_xn = t;
      break;
    }
    case GGO_SSSP: {
      uint32_t* t = r->d_x;
      r->d_x = r->d_xn;
      r->d_xn = t;
      break;
    }
    case GGO_CC: {
      int32_t* t = r->l_x;
      r->l_x = r->l_xn;
      r->l_xn = t;
      break;
    }
  }
  info->iter = i;
  info->kind = kind;
  info->accurate = kind == GGO_KIND_ACCURATE || kind == GGO_KIND_FULL;
  info->superstep = kind == GGO_KIND_FULL || kind == GGO_KIND_PARTIAL;
  info->edges = edges;
  info->changed = changed;
  info->selected = selected;
  r->iter = i;
  r->edges_total += edges;
  int64_t act = 0;
  for (int64_t e = 0; e < r->g.m; ++e) act += r->active[e];
  info->active_edges = p->kind == GGO_EXACT ? r->g.m : act;

  /* Termination. */
  const int app = r->app.app;
  if (app == GGO_PR || app == GGO_PPR || app == GGO_BP) {
    if (i >= r->app.iters) r->done = 1;
  } else if (p->kind == GGO_EXACT) {
    if (changed == 0) r->converged = 1;
    if (changed == 0 || i >= r->app.max_iters) r->done = 1;
  } else if (p->stop == GGO_STOP_FIXED_ITERS) {
    if (i >= r->app.iters) r->done = 1;
  } else {
    /* Fixed point: a no-change iteration ends the run when no later
       iteration can differ from it (an iteration over every edge, or any
       iteration of SP, whose edge set never changes). */
    const int final_kind = info->accurate || p->kind == GGO_SP;
    if ((changed == 0 && final_kind) || i >= r->app.max_iters) r->done = 1;
  }
  return 1;
}

int ggo_done(const ggo_run* r) { return r->done; }

/* ---------------------------------------------------------------------------
 * Dynamic graphs. An SSSP/CC value at a converged exact run is the length of
 * a shortest path (the smallest label that reaches the vertex). Edge s -> d
 * "supports" d when it realises d's value: x_s + w = x_d for SSSP (d not the
 * source, both finite), l_s = l_d for CC (l_d not d's own id). After
 * deletions a value can only be wrong if every path realising it used a
 * deleted edge; walking such a path back from the vertex meets a deleted
 * supporting edge, so the closure below (seeded at the targets of deleted
 * supporting edges, grown along supporting edges of the new graph) contains
 * every vertex whose value may have become too small. Those restart from
 * their initial values; every other value is still exact.
 * ------------------------------------------------------------------------- */
static int supports(const ggo_run* r, int32_t s, int32_t d, int32_t w) {
  if (r->app.app == GGO_SSSP) {
    if (d == r->app.source || r->d_x[s] == GGO_INF_U32 || r->d_x[d] == GGO_INF_U32) return 0;
    return (uint64_t)r->d_x[s] + (uint64_t)w == (uint64_t)r->d_x[d];
  }
  return r->l_x[s] == r->l_x[d] && r->l_x[d] != d;
}

int ggo_run_update(ggo_run* r, const ggo_csr* gn, const int64_t* old_of_new, const uint8_t* deleted_old,
                   int32_t more_iters) {
  if (!r || !gn || (gn->m > 0 && !old_of_new) || (r->g.m > 0 && !deleted_old)) { set_err("null argument"); return -1; }
  if (gn->n != r->g.n) { set_err("the vertex set of an update is fixed"); return -1; }
  if (more_iters < 0) { set_err("more_iters < 0"); return -1; }
  if (r->pol.kind == GGO_LEARNED || r->pol.trace || r->pol.vstatus != GGO_VSTATUS_NONE ||
      r->app.pr_degree != GGO_DEGREE_FULL) {
    set_err("updates of LEARNED, traced, vertex-status or ACTIVE-degree runs");
    return -1;
  }
  if ((r->g.weight != NULL) != (gn->weight != NULL)) { set_err("weights on one side only"); return -1; }
  const int32_t n = gn->n;
  const int64_t m0 = r->g.m, m1 = gn->m;
  for (int64_t e = 0; e < m1; ++e)
    if (old_of_new[e] < -1 || old_of_new[e] >= m0) { set_err("old_of_new out of range"); return -1; }
  const int app = r->app.app;
  int any_deleted = 0;
  for (int64_t e = 0; e < m0; ++e) any_deleted |= deleted_old[e] != 0;
  memset(r->reset, 0, (size_t)n + 1);
  if ((app == GGO_SSSP || app == GGO_CC) && any_deleted) {
    if (r->pol.kind == GGO_EXACT && r->converged) {
      /* seeds: targets of deleted supporting edges (old graph) */
      for (int32_t u = 0; u < n; ++u)
        for (int32_t e = r->g.rowptr[u]; e < r->g.rowptr[u + 1]; ++e)
          if (deleted_old[e] && supports(r, r->g.col[e], u, r->g.weight ? r->g.weight[e] : 0)) r->reset[u] = 1;
      /* closure along supporting edges of the new graph */
      int grew = 1;
      while (grew) {
        grew = 0;
        for (int32_t v = 0; v < n; ++v) {
          if (r->reset[v]) continue;
          for (int32_t e = gn->rowptr[v]; e < gn->rowptr[v + 1]; ++e) {
            const int32_t p = gn->col[e];
            if (r->reset[p] && supports(r, p, v, gn->weight ? gn->weight[e] : 0)) {
              r->reset[v] = 1;
              grew = 1;
              break;
            }
          }
        }
      }
    } else {
      memset(r->reset, 1, (size_t)n);
    }
    for (int32_t v = 0; v < n; ++v) {
      if (!r->reset[v]) continue;
      if (app == GGO_SSSP) r->d_x[v] = v == r->app.source ? 0u : GGO_INF_U32;
      else r->l_x[v] = v;
    }
  }
  /* edge flags: a surviving edge keeps its flag, an inserted edge is active */
  uint8_t* act = (uint8_t*)calloc((size_t)m1 + 1, 1);
  for (int64_t e = 0; e < m1; ++e) act[e] = old_of_new[e] >= 0 ? r->active[old_of_new[e]] : 1;
  free(r->active);
  r->active = act;
  free(r->infl);
  r->infl = (double*)calloc((size_t)m1 + 1, sizeof(double));
  r->g = *gn;
  memset(r->outdeg, 0, sizeof(int32_t) * ((size_t)n + 1));
  for (int64_t e = 0; e < m1; ++e) r->outdeg[gn->col[e]]++;
  for (int32_t u = 0; u < n; ++u) r->indeg[u] = gn->rowptr[u + 1] - gn->rowptr[u];
  r->converged = 0;
  const int fixed_iters = app == GGO_PR || app == GGO_PPR || app == GGO_BP || r->pol.stop == GGO_STOP_FIXED_ITERS;
  if (fixed_iters) {
    if (r->app.iters < r->iter) r->app.iters = r->iter;
    r->app.iters += more_iters;
    r->done = r->iter >= r->app.iters;
  } else {
    if (r->app.max_iters < r->iter) r->app.max_iters = r->iter;
    r->app.max_iters += more_iters;
    r->done = r->iter >= r->app.max_iters;
  }
  return 0;
}

void ggo_get_reset(const ggo_run* r, uint8_t* out) { memcpy(out, r->reset, (size_t)r->g.n); }
int32_t ggo_iterations(const ggo_run* r) { return r->iter; }
int64_t ggo_edges_total(const ggo_run* r) { return r->edges_total; }

void ggo_get_values(const ggo_run* r, void* out) {
  const size_t n = (size_t)r->g.n;
  switch (r->app.app) {
    case GGO_PR:
    case GGO_PPR:
    case GGO_BP: memcpy(out, r->pr_x, n * sizeof(double)); break;
    case GGO_SSSP: memcpy(out, r->d_x, n * sizeof(uint32_t)); break;
    case GGO_CC: memcpy(out, r->l_x, n * sizeof(int32_t)); break;
  }
}

void ggo_get_mask(const ggo_run* r, uint8_t* out) { memcpy(out, r->active, (size_t)r->g.m); }

void ggo_set_mask(ggo_run* r, const uint8_t* mask) {
  for (int64_t e = 0; e < r->g.m; ++e) r->active[e] = mask[e] != 0;
}

void ggo_get_vactive(const ggo_run* r, uint8_t* out) { memcpy(out, r->vact, (size_t)r->g.n); }

void ggo_set_vactive(ggo_run* r, const uint8_t* in) {
  for (int32_t u = 0; u < r->g.n; ++u) r->vact[u] = in[u] != 0;
}

void ggo_get_influence(const ggo_run* r, double* out) {
  memcpy(out, r->infl, (size_t)r->g.m * sizeof(double));
}

void ggo_get_features(const ggo_run* r, uint16_t* out) {
  memcpy(out, r->feat, (size_t)r->g.n * GGO_MLP_IN * sizeof(uint16_t));
}

int ggo_get_selection(const ggo_run* r, uint8_t* sel, double* logits) {
  if (!r->have_sel) return 0;
  if (sel) memcpy(sel, r->sel, (size_t)r->g.n);
  if (logits) memcpy(logits, r->logit, (size_t)r->g.n * sizeof(double));
  return 1;
}

int ggo_get_labels(const ggo_run* r, uint8_t* out) {
  if (!r->have_label) return 0;
  memcpy(out, r->label, (size_t)r->g.n);
  return 1;
}

void ggo_end(ggo_run* r) {
  if (!r) return;
  free(r->outdeg);
  free(r->indeg);
  free(r->active);
  free(r->infl);
  free(r->mode);
  for (int k = 0; k < 2; ++k) free(r->hist[k]);
  free(r->feat);
  free(r->logit);
  free(r->sel);
  free(r->label);
  free(r->odeg_act);
  free(r->vact);
  free(r->skip);
  free(r->reset);
  free(r->pr_x);
  free(r->pr_xn);
  free(r->pr_sh);
  free(r->d_x);
  free(r->d_xn);
  free(r->d_sh);
  free(r->l_x);
  free(r->l_xn);
  free(r->l_sh);
  free(r);
}
