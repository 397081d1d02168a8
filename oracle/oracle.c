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

/* ------------------------------------------------------------------------- */

struct ggo_run {
  ggo_csr g;
  ggo_app_params app;
  ggo_policy pol;
  int32_t* outdeg;
  uint8_t* active; /* edge flags */
  double* infl;    /* influence at the last superstep (diagnostics) */
  /* values: x (current, iteration i-1) and xn (next) */
  double* pr_x;
  double* pr_xn;
  uint32_t* d_x;
  uint32_t* d_xn;
  int32_t* l_x;
  int32_t* l_xn;
  int32_t iter;
  int32_t done;
  int64_t edges_total;
};

static int is_accurate(const ggo_policy* p, int32_t i) {
  switch (p->kind) {
    case GGO_EXACT: return 1;
    case GGO_SP: return 0;
    case GGO_SMS: return i >= p->alpha + 1;
    case GGO_GG: return (i % (p->alpha + 1)) == 0;
  }
  return 1;
}

/* Edge flags are re-selected after an accurate iteration of GG only (for SMS
   the flags are never read again after its switch). */
static int is_superstep(const ggo_policy* p, int32_t i) {
  return p->kind == GGO_GG && is_accurate(p, i);
}

ggo_run* ggo_begin(const ggo_csr* g, const ggo_app_params* app, const ggo_policy* pol) {
  if (!g || !app || !pol) { set_err("null argument"); return NULL; }
  if (g->n < 0 || g->m < 0 || !g->rowptr || (g->m > 0 && !g->col)) { set_err("bad csr"); return NULL; }
  if (g->rowptr[0] != 0 || g->rowptr[g->n] != g->m) { set_err("rowptr ends"); return NULL; }
  for (int32_t u = 0; u < g->n; ++u)
    if (g->rowptr[u + 1] < g->rowptr[u]) { set_err("rowptr not monotone"); return NULL; }
  for (int64_t e = 0; e < g->m; ++e)
    if (g->col[e] < 0 || g->col[e] >= g->n) { set_err("col out of range"); return NULL; }
  if (app->app < GGO_PR || app->app > GGO_PPR) { set_err("bad app"); return NULL; }
  if (pol->kind < GGO_EXACT || pol->kind > GGO_GG) { set_err("bad policy"); return NULL; }
  if (pol->alpha < 0 || !(pol->theta >= 0) || !(pol->sigma >= 0 && pol->sigma <= 1)) {
    set_err("bad alpha/theta/sigma");
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

  ggo_run* r = (ggo_run*)calloc(1, sizeof(ggo_run));
  r->g = *g;
  r->app = *app;
  r->pol = *pol;
  int32_t n = g->n;
  int64_t m = g->m;
  r->outdeg = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  for (int64_t e = 0; e < m; ++e) r->outdeg[g->col[e]]++;
  r->active = (uint8_t*)calloc((size_t)m + 1, 1);
  r->infl = (double*)calloc((size_t)m + 1, sizeof(double));

  /* Initial sparsification [Sec. 3.4]: each edge kept iff its draw falls
     below floor(sigma * 2^32 + 1/2). The exact baseline ignores the flags. */
  uint64_t keep = ggo_keep_threshold(pol->sigma);
  for (int64_t e = 0; e < m; ++e)
    r->active[e] = pol->kind == GGO_EXACT ? 1 : ((uint64_t)ggo_sample_draw(pol->seed, 0, e) < keep);

  /* Initial values. */
  switch (app->app) {
    case GGO_PR:
      r->pr_x = (double*)malloc(sizeof(double) * ((size_t)n + 1));
      r->pr_xn = (double*)malloc(sizeof(double) * ((size_t)n + 1));
      for (int32_t u = 0; u < n; ++u) r->pr_x[u] = 1.0 / n;
      break;
    case GGO_PPR:
      r->pr_x = (double*)calloc((size_t)n + 1, sizeof(double));
      r->pr_xn = (double*)calloc((size_t)n + 1, sizeof(double));
      r->pr_x[app->source] = 1.0;
      break;
    case GGO_SSSP:
      r->d_x = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
      r->d_xn = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
      for (int32_t u = 0; u < n; ++u) r->d_x[u] = GGO_INF_U32;
      r->d_x[app->source] = 0;
      break;
    case GGO_CC:
      r->l_x = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
      r->l_xn = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
      for (int32_t u = 0; u < n; ++u) r->l_x[u] = u;
      break;
  }
  r->iter = 0;
  r->done = (app->app == GGO_PR || app->app == GGO_PPR || pol->stop == GGO_STOP_FIXED_ITERS) &&
            app->iters <= 0;
  return r;
}

/* ---------------------------------------------------------------------------
 * One PageRank / personalized PageRank iteration [Alg. 2]. Gather sums the
 * contributions x_v / outdeg_v over the row's edge set; Apply computes
 * (1-d)/N + d * (sum + D/N) (PPR: teleport and dangling mass go to the
 * source). On a superstep, each edge's influence is computed during the
 * gather from the running sum, and GG-EStatus sets its flag.
 * ------------------------------------------------------------------------- */
static void step_pr(ggo_run* r, int accurate, int superstep, ggo_step_info* info) {
  const ggo_csr* g = &r->g;
  const int32_t n = g->n;
  const double d = r->app.damping;
  const int ppr = r->app.app == GGO_PPR;
  const int32_t s = r->app.source;
  double D = 0.0;
  if (r->app.dangling == GGO_DANGLING_UNIFORM)
    for (int32_t v = 0; v < n; ++v)
      if (r->outdeg[v] == 0) D += r->pr_x[v];

  int64_t edges = 0, changed = 0;
  for (int32_t u = 0; u < n; ++u) {
    double sum = 0.0;   /* gather accumulator */
    double P = 0.0;     /* running sum of binary32 contributions (influence) */
    const int32_t b = g->rowptr[u], e_end = g->rowptr[u + 1];
    for (int32_t e = b; e < e_end; ++e) {
      if (!accurate && !r->active[e]) continue;
      const int32_t v = g->col[e];
      sum += r->pr_x[v] / r->outdeg[v];
      ++edges;
    }
    if (superstep) {
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
    r->pr_xn[u] = xn;
  }
  double* t = r->pr_x;
  r->pr_x = r->pr_xn;
  r->pr_xn = t;
  info->edges = edges;
  info->changed = changed;
}

/* ---------------------------------------------------------------------------
 * One SSSP iteration: x_u <- min(x_u, min over the edge set of x_v + w_e),
 * unreached sources (INF) contribute nothing. On a superstep the running
 * minimum r over the row (starting at INF) gives each assessable edge its
 * influence.
 * ------------------------------------------------------------------------- */
static void step_sssp(ggo_run* r, int accurate, int superstep, ggo_step_info* info) {
  const ggo_csr* g = &r->g;
  const int32_t n = g->n;
  int64_t edges = 0, changed = 0;
  for (int32_t u = 0; u < n; ++u) {
    uint32_t best = r->d_x[u];
    const int32_t b = g->rowptr[u], e_end = g->rowptr[u + 1];
    for (int32_t e = b; e < e_end; ++e) {
      if (!accurate && !r->active[e]) continue;
      ++edges;
      const uint32_t xv = r->d_x[g->col[e]];
      if (xv == GGO_INF_U32) continue;
      const uint64_t cand = (uint64_t)xv + (uint64_t)g->weight[e];
      if (cand < best) best = (uint32_t)cand;
    }
    if (superstep) {
      uint64_t run = GGO_INF_U32; /* running minimum, starts at INF */
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
    r->d_xn[u] = best;
  }
  uint32_t* t = r->d_x;
  r->d_x = r->d_xn;
  r->d_xn = t;
  info->edges = edges;
  info->changed = changed;
}

/* ---------------------------------------------------------------------------
 * One CC (label propagation) iteration on the symmetrized graph:
 * x_u <- min(x_u, min over the edge set of x_v). Superstep influence is
 * binary: 1 iff x_v lowers the running minimum of the row.
 * ------------------------------------------------------------------------- */
static void step_cc(ggo_run* r, int accurate, int superstep, ggo_step_info* info) {
  const ggo_csr* g = &r->g;
  const int32_t n = g->n;
  int64_t edges = 0, changed = 0;
  for (int32_t u = 0; u < n; ++u) {
    int32_t best = r->l_x[u];
    const int32_t b = g->rowptr[u], e_end = g->rowptr[u + 1];
    for (int32_t e = b; e < e_end; ++e) {
      if (!accurate && !r->active[e]) continue;
      ++edges;
      const int32_t xv = r->l_x[g->col[e]];
      if (xv < best) best = xv;
    }
    if (superstep) {
      int64_t run = INT64_MAX;
      for (int32_t e = b; e < e_end; ++e) {
        const int32_t xv = r->l_x[g->col[e]];
        r->infl[e] = xv < run ? 1.0 : 0.0;
        if (xv < run) run = xv;
      }
    }
    if (best != r->l_x[u]) ++changed;
    r->l_xn[u] = best;
  }
  int32_t* t = r->l_x;
  r->l_x = r->l_xn;
  r->l_xn = t;
  info->edges = edges;
  info->changed = changed;
}

/* GG-EStatus [Alg. 2] applied after a superstep: an assessed edge is active
   iff its influence exceeds theta; every other edge is deactivated whether or
   not it was active before [Sec. 3.4] (the UNION variant keeps old flags). */
static void estatus(ggo_run* r) {
  for (int64_t e = 0; e < r->g.m; ++e) {
    const int flag = r->infl[e] > r->pol.theta;
    r->active[e] = r->pol.mask_update == GGO_MASK_UNION ? (uint8_t)(r->active[e] | flag) : (uint8_t)flag;
  }
}

/* SSSP EStatus needs the values the superstep gathered from (iteration i-1),
   so it runs before the values are swapped; see ggo_step. */
static void estatus_sssp(ggo_run* r, const uint32_t* x_prev) {
  const ggo_csr* g = &r->g;
  const uint64_t theta_q = (uint64_t)floor(r->pol.theta * 65536.0 + 0.5);
  for (int32_t u = 0; u < g->n; ++u) {
    uint64_t run = GGO_INF_U32;
    for (int32_t e = g->rowptr[u]; e < g->rowptr[u + 1]; ++e) {
      const uint32_t xv = x_prev[g->col[e]];
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

int ggo_step(ggo_run* r, ggo_step_info* info) {
  ggo_step_info tmp;
  if (!info) info = &tmp;
  memset(info, 0, sizeof(*info));
  if (r->done) return 0;
  const int32_t i = r->iter + 1;
  const int accurate = is_accurate(&r->pol, i);
  const int superstep = is_superstep(&r->pol, i);
  info->iter = i;
  info->accurate = accurate;
  info->superstep = superstep;
  switch (r->app.app) {
    case GGO_PR:
    case GGO_PPR:
      step_pr(r, accurate, superstep, info);
      if (superstep) estatus(r);
      break;
    case GGO_SSSP:
      step_sssp(r, accurate, superstep, info);
      if (superstep) estatus_sssp(r, r->d_xn); /* d_xn now holds iteration i-1 */
      break;
    case GGO_CC:
      step_cc(r, accurate, superstep, info);
      if (superstep) estatus(r);
      break;
  }
  r->iter = i;
  r->edges_total += info->edges;
  int64_t act = 0;
  for (int64_t e = 0; e < r->g.m; ++e) act += r->active[e];
  info->active_edges = r->pol.kind == GGO_EXACT ? r->g.m : act;

  /* Termination. */
  const int app = r->app.app;
  if (app == GGO_PR || app == GGO_PPR) {
    if (i >= r->app.iters) r->done = 1;
  } else if (r->pol.kind == GGO_EXACT) {
    if (info->changed == 0 || i >= r->app.max_iters) r->done = 1;
  } else if (r->pol.stop == GGO_STOP_FIXED_ITERS) {
    if (i >= r->app.iters) r->done = 1;
  } else {
    /* Fixed point: a no-change iteration ends the run when no later
       iteration can differ from it (an accurate iteration, or any iteration
       of SP, whose edge set never changes). */
    const int final_kind = accurate || r->pol.kind == GGO_SP;
    if ((info->changed == 0 && final_kind) || i >= r->app.max_iters) r->done = 1;
  }
  return 1;
}

int ggo_done(const ggo_run* r) { return r->done; }
int32_t ggo_iterations(const ggo_run* r) { return r->iter; }
int64_t ggo_edges_total(const ggo_run* r) { return r->edges_total; }

void ggo_get_values(const ggo_run* r, void* out) {
  const size_t n = (size_t)r->g.n;
  switch (r->app.app) {
    case GGO_PR:
    case GGO_PPR: memcpy(out, r->pr_x, n * sizeof(double)); break;
    case GGO_SSSP: memcpy(out, r->d_x, n * sizeof(uint32_t)); break;
    case GGO_CC: memcpy(out, r->l_x, n * sizeof(int32_t)); break;
  }
}

void ggo_get_mask(const ggo_run* r, uint8_t* out) { memcpy(out, r->active, (size_t)r->g.m); }

void ggo_get_influence(const ggo_run* r, double* out) {
  memcpy(out, r->infl, (size_t)r->g.m * sizeof(double));
}

void ggo_end(ggo_run* r) {
  if (!r) return;
  free(r->outdeg);
  free(r->active);
  free(r->infl);
  free(r->pr_x);
  free(r->pr_xn);
  free(r->d_x);
  free(r->d_xn);
  free(r->l_x);
  free(r->l_xn);
  free(r);
}
