/*
 * Seeded synthetic graph inputs: R-MAT and Erdos-Renyi edge lists, vertex
 * permutation, edge weights, source selection, and the canonical in-CSR
 * (rows = destinations, each row sorted by (source, generation index),
 * self-loops removed, duplicate edges kept).
 *
 * This module produces inputs only. It holds none of the graph method's
 * arithmetic (no sampling, gathering, influence or correction), and it is
 * shared by the oracle-side tests and the GPU-side tests alike.
 *
 * Randomness: every draw is SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014) evaluated at a
 * counter, so the output does not depend on the thread count.
 *
 * R-MAT follows Chakrabarti, Zhan and Faloutsos (SDM 2004): at each of
 * `scale` levels, most significant bit first, a quadrant is chosen with
 * probabilities a (src bit 0, dst bit 0), b (0,1), c (1,0), d (1,1). No noise.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Element `idx` of the SplitMix64 sequence started at state `seed`. */
static inline uint64_t sm64_at(uint64_t seed, uint64_t idx) {
  return sm64_mix(seed + (idx + 1) * SM64_GAMMA);
}

/* Draw for (stream seed, item k, sub-draw l), l < 64. */
static inline uint64_t draw(uint64_t seed, uint64_t k, uint32_t l) {
  return sm64_at(seed, (k << 6) | (uint64_t)l);
}

/* Uniform integer in [0, n) by 64x64 multiply-high. */
static inline uint64_t mulshift(uint64_t x, uint64_t n) {
  return (uint64_t)(((unsigned __int128)x * (unsigned __int128)n) >> 64);
}

uint64_t graphgen_draw(uint64_t seed, uint64_t k, uint32_t l) { return draw(seed, k, l); }

/* out[k] = draw(seed, k, l) for k in [0, count). */
void graphgen_draws(uint64_t seed, uint32_t l, int64_t count, uint64_t* out) {
  for (int64_t k = 0; k < count; ++k) out[k] = draw(seed, (uint64_t)k, l);
}

/* R-MAT edge list: m pairs on n = 2^scale vertices (ids before permutation). */
void graphgen_rmat_edges(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed,
                         int32_t* src, int32_t* dst) {
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    uint32_t s = 0, d = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double u = (double)(draw(seed, (uint64_t)k, (uint32_t)l) >> 11) * (1.0 / 9007199254740992.0);
      uint32_t sb, db;
      if (u < a) { sb = 0; db = 0; }
      else if (u < ab) { sb = 0; db = 1; }
      else if (u < abc) { sb = 1; db = 0; }
      else { sb = 1; db = 1; }
      s = (s << 1) | sb;
      d = (d << 1) | db;
    }
    src[k] = (int32_t)s;
    dst[k] = (int32_t)d;
  }
}

/* Erdos-Renyi-style multigraph: m pairs with independent uniform endpoints. */
void graphgen_er_edges(int32_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    src[k] = (int32_t)mulshift(draw(seed, (uint64_t)k, 0), (uint64_t)n);
    dst[k] = (int32_t)mulshift(draw(seed, (uint64_t)k, 1), (uint64_t)n);
  }
}

/* Seeded uniform permutation of [0, n) (Fisher-Yates). */
void graphgen_permutation(int32_t n, uint64_t seed, int32_t* perm) {
  for (int32_t i = 0; i < n; ++i) perm[i] = i;
  for (int64_t i = (int64_t)n - 1; i > 0; --i) {
    int64_t j = (int64_t)mulshift(draw(seed, (uint64_t)i, 0), (uint64_t)(i + 1));
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

void graphgen_apply_permutation(int64_t m, const int32_t* perm, int32_t* src, int32_t* dst) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    src[k] = perm[src[k]];
    dst[k] = perm[dst[k]];
  }
}

/* Integer weights in [1, 255], one per generated edge k. */
void graphgen_weights(int64_t m, uint64_t seed, int32_t* w) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) w[k] = 1 + (int32_t)mulshift(draw(seed, (uint64_t)k, 0), 255);
}

static int cmp_u64(const void* x, const void* y) {
  uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
  return (a > b) - (a < b);
}

/*
 * Canonical in-CSR. Arc list: generated pair k gives arc (src[k] -> dst[k])
 * with generation index k; if `symmetrize`, it also gives (dst[k] -> src[k])
 * with generation index m + k. Self-loops are dropped; duplicates are kept.
 * Row u lists the sources of arcs into u sorted by (source, generation index).
 * rowptr has n+1 entries; col and genidx (nullable) have room for the returned
 * arc count (at most m, or 2m when symmetrizing). Returns the arc count, or -1
 * on allocation failure, or -2 if a generation index does not fit 32 bits.
 */
int64_t graphgen_build_in_csr(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                              int32_t symmetrize, int32_t* rowptr, int32_t* col, int64_t* genidx) {
  const int64_t narcs_gen = symmetrize ? 2 * m : m;
  if (narcs_gen >= ((int64_t)1 << 32)) return -2;
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    if (src[k] == dst[k]) continue;
    __atomic_fetch_add(&cnt[dst[k]], 1, __ATOMIC_RELAXED);
    if (symmetrize) __atomic_fetch_add(&cnt[src[k]], 1, __ATOMIC_RELAXED);
  }
  int64_t total = 0;
  for (int32_t u = 0; u < n; ++u) {
    int64_t cu = cnt[u];
    cnt[u] = total;
    rowptr[u] = (int32_t)total;
    total += cu;
  }
  rowptr[n] = (int32_t)total;
  uint64_t* key = (uint64_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(uint64_t));
  if (!key) { free(cnt); return -1; }
  /* Scatter (source, generation index) keys into rows; the order inside a
     row is fixed afterwards by sorting the keys. */
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    if (src[k] == dst[k]) continue;
    int64_t p = __atomic_fetch_add(&cnt[dst[k]], 1, __ATOMIC_RELAXED);
    key[p] = ((uint64_t)(uint32_t)src[k] << 32) | (uint64_t)k;
    if (symmetrize) {
      int64_t q = __atomic_fetch_add(&cnt[src[k]], 1, __ATOMIC_RELAXED);
      key[q] = ((uint64_t)(uint32_t)dst[k] << 32) | (uint64_t)(m + k);
    }
  }
  free(cnt);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t u = 0; u < n; ++u) {
    int64_t b = rowptr[u], e = rowptr[u + 1], len = e - b;
    uint64_t* r = key + b;
    if (len < 32) {
      for (int64_t i = 1; i < len; ++i) {
        uint64_t v = r[i];
        int64_t j = i - 1;
        while (j >= 0 && r[j] > v) { r[j + 1] = r[j]; --j; }
        r[j + 1] = v;
      }
    } else {
      qsort(r, (size_t)len, sizeof(uint64_t), cmp_u64);
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < total; ++e) {
    col[e] = (int32_t)(key[e] >> 32);
    if (genidx) genidx[e] = (int64_t)(key[e] & 0xffffffffULL);
  }
  free(key);
  return total;
}

/* Out-degree of every vertex from an in-CSR column array. */
void graphgen_outdeg(int32_t n, int64_t m, const int32_t* col, int32_t* outdeg) {
  memset(outdeg, 0, sizeof(int32_t) * (size_t)n);
  for (int64_t e = 0; e < m; ++e) outdeg[col[e]]++;
}

/*
 * Query sources: v_j = mulshift(draw(seed, j, 0), n) for j = 0, 1, ..., keeping
 * those with outdeg > 0, drawn with replacement, until `count` are found or
 * `max_tries` draws are spent. Returns the number found.
 */
int32_t graphgen_pick_sources(int32_t n, const int32_t* outdeg, int32_t count, uint64_t seed,
                              int64_t max_tries, int32_t* out) {
  int32_t found = 0;
  for (int64_t j = 0; j < max_tries && found < count; ++j) {
    int32_t v = (int32_t)mulshift(draw(seed, (uint64_t)j, 0), (uint64_t)n);
    if (outdeg[v] > 0) out[found++] = v;
  }
  return found;
}
