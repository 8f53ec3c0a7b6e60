/*
 * Seeded synthetic inputs: Erdos-Renyi G(n,M), Barabasi-Albert and R-MAT graphs
 * as CSR, plus random vertex groups.
 *
 * This file holds no part of the walk-count method; it only produces inputs.
 * Both the CPU oracle and the GPU path consume what it emits, so every random
 * number comes from generators with published definitions, identical on any
 * compiler and thread count:
 *   - splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 *     generators", OOPSLA 2014) as a counter-based stream and as a seeder;
 *   - xoshiro256** (Blackman, Vigna, "Scrambled linear pseudorandom number
 *     generators", 2018) for the sequential generators;
 *   - Lemire's multiply-shift bounded integers ("Fast random integer generation
 *     in an interval", ACM TOMACS 2019);
 *   - Floyd's algorithm for k distinct integers (Bentley & Floyd, CACM 1987).
 *
 * Generator families and R-MAT parameters follow the paper's experimental
 * setup appendix (Erdos-Renyi, R-MAT with Graph500 parameters, Barabasi-Albert).
 * Every graph is simple and undirected: self-loops dropped, duplicate edges
 * merged, each edge stored as two arcs; rows are sorted by column id.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *row_ptr; /* [n+1] */
  int32_t *col_idx; /* [nnz] */
} gg_csr;

/* ---------------------------------------------------------------- RNG --- */

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_next(uint64_t *s) {
  *s += SM64_GAMMA;
  return sm64_mix(*s);
}

typedef struct {
  uint64_t s[4];
} xo256;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void xo_seed(xo256 *r, uint64_t seed) {
  uint64_t sm = seed;
  for (int i = 0; i < 4; ++i) r->s[i] = sm64_next(&sm);
}

static inline uint64_t xo_next(xo256 *r) {
  uint64_t *s = r->s;
  const uint64_t result = rotl64(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl64(s[3], 45);
  return result;
}

/* Uniform integer in [0, range), range >= 1 (Lemire 2019). */
static inline uint64_t xo_bounded(xo256 *r, uint64_t range) {
  uint64_t x = xo_next(r);
  __uint128_t m = (__uint128_t)x * range;
  uint64_t l = (uint64_t)m;
  if (l < range) {
    uint64_t t = (0 - range) % range;
    while (l < t) {
      x = xo_next(r);
      m = (__uint128_t)x * range;
      l = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

static inline double u01_from64(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------- CSR assembly --- */

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Build a CSR from an edge list.  symmetrize != 0: every (u,v) is stored as
 * arcs u->v and v->u.  Rows are sorted; duplicates and self-loops dropped.
 * Row v of the result lists the sources u of arcs u->v when symmetrize == 0
 * and transpose != 0, else the targets of arcs v->u.
 */
static int build_csr(int64_t n, int64_t ne, const int32_t *src, const int32_t *dst, int symmetrize,
                     int transpose, gg_csr *out) {
  memset(out, 0, sizeof(*out));
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -6;
  for (int64_t e = 0; e < ne; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    if (symmetrize) {
      cnt[u + 1]++;
      cnt[v + 1]++;
    } else {
      cnt[(transpose ? v : u) + 1]++;
    }
  }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  int64_t total = cnt[n];
  int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!col || !pos) {
    free(cnt);
    free(col);
    free(pos);
    return -6;
  }
  memcpy(pos, cnt, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t e = 0; e < ne; ++e) {
    int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    if (symmetrize) {
      col[pos[u]++] = v;
      col[pos[v]++] = u;
    } else if (transpose) {
      col[pos[v]++] = u;
    } else {
      col[pos[u]++] = v;
    }
  }
  free(pos);
  /* sort each row, then compact duplicates in place */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096)
#endif
  for (int64_t r = 0; r < n; ++r) {
    int64_t b = cnt[r], e = cnt[r + 1];
    if (e - b > 1) qsort(col + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
  }
  int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!rp) {
    free(cnt);
    free(col);
    return -6;
  }
  int64_t w = 0;
  rp[0] = 0;
  for (int64_t r = 0; r < n; ++r) {
    int64_t b = cnt[r], e = cnt[r + 1];
    for (int64_t j = b; j < e; ++j) {
      if (j > b && col[j] == col[j - 1]) continue;
      col[w++] = col[j];
    }
    rp[r + 1] = w;
  }
  free(cnt);
  int32_t *shrunk = (int32_t *)realloc(col, sizeof(int32_t) * (size_t)(w > 0 ? w : 1));
  out->n = n;
  out->nnz = w;
  out->row_ptr = rp;
  out->col_idx = shrunk ? shrunk : col;
  return 0;
}

void gg_free(gg_csr *g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col_idx);
  g->row_ptr = NULL;
  g->col_idx = NULL;
}

int gg_from_edges(int64_t n, int64_t ne, const int32_t *src, const int32_t *dst, int symmetrize,
                  int transpose, gg_csr *out) {
  if (n < 1 || n > INT32_MAX || ne < 0) return -1;
  for (int64_t e = 0; e < ne; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -2;
  return build_csr(n, ne, src, dst, symmetrize, transpose, out);
}

/* ------------------------------------------------------ Erdos-Renyi --- */

/*
 * G(n, M): M distinct unordered non-loop pairs drawn uniformly (sequential
 * rejection against a hash set of the pairs drawn so far).
 */
int gg_er(int64_t n, int64_t m, uint64_t seed, gg_csr *out) {
  if (n < 2 || n > INT32_MAX) return -1;
  double maxm = (double)n * (double)(n - 1) / 2.0;
  if (m < 0 || (double)m > maxm) return -1;
  uint64_t cap = 16;
  while (cap < (uint64_t)m * 2 + 16) cap <<= 1;
  uint64_t *tab = (uint64_t *)malloc(sizeof(uint64_t) * cap);
  int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!tab || !src || !dst) {
    free(tab);
    free(src);
    free(dst);
    return -6;
  }
  memset(tab, 0xff, sizeof(uint64_t) * cap);
  xo256 r;
  xo_seed(&r, seed);
  int64_t got = 0;
  while (got < m) {
    uint64_t u = xo_bounded(&r, (uint64_t)n);
    uint64_t v = xo_bounded(&r, (uint64_t)n);
    if (u == v) continue;
    uint64_t a = u < v ? u : v, b = u < v ? v : u;
    uint64_t key = a * (uint64_t)n + b;
    uint64_t h = sm64_mix(key) & (cap - 1);
    int dup = 0;
    while (tab[h] != UINT64_MAX) {
      if (tab[h] == key) {
        dup = 1;
        break;
      }
      h = (h + 1) & (cap - 1);
    }
    if (dup) continue;
    tab[h] = key;
    src[got] = (int32_t)a;
    dst[got] = (int32_t)b;
    ++got;
  }
  free(tab);
  int rc = build_csr(n, m, src, dst, 1, 0, out);
  free(src);
  free(dst);
  return rc;
}

/* -------------------------------------------------- Barabasi-Albert --- */

/*
 * Preferential attachment: seed clique on m+1 vertices, then each new vertex
 * takes m distinct targets, each drawn with probability proportional to the
 * current degree (uniform draw from the list of all arc endpoints so far,
 * duplicates within one vertex's targets rejected).
 */
int gg_ba(int64_t n, int32_t m, uint64_t seed, gg_csr *out) {
  if (m < 1 || n < (int64_t)m + 1 || n > INT32_MAX) return -1;
  int64_t seed_edges = (int64_t)(m + 1) * m / 2;
  int64_t ne = seed_edges + (n - (m + 1)) * (int64_t)m;
  int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne);
  int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne);
  int32_t *ends = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * ne));
  int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  if (!src || !dst || !ends || !pick) {
    free(src);
    free(dst);
    free(ends);
    free(pick);
    return -6;
  }
  int64_t e = 0, ne_ends = 0;
  for (int32_t a = 0; a <= m; ++a)
    for (int32_t b = a + 1; b <= m; ++b) {
      src[e] = a;
      dst[e] = b;
      ++e;
      ends[ne_ends++] = a;
      ends[ne_ends++] = b;
    }
  xo256 r;
  xo_seed(&r, seed);
  for (int64_t v = m + 1; v < n; ++v) {
    int32_t got = 0;
    while (got < m) {
      int32_t t = ends[xo_bounded(&r, (uint64_t)ne_ends)];
      int dup = 0;
      for (int32_t q = 0; q < got; ++q)
        if (pick[q] == t) {
          dup = 1;
          break;
        }
      if (!dup) pick[got++] = t;
    }
    for (int32_t q = 0; q < m; ++q) {
      src[e] = (int32_t)v;
      dst[e] = pick[q];
      ++e;
      ends[ne_ends++] = (int32_t)v;
      ends[ne_ends++] = pick[q];
    }
  }
  free(ends);
  free(pick);
  int rc = build_csr(n, ne, src, dst, 1, 0, out);
  free(src);
  free(dst);
  return rc;
}

/* ------------------------------------------------------------ R-MAT --- */

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): 2^scale vertices,
 * edge_factor * 2^scale sampled edges; each edge descends `scale` levels of
 * the adjacency matrix choosing a quadrant with probabilities (a, b, c, d).
 * Sample e, level j draws splitmix64 at counter e*scale + j of the stream
 * keyed by `seed`, so the graph does not depend on the thread count.
 * Self-loops dropped, edges symmetrized and deduplicated; no noise, no
 * relabeling, isolated vertices kept.
 */
int gg_rmat(int32_t scale, int32_t edge_factor, double a, double b, double c, uint64_t seed,
            gg_csr *out) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return -1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
  int64_t n = (int64_t)1 << scale;
  int64_t ne = (int64_t)edge_factor * n;
  int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne);
  int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne);
  if (!src || !dst) {
    free(src);
    free(dst);
    return -6;
  }
  const uint64_t base = sm64_mix(seed ^ 0x5DEECE66DULL);
  const double ab = a + b, abc = a + b + c;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t e = 0; e < ne; ++e) {
    uint32_t u = 0, v = 0;
    uint64_t ctr = (uint64_t)e * (uint64_t)scale;
    for (int32_t j = 0; j < scale; ++j) {
      double p = u01_from64(sm64_mix(base + (ctr + (uint64_t)j + 1) * SM64_GAMMA));
      uint32_t bu, bv;
      if (p < a) {
        bu = 0;
        bv = 0;
      } else if (p < ab) {
        bu = 0;
        bv = 1;
      } else if (p < abc) {
        bu = 1;
        bv = 0;
      } else {
        bu = 1;
        bv = 1;
      }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    src[e] = (int32_t)u;
    dst[e] = (int32_t)v;
  }
  int rc = build_csr(n, ne, src, dst, 1, 0, out);
  free(src);
  free(dst);
  return rc;
}

/* -------------------------------------------------------------- groups --- */

/*
 * n_groups groups with sizes uniform in [smin, smax]; members are distinct and
 * uniform over [0, n) (Floyd's algorithm), emitted sorted.  offsets has
 * n_groups+1 entries; members must hold at least n_groups*smax entries.
 */
int gg_groups(int64_t n, int32_t n_groups, int32_t smin, int32_t smax, uint64_t seed,
              int64_t *offsets, int32_t *members) {
  if (n < 1 || n_groups < 0 || smin < 0 || smax < smin || smax > n) return -1;
  xo256 r;
  xo_seed(&r, seed);
  int64_t w = 0;
  offsets[0] = 0;
  for (int32_t g = 0; g < n_groups; ++g) {
    int32_t sz = smin + (int32_t)xo_bounded(&r, (uint64_t)(smax - smin + 1));
    int32_t *grp = members + w;
    int32_t got = 0;
    for (int64_t j = n - sz; j < n; ++j) {
      int32_t t = (int32_t)xo_bounded(&r, (uint64_t)(j + 1));
      int dup = 0;
      for (int32_t q = 0; q < got; ++q)
        if (grp[q] == t) {
          dup = 1;
          break;
        }
      grp[got++] = dup ? (int32_t)j : t;
    }
    qsort(grp, (size_t)sz, sizeof(int32_t), cmp_i32);
    w += sz;
    offsets[g + 1] = w;
  }
  return 0;
}

/* Uniform integers in [0, range) from the xoshiro stream keyed by seed. */
int gg_uniform_ints(int64_t count, int64_t range, uint64_t seed, int64_t *out) {
  if (count < 0 || range < 1) return -1;
  xo256 r;
  xo_seed(&r, seed);
  for (int64_t i = 0; i < count; ++i) out[i] = (int64_t)xo_bounded(&r, (uint64_t)range);
  return 0;
}

/* Uniform doubles in [0, 1) from the xoshiro stream keyed by seed. */
int gg_uniform_doubles(int64_t count, uint64_t seed, double *out) {
  if (count < 0) return -1;
  xo256 r;
  xo_seed(&r, seed);
  for (int64_t i = 0; i < count; ++i) out[i] = u01_from64(xo_next(&r));
  return 0;
}
