/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of GED-Walk group
 * centrality (Angriman, van der Grinten, Bojchevski, Zuegner, Guennemann,
 * Meyerhenke, "Group Centrality Maximization for Large-scale Graphs").  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the GPU library never does.  It shares no code with the GPU path.
 *
 * Graph convention: CSR whose row v lists the in-neighbours u of v (arcs
 * u -> v).  The paper's recurrences sum over the edges (u, v) entering v, so
 * every recurrence below is a pull over a row.  An undirected graph stores each
 * edge as two arcs.  The reverse graph (rows = out-neighbours) is passed
 * separately where walks must be counted from their start (psi^miss).
 *
 * Representation: every per-level vector is stored "decayed", i.e. level i
 * holds alpha^i times the walk count of the paper.  The recurrences are the
 * paper's, multiplied through by alpha once per level; this keeps the numbers
 * in range for any walk length.  Sums over vertices and over a row use
 * Neumaier's compensated summation (Neumaier 1974).
 *
 * Every function cites the part of the paper it follows.  The greedy driver is
 * the lazy greedy algorithm of Section 3.2.2 with the priority initialisation of
 * Lemma "initialize"; an eager variant (exact gains for every candidate) is
 * provided for cross-checks.  Readings of points the paper leaves open:
 *   - the base case of the recurrences is walk length 0 (hit_0 = 1_S,
 *     miss_0 = 1_{V\S}), which reproduces the paper's length-1 counts;
 *   - the loop index of the score algorithm is the walk length (its bound is
 *     printed as B_ell; read ell == i) and the stopping test is strict;
 *   - ties in the priority queues go to the larger value, then the smaller id;
 *   - if only one candidate remains it is accepted without a separation test;
 *   - max degree for the combinatorial bound is the maximum out-degree (equal
 *     to the maximum degree for undirected graphs);
 *   - the spectral bound needs sigma_max itself; an upper estimate replaces it
 *     (any value >= sigma_max keeps the bound valid), computed by
 *     or_sigma_max.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  OR_OK = 0,
  OR_ERR_ARG = -1,
  OR_ERR_VERTEX = -2,
  OR_ERR_ALPHA = -3,
  OR_ERR_EPS = -4,
  OR_ERR_NOMEM = -6,
  OR_ERR_ELL = -9
};

/* ------------------------------------------------------------ summation --- */

typedef struct {
  double s, c;
} nsum;

static inline void nsum_add(nsum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static inline double nsum_get(const nsum *a) { return a->s + a->c; }

static double vec_sum(int64_t n, const double *x) {
  nsum acc = {0, 0};
  for (int64_t i = 0; i < n; ++i) nsum_add(&acc, x[i]);
  return nsum_get(&acc);
}

/*
 * Arc weights for the weighted variant (Section 4.4: a walk contributes
 * alpha^i times the product of its arc weights; the recurrences only gain a
 * coefficient per arc).  NULL means every weight is 1.  Set for the duration
 * of one public call by or_set_weights (single-threaded oracle).
 */
static const double *g_w = NULL;
static const double *g_w_rev = NULL;

void or_set_weights(const double *w, const double *w_rev) {
  g_w = w;
  g_w_rev = w_rev;
}

/* sum of w(u,v) x[u] over the in-neighbours u of v */
static inline double row_sum_w(const int64_t *rp, const int32_t *ci, const double *w, int64_t v,
                               const double *x) {
  nsum acc = {0, 0};
  if (w) {
    for (int64_t j = rp[v]; j < rp[v + 1]; ++j) nsum_add(&acc, w[j] * x[ci[j]]);
  } else {
    for (int64_t j = rp[v]; j < rp[v + 1]; ++j) nsum_add(&acc, x[ci[j]]);
  }
  return nsum_get(&acc);
}

static inline double row_sum(const int64_t *rp, const int32_t *ci, int64_t v, const double *x) {
  return row_sum_w(rp, ci, g_w, v, x);
}

/* ---------------------------------------------------------- graph facts --- */

/*
 * Maximum degree deg_max of the combinatorial bound (Section 3.1.2).  For a
 * directed graph the walk-extension argument behind that bound needs the
 * maximum out-degree; with in-neighbour rows that is the largest number of
 * occurrences of a vertex in ci.
 */
/*
 * Weighted graphs: the same walk-extension argument with arc weights bounds
 * sum_x omega_{l+1}(x) by max_v (sum of the weights of the arcs leaving v)
 * times sum_x omega_l(x); that maximum replaces deg_max (the paper states the
 * bound for unweighted graphs only; this is the reading used here).
 */
double or_max_weighted_out_degree(int64_t n, const int64_t *rp, const int32_t *ci,
                                  const double *w) {
  double *acc = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  if (!acc) return -1.0;
  for (int64_t v = 0; v < n; ++v)
    for (int64_t j = rp[v]; j < rp[v + 1]; ++j) acc[ci[j]] += w ? w[j] : 1.0;
  double m = 0.0;
  for (int64_t v = 0; v < n; ++v)
    if (acc[v] > m) m = acc[v];
  free(acc);
  return m;
}

int64_t or_max_out_degree(int64_t n, const int64_t *rp, const int32_t *ci) {
  int64_t *cnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
  if (!cnt) return -1;
  for (int64_t j = 0; j < rp[n]; ++j) cnt[ci[j]]++;
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v)
    if (cnt[v] > m) m = cnt[v];
  free(cnt);
  return m;
}

/*
 * Decayed total walk counts W[i] = alpha^i * sum_x omega_i(x), i = 0..ell,
 * where omega_i(x) = sum_z (A^i)_{xz} is the Katz walk count (Section 2.1,
 * Katz definition).  sum_x omega_i(x) = 1^T A^i 1 also counts the i-walks by
 * their end vertex, which is what the pull below does.
 */
int or_walk_totals(int64_t n, const int64_t *rp, const int32_t *ci, double alpha, int32_t ell,
                   double *W) {
  if (n < 1 || ell < 0) return OR_ERR_ARG;
  double *a = (double *)malloc(sizeof(double) * (size_t)n);
  double *b = (double *)malloc(sizeof(double) * (size_t)n);
  if (!a || !b) {
    free(a);
    free(b);
    return OR_ERR_NOMEM;
  }
  for (int64_t v = 0; v < n; ++v) a[v] = 1.0;
  W[0] = (double)n;
  for (int32_t i = 1; i <= ell; ++i) {
    for (int64_t v = 0; v < n; ++v) b[v] = alpha * row_sum(rp, ci, v, a);
    W[i] = vec_sum(n, b);
    double *t = a;
    a = b;
    b = t;
  }
  free(a);
  free(b);
  return OR_OK;
}

/*
 * Combinatorial bound on the tail GED_{>ell}(V) (Section 3.1.2, Eq.
 * comb-bound): alpha^{ell+1} * deg_max / (1 - alpha*deg_max) * sum_x omega_ell(x).
 * W_ell is the decayed total alpha^ell * sum_x omega_ell(x).
 */
double or_comb_bound(double alpha, double deg_max, double W_ell) {
  double ad = alpha * deg_max;
  return alpha * (deg_max / (1.0 - ad)) * W_ell;
}

/* ------------------------------------------------------- spectral bound --- */

/*
 * Tail bound selector (Section 3.1.2): g_sigma = 0 selects the combinatorial
 * bound (Eq. comb-bound, needs alpha < 1/deg_max); g_sigma > 0 selects the
 * spectral bound (Lemma "spectral-bound", Eq. spectral-bound) with that upper
 * estimate of sigma_max, which needs only alpha < 1/sigma.  Set for one public
 * call by or_set_spectral (single-threaded oracle).
 */
static double g_sigma = 0.0;

void or_set_spectral(double sigma) { g_sigma = sigma; }

/* sqrt(|V|) * alpha^{ell+1} * sigma / (1 - alpha sigma) * sum_x omega_ell(x), with
 * the decayed total W_ell = alpha^ell sum_x omega_ell(x) */
double or_spectral_bound(double alpha, double sigma, int64_t n, double W_ell) {
  return sqrt((double)n) * alpha * (sigma / (1.0 - alpha * sigma)) * W_ell;
}

static double tail_bound(double alpha, double deg_max, int64_t n, double W_ell) {
  if (g_sigma > 0.0) return or_spectral_bound(alpha, g_sigma, n, W_ell);
  return or_comb_bound(alpha, deg_max, W_ell);
}

static int check_alpha(double alpha, double deg_max) {
  if (!(alpha > 0.0) || !isfinite(alpha)) return OR_ERR_ALPHA;
  if (g_sigma > 0.0) return alpha * g_sigma < 1.0 ? OR_OK : OR_ERR_ALPHA;
  if (deg_max > 0 && !(alpha * deg_max < 1.0)) return OR_ERR_ALPHA;
  return OR_OK;
}

/*
 * Upper estimate of sigma_max = ||A||_2, the largest singular value of the
 * adjacency matrix (Section 2.1; the spectral bound needs a value >= it).
 * sigma_max^2 is the Perron root of the nonnegative symmetric B = A^T A, and
 * for every positive vector x the Collatz-Wielandt inequality gives
 * rho(B) <= max_v (B x)_v / x_v.  So, from x_0 = 1, for k = 1..iters:
 *     z   = B x_{k-1}
 *     c_k = max_v z_v / x_{k-1,v}
 *     x_k = max((z + x_{k-1}) / max_v (z_v + x_{k-1,v}), 2^-990)
 * (a power step on B + I, which converges also on bipartite graphs, clamped
 * so every entry stays positive), and
 *     sigma_hat = sqrt(min_k c_k * (1 + 2^-40)),
 * the factor covering the rounding of the sums.  (rp_r, ci_r) are the rows of
 * A^T (out-neighbours); an undirected graph passes (rp, ci) again.  Weights,
 * when set, are w for A and w_rev for A^T.
 */
int or_sigma_max(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rp_r,
                 const int32_t *ci_r, int32_t iters, double *out) {
  if (n < 1 || iters < 1) return OR_ERR_ARG;
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  double *z = (double *)malloc(sizeof(double) * (size_t)n);
  if (!x || !y || !z) {
    free(x);
    free(y);
    free(z);
    return OR_ERR_NOMEM;
  }
  const double floor_v = ldexp(1.0, -990);
  for (int64_t v = 0; v < n; ++v) x[v] = 1.0;
  double best = INFINITY;
  for (int32_t k = 1; k <= iters; ++k) {
    for (int64_t v = 0; v < n; ++v) y[v] = row_sum_w(rp, ci, g_w, v, x);       /* A x */
    for (int64_t v = 0; v < n; ++v) z[v] = row_sum_w(rp_r, ci_r, g_w_rev, v, y); /* A^T A x */
    double c = 0.0, m = 0.0;
    for (int64_t v = 0; v < n; ++v) {
      const double r = z[v] / x[v];
      if (r > c) c = r;
      const double s = z[v] + x[v];
      if (s > m) m = s;
    }
    if (c < best) best = c;
    for (int64_t v = 0; v < n; ++v) {
      const double t = (z[v] + x[v]) / m;
      x[v] = t > floor_v ? t : floor_v;
    }
  }
  *out = sqrt(best * (1.0 + ldexp(1.0, -40)));
  free(x);
  free(y);
  free(z);
  return OR_OK;
}

/* deg_max of the bound: structural, or weighted when weights are set */
static double bound_degree(int64_t n, const int64_t *rp, const int32_t *ci) {
  if (g_w) return or_max_weighted_out_degree(n, rp, ci, g_w);
  return (double)or_max_out_degree(n, rp, ci);
}

/* ------------------------------------------------------------- scoring --- */

/*
 * GED-Walk score of a group S (Section 3.1, Algorithm "GED-Walk Computation").
 *
 * For walk length i = 1, 2, ...:
 *   phi^hit_i(v)  = sum_{(u,v) in E} phi^hit_{i-1}(u) + [v in S] phi^miss_{i-1}(u)
 *   phi^miss_i(v) = [v not in S] sum_{(u,v) in E} phi^miss_{i-1}(u)
 *   phi_i(S)      = sum_v phi^hit_i(v)                       (Eq. phisum)
 *   c            += alpha^i phi_i(S)
 *   B_i           = combinatorial bound with sum_x omega_i(x); every i-walk
 *                   ends somewhere, so sum_x omega_i(x) = sum_v (hit + miss).
 *   stop when B_i < eps and return c.
 * Outputs: *out_c = c (the partial sum GED_{<=ell}(S)), *out_ell = the final
 * i, *out_bound = B at that i, phi[i] = alpha^i phi_i(S) for i = 1..ell
 * (phi may be NULL; it must hold max_ell + 1 entries).
 */
int or_score(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *S, int32_t s_len,
             double alpha, double eps, int32_t max_ell, double *out_c, int32_t *out_ell,
             double *out_bound, double *phi) {
  if (n < 1 || s_len < 0 || max_ell < 1) return OR_ERR_ARG;
  if (!(eps > 0.0) || !isfinite(eps)) return OR_ERR_EPS;
  double deg_max = bound_degree(n, rp, ci);
  int rc = check_alpha(alpha, deg_max);
  if (rc) return rc;
  uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
  double *hit = (double *)malloc(sizeof(double) * (size_t)n);
  double *miss = (double *)malloc(sizeof(double) * (size_t)n);
  double *hit2 = (double *)malloc(sizeof(double) * (size_t)n);
  double *miss2 = (double *)malloc(sizeof(double) * (size_t)n);
  if (!inS || !hit || !miss || !hit2 || !miss2) {
    rc = OR_ERR_NOMEM;
    goto done;
  }
  for (int32_t q = 0; q < s_len; ++q) {
    if (S[q] < 0 || S[q] >= n) {
      rc = OR_ERR_VERTEX;
      goto done;
    }
    inS[S[q]] = 1;
  }
  /* walk length 0: the single vertex v is a 0-walk; it hits S iff v in S */
  for (int64_t v = 0; v < n; ++v) {
    hit[v] = inS[v] ? 1.0 : 0.0;
    miss[v] = inS[v] ? 0.0 : 1.0;
  }
  nsum c = {0, 0};
  if (phi) phi[0] = 0.0;
  for (int32_t i = 1;; ++i) {
    if (i > max_ell) {
      rc = OR_ERR_ELL;
      goto done;
    }
    for (int64_t v = 0; v < n; ++v) {
      double h = row_sum(rp, ci, v, hit);
      if (inS[v]) {
        h += row_sum(rp, ci, v, miss);
        miss2[v] = 0.0;
      } else {
        miss2[v] = alpha * row_sum(rp, ci, v, miss);
      }
      hit2[v] = alpha * h;
    }
    double *t = hit;
    hit = hit2;
    hit2 = t;
    t = miss;
    miss = miss2;
    miss2 = t;
    double phi_i = vec_sum(n, hit);
    nsum_add(&c, phi_i);
    if (phi) phi[i] = phi_i;
    nsum w = {0, 0};
    for (int64_t v = 0; v < n; ++v) {
      nsum_add(&w, hit[v]);
      nsum_add(&w, miss[v]);
    }
    double B = tail_bound(alpha, deg_max, n, nsum_get(&w));
    if (B < eps) {
      *out_c = nsum_get(&c);
      *out_ell = i;
      *out_bound = B;
      rc = OR_OK;
      goto done;
    }
  }
done:
  free(inS);
  free(hit);
  free(miss);
  free(hit2);
  free(miss2);
  return rc;
}

/*
 * The truncated score GED_{<=ell}(S) = sum_{i=1}^{ell} alpha^i phi_i(S) at a
 * fixed ell (the partial sum defined in Section 3.1), by the same recurrences.
 */
int or_score_fixed(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *S,
                   int32_t s_len, double alpha, int32_t ell, double *out_c, double *phi) {
  if (n < 1 || s_len < 0 || ell < 0) return OR_ERR_ARG;
  uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
  double *hit = (double *)malloc(sizeof(double) * (size_t)n);
  double *miss = (double *)malloc(sizeof(double) * (size_t)n);
  double *hit2 = (double *)malloc(sizeof(double) * (size_t)n);
  double *miss2 = (double *)malloc(sizeof(double) * (size_t)n);
  int rc = OR_OK;
  if (!inS || !hit || !miss || !hit2 || !miss2) {
    rc = OR_ERR_NOMEM;
    goto done;
  }
  for (int32_t q = 0; q < s_len; ++q) {
    if (S[q] < 0 || S[q] >= n) {
      rc = OR_ERR_VERTEX;
      goto done;
    }
    inS[S[q]] = 1;
  }
  for (int64_t v = 0; v < n; ++v) {
    hit[v] = inS[v] ? 1.0 : 0.0;
    miss[v] = inS[v] ? 0.0 : 1.0;
  }
  nsum c = {0, 0};
  if (phi) phi[0] = 0.0;
  for (int32_t i = 1; i <= ell; ++i) {
    for (int64_t v = 0; v < n; ++v) {
      double h = row_sum(rp, ci, v, hit);
      if (inS[v]) {
        h += row_sum(rp, ci, v, miss);
        miss2[v] = 0.0;
      } else {
        miss2[v] = alpha * row_sum(rp, ci, v, miss);
      }
      hit2[v] = alpha * h;
    }
    double *t = hit;
    hit = hit2;
    hit2 = t;
    t = miss;
    miss = miss2;
    miss2 = t;
    double phi_i = vec_sum(n, hit);
    if (phi) phi[i] = phi_i;
    nsum_add(&c, phi_i);
  }
  *out_c = nsum_get(&c);
done:
  free(inS);
  free(hit);
  free(miss);
  free(hit2);
  free(miss2);
  return rc;
}

/* -------------------------------------------------------- marginal gain --- */

/*
 * L_ell(S, x) = GED_{<=ell}(S u {x}) - GED_{<=ell}(S) (Section 3.2.1).
 *
 * The proof of submodularity (Section 2.2) identifies the marginal gain with
 * the alpha-weighted number of walks that contain x and no vertex of S.  Those
 * are exactly the walks of the graph G - S (S deleted) that contain x, so the
 * gain is the ED-Walk partial sum of {x} in G - S, computed here with the same
 * hit/miss recurrences as the score (no subtraction of two large scores).
 * inS is a 0/1 flag per vertex; x must not be in S.
 */
double or_gain(int64_t n, const int64_t *rp, const int32_t *ci, const uint8_t *inS, int32_t x,
               double alpha, int32_t ell, double *work /* 4n doubles */) {
  double *hit = work, *miss = work + n, *hit2 = work + 2 * n, *miss2 = work + 3 * n;
  for (int64_t v = 0; v < n; ++v) {
    hit[v] = (v == x) ? 1.0 : 0.0;
    miss[v] = (v == x || inS[v]) ? 0.0 : 1.0;
  }
  nsum L = {0, 0};
  for (int32_t i = 1; i <= ell; ++i) {
    for (int64_t v = 0; v < n; ++v) {
      if (inS[v]) {
        hit2[v] = 0.0;
        miss2[v] = 0.0;
      } else if (v == x) {
        hit2[v] = alpha * (row_sum(rp, ci, v, hit) + row_sum(rp, ci, v, miss));
        miss2[v] = 0.0;
      } else {
        hit2[v] = alpha * row_sum(rp, ci, v, hit);
        miss2[v] = alpha * row_sum(rp, ci, v, miss);
      }
    }
    double *t = hit;
    hit = hit2;
    hit2 = t;
    t = miss;
    miss = miss2;
    miss2 = t;
    nsum_add(&L, vec_sum(n, hit));
  }
  return nsum_get(&L);
}

int or_gain_ext(int64_t n, const int64_t *rp, const int32_t *ci, const int32_t *S, int32_t s_len,
                int32_t x, double alpha, int32_t ell, double *out) {
  if (x < 0 || x >= n) return OR_ERR_VERTEX;
  uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
  double *work = (double *)malloc(sizeof(double) * 4 * (size_t)n);
  if (!inS || !work) {
    free(inS);
    free(work);
    return OR_ERR_NOMEM;
  }
  for (int32_t q = 0; q < s_len; ++q) {
    if (S[q] < 0 || S[q] >= n) {
      free(inS);
      free(work);
      return OR_ERR_VERTEX;
    }
    inS[S[q]] = 1;
  }
  *out = inS[x] ? 0.0 : or_gain(n, rp, ci, inS, x, alpha, ell, work);
  free(inS);
  free(work);
  return OR_OK;
}

/* ------------------------------------------------- priority initialiser --- */

/*
 * Decayed miss counts for levels 0..ell: M[i*n + v] = alpha^i phi^miss_i(v, S)
 * (Section 3.1.1).  On the reverse graph the same pull gives
 * alpha^j psi^miss_j(v, S), the walks that start at v and avoid S (Lemma
 * "initialize").
 */
static void miss_levels(int64_t n, const int64_t *rp, const int32_t *ci, const double *w,
                        const uint8_t *inS, double alpha, int32_t ell, double *M) {
  for (int64_t v = 0; v < n; ++v) M[v] = inS[v] ? 0.0 : 1.0;
  for (int32_t i = 1; i <= ell; ++i) {
    const double *prev = M + (int64_t)(i - 1) * n;
    double *cur = M + (int64_t)i * n;
    for (int64_t v = 0; v < n; ++v)
      cur[v] = inS[v] ? 0.0 : alpha * row_sum_w(rp, ci, w, v, prev);
  }
}

/*
 * Initial priorities (Lemma "initialize"):
 *   P_i(S, x) = sum_{j=0}^{i} phi^miss_{i-j}(x, S) psi^miss_j(x, S)
 *   I(x)      = sum_{i=1}^{ell} alpha^i P_i(S, x)   >=  L_ell(S, x).
 * With decayed levels alpha^i P_i = sum_j m_{i-j}(x) b_j(x).  I[x] = 0 for x in S.
 * rp_r/ci_r is the reverse graph (the same arrays for an undirected graph).
 */
int or_pinit(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rp_r,
             const int32_t *ci_r, const uint8_t *inS, double alpha, int32_t ell, double *I) {
  double *m = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(ell + 1));
  double *b = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(ell + 1));
  if (!m || !b) {
    free(m);
    free(b);
    return OR_ERR_NOMEM;
  }
  miss_levels(n, rp, ci, g_w, inS, alpha, ell, m);
  miss_levels(n, rp_r, ci_r, g_w ? g_w_rev : NULL, inS, alpha, ell, b);
  for (int64_t x = 0; x < n; ++x) {
    if (inS[x]) {
      I[x] = 0.0;
      continue;
    }
    nsum acc = {0, 0};
    for (int32_t i = 1; i <= ell; ++i)
      for (int32_t j = 0; j <= i; ++j)
        nsum_add(&acc, m[(int64_t)(i - j) * n + x] * b[(int64_t)j * n + x]);
    I[x] = nsum_get(&acc);
  }
  free(m);
  free(b);
  return OR_OK;
}

int or_pinit_ext(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rp_r,
                 const int32_t *ci_r, const int32_t *S, int32_t s_len, double alpha, int32_t ell,
                 double *I) {
  uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
  if (!inS) return OR_ERR_NOMEM;
  for (int32_t q = 0; q < s_len; ++q) {
    if (S[q] < 0 || S[q] >= n) {
      free(inS);
      return OR_ERR_VERTEX;
    }
    inS[S[q]] = 1;
  }
  int rc = or_pinit(n, rp, ci, rp_r, ci_r, inS, alpha, ell, I);
  free(inS);
  return rc;
}

/* ----------------------------------------------------- priority queues --- */

/* Indexed binary max-heap over vertex ids keyed by key[]: larger key first,
 * then smaller id. */
typedef struct {
  int32_t *h;   /* heap array of vertex ids */
  int32_t *pos; /* position of a vertex in h, -1 if absent */
  int32_t size;
  const double *key;
} iheap;

static inline int hbefore(const iheap *q, int32_t a, int32_t b) {
  double ka = q->key[a], kb = q->key[b];
  return ka > kb || (ka == kb && a < b);
}
static void hswap(iheap *q, int32_t i, int32_t j) {
  int32_t a = q->h[i], b = q->h[j];
  q->h[i] = b;
  q->h[j] = a;
  q->pos[b] = i;
  q->pos[a] = j;
}
static void hup(iheap *q, int32_t i) {
  while (i > 0) {
    int32_t p = (i - 1) / 2;
    if (!hbefore(q, q->h[i], q->h[p])) break;
    hswap(q, i, p);
    i = p;
  }
}
static void hdown(iheap *q, int32_t i) {
  for (;;) {
    int32_t l = 2 * i + 1, r = l + 1, best = i;
    if (l < q->size && hbefore(q, q->h[l], q->h[best])) best = l;
    if (r < q->size && hbefore(q, q->h[r], q->h[best])) best = r;
    if (best == i) break;
    hswap(q, i, best);
    i = best;
  }
}
static void hupdate(iheap *q, int32_t x) {
  int32_t i = q->pos[x];
  if (i < 0) return;
  hup(q, i);
  hdown(q, q->pos[x]);
}
static void hinsert(iheap *q, int32_t x) {
  q->h[q->size] = x;
  q->pos[x] = q->size;
  q->size++;
  hup(q, q->size - 1);
}
static void hremove(iheap *q, int32_t x) {
  int32_t i = q->pos[x];
  if (i < 0) return;
  int32_t last = q->size - 1;
  if (i != last) {
    hswap(q, i, last);
    q->size--;
    q->pos[x] = -1;
    hup(q, i);
    hdown(q, q->pos[q->h[i]]);
  } else {
    q->size--;
    q->pos[x] = -1;
  }
}
static void hrebuild(iheap *q, int64_t n, const uint8_t *member) {
  q->size = 0;
  for (int64_t v = 0; v < n; ++v) q->pos[v] = -1;
  for (int64_t v = 0; v < n; ++v)
    if (member[v]) {
      q->h[q->size] = (int32_t)v;
      q->pos[v] = q->size;
      q->size++;
    }
  for (int32_t i = q->size / 2 - 1; i >= 0; --i) hdown(q, i);
}

/* --------------------------------------------------------------- greedy --- */

typedef struct {
  int64_t n;
  const int64_t *rp;
  const int32_t *ci;
  uint8_t *inS;
  double alpha;
  int32_t ell;
  double B;
  double *L, *U;
  int32_t *fresh; /* L[x], U[x] exact for the current (S, ell) iff fresh[x] == stamp */
  int32_t stamp;
  double *work;
  int64_t evals;
  iheap QL, QU;
} gstate;

static void evaluate(gstate *g, int32_t x) {
  g->L[x] = or_gain(g->n, g->rp, g->ci, g->inS, x, g->alpha, g->ell, g->work);
  g->U[x] = g->L[x] + g->B;
  g->fresh[x] = g->stamp;
  g->evals++;
}

/* Procedure lazyUpdate (Algorithm "lazy greedy"): refresh the top of Q until
 * the top element carries its exact L_ell and U_ell. */
static int32_t lazy_update(gstate *g, iheap *Q) {
  for (;;) {
    if (Q->size == 0) return -1;
    int32_t x = Q->h[0];
    if (g->fresh[x] == g->stamp) return x; /* re-evaluating gives the same value */
    evaluate(g, x);
    hupdate(&g->QL, x);
    hupdate(&g->QU, x);
    if (Q->h[0] == x) return x;
  }
}

/*
 * Greedy GED-Walk maximisation (Section 3.2.2, Algorithm "lazy greedy"), with
 * (eps/k)-separation between the best and the runner-up candidate and ell
 * doubled on failure.  lazy != 0 uses the two priority queues with the
 * initialisation of Lemma "initialize"; lazy == 0 evaluates L_ell for every
 * candidate (same decisions, used to cross-check the lazy bookkeeping).
 *
 * A forced prefix (forced[0..n_forced)) is added to S first without any test,
 * after which ell starts at forced_ell (>= 1); this replays a decision sequence.
 *
 * Per pick p the trace holds the walk length, L(u), U(v) (or NaN when no
 * runner-up exists), L(v), the bound B_ell and the running number of gain
 * evaluations.  out_score is GED_{<=ell*}(S) of the final group via or_score.
 */
/*
 * Stochastic greedy sample (appendix "Dealing with large k"): for addition p
 * (|S| = p), m = ceil((n/k) ln(1/eta)) vertices (at most |V \ S|) drawn
 * without replacement from V \ S by a partial Fisher-Yates shuffle (Durstenfeld
 * 1964) of the vertices outside S in increasing id order.  Draw j uses the
 * splitmix64 output (Steele, Lea, Flood 2014) at position (p << 32) + j + 1 of
 * the stream keyed by seed, scaled into [j, rest) by a 64x64->128-bit multiply.
 * mark[v] = p for sampled v.
 */
static void draw_sample(int64_t n, const uint8_t *inS, int32_t k, double eta, uint64_t seed,
                        int32_t p, int32_t *pool, int32_t *mark) {
  int64_t rest = 0;
  for (int64_t v = 0; v < n; ++v)
    if (!inS[v]) pool[rest++] = (int32_t)v;
  int64_t m = (int64_t)ceil((double)n / k * log(1.0 / eta));
  if (m > rest) m = rest;
  for (int64_t j = 0; j < m; ++j) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL * (((uint64_t)p << 32) + (uint64_t)j + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    int64_t q = j + (int64_t)(((__uint128_t)z * (uint64_t)(rest - j)) >> 64);
    int32_t t = pool[j];
    pool[j] = pool[q];
    pool[q] = t;
  }
  for (int64_t j = 0; j < m; ++j) mark[pool[j]] = p;
}

int or_greedy_ex(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rp_r,
                 const int32_t *ci_r, int32_t k, double alpha, double eps, int32_t lazy,
                 int32_t stochastic, double eta, uint64_t seed, const int32_t *forced,
                 int32_t n_forced, int32_t forced_ell, int32_t max_ell, int32_t stop_after,
                 int32_t *out_group, int32_t *tr_ell, double *tr_L1, double *tr_U2,
                 double *tr_L2, double *tr_B, int64_t *tr_evals, double *out_score,
                 int32_t *out_score_ell);

/* The sample of addition p for group S (test helper): writes the sampled ids
 * (increasing) to out and returns their number. */
int64_t or_sample(int64_t n, const int32_t *S, int32_t s_len, int32_t k, double eta, uint64_t seed,
                  int32_t p, int32_t *out) {
  uint8_t *inS = (uint8_t *)calloc((size_t)n, 1);
  int32_t *pool = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!inS || !pool || !mark) {
    free(inS);
    free(pool);
    free(mark);
    return -1;
  }
  for (int32_t q = 0; q < s_len; ++q) inS[S[q]] = 1;
  for (int64_t v = 0; v < n; ++v) mark[v] = -1;
  draw_sample(n, inS, k, eta, seed, p, pool, mark);
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v)
    if (mark[v] == p) out[m++] = (int32_t)v;
  free(inS);
  free(pool);
  free(mark);
  return m;
}

int or_greedy(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rp_r,
              const int32_t *ci_r, int32_t k, double alpha, double eps, int32_t lazy,
              const int32_t *forced, int32_t n_forced, int32_t forced_ell, int32_t max_ell,
              int32_t *out_group, int32_t *tr_ell, double *tr_L1, double *tr_U2, double *tr_L2,
              double *tr_B, int64_t *tr_evals, double *out_score, int32_t *out_score_ell) {
  return or_greedy_ex(n, rp, ci, rp_r, ci_r, k, alpha, eps, lazy, 0, 0.0, 0, forced, n_forced,
                      forced_ell, max_ell, 0, out_group, tr_ell, tr_L1, tr_U2, tr_L2, tr_B,
                      tr_evals, out_score, out_score_ell);
}

int or_greedy_ex(int64_t n, const int64_t *rp, const int32_t *ci, const int64_t *rp_r,
                 const int32_t *ci_r, int32_t k, double alpha, double eps, int32_t lazy,
                 int32_t stochastic, double eta, uint64_t seed, const int32_t *forced,
                 int32_t n_forced, int32_t forced_ell, int32_t max_ell, int32_t stop_after,
                 int32_t *out_group, int32_t *tr_ell, double *tr_L1, double *tr_U2,
                 double *tr_L2, double *tr_B, int64_t *tr_evals, double *out_score,
                 int32_t *out_score_ell) {
  if (n < 1 || k < 1 || k > n || n_forced < 0 || n_forced > k || max_ell < 1) return OR_ERR_ARG;
  if (stop_after < 0 || stop_after > k) return OR_ERR_ARG;
  /* stop_after = m in [1, k) returns after the first m picks of the k-pick
   * run (the separation threshold stays eps/k); 0 runs all k picks */
  const int32_t stop = stop_after > 0 ? stop_after : k;
  if (stochastic && !(eta > 0.0 && eta < 1.0)) return OR_ERR_ARG;
  if (!(eps > 0.0) || !isfinite(eps)) return OR_ERR_EPS;
  double deg_max = bound_degree(n, rp, ci);
  int rc = check_alpha(alpha, deg_max);
  if (rc) return rc;

  gstate g;
  memset(&g, 0, sizeof(g));
  g.n = n;
  g.rp = rp;
  g.ci = ci;
  g.alpha = alpha;
  g.inS = (uint8_t *)calloc((size_t)n, 1);
  uint8_t *cand = (uint8_t *)calloc((size_t)n, 1);
  g.L = (double *)malloc(sizeof(double) * (size_t)n);
  g.U = (double *)malloc(sizeof(double) * (size_t)n);
  g.fresh = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  g.work = (double *)malloc(sizeof(double) * 4 * (size_t)n);
  double *W = (double *)malloc(sizeof(double) * (size_t)(max_ell + 1));
  g.QL.h = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  g.QL.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  g.QU.h = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  g.QU.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  g.QL.key = g.L;
  g.QU.key = g.U;
  int32_t *pool = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t sampled_for = -1;
  int32_t s_size = 0;
  if (!g.inS || !cand || !g.L || !g.U || !g.fresh || !g.work || !W || !g.QL.h || !g.QL.pos ||
      !g.QU.h || !g.QU.pos || !pool || !mark) {
    rc = OR_ERR_NOMEM;
    goto done;
  }
  for (int64_t v = 0; v < n; ++v) {
    g.fresh[v] = -1;
    mark[v] = -1;
  }
  g.stamp = 0;

  for (int32_t p = 0; p < n_forced; ++p) {
    int32_t u = forced[p];
    if (u < 0 || u >= n || g.inS[u]) {
      rc = OR_ERR_VERTEX;
      goto done;
    }
    g.inS[u] = 1;
    out_group[s_size] = u;
    if (tr_ell) tr_ell[s_size] = -1;
    if (tr_L1) tr_L1[s_size] = NAN;
    if (tr_U2) tr_U2[s_size] = NAN;
    if (tr_L2) tr_L2[s_size] = NAN;
    if (tr_B) tr_B[s_size] = NAN;
    if (tr_evals) tr_evals[s_size] = 0;
    s_size++;
  }
  g.ell = n_forced > 0 ? (forced_ell >= 1 ? forced_ell : 1) : 1;

  while (s_size < stop) {
    /* reset: new walk length, fresh priorities */
    if (g.ell > max_ell) {
      rc = OR_ERR_ELL;
      goto done;
    }
    rc = or_walk_totals(n, rp, ci, alpha, g.ell, W);
    if (rc) goto done;
    g.B = tail_bound(alpha, deg_max, n, W[g.ell]);
    g.stamp++;
    if (lazy) {
      rc = or_pinit(n, rp, ci, rp_r, ci_r, g.inS, alpha, g.ell, g.L);
      if (rc) goto done;
      for (int64_t v = 0; v < n; ++v) g.U[v] = g.L[v] + g.B;
    }
    int32_t heaps_for = -1; /* addition whose candidate set the heaps hold */
    for (;;) {
      if (s_size >= stop) break;
      if (stochastic && sampled_for != s_size) {
        draw_sample(n, g.inS, k, eta, seed, s_size, pool, mark);
        sampled_for = s_size;
      }
      if (lazy && heaps_for != s_size) {
        /* stale L, U stay valid upper bounds (non-increasing in S) */
        for (int64_t v = 0; v < n; ++v)
          cand[v] = (!g.inS[v] && (!stochastic || mark[v] == s_size)) ? 1 : 0;
        hrebuild(&g.QL, n, cand);
        hrebuild(&g.QU, n, cand);
        heaps_for = s_size;
      }
      int32_t u = -1, v = -1;
      if (lazy) {
        u = lazy_update(&g, &g.QL);
        hremove(&g.QL, u);
        hremove(&g.QU, u);
        v = lazy_update(&g, &g.QU);
      } else {
        for (int64_t x = 0; x < n; ++x) {
          if (g.inS[x] || (stochastic && mark[x] != s_size)) continue;
          if (g.fresh[x] != g.stamp) evaluate(&g, (int32_t)x);
          if (u < 0 || g.L[x] > g.L[u] || (g.L[x] == g.L[u] && x < u)) {
            v = u;
            u = (int32_t)x;
          } else if (v < 0 || g.L[x] > g.L[v] || (g.L[x] == g.L[v] && x < v)) {
            v = (int32_t)x;
          }
        }
      }
      /* (eps/k)-separation test between u and the runner-up v */
      if (v >= 0 && g.L[u] <= g.U[v] - eps / (double)k) {
        if (lazy) {
          hinsert(&g.QL, u);
          hinsert(&g.QU, u);
        }
        break;
      }
      g.inS[u] = 1;
      out_group[s_size] = u;
      if (tr_ell) tr_ell[s_size] = g.ell;
      if (tr_L1) tr_L1[s_size] = g.L[u];
      if (tr_U2) tr_U2[s_size] = v >= 0 ? g.U[v] : NAN;
      if (tr_L2) tr_L2[s_size] = v >= 0 ? g.L[v] : NAN;
      if (tr_B) tr_B[s_size] = g.B;
      if (tr_evals) tr_evals[s_size] = g.evals;
      s_size++;
      g.stamp++; /* S changed: every value is stale (still an upper bound) */
    }
    if (s_size >= stop) break;
    g.ell *= 2;
  }
  if (out_score) {
    int32_t ell_s = 0;
    double Bs = 0.0;
    rc = or_score(n, rp, ci, out_group, s_size, alpha, eps, 1 << 20, out_score, &ell_s, &Bs,
                  NULL);
    if (out_score_ell) *out_score_ell = ell_s;
    if (rc) goto done;
  }
  rc = OR_OK;
done:
  free(g.inS);
  free(cand);
  free(g.L);
  free(g.U);
  free(g.fresh);
  free(g.work);
  free(W);
  free(g.QL.h);
  free(g.QL.pos);
  free(g.QU.h);
  free(g.QU.pos);
  free(pool);
  free(mark);
  return rc;
}
