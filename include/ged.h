/*
 * ged.h -- C ABI of the GED-Walk library for AMD Instinct MI355X (gfx950).
 *
 * GED-Walk group centrality (Angriman et al., "Group Centrality Maximization
 * for Large-scale Graphs"): for a group S of vertices,
 *     GED(S) = sum_{i>=1} alpha^i * phi_i(S),
 * phi_i(S) = number of walks of length i that contain at least one vertex of S
 * (Section 2.1, Definition "GED-Walk").  The library computes the partial sum
 * up to the walk length ell* at which the combinatorial tail bound drops below
 * eps (Section 3.1, Algorithm "GED-Walk Computation"), and maximises it
 * greedily with (eps/k)-separation (Section 3.2.2, Algorithm "lazy greedy").
 * Every step runs in HIP kernels on the GPU in FP64.
 *
 * Conventions shared by every entry point:
 *  - Graphs are CSR whose row v lists the in-neighbours u of v (arcs u -> v).
 *    An undirected graph stores each edge as two arcs, so its rows are
 *    neighbour lists.  Vertex ids are 0..n-1; col_idx is int32.
 *  - Pointers are host pointers unless the name starts with d_.  The caller
 *    owns every input array; the library copies what it keeps before the call
 *    returns.  Outputs go to caller-allocated buffers of the stated length.
 *  - Return value: GED_OK (0) or a negative GED_ERR_* code; ged_last_error()
 *    returns a message for the last failure of the calling thread.  No C++
 *    exception crosses this boundary.
 *  - alpha: 0 < alpha < 1/deg_max (the combinatorial bound needs
 *    alpha * deg_max < 1, Section 3.1.2); deg_max is the maximum out-degree
 *    (the maximum degree for undirected graphs).  Otherwise GED_ERR_ALPHA.
 *  - eps: finite and > 0, otherwise GED_ERR_EPS.
 *  - Groups have set semantics: duplicate ids are ignored and order does not
 *    matter; an id outside [0, n) gives GED_ERR_VERTEX.
 *  - Calls on one graph handle are serialised by the library; different
 *    handles may be used from different threads.
 */
#ifndef GED_H
#define GED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ged_status {
  GED_OK = 0,
  GED_ERR_ARG = -1,    /* bad size, null pointer or unsupported flag */
  GED_ERR_VERTEX = -2, /* vertex id out of range, or duplicate where forbidden */
  GED_ERR_ALPHA = -3,  /* alpha not in (0, 1/deg_max) */
  GED_ERR_EPS = -4,    /* eps not finite and positive */
  GED_ERR_GRAPH = -5,  /* malformed CSR */
  GED_ERR_NOMEM = -6,  /* device allocation failed, or over the serving budget */
  GED_ERR_DEVICE = -7, /* a HIP call failed (message in ged_last_error) */
  GED_ERR_BUSY = -8,   /* serving queue full; or the graph is registered with a server */
  GED_ERR_ELL = -9,    /* walk length limit (65536) reached */
  GED_ERR_CANCELLED = -10, /* serving: the request was cancelled */
  GED_ERR_DEADLINE = -11   /* serving: the request passed its deadline */
};

#define GED_UNDIRECTED 1u /* col_idx is symmetric: rows are neighbour lists */
#define GED_DIRECTED 2u   /* rows are in-neighbour lists of a directed graph */
#define GED_WEIGHTED 4u   /* per-arc weights given (ged_graph_create_weighted) */
#define GED_KEEP_ORDER 8u /* keep the caller's vertex order on the device (default:
                             vertices are stored by decreasing out-degree, which
                             concentrates the gathers of hub values in cache;
                             results and ids seen by the caller are unchanged) */

typedef struct ged_graph ged_graph;

/*
 * Create a graph handle from a host CSR (row_ptr int64[n+1], col_idx
 * int32[nnz]); the arrays are copied to device memory owned by the handle.
 * flags: exactly one of GED_UNDIRECTED / GED_DIRECTED, optionally OR-ed with
 * GED_KEEP_ORDER.  Validation
 * (GED_ERR_GRAPH): row_ptr[0] == 0, non-decreasing, row_ptr[n] == nnz,
 * 0 <= col_idx < n, no self-loops, nnz < 2^31; for GED_UNDIRECTED the arc set
 * must be symmetric.  Duplicate arcs count as parallel edges.
 * n must be in [1, 2^31 - 2].  The host side of the construction (validation,
 * the vertex order, sorted rows) runs on up to 16 host threads for graphs of
 * 2^20 arcs and more; the handle is the same at any thread count.
 */
int ged_graph_create(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                     uint32_t flags, ged_graph **out);

/*
 * Weighted variant (Section 4.4: a walk contributes alpha^i times the product
 * of its arc weights).  weights float64[nnz], each in (0, 1], aligned with
 * col_idx.  The tail bound uses the maximum weighted out-degree in place of
 * deg_max, so alpha must satisfy alpha * max_v sum_{v->w} w(v,w) < 1.
 */
int ged_graph_create_weighted(int64_t n, int64_t nnz, const int64_t *row_ptr,
                              const int32_t *col_idx, const double *weights, uint32_t flags,
                              ged_graph **out);

/* Release the handle and all device memory it owns.  NULL is accepted. */
int ged_graph_destroy(ged_graph *g);

/* n, nnz (stored arcs) and deg_max (maximum out-degree) of the graph. */
int ged_graph_info(const ged_graph *g, int64_t *n, int64_t *nnz, int32_t *max_deg);

/* 1 / (deg_max + 1), the alpha every benchmark workload uses; for a weighted
 * graph, 1 / (max weighted out-degree + 1). */
double ged_default_alpha(const ged_graph *g);

/*
 * Make the library launch this graph's work on `hip_stream` (a hipStream_t;
 * NULL selects the handle's own stream).  The stream must belong to the
 * current device and outlive its use.
 */
int ged_set_stream(ged_graph *g, void *hip_stream);

/*
 * Tail bound used to choose ell* and, in the greedy, U = L + B_ell
 * (Section 3.1.2).  GED_BOUND_COMBINATORIAL (the default) is Eq. comb-bound
 * and needs alpha * deg_max < 1.  GED_BOUND_SPECTRAL is Lemma
 * "spectral-bound", sqrt(n) alpha sigma / (1 - alpha sigma) * sum(t_ell), which
 * needs only alpha * sigma < 1; sigma is an upper estimate of sigma_max
 * (ged_sigma_max).  Changing the bound drops the cached precomputation.
 * Returns GED_ERR_ARG for an unknown kind.
 */
#define GED_BOUND_COMBINATORIAL 0
#define GED_BOUND_SPECTRAL 1
int ged_set_tail_bound(ged_graph *g, int32_t kind);

/*
 * Upper estimate of sigma_max, the largest singular value of the (weighted)
 * adjacency matrix (Section 2.1; the spectral bound is valid with any value
 * >= sigma_max).  sigma_max^2 is the Perron root of B = A^T A, and for every
 * positive x the Collatz-Wielandt inequality bounds it by max_v (Bx)_v / x_v;
 * from x = 1 the library takes 100 power steps on B + I (entries kept
 * >= 2^-990) and returns sqrt(min over the steps of that maximum * (1 + 2^-40)).
 * Computed on the device on first use and cached on the handle.
 */
int ged_sigma_max(ged_graph *g, double *out_sigma);

typedef struct {
  int32_t ell;       /* ell*: first walk length whose tail bound is < eps */
  double bound;      /* B_{ell*} of the selected tail bound */
  double walk_total; /* alpha^{ell*} * sum_x omega_{ell*}(x) */
} ged_score_info;

/*
 * Per-(graph, alpha, eps) precomputation: the decayed total-walk levels
 * t_i = alpha * A t_{i-1}, t_0 = 1 (Katz walk counts, Section 2.1), their sums
 * and the tail bound B_i (combinatorial: alpha*deg_max/(1 - alpha*deg_max) *
 * sum(t_i), Eq. comb-bound; or spectral, see ged_set_tail_bound) until
 * B_i < eps.  ell* does not depend on S because the
 * bound is taken on the whole vertex set (Eq. katz-bound).  Called implicitly
 * by the score entry points; cached on the handle.  info may be NULL.
 */
int ged_prepare(ged_graph *g, double alpha, double eps, ged_score_info *info);

/* Drop the cached per-(alpha, eps) precomputation; the next call recomputes it. */
int ged_invalidate(ged_graph *g);

/*
 * GED_{<=ell*}(S) for one group (Section 3.1, Algorithm "GED-Walk
 * Computation").  GED(S) - eps < *out_score <= GED(S).  s_len == 0 gives 0;
 * duplicate members count once.  On undirected graphs the sum is formed from
 * the hit chain up to ceil(ell* / 2) by cutting each walk in two (both halves
 * are counted by the hit and total-walk chains); the result agrees with the
 * level-by-level sum to rounding.  info may be NULL.  Blocks until the result
 * is on the host.
 */
int ged_score(ged_graph *g, const int32_t *S, int32_t s_len, double alpha, double eps,
              double *out_score, ged_score_info *info);

/*
 * Scores of n_groups groups in one batched pass (group j is
 * members[offsets[j] .. offsets[j+1])), all at the shared ell*.  Groups run as
 * columns of a masked sparse-matrix x dense-matrix product, in tiles whose
 * width is chosen per graph by an autotuner; out_scores float64[n_groups].
 * Each result equals ged_score on the same group to ~1e-12 relative.
 */
int ged_score_batch(ged_graph *g, const int64_t *offsets, const int32_t *members,
                    int32_t n_groups, double alpha, double eps, double *out_scores);

/* Tile width (columns) the autotuner picked for ged_score_batch on this graph
 * (0 if not tuned yet). */
int32_t ged_batch_tile(const ged_graph *g);

/* Fix the tile width of ged_score_batch (a power of two <= 64), or 0 to let
 * the autotuner choose it (and the row-split threshold) on the next call. */
int ged_set_batch_tile(ged_graph *g, int32_t tile);

/*
 * Row-split threshold of ged_score_batch's tiles, as a divisor cut_div of a
 * step block's staging capacity (2048 FP64 values, i.e. 2048 / C arcs at C
 * columns, twice that for 32-bit counts gathered as column pairs): rows with
 * more arcs than capacity / cut_div are cut into fixed segments summed by a
 * fix-up pass, and no block takes more arcs than that.  cut_div 1, 2 or 4,
 * or 0 to let the autotuner choose it after the tile width (it races 2 and 4
 * against 1 at the chosen width).  Results are the same to rounding for any
 * threshold; a graph's batch scores are reproducible bit for bit while it is
 * fixed.  ged_batch_row_cut returns the divisor in use (0 before tuning).
 */
int ged_set_batch_row_cut(ged_graph *g, int32_t cut_div);
int32_t ged_batch_row_cut(const ged_graph *g);

/*
 * Width of the level-2 walk counts in ged_score_batch's tiles (undirected
 * unweighted graphs; the second level of the hit chain of Section 3.1.1,
 * pushed as exact integers).  On such a graph the level-2 count at v is at
 * most omega_2(v), the number of length-2 walks ending at v, so it fits 16
 * bits wherever omega_2(v) <= 2^16 - 2 (2^16 - 1 marks the rows below the
 * cut in the gather's staging).  The library keeps vertices in
 * decreasing-degree order; the rows below a cut `hub` (which must include
 * every vertex with omega_2 > 2^16 - 2) keep 32-bit counts and all others
 * are stored in 16 bits, halving the bytes the next level gathers per arc.
 * hub = 0 (default): the least such cut, when it is at most n/8, for tiles
 * of at least 4 columns whose plan stores its deeper levels as 32-bit counts
 * (or has none); -1: never; hub > 0: that cut (GED_ERR_ARG if it is below
 * the least cut or not below n).  With the layout the last stored level
 * (above 2) also keeps a 16-bit copy of its exact counts, marking those
 * above 2^16 - 2, and the combining step gathers that copy.  The counts are
 * exact integers either way, but the 16-bit steps sum rows in blocks of
 * more arcs, so scores with and without the layout differ by the rounding of
 * the column sums (~1e-16 relative); they are bit-identical among the 16-bit
 * settings.  ged_count16_hub returns the cut the last ged_score_batch used,
 * -1 for 32-bit counts.
 */
int ged_set_count16(ged_graph *g, int32_t hub);
int32_t ged_count16_hub(const ged_graph *g);

/*
 * Layout of the rows above the row-split threshold in every step (the
 * per-level pull of Section 3.1.1).  Their arcs can be grouped by source:
 * the vertex range is cut into buckets of `bytes` of gathered vector, each
 * row's arcs in one bucket form pieces, and the blocks summing the pieces
 * are dealt bucket range by bucket range to the device's XCDs, so that the
 * slice each XCD gathers from stays in its L2 (the long rows' col_idx
 * entries are copied once per partition for this).  bytes 0 (the default)
 * does so with 3 MiB buckets on unweighted graphs whose gathered vector
 * exceeds 24 MiB, for gathers of 16 to 32 bytes per arc; bytes < 0 never
 * does; bytes > 0 always does (gathers of at most 32 bytes per arc), with
 * that bucket size (any graph, any size: for tests and tuning).  Results are the same to rounding for any layout
 * and reproducible bit for bit under one.  Set it before the first call
 * that computes anything: GED_ERR_BUSY once a step partition exists.
 * ged_source_buckets returns the setting.
 */
int ged_set_source_buckets(ged_graph *g, int64_t bytes);
int64_t ged_source_buckets(const ged_graph *g);

/*
 * Host-only diagnostic (touches no device): the step partition the library
 * builds for a CSR whose rows it would store as given (row_ptr [n+1],
 * col_idx [nnz], rows sorted), gathering `units` 8-byte units per arc, with
 * row-split divisor cut_div (1, 2, 4) and source buckets of bucket_rows
 * vertices (0: segments).  counts is always filled; each non-NULL array
 * receives its part of the plan, sized from the counts of a first call:
 *   blocks [4*n_blocks]  row blocks (row0, row1, arc0, arc1)
 *   grid2 [4*n_grid2]    segments (row, arc0, arc1, long index), or bucket
 *                        blocks (piece0, piece1, arc0, arc1) in launch order
 *   long_rows [n_long], long_first [n_long+1]
 *   bk_ptr [n_segs+1], bk_lsub [n_segs], bk_ci [bk_arcs]  (buckets only)
 * The CPU tests check every index of the step kernels against it.
 */
typedef struct {
  int32_t n_blocks, n_grid2, n_segs, n_long, cut, bucketed;
  int64_t bucket_rows, bk_arcs;
} ged_partition_counts;
int ged_partition_plan(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t units,
                       int32_t cut_div, int64_t bucket_rows, ged_partition_counts *counts,
                       int32_t *blocks, int32_t *grid2, int32_t *long_rows,
                       int32_t *long_first, int32_t *bk_ptr, int32_t *bk_lsub, int32_t *bk_ci);

typedef struct {
  /* per-pick outputs, arrays of length k (any may be NULL) */
  int32_t *ell;  /* walk length at which the pick was separated */
  double *L1;    /* L_ell(S, u) of the pick u */
  double *U2;    /* U_ell(S, v) = L_ell(S, v) + B_ell of the runner-up v (NaN if none) */
  double *L2;    /* L_ell(S, v) (NaN if none) */
  double *B;     /* B_ell(V) */
  int64_t *evals; /* running count of exact gain evaluations */
  /* optional forced prefix: these picks are taken first without tests, then
   * the search continues from walk length forced_ell (>= 1) */
  const int32_t *forced;
  int32_t n_forced;
  int32_t forced_ell;
  /* outputs */
  int32_t score_ell; /* ell* used for *out_score */
  int32_t n_rounds;  /* separation attempts (accepted + failed) */
} ged_greedy_trace;

/*
 * Greedy maximisation (Section 3.2.2): repeatedly add the vertex u with the
 * largest L_ell(S, u) once it is (eps/k)-separated from the runner-up v, i.e.
 * L(u) > L(v) + B_ell - eps/k; otherwise double ell.  Priorities start from the
 * upper bounds of Lemma "initialize".  Ties go to the larger value, then the
 * smaller vertex id.  out_group int32[k] in pick order.  out_score (nullable)
 * receives GED_{<=ell*}(S) of the final group, as ged_score would return it.
 * k in [1, n]; trace may be NULL.
 */
int ged_greedy(ged_graph *g, int32_t k, double alpha, double eps, int32_t *out_group,
               double *out_score, ged_greedy_trace *trace);

/*
 * Stochastic greedy (appendix "Dealing with large k"): per addition, sample
 * ceil((n/k) * ln(1/eta)) candidates uniformly without replacement from
 * V \ S (seeded, splitmix64 counter stream keyed by `seed`), and separate only
 * among them.  eta in (0, 1).  Other arguments as ged_greedy.
 */
int ged_greedy_stochastic(ged_graph *g, int32_t k, double alpha, double eps, double eta,
                          uint64_t seed, int32_t *out_group, double *out_score,
                          ged_greedy_trace *trace);

/*
 * Candidate batch width of the greedy: the number of candidates whose exact
 * gains one walk-count SpMM evaluates (one column each).  The decisions do
 * not depend on it (every batch width finds the same exact top two of L_ell,
 * Section 3.2.2); it sets how much of each level's gather traffic a batch
 * shares and how many gains a pick evaluates.  width 2, 4, 8 or 16 makes
 * every batch that wide; 0 (the default) starts each separation round with a
 * batch of 2 (of 8 on graphs of at most 2^20 arcs, whose steps cost the same
 * at any width) and doubles the width of the round's later batches up to 16.
 * GED_ERR_ARG for another value.
 */
int ged_set_greedy_width(ged_graph *g, int32_t width);

/*
 * Device memory of the greedy, for callers that plan it: *estimate receives
 * an upper bound of the bytes a ged_greedy call of k picks at (alpha, eps)
 * can leave allocated on the handle (its workspace, grown to the largest walk
 * length k can reach -- the first power of two whose tail bound is below
 * eps/k, where every round separates -- and the widest candidate batch, and
 * the total-walk levels beyond ell*), counted from nothing; *held (nullable)
 * the bytes that workspace holds now.  The handle keeps the workspace for
 * later calls.  The single-group score of the final group uses the handle's
 * score workspace, which is not included.  May run the precomputation.
 */
int ged_greedy_footprint(ged_graph *g, int32_t k, double alpha, double eps, int64_t *estimate,
                         int64_t *held);

/* The width of a round's first candidate batch on this graph: the value set
 * with ged_set_greedy_width, or the default's first width when that is 0. */
int32_t ged_greedy_width(const ged_graph *g);

/*
 * For callers that cannot allocate device memory (code between other work
 * that must not call hipMalloc, tight serving loops, harnesses that forbid
 * allocation): GED_{<=ell*}(S) of one group, like ged_score, computed by the
 * level-by-level hit chain (Section 3.1.1, Eq. phisum; Algorithm "GED-Walk
 * Computation") with every per-call buffer in a fixed 80 MiB region of device
 * memory that the library holds on each device it runs on until the process
 * ends.  The call allocates nothing: ged_prepare(g, alpha, eps) must have
 * been called on the handle first (otherwise GED_ERR_ARG), and a graph and
 * group whose working memory -- about 16 bytes per vertex plus the group --
 * exceeds the region give GED_ERR_NOMEM with the sizes in ged_last_error()
 * (graphs up to about 5 million vertices fit).  Arguments, set semantics and
 * errors otherwise as ged_score; the result equals ged_score's to rounding.
 * Calls are serialised by the library (they share the region); calls made
 * through other means that overlap on one GPU would race on it.  Blocks until
 * the result is on the host.
 */
int ged_score_noalloc(ged_graph *g, const int32_t *S, int32_t s_len, double alpha, double eps,
                      double *out_score, ged_score_info *info);

/* ------------------------------------------------------------ profiling --- */

typedef struct {
  int64_t launches;        /* walk-count step launches (SpMV/SpMM) recorded */
  double total_ms;         /* sum of their durations (HIP events, launch stream) */
  double bytes;            /* algorithmic bytes they moved */
  double edges;            /* arcs x columns they traversed */
  int64_t dominant_launches; /* launches of the most time-consuming step kernel */
  double dominant_ms;        /* their summed duration */
  double dominant_bytes;     /* their summed algorithmic bytes */
  int32_t dominant_columns;  /* its column count C */
  int32_t dominant_kind;     /* its gather/epilogue variant (input mode * 16 + output mode) */
} ged_profile;

/* Start (on != 0) or stop timing every walk-count step launch of this handle
 * with a pair of HIP events on its stream; starting clears the counters. */
int ged_profile_enable(ged_graph *g, int on);
/* Read the counters (synchronises the handle's stream). */
int ged_profile_read(ged_graph *g, ged_profile *out);

/* ------------------------------------------------------------- serving --- */

typedef struct ged_server ged_server;

typedef struct {
  int64_t hbm_budget_bytes; /* admission limit for request working memory */
  int32_t score_slots;      /* columns per resident graph for score requests: 0 or a
                               power of two <= 64; 0 picks 64 (undirected, n <= 1e6),
                               32 (undirected, larger), or 64/32/16/8 for directed
                               column pools by n (<= 2e5, 1e6, 2e6, beyond) */
  int32_t max_queue;        /* requests waiting for a column or a worker before GED_ERR_BUSY */
  int32_t greedy_workers;   /* concurrent greedy requests */
} ged_server_config;

typedef struct {
  uint64_t id;
  int32_t kind;       /* 0 = score, 1 = greedy */
  int32_t status;     /* GED_OK or an error code */
  double score;       /* score, or GED_{<=ell*} of the greedy group */
  int32_t k;          /* greedy group size (group in ged_server_group) */
  int32_t graph;
  double t_submit_us; /* arrival, completion (steady clock, microseconds) */
  double t_done_us;
} ged_result;

/*
 * Continuous-batching request server.  Resident graphs keep their CSR and
 * walk-count levels in device memory.  Score requests on one graph run
 * together as the columns of a tile: on undirected graphs each launch takes
 * the waiting requests (up to score_slots) through a whole split scoring tile,
 * run at the narrowest power-of-two width that holds them, and requests
 * arriving meanwhile join the next one; on directed graphs a
 * pool of columns advances one walk length per step and admits new requests
 * into free columns between steps.  Greedy requests run on worker threads
 * (one at a time per graph) once their working memory fits the HBM budget.
 * Every result equals the same request run alone (scores to ~1e-12).
 */
int ged_server_create(const ged_server_config *cfg, ged_server **out);
/* Register a graph at (alpha, eps); *graph_id receives its index.  The handle
 * stays owned by the caller and must outlive the server; until
 * ged_server_destroy the server's threads read its precomputation, so calls
 * on the handle through other entry points must use the same alpha and eps
 * (others, and ged_invalidate / ged_set_tail_bound, give GED_ERR_BUSY).  A
 * handle serves one server at a time. */
int ged_server_add_graph(ged_server *s, ged_graph *g, double alpha, double eps, int32_t *graph_id);
int ged_server_submit_score(ged_server *s, int32_t graph_id, const int32_t *S, int32_t s_len,
                            uint64_t *req_id);
int ged_server_submit_greedy(ged_server *s, int32_t graph_id, int32_t k, uint64_t *req_id);
/* Move up to max finished results into out; waits up to timeout_us for the
 * first one (0 = do not wait). */
int ged_server_poll(ged_server *s, ged_result *out, int32_t max, int32_t *n_out,
                    int64_t timeout_us);
/* Picks of a finished greedy request (out int32[k]); valid until destroy. */
int ged_server_group(ged_server *s, uint64_t req_id, int32_t *out, int32_t k);
/*
 * Ask a request to stop.  GED_OK: it will complete with status
 * GED_ERR_CANCELLED -- a waiting request is dropped by the scheduler's next
 * pass, a running greedy stops before its next separation round (its device
 * memory stays with the graph for later requests).  GED_ERR_BUSY: a score
 * already on the device, which completes normally.  GED_ERR_ARG: unknown or
 * finished id.
 */
int ged_server_cancel(ged_server *s, uint64_t req_id);
/*
 * Absolute deadline of a request, in the clock of ged_result.t_submit_us
 * (steady clock, microseconds); 0 removes it.  A request not finished by its
 * deadline stops as ged_server_cancel would stop it and completes with
 * GED_ERR_DEADLINE (scores already on the device complete normally).
 * Deadlines are checked about every half millisecond.  GED_ERR_ARG for an
 * unknown or finished id.
 */
int ged_server_set_deadline(ged_server *s, uint64_t req_id, double deadline_us);
/* Counters: [0] admitted, [1] completed, [2] steps launched, [3] peak bytes
 * counted against the budget (lane pools, the graphs' single-score
 * workspaces, greedy working memory held with each graph, reservations of
 * running greedy requests), [4] peak active score columns, [5] rejected
 * (budget). */
int ged_server_stats(ged_server *s, int64_t *out6);
int ged_server_destroy(ged_server *s);

/* Message for the last failing call on this thread ("" if none). */
const char *ged_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GED_H */
