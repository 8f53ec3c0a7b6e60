// C ABI: graph handles, per-(alpha, eps) precomputation, single-group scoring,
// profiling.  Scoring follows Section 3.1 (Algorithm "GED-Walk Computation"):
// the walks of length i that touch S are counted by the hit chain
//     h_0 = 1_S,  h_i(v) = t_i(v) if v in S else alpha * sum_{u->v} h_{i-1}(u),
// where t_i = alpha * A t_{i-1} (t_0 = 1) counts all decayed i-walks ending at
// v.  It is the paper's phi^hit recurrence with phi^hit + phi^miss replaced by
// the total walk count (every walk either hits S or misses it), which leaves a
// single vector per level and only non-negative sums.  The score is
// sum_{i=1}^{ell*} sum_v h_i(v); ell* is the first length whose combinatorial
// bound (Eq. comb-bound) is below eps and does not depend on S.
#include <math.h>

#include <algorithm>
#include <cstring>

#include "ged_internal.h"
#include "graph_build.h"

namespace ged {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

// Partitions are kept under key C * 8 + cut_div (narrow ones negated).
static int part_key(int C, int cut_div) { return C * 8 + cut_div; }

static void check_cut(int cut_div) {
  if (cut_div != 1 && cut_div != 2 && cut_div != 4)
    throw HipError{GED_ERR_ARG, "row-split threshold divisor must be 1, 2 or 4"};
}

// Source-bucket size (in vertices) of a partition gathering `units` 8-byte
// units per arc, 0 for segments; copies col_idx to the host the first time.
// Called with parts_mu held.
static int64_t bucket_rows_for(ged_graph *g, int units, bool reverse) {
  if (g->weighted || units > kBucketMaxUnits || g->bucket_bytes < 0 || g->nnz == 0) return 0;
  if (g->bucket_bytes == 0 &&
      ((int64_t)g->n * 8 * units <= kBucketAutoBytes || units < kBucketMinUnits))
    return 0;
  const int64_t bytes = g->bucket_bytes > 0 ? g->bucket_bytes : kBucketBytes;
  std::vector<int> &h = reverse ? g->h_ci_r : g->h_ci;
  if (h.size() != (size_t)g->nnz) {
    std::vector<int> t((size_t)g->nnz);
    GED_HIP(hipMemcpy(t.data(), (reverse ? g->ci_r : g->ci).p, sizeof(int) * t.size(),
                      hipMemcpyDeviceToHost));
    h.swap(t);
  }
  return std::max<int64_t>(1, bytes / (8 * units));
}

static void build_for(ged_graph *g, Partition &p, int C, int units, bool reverse, int cut_div,
                      bool buckets = true) {
  const int64_t br = buckets ? bucket_rows_for(g, units, reverse) : 0;
  build_partition(p, reverse ? g->h_rp_r : g->h_rp, C, units, cut_div,
                  br > 0 ? (reverse ? g->h_ci_r : g->h_ci).data() : nullptr, br);
}

Partition &partition(ged_graph *g, int C, bool reverse, int cut_div) {
  check_cut(cut_div);
  std::lock_guard<std::mutex> lk(g->parts_mu);
  auto &m = reverse ? g->parts_r : g->parts;
  const int key = part_key(C, cut_div);
  auto it = m.find(key);
  if (it != m.end()) return *it->second;
  auto p = std::make_unique<Partition>();
  build_for(g, *p, C, C, reverse, cut_div);
  Partition &ref = *p;
  m[key] = std::move(p);
  return ref;
}

Partition &partition_narrow(ged_graph *g, int C, int cut_div) {
  if (C < 2) return partition(g, C, false, cut_div);
  check_cut(cut_div);
  std::lock_guard<std::mutex> lk(g->parts_mu);
  auto &m = g->parts;
  const int key = -part_key(C, cut_div);
  auto it = m.find(key);
  if (it != m.end()) return *it->second;
  auto p = std::make_unique<Partition>();
  build_for(g, *p, C, C / 2, false, cut_div);
  Partition &ref = *p;
  m[key] = std::move(p);
  return ref;
}

Partition &partition_quad(ged_graph *g, int C, int cut_div) {
  if (C < 4) throw HipError{GED_ERR_ARG, "16-bit gathers need at least 4 columns"};
  check_cut(cut_div);
  std::lock_guard<std::mutex> lk(g->parts_mu);
  auto &m = g->parts;
  const int key = -(1 << 16) - part_key(C, cut_div);
  auto it = m.find(key);
  if (it != m.end()) return *it->second;
  auto p = std::make_unique<Partition>();
  // the bucket fix-up sums at most 8 columns per row
  build_for(g, *p, C, C / 4, false, cut_div, C <= 8);
  Partition &ref = *p;
  m[key] = std::move(p);
  return ref;
}

const Partition *partition_if_built(ged_graph *g, int C) {
  std::lock_guard<std::mutex> lk(g->parts_mu);
  auto it = g->parts.find(part_key(C, 1));
  return it == g->parts.end() ? nullptr : it->second.get();
}

StepArgs base_args(ged_graph *g, bool reverse) {
  StepArgs a;
  a.rp = (reverse ? g->rp_r : g->rp).as<const int>();
  a.ci = (reverse ? g->ci_r : g->ci).as<const int>();
  a.w = g->weighted ? (reverse ? g->w_r : g->w).as<const double>() : nullptr;
  a.n = (int)g->n;
  a.hc_rows = reverse ? 0 : g->hc_rows;
  return a;
}

double algo_bytes(const ged_graph *g, int C, int in, int out, double extra_rows) {
  const double n = (double)g->n, nnz = (double)g->nnz;
  double b = 4.0 * (n + 1) + 4.0 * nnz;  // row_ptr, col_idx
  if (out == OUT_TILE32 || out == OUT_GAIN32 || out == OUT_GAINCOMB32S)
    b += 4.0 * n * C;  // Y32
  else if (out == OUT_TILE32H)
    b += 6.0 * n * C;  // Y32 and Y16
  else if (out == OUT_ZERO32 || out == OUT_GAIN32D)
    b += 12.0 * n * C;  // Y32 and Y
  else if (out != OUT_COMBINE && out != OUT_COMBINE32 && out != OUT_COMBINE32L &&
           out != OUT_COMBINE16 &&
           out != OUT_GAINCOMB && out != OUT_GAINCOMB32L && out != OUT_GAINCOMB32S)
    b += 8.0 * n * C;  // Y
  if (g->weighted) b += 8.0 * nnz;
  switch (in) {
    case IN_VEC:
    case IN_CNT: b += 8.0 * n * C; break;
    case IN_CNT32: b += 4.0 * n * C; break;
    case IN_CNT16: b += 2.0 * n * C; break;
    case IN_MASK:
    case IN_NOTMASK: b += n / 8.0; break;
    case IN_TILEMASK: b += 8.0 * n; break;
    case IN_ONEHOT: b += 4.0 * n; break;
    case IN_FRESH: b += 8.0 * n * C + 8.0 * n; break;
    default: break;  // IN_ONES reads nothing
  }
  switch (out) {
    case OUT_INJ:
    case OUT_ZERO:
    case OUT_ZERO32: b += n / 8.0; break;
    case OUT_TILE:
    case OUT_TILE32:
    case OUT_TILE32H:
    case OUT_POOL: b += 8.0 * n; break;
    case OUT_GAIN:
    case OUT_GAIN32:
    case OUT_GAIN32D: b += n / 8.0 + 4.0 * n; break;
    case OUT_COMBINE:
    case OUT_COMBINE32:
    case OUT_COMBINE32L:
    case OUT_COMBINE16: b += 8.0 * n * 3; break;  // tmask, t_a, tr
    case OUT_GAINCOMB:
    case OUT_GAINCOMB32L:
    case OUT_GAINCOMB32S: b += n / 8.0 + 4.0 * n + 16.0 * n; break;  // S bits, candidates, m_a, M_r
    default: break;
  }
  return b + 8.0 * n * C * extra_rows;
}

double comb_bound(ged_graph *g, double alpha, double W_ell) {
  if (g->bound_kind == GED_BOUND_SPECTRAL) {
    // Lemma "spectral-bound": sqrt(n) alpha^{ell+1} sigma / (1 - alpha sigma) *
    // sum_x omega_ell(x)
    const double sg = sigma_max(g);
    return sqrt((double)g->n) * alpha * (sg / (1.0 - alpha * sg)) * W_ell;
  }
  // Eq. comb-bound: alpha^{ell+1} * D/(1 - alpha D) * sum_x omega_ell(x), with the
  // decayed total W_ell = alpha^ell sum_x omega_ell(x).
  const double D = g->weighted ? g->max_wdeg : (double)g->max_deg;
  return alpha * (D / (1.0 - alpha * D)) * W_ell;
}

size_t score_bytes_held(const ged_graph *g) {
  size_t b = 0;
  for (const DBuf *d : {&g->mask, &g->vec[0], &g->vec[1], &g->s_levels, &g->acc, &g->s_dev,
                        &g->sws.blk, &g->sws.seg, &g->sws.lng, &g->sws.red2,
                        &g->split_ws.cnt1, &g->split_ws.cnt2, &g->split_ws.lv, &g->split_ws.wl,
                        &g->split_ws.wl_n, &g->split_ws.wl3, &g->split_ws.wl3_n,
                        &g->split_ws.ws.blk, &g->split_ws.ws.seg, &g->split_ws.ws.lng,
                        &g->split_ws.ws.red2, &g->split_tmask, &g->split_in})
    b += d->bytes;
  return b;
}

int check_alpha_eps(ged_graph *g, double alpha, double eps) {
  const double D = g->weighted ? g->max_wdeg : (double)g->max_deg;
  if (!(alpha > 0.0) || !isfinite(alpha)) return fail(GED_ERR_ALPHA, "alpha must be > 0");
  if (g->bound_kind == GED_BOUND_SPECTRAL) {
    if (!(alpha * sigma_max(g) < 1.0))
      return fail(GED_ERR_ALPHA, "alpha * sigma_max must be < 1 (spectral bound)");
  } else if (D > 0 && !(alpha * D < 1.0)) {
    return fail(GED_ERR_ALPHA, "alpha * max out-degree must be < 1 (combinatorial bound)");
  }
  if (!(eps > 0.0) || !isfinite(eps)) return fail(GED_ERR_EPS, "eps must be finite and > 0");
  return GED_OK;
}

// ------------------------------------------------------------- profiling --

static hipEvent_t prof_event(ged_graph *g) {
  if (g->prof.pool.empty()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      GED_HIP(hipEventCreate(&e));
      g->prof.pool.push_back(e);
    }
  }
  hipEvent_t e = g->prof.pool.back();
  g->prof.pool.pop_back();
  return e;
}

void run_step(ged_graph *g, const Partition &p, const StepArgs &a, int in, int out,
              hipStream_t st, double extra_rows) {
  if (!g->prof.on) {
    launch_step(p, a, in, out, st);
    return;
  }
  hipEvent_t e0 = prof_event(g), e1 = prof_event(g);
  GED_HIP(hipEventRecord(e0, st));
  launch_step(p, a, in, out, st, e1);
  double bytes = algo_bytes(g, a.C, in, out, extra_rows);
  if (out == OUT_TILE32H && a.y32_marked)
    bytes -= 4.0 * (double)g->n * a.C;  // Y32 only for the counts the copy marks
  g->prof.recs.push_back({e0, e1, a.C, bytes, (double)g->nnz * a.C, in * kKindBase + out});
}

// -------------------------------------------------------- precomputation --

static void ensure_levels(PrepCache &pc, int64_t n, int levels_needed, hipStream_t st) {
  const size_t need = sizeof(double) * (size_t)n * (size_t)levels_needed;
  if (pc.t_levels.bytes >= need) return;
  DBuf nb;
  nb.ensure(std::max(need, pc.t_levels.bytes * 2));
  if (pc.t_levels.p) {
    GED_HIP(hipMemcpyAsync(nb.p, pc.t_levels.p, pc.t_levels.bytes, hipMemcpyDeviceToDevice, st));
    GED_HIP(hipStreamSynchronize(st));
  }
  std::swap(pc.t_levels.p, nb.p);
  std::swap(pc.t_levels.bytes, nb.bytes);
}

// Sum of one step's single column, reduced straight into coherent host
// memory (slot 1 of out_host; a single score's result takes slot 0), after
// waiting for the stream.
static double level_sum_to_host(ged_graph *g, const Partition &p, const StepArgs &a,
                                hipStream_t st) {
  g->out_host.ensure(64, hipHostMallocCoherent);
  double *hw = g->out_host.as<double>() + 1;
  launch_reduce(p, a, hw, nullptr, nullptr, st, g->pws.scratch());
  GED_HIP(hipStreamSynchronize(st));
  return *hw;
}

// t_i = alpha * A t_{i-1} with t_0 = 1; W[i] = sum_v t_i(v) = alpha^i sum_x omega_i(x).
// Levels whose exact walk counts omega_i the graph already holds are written
// as alpha^i omega_i with W_i from the integer sums (no step, no reduction, no
// host round trip); the rest follow by steps.
int prepare(ged_graph *g, double alpha, double eps) {
  int rc = check_alpha_eps(g, alpha, eps);
  if (rc) return rc;
  if (g->served && (alpha != g->served_alpha || eps != g->served_eps))
    return fail(GED_ERR_BUSY, "the graph is registered with a server at another alpha and eps");
  PrepCache &pc = g->prep;
  if (pc.valid && pc.alpha == alpha && pc.eps == eps) return GED_OK;
  hipStream_t st = g->stream;
  const int64_t n = g->n;
  Partition &p = partition(g, 1);
  g->pws.fit(p);
  pc.valid = false;
  pc.tr_r = -1;
  pc.W.clear();
  pc.W.push_back((double)n);
  const int held = omega_prefix_levels(g);
  ensure_levels(pc, n, std::max(16, held + 1), st);
  double *T = pc.t_levels.as<double>();
  launch_fill_f64(T, 1.0, (size_t)n, st);
  const int i0 = t_levels_from_omega(g, alpha, eps, held, T, pc.W, st);
  bool done = false;
  if (i0 > 0) {
    const double B = comb_bound(g, alpha, pc.W.back());
    if (B < eps) {
      pc.ell = i0;
      pc.bound = B;
      done = true;
    }
  }
  double W_host = 0.0;
  for (int i = i0 + 1; !done; ++i) {
    if (i > 65536) return fail(GED_ERR_ELL, "walk length limit reached in precomputation");
    ensure_levels(pc, n, i + 1, st);
    T = pc.t_levels.as<double>();
    StepArgs a = base_args(g);
    g->pws.into(a);
    a.C = 1;
    a.alpha = alpha;
    a.X = T + (size_t)(i - 1) * n;
    a.Y = T + (size_t)i * n;
    run_step(g, p, a, i == 1 ? IN_ONES : IN_VEC, OUT_PLAIN, st);
    W_host = level_sum_to_host(g, p, a, st);
    pc.W.push_back(W_host);
    const double B = comb_bound(g, alpha, W_host);
    if (B < eps) {
      pc.ell = i;
      pc.bound = B;
      done = true;
    }
  }
  pc.alpha = alpha;
  pc.eps = eps;
  pc.tail_level = -1;
  pc.t_ext_count = 0;
  pc.valid = true;
  return GED_OK;
}

void t_levels_to(ged_graph *g, int L) {
  PrepCache &pc = g->prep;
  const int have = pc.ell + pc.t_ext_count;  // highest level stored
  if (L <= have) return;
  hipStream_t st = g->stream;
  const int64_t n = g->n;
  Partition &p = partition(g, 1);
  g->pws.fit(p);
  const size_t need = sizeof(double) * (size_t)n * (size_t)(L - pc.ell);
  if (pc.t_ext.bytes < need) {
    DBuf nb;
    nb.ensure(std::max(need, 2 * pc.t_ext.bytes));
    if (pc.t_ext_count > 0) {
      GED_HIP(hipMemcpyAsync(nb.p, pc.t_ext.p, sizeof(double) * (size_t)n * pc.t_ext_count,
                             hipMemcpyDeviceToDevice, st));
      GED_HIP(hipStreamSynchronize(st));
    }
    std::swap(pc.t_ext.p, nb.p);
    std::swap(pc.t_ext.bytes, nb.bytes);
  }
  for (int i = have + 1; i <= L; ++i) {
    StepArgs a = base_args(g);
    g->pws.into(a);
    a.C = 1;
    a.alpha = pc.alpha;
    a.X = t_level(g, i - 1);
    a.Y = pc.t_ext.as<double>() + (size_t)(i - pc.ell - 1) * n;
    run_step(g, p, a, IN_VEC, OUT_PLAIN, st);
    pc.t_ext_count = i - pc.ell;
  }
}

const double *t_level(const ged_graph *g, int j) {
  const PrepCache &pc = g->prep;
  if (j <= pc.ell) return pc.t_levels.as<const double>() + (size_t)j * g->n;
  return pc.t_ext.as<const double>() + (size_t)(j - pc.ell - 1) * g->n;
}

double walk_total(ged_graph *g, int ell) {
  PrepCache &pc = g->prep;
  if (ell < (int)pc.W.size()) return pc.W[ell];
  hipStream_t st = g->stream;
  const int64_t n = g->n;
  Partition &p = partition(g, 1);
  g->pws.fit(p);
  pc.t_tail[0].ensure(sizeof(double) * n);
  pc.t_tail[1].ensure(sizeof(double) * n);
  if (pc.tail_level < 0) {
    launch_copy_f64(pc.t_tail[0].as<double>(), pc.t_levels.as<double>() + (size_t)pc.ell * n,
                    (size_t)n, st);
    pc.tail_level = pc.ell;
    pc.tail_cur = 0;
  }
  double W_host = 0.0;
  while ((int)pc.W.size() <= ell) {
    StepArgs a = base_args(g);
    g->pws.into(a);
    a.C = 1;
    a.alpha = pc.alpha;
    a.X = pc.t_tail[pc.tail_cur].as<double>();
    a.Y = pc.t_tail[pc.tail_cur ^ 1].as<double>();
    run_step(g, p, a, IN_VEC, OUT_PLAIN, st);
    W_host = level_sum_to_host(g, p, a, st);
    pc.tail_cur ^= 1;
    pc.tail_level++;
    pc.W.push_back(W_host);
  }
  return pc.W[ell];
}

// ---------------------------------------------------------------- scoring --

// Enqueue the hit chain for the group held in g->s_dev (length at s_dev[0],
// members from s_dev[1]); the score accumulates in g->acc[0] and the mask is
// cleared again at the end, so it is all zero between calls.
static void enqueue_score(ged_graph *g, hipStream_t st, bool timed) {
  const int64_t n = g->n;
  const PrepCache &pc = g->prep;
  Partition &p = partition(g, 1);
  int *sd = g->s_dev.as<int>();
  launch_mask_set(g->mask.as<uint32_t>(), sd + 1, sd, g->s_cap, 1, st);
  const double *T = pc.t_levels.as<const double>();
  StepArgs a = base_args(g);
  g->sws.into(a);
  for (int i = 1; i <= pc.ell; ++i) {
    a.C = 1;
    a.alpha = pc.alpha;
    a.accum = i > 1;  // block partials of all levels add up to the score
    a.smask = g->mask.as<const uint32_t>();
    a.X = g->vec[(i - 1) & 1].as<const double>();
    a.Y = g->vec[i & 1].as<double>();
    a.inj = T + (size_t)i * n;
    if (timed)
      run_step(g, p, a, i == 1 ? IN_MASK : IN_VEC, OUT_INJ, st);
    else
      launch_step(p, a, i == 1 ? IN_MASK : IN_VEC, OUT_INJ, st);
  }
  launch_reduce(p, a, g->acc.as<double>(), nullptr, nullptr, st, g->sws.scratch());
  launch_mask_set(g->mask.as<uint32_t>(), sd + 1, sd, g->s_cap, 0, st);
}

static void drop_score_graph(ged_graph *g) {
  if (g->score_exec) (void)hipGraphExecDestroy(g->score_exec);
  if (g->score_graph) (void)hipGraphDestroy(g->score_graph);
  g->score_exec = nullptr;
  g->score_graph = nullptr;
  g->score_sig.clear();
}

static void ensure_score_buffers(ged_graph *g, int s_len, hipStream_t st) {
  const int64_t n = g->n;
  const size_t mbytes = sizeof(uint32_t) * (size_t)((n + 31) / 32 + 1);
  if (g->mask.bytes < mbytes || !g->mask.p) {
    g->mask.ensure(mbytes);
    g->mask_ready = false;
  }
  if (!g->mask_ready) {
    launch_fill_i32(g->mask.as<int>(), 0, g->mask.bytes / sizeof(int), st);
    g->mask_ready = true;
  }
  g->vec[0].ensure(sizeof(double) * (size_t)n);
  g->vec[1].ensure(sizeof(double) * (size_t)n);
  g->acc.ensure(sizeof(double) * 64);
  g->s_levels.ensure(sizeof(double) * (size_t)(g->prep.ell + 2));
  g->out_host.ensure(64, hipHostMallocCoherent);
  g->sws.fit(partition(g, 1));
  if (s_len > g->s_cap) {
    int cap = std::max(256, g->s_cap);
    while (cap < s_len) cap *= 2;
    g->s_dev.ensure(sizeof(int) * (size_t)(cap + 1));
    g->s_host.ensure(sizeof(int) * (size_t)(cap + 1));
    g->s_cap = cap;
  }
}

// Everything the captured score graph bakes in; a change forces a recapture.
static std::vector<const void *> score_signature(ged_graph *g) {
  const PrepCache &pc = g->prep;
  double a = pc.alpha;
  const void *abits;
  std::memcpy(&abits, &a, sizeof(a));
  return {g->mask.p, g->vec[0].p, g->vec[1].p, g->acc.p, g->s_levels.p, g->s_dev.p,
          g->sws.blk.p, g->sws.seg.p, g->sws.lng.p, g->sws.red2.p, pc.t_levels.p,
          (const void *)g->stream,
          abits, (const void *)(intptr_t)pc.ell, (const void *)(intptr_t)g->s_cap,
          (const void *)(intptr_t)0 /* level-by-level chain */};
}

int score_group(ged_graph *g, const int32_t *S, int32_t s_len, double alpha, double eps,
                double *out, ged_score_info *info) {
  for (int32_t q = 0; q < s_len; ++q)
    if (S[q] < 0 || S[q] >= g->n) return fail(GED_ERR_VERTEX, "group member out of range");
  int rc = prepare(g, alpha, eps);
  if (rc) return rc;
  if (info) {
    info->ell = g->prep.ell;
    info->bound = g->prep.bound;
    info->walk_total = g->prep.W[g->prep.ell];
  }
  if (s_len == 0) {
    *out = 0.0;
    return GED_OK;
  }
  if (split_ok(g)) return split_score(g, S, s_len, out);
  hipStream_t st = g->stream;
  ensure_score_buffers(g, s_len, st);
  int *hs = g->s_host.as<int>();
  hs[0] = s_len;
  for (int32_t q = 0; q < s_len; ++q) hs[1 + q] = g->new_id[S[q]];
  GED_HIP(hipMemcpyAsync(g->s_dev.p, hs, sizeof(int) * (size_t)(s_len + 1),
                         hipMemcpyHostToDevice, st));
  if (g->prof.on) {
    enqueue_score(g, st, true);
  } else {
    std::vector<const void *> sig = score_signature(g);
    if (g->score_exec && sig != g->score_sig) drop_score_graph(g);
    if (!g->score_exec) {
      GED_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        enqueue_score(g, st, false);
      } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(st, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
      }
      GED_HIP(hipStreamEndCapture(st, &g->score_graph));
      GED_HIP(hipGraphInstantiate(&g->score_exec, g->score_graph, nullptr, nullptr, 0));
      g->score_sig = sig;
    }
    GED_HIP(hipGraphLaunch(g->score_exec, st));
  }
  double *ho = g->out_host.as<double>();
  GED_HIP(hipMemcpyAsync(ho, g->acc.p, sizeof(double), hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  *out = ho[0];
  return GED_OK;
}

}  // namespace ged

using namespace ged;

ged_graph::~ged_graph() {
  if (score_exec) (void)hipGraphExecDestroy(score_exec);
  if (score_graph) (void)hipGraphDestroy(score_graph);
  for (auto &x : split_exec) x.drop();
  if (score_done) (void)hipEventDestroy(score_done);
  for (auto e : prof.pool) (void)hipEventDestroy(e);
  for (auto &r : prof.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  if (own_stream) (void)hipStreamDestroy(own_stream);
}

// ------------------------------------------------------------------ C ABI --

extern "C" const char *ged_last_error(void) { return g_err.c_str(); }

static int create_impl(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                       const double *weights, uint32_t flags, ged_graph **out) {
  if (!out) return fail(GED_ERR_ARG, "out is null");
  *out = nullptr;
  if (n < 1 || n > INT32_MAX - 1) return fail(GED_ERR_ARG, "n must be in [1, 2^31-2]");
  if (nnz < 0 || nnz >= (int64_t)INT32_MAX) return fail(GED_ERR_GRAPH, "nnz must be < 2^31");
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(GED_ERR_ARG, "null CSR array");
  const bool keep_order = (flags & GED_KEEP_ORDER) != 0;
  flags &= ~GED_KEEP_ORDER;
  if (flags != GED_UNDIRECTED && flags != GED_DIRECTED)
    return fail(GED_ERR_ARG, "flags must be GED_UNDIRECTED or GED_DIRECTED (| GED_KEEP_ORDER)");
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return fail(GED_ERR_GRAPH, "row_ptr ends mismatch");
  // validation, internal order and sorted in/out rows on the host's threads
  HostCsr hc;
  const int brc = guarded([&]() -> int {
    if (const char *m = build_host_csr(n, nnz, row_ptr, col_idx, weights,
                                       flags == GED_UNDIRECTED, keep_order, 0, hc))
      return fail(GED_ERR_GRAPH, m);
    return GED_OK;
  });
  if (brc != GED_OK) return brc;
  auto g = std::make_unique<ged_graph>();
  g->n = n;
  g->nnz = nnz;
  g->flags = flags;
  g->weighted = weights != nullptr;
  g->max_deg = hc.max_deg;
  if (weights) g->max_wdeg = hc.max_wdeg;
  g->simple = hc.simple;
  g->new_id = std::move(hc.new_id);
  g->old_id = std::move(hc.old_id);
  {
    // the LDS copy of the first rows pays where they are the sources of a
    // large share of the arcs (skewed degrees, stored by decreasing degree)
    const int h = (int)std::min<int64_t>(kHubRows, n);
    if (flags == GED_UNDIRECTED && !weights && nnz > 0 &&
        (int64_t)hc.irp[(size_t)h] * kHubShareDiv >= nnz)
      g->hc_rows = h;
  }
  const std::vector<int> &irp = hc.irp, &ici = hc.ici, &orp = hc.orp, &oci = hc.oci;
  const std::vector<double> &iw = hc.iw, &ow = hc.ow;
  return guarded([&]() -> int {
    GED_HIP(hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking));
    g->stream = g->own_stream;
    g->h_rp = irp;
    g->rp.ensure(sizeof(int) * (size_t)(n + 1));
    g->ci.ensure(sizeof(int) * (size_t)std::max<int64_t>(1, nnz));
    GED_HIP(hipMemcpy(g->rp.p, irp.data(), sizeof(int) * (size_t)(n + 1), hipMemcpyHostToDevice));
    if (nnz > 0)
      GED_HIP(hipMemcpy(g->ci.p, ici.data(), sizeof(int) * (size_t)nnz, hipMemcpyHostToDevice));
    if (weights) {
      g->w.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, nnz));
      if (nnz > 0)
        GED_HIP(hipMemcpy(g->w.p, iw.data(), sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice));
    }
    g->d_old_id.ensure(sizeof(int) * (size_t)n);
    GED_HIP(hipMemcpy(g->d_old_id.p, g->old_id.data(), sizeof(int) * (size_t)n,
                      hipMemcpyHostToDevice));
    if (flags == GED_DIRECTED) {
      g->h_rp_r = orp;
      g->rp_r.ensure(sizeof(int) * (size_t)(n + 1));
      g->ci_r.ensure(sizeof(int) * oci.size());
      GED_HIP(hipMemcpy(g->rp_r.p, orp.data(), sizeof(int) * orp.size(), hipMemcpyHostToDevice));
      GED_HIP(hipMemcpy(g->ci_r.p, oci.data(), sizeof(int) * oci.size(), hipMemcpyHostToDevice));
      if (weights) {
        g->w_r.ensure(sizeof(double) * ow.size());
        GED_HIP(hipMemcpy(g->w_r.p, ow.data(), sizeof(double) * ow.size(),
                          hipMemcpyHostToDevice));
      }
    }
    *out = g.release();
    return GED_OK;
  });
}

extern "C" int ged_graph_create(int64_t n, int64_t nnz, const int64_t *row_ptr,
                                const int32_t *col_idx, uint32_t flags, ged_graph **out) {
  return create_impl(n, nnz, row_ptr, col_idx, nullptr, flags, out);
}

extern "C" int ged_graph_create_weighted(int64_t n, int64_t nnz, const int64_t *row_ptr,
                                         const int32_t *col_idx, const double *weights,
                                         uint32_t flags, ged_graph **out) {
  if (!weights) return fail(GED_ERR_ARG, "weights is null");
  return create_impl(n, nnz, row_ptr, col_idx, weights, flags, out);
}

extern "C" int ged_graph_destroy(ged_graph *g) {
  if (!g) return GED_OK;
  {
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
  }
  batch_forget(g);
  greedy_forget(g);
  delete g;
  return GED_OK;
}

extern "C" int ged_graph_info(const ged_graph *g, int64_t *n, int64_t *nnz, int32_t *max_deg) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (max_deg) *max_deg = g->max_deg;
  return GED_OK;
}

extern "C" double ged_default_alpha(const ged_graph *g) {
  if (!g) return 0.0;
  if (g->weighted) return 1.0 / (g->max_wdeg + 1.0);
  return 1.0 / ((double)g->max_deg + 1.0);
}

extern "C" int ged_set_stream(ged_graph *g, void *hip_stream) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() -> int {
    GED_HIP(hipStreamSynchronize(g->stream));
    g->stream = hip_stream ? (hipStream_t)hip_stream : g->own_stream;
    return GED_OK;
  });
}

extern "C" int ged_prepare(ged_graph *g, double alpha, double eps, ged_score_info *info) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() -> int {
    int rc = prepare(g, alpha, eps);
    if (rc) return rc;
    if (info) {
      info->ell = g->prep.ell;
      info->bound = g->prep.bound;
      info->walk_total = g->prep.W[g->prep.ell];
    }
    return GED_OK;
  });
}

extern "C" int ged_set_tail_bound(ged_graph *g, int32_t kind) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  if (kind != GED_BOUND_COMBINATORIAL && kind != GED_BOUND_SPECTRAL)
    return fail(GED_ERR_ARG, "unknown tail bound");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  if (g->served) return fail(GED_ERR_BUSY, "the graph is registered with a server");
  return guarded([&]() -> int {
    GED_HIP(hipStreamSynchronize(g->stream));
    if (g->bound_kind != kind) {
      g->bound_kind = kind;
      g->prep.valid = false;
      g->prep.tr_r = -1;
      g->prep.W.clear();
      g->prep.tail_level = -1;
    }
    return GED_OK;
  });
}

extern "C" int ged_sigma_max(ged_graph *g, double *out_sigma) {
  if (!g || !out_sigma) return fail(GED_ERR_ARG, "null argument");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() -> int {
    *out_sigma = sigma_max(g);
    return GED_OK;
  });
}

extern "C" int ged_set_source_buckets(ged_graph *g, int64_t bytes) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  std::lock_guard<std::mutex> pk(g->parts_mu);
  if (!g->parts.empty() || !g->parts_r.empty())
    return fail(GED_ERR_BUSY, "the graph's step partitions are already built");
  g->bucket_bytes = bytes;
  return GED_OK;
}

extern "C" int64_t ged_source_buckets(const ged_graph *g) { return g ? g->bucket_bytes : 0; }

extern "C" int ged_partition_plan(const int32_t *row_ptr, const int32_t *col_idx, int32_t n,
                                  int32_t units, int32_t cut_div, int64_t bucket_rows,
                                  ged_partition_counts *counts, int32_t *blocks, int32_t *grid2,
                                  int32_t *long_rows, int32_t *long_first, int32_t *bk_ptr,
                                  int32_t *bk_lsub, int32_t *bk_ci) {
  if (!row_ptr || !counts || n < 0 || units < 1 || bucket_rows < 0 ||
      (bucket_rows > 0 && !col_idx))
    return fail(GED_ERR_ARG, "bad argument to ged_partition_plan");
  if (cut_div != 1 && cut_div != 2 && cut_div != 4)
    return fail(GED_ERR_ARG, "cut_div must be 1, 2 or 4");
  if (row_ptr[0] != 0) return fail(GED_ERR_GRAPH, "row_ptr[0] must be 0");
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return fail(GED_ERR_GRAPH, "row_ptr must not decrease");
  if (col_idx)
    for (int32_t j = 0; j < row_ptr[n]; ++j)
      if (col_idx[j] < 0 || col_idx[j] >= n) return fail(GED_ERR_GRAPH, "col_idx out of range");
  return guarded([&]() -> int {
    PartitionPlan pl;
    plan_partition(pl, row_ptr, col_idx, n, units, cut_div, bucket_rows);
    counts->n_blocks = pl.n_blocks;
    counts->n_grid2 = pl.n_grid2;
    counts->n_segs = pl.n_segs;
    counts->n_long = pl.n_long;
    counts->cut = pl.cut;
    counts->bucketed = pl.bucket_rows > 0 ? 1 : 0;
    counts->bucket_rows = pl.bucket_rows;
    counts->bk_arcs = pl.bucket_rows > 0 ? (int64_t)pl.bk_ptr[(size_t)pl.n_segs] : 0;
    auto out = [](int32_t *dst, const std::vector<int> &v, size_t count) {
      if (dst && count) std::copy(v.begin(), v.begin() + count, dst);
    };
    out(blocks, pl.blocks, 4 * (size_t)pl.n_blocks);
    out(grid2, pl.grid2, 4 * (size_t)pl.n_grid2);
    out(long_rows, pl.long_rows, (size_t)pl.n_long);
    out(long_first, pl.long_first, (size_t)pl.n_long + 1);
    if (pl.bucket_rows > 0) {
      out(bk_ptr, pl.bk_ptr, (size_t)pl.n_segs + 1);
      out(bk_lsub, pl.bk_lsub, (size_t)pl.n_segs);
      out(bk_ci, pl.bk_ci, (size_t)counts->bk_arcs);
    }
    return GED_OK;
  });
}

extern "C" int ged_invalidate(ged_graph *g) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  if (g->served) return fail(GED_ERR_BUSY, "the graph is registered with a server");
  return guarded([&]() -> int {
    GED_HIP(hipStreamSynchronize(g->stream));
    g->prep.valid = false;
    g->prep.tr_r = -1;
    g->prep.W.clear();
    g->prep.tail_level = -1;
    return GED_OK;
  });
}

extern "C" int ged_score(ged_graph *g, const int32_t *S, int32_t s_len, double alpha, double eps,
                         double *out_score, ged_score_info *info) {
  if (!g || !out_score || (s_len > 0 && !S) || s_len < 0)
    return fail(GED_ERR_ARG, "bad argument to ged_score");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() { return score_group(g, S, s_len, alpha, eps, out_score, info); });
}

extern "C" int ged_profile_enable(ged_graph *g, int on) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() -> int {
    GED_HIP(hipStreamSynchronize(g->stream));
    for (auto &r : g->prof.recs) {
      g->prof.pool.push_back(r.a);
      g->prof.pool.push_back(r.b);
    }
    g->prof.recs.clear();
    g->prof.on = on != 0;
    return GED_OK;
  });
}

extern "C" int ged_profile_read(ged_graph *g, ged_profile *out) {
  if (!g || !out) return fail(GED_ERR_ARG, "bad argument");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() -> int {
    GED_HIP(hipStreamSynchronize(g->stream));
    std::memset(out, 0, sizeof(*out));
    std::map<std::pair<int, int>, std::tuple<int64_t, double, double>> by_kernel;
    for (auto &r : g->prof.recs) {
      float ms = 0.f;
      GED_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      out->launches++;
      out->total_ms += ms;
      out->bytes += r.bytes;
      out->edges += r.edges;
      auto &e = by_kernel[{r.C, r.kind}];
      std::get<0>(e)++;
      std::get<1>(e) += ms;
      std::get<2>(e) += r.bytes;
    }
    double best = -1;
    for (auto &kv : by_kernel) {
      if (std::get<1>(kv.second) > best) {
        best = std::get<1>(kv.second);
        out->dominant_columns = kv.first.first;
        out->dominant_kind = kv.first.second;
        out->dominant_launches = std::get<0>(kv.second);
        out->dominant_ms = std::get<1>(kv.second);
        out->dominant_bytes = std::get<2>(kv.second);
      }
    }
    return GED_OK;
  });
}
