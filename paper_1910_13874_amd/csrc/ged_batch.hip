// Batched scoring: many groups at once as the columns of one masked SpMM.
//
// Every score query on a graph stops at the same ell* (the tail bound is taken
// on the whole vertex set, Eq. katz-bound), so the hit chains of C groups run
// in lock-step: column c holds h_i for group g0 + c, a per-vertex 64-bit word
// marks which columns have v in their group (injection of t_i(v) there), and
// one pass over col_idx serves all C columns.  Undirected graphs run each tile
// as a split tile (ged_split.hip: integer levels 1-2, dense levels up to
// ceil(ell*/2), combining epilogue); directed graphs run all ell* levels.  The
// whole batch -- every tile, every level -- is captured into one hipGraph and
// replayed, so the host issues one launch per call.  The tile width C is chosen
// per graph by timing the dense phase for each candidate width (autotuner).
#include <algorithm>
#include <cstring>

#include "ged_internal.h"

namespace ged {

struct BatchWs {
  DBuf tmask;       // uint64 [n], all zero between calls
  bool tmask_ready = false;
  DBuf X, Y;        // double [n*C]
  DBuf offsets;     // int64 [cap_g+1]
  DBuf members;     // int [cap_m] (internal ids, duplicates dropped)
  DBuf mcol;        // int [cap_m] group of each member
  std::vector<int64_t> h_offsets;
  std::vector<int> h_members, h_mcol;
  // split tiles (undirected graphs): tile t uses counts sw / sw2 and member bits
  // tmask / tmask2 by the parity of t, so the pushes of tile t+1 and the
  // clearing of tile t-1 (side stream) overlap the dense levels of tile t
  SplitWs sw, sw2;
  DBuf tmask2;
  bool tmask2_ready = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_push[2] = {}, ev_dense[2] = {};
  DBuf scores;      // double [cap_g + 64]
  HBuf h_scores;
  size_t cap_g = 0, cap_m = 0;
  StepWs ws;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void *> sig;
  ~BatchWs() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : {ev_fork, ev_join, ev_push[0], ev_push[1], ev_dense[0], ev_dense[1]})
      if (e) (void)hipEventDestroy(e);
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
  }
};

static std::mutex g_batch_mu;
static std::map<const ged_graph *, std::unique_ptr<BatchWs>> g_batch;

static BatchWs &batch_ws(ged_graph *g) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto &p = g_batch[g];
  if (!p) p = std::make_unique<BatchWs>();
  return *p;
}

void batch_forget(const ged_graph *g) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_batch.erase(g);
}

// The race both autotuners run: every candidate width at the threshold the
// caller fixed (or the full LDS capacity), then -- when the threshold is left
// to the tuner -- thresholds of 1/2 and 1/4 of the capacity at the chosen
// width.  time_per_col(C, cut_div) returns milliseconds per column, or throws
// HipError{GED_ERR_NOMEM} when the width does not fit (wider ones are then
// skipped).  A candidate replaces the best so far only if it is faster per
// column by the factor `margin` (wider tiles hold more memory and leave more
// columns idle in a batch's last tile; lower thresholds add segments).
template <class F>
static int race_tile(ged_graph *g, std::initializer_list<int> widths, double margin,
                     F &&time_per_col) {
  const int cut0 = g->batch_cut_div > 0 ? g->batch_cut_div : 1;
  double best = 1e300;
  int best_c = g->batch_tile > 0 ? g->batch_tile : 16, best_cut = cut0;
  std::vector<int> ws;
  if (g->batch_tile > 0)
    ws.push_back(g->batch_tile);
  else
    ws.assign(widths.begin(), widths.end());
  for (int C : ws) {
    double t;
    try {
      t = time_per_col(C, cut0);
    } catch (const HipError &e) {
      if (e.code != GED_ERR_NOMEM) throw;
      break;  // wider tiles do not fit either
    }
    if (t < best * margin) {
      best = t;
      best_c = C;
    }
  }
  if (g->batch_cut_div == 0)
    for (int d : {2, 4}) {
      const double t = time_per_col(best_c, d);
      if (t < best * 0.97) {
        best = t;
        best_cut = d;
      }
    }
  g->batch_tile = best_c;
  g->batch_cut_div = best_cut;
  return best_c;
}

// Step time per column for each candidate tile width; the fastest wins.  Each
// candidate runs three ping-pong steps (X -> Y -> X -> Y) and the last two
// are timed, so the cache state (the dense tiles of a step stay in the
// Infinity Cache only when they fit) is that of a running batch.
static int autotune_tile(ged_graph *g, BatchWs &b) {
  if (g->batch_tile > 0 && g->batch_cut_div > 0) return g->batch_tile;
  const int n = (int)g->n;
  hipStream_t st = g->stream;
  hipEvent_t e0, e1;
  GED_HIP(hipEventCreate(&e0));
  GED_HIP(hipEventCreate(&e1));
  auto timed = [&](int C, int cut) -> double {
    Partition &p = partition(g, C, false, cut);
    StepWs ws;
    ws.fit(p);
    b.X.ensure(sizeof(double) * (size_t)n * C);
    b.Y.ensure(sizeof(double) * (size_t)n * C);
    launch_fill_f64(b.X.as<double>(), 0.0, (size_t)n * C, st);
    StepArgs a = base_args(g);
    ws.into(a);
    a.C = C;
    a.alpha = g->prep.alpha;
    a.tmask = b.tmask.as<const uint64_t>();
    a.inj = g->prep.t_levels.as<const double>();
    for (int r = 0; r < 3; ++r) {
      if (r == 1) GED_HIP(hipEventRecord(e0, st));
      a.X = ((r & 1) ? b.Y : b.X).as<const double>();
      a.Y = ((r & 1) ? b.X : b.Y).as<double>();
      a.accum = r > 0;
      launch_step(p, a, IN_VEC, OUT_TILE, st);
    }
    launch_reduce(p, a, nullptr, nullptr, nullptr, st, ws.scratch());
    GED_HIP(hipEventRecord(e1, st));
    GED_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GED_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms / C;
  };
  try {
    const int C = race_tile(g, {4, 8, 16, 32, 64}, 1.0, timed);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return C;
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
}

// Split scoring: the same race over the dense levels of a split tile (the
// level-(s+1) step on count rows and the combining step), at C = 8..64; best
// of two timed passes after a warm-up.
static int autotune_split(ged_graph *g, BatchWs &b, const SplitPlan &pl0) {
  if (g->batch_tile > 0 && g->batch_cut_div > 0) return g->batch_tile;
  hipStream_t st = g->stream;
  hipEvent_t e0, e1;
  GED_HIP(hipEventCreate(&e0));
  GED_HIP(hipEventCreate(&e1));
  auto timed = [&](int C, int cut) -> double {
    SplitPlan pl = pl0;
    pl.cut_div = cut;
    pl.c16_hub = split_c16_hub(g, pl, C, st);
    split_fit(g, b.sw, pl, C, 1, st);
    split_dense(g, b.sw, pl, C, b.tmask.as<const uint64_t>(), st);  // warm-up
    float ms = 1e30f;
    for (int r = 0; r < 2; ++r) {
      GED_HIP(hipEventRecord(e0, st));
      split_dense(g, b.sw, pl, C, b.tmask.as<const uint64_t>(), st);
      GED_HIP(hipEventRecord(e1, st));
      GED_HIP(hipEventSynchronize(e1));
      float t = 0.f;
      GED_HIP(hipEventElapsedTime(&t, e0, e1));
      ms = std::min(ms, t);
    }
    return ms / C;
  };
  try {
    const int C = race_tile(g, {8, 16, 32, 64}, 0.97, timed);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return C;
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
}

static void enqueue_batch(ged_graph *g, BatchWs &b, int G, int C, hipStream_t st) {
  const int64_t n = g->n;
  const PrepCache &pc = g->prep;
  Partition &p = partition(g, C, false, g->batch_cut_div);
  const double *T = pc.t_levels.as<const double>();
  for (int g0 = 0; g0 < G; g0 += C) {
    const int nc = std::min(C, G - g0);
    launch_tmask_set(b.tmask.as<uint64_t>(), b.offsets.as<const int64_t>(),
                     b.members.as<const int>(), g0, nc, 1, st);
    StepArgs a = base_args(g);
    b.ws.into(a);
    for (int i = 1; i <= pc.ell; ++i) {
      a.C = C;
      a.alpha = pc.alpha;
      a.accum = i > 1;  // all levels add into the block partials
      a.tmask = b.tmask.as<const uint64_t>();
      a.X = ((i & 1) ? b.X : b.Y).as<const double>();
      a.Y = ((i & 1) ? b.Y : b.X).as<double>();
      a.inj = T + (size_t)i * n;
      run_step(g, p, a, i == 1 ? IN_TILEMASK : IN_VEC, OUT_TILE, st);
    }
    // scores of this tile's columns (the buffer has C entries of slack)
    launch_reduce(p, a, b.scores.as<double>() + g0, nullptr, nullptr, st, b.ws.scratch());
    launch_tmask_set(b.tmask.as<uint64_t>(), b.offsets.as<const int64_t>(),
                     b.members.as<const int>(), g0, nc, 0, st);
  }
}

int score_batch(ged_graph *g, const int64_t *offsets, const int32_t *members, int32_t G,
                double alpha, double eps, double *out) {
  if (G < 0 || (G > 0 && (!offsets || !out))) return fail(GED_ERR_ARG, "bad batch arguments");
  if (G == 0) return GED_OK;
  if (offsets[0] != 0) return fail(GED_ERR_ARG, "offsets[0] must be 0");
  for (int j = 0; j < G; ++j)
    if (offsets[j + 1] < offsets[j]) return fail(GED_ERR_ARG, "offsets must be non-decreasing");
  const int64_t M = offsets[G];
  if (M > 0 && !members) return fail(GED_ERR_ARG, "members is null");
  for (int64_t j = 0; j < M; ++j)
    if (members[j] < 0 || members[j] >= g->n) return fail(GED_ERR_VERTEX, "member out of range");
  int rc = prepare(g, alpha, eps);
  if (rc) return rc;
  hipStream_t st = g->stream;
  BatchWs &b = batch_ws(g);
  const int64_t n = g->n;
  b.tmask.ensure(sizeof(uint64_t) * (size_t)n);
  if (!b.tmask_ready) {
    launch_fill_i32(b.tmask.as<int>(), 0, (size_t)n * 2, st);
    b.tmask_ready = true;
  }
  const bool split = split_ok(g);
  SplitPlan pl;
  if (split) {
    pl = split_plan(g, g->prep.ell);
    split_tables(g, pl, st);
  }
  const int C = split ? autotune_split(g, b, pl) : autotune_tile(g, b);
  pl.cut_div = g->batch_cut_div;
  if (split) pl.c16_hub = split_c16_hub(g, pl, C, st);
  g->c16_used = pl.c16_hub;
  Partition &p = partition(g, C, false, g->batch_cut_div);
  b.ws.fit(p);
  // internal ids, duplicates inside a group dropped; column of every member
  std::vector<int64_t> &hoff = b.h_offsets;
  std::vector<int> &hmem = b.h_members;
  std::vector<int> &hcol = b.h_mcol;
  hoff.assign((size_t)G + 1, 0);
  hmem.clear();
  hmem.reserve((size_t)M);
  std::vector<int64_t> degsum((size_t)G);
  for (int j = 0; j < G; ++j) {
    hoff[j] = (int64_t)hmem.size();
    degsum[j] = map_group(g, members + offsets[j], offsets[j + 1] - offsets[j], hmem);
  }
  hoff[G] = (int64_t)hmem.size();
  const int64_t Md = hoff[G];
  hcol.resize((size_t)Md);
  for (int j = 0; j < G; ++j)
    for (int64_t q = hoff[j]; q < hoff[j + 1]; ++q) hcol[q] = j;
  if ((size_t)G + 1 > b.cap_g) {
    b.cap_g = std::max<size_t>((size_t)G + 1, 2 * b.cap_g);
    b.offsets.ensure(sizeof(int64_t) * b.cap_g);
    b.scores.ensure(sizeof(double) * (b.cap_g + 64));
    b.h_scores.ensure(sizeof(double) * (b.cap_g + 64));
  }
  if ((size_t)std::max<int64_t>(Md, 1) > b.cap_m) {
    b.cap_m = std::max<size_t>((size_t)std::max<int64_t>(Md, 1), 2 * b.cap_m);
    b.members.ensure(sizeof(int) * b.cap_m);
    b.mcol.ensure(sizeof(int) * b.cap_m);
  }
  GED_HIP(hipMemcpyAsync(b.offsets.p, hoff.data(), sizeof(int64_t) * (size_t)(G + 1),
                         hipMemcpyHostToDevice, st));
  if (Md > 0) {
    GED_HIP(hipMemcpyAsync(b.members.p, hmem.data(), sizeof(int) * (size_t)Md,
                           hipMemcpyHostToDevice, st));
    GED_HIP(hipMemcpyAsync(b.mcol.p, hcol.data(), sizeof(int) * (size_t)Md,
                           hipMemcpyHostToDevice, st));
  }
  if (split) {
    size_t wl_need = 1;
    int64_t deg_tile = 1;  // largest member-degree sum of a tile: about its worklist size
    for (int g0 = 0; g0 < G; g0 += C) {
      size_t need = 0;
      int64_t ds = 0;
      for (int j = g0; j < std::min(G, g0 + C); ++j) {
        need += split_wl_need(g, degsum[j]);
        ds += degsum[j];
      }
      wl_need = std::max(wl_need, need);
      deg_tile = std::max(deg_tile, ds);
    }
    split_fit(g, b.sw, pl, C, wl_need, st);
    split_fit(g, b.sw2, pl, C, wl_need, st, true);
    b.sw.wl_blocks = b.sw2.wl_blocks = split_wl_blocks(deg_tile);
    b.tmask2.ensure(sizeof(uint64_t) * (size_t)n);
    if (!b.tmask2_ready) {
      launch_fill_i32(b.tmask2.as<int>(), 0, (size_t)n * 2, st);
      b.tmask2_ready = true;
    }
    if (!b.side) {
      GED_HIP(hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking));
      for (hipEvent_t *e : {&b.ev_fork, &b.ev_join, &b.ev_push[0], &b.ev_push[1], &b.ev_dense[0],
                            &b.ev_dense[1]})
        GED_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    }
    b.sw.zero = false;
    b.sw2.zero = false;
  } else {
    b.X.ensure(sizeof(double) * (size_t)n * C);
    b.Y.ensure(sizeof(double) * (size_t)n * C);
  }
  // per tile: clear its count levels by a fill where replaying its pushes
  // would cost more (members' omega_2 sum against the levels' size); decided
  // before any capture (the host table may need a synchronisation once).  A
  // captured batch keeps the choices of the call that captured it: both
  // clear everything the pushes wrote, so later groups only differ in speed.
  std::vector<char> fill((size_t)(G + C - 1) / C, 0);
  if (split && pl.s >= 2 && !pl.push3) {
    const std::vector<double> &om2 = omega2_host(g, st);
    for (size_t t = 0; t < fill.size(); ++t) {
      double v = 0.0;
      for (int64_t q = hoff[t * C]; q < hoff[std::min(G, (int)(t + 1) * C)]; ++q) v += om2[hmem[q]];
      fill[t] = split_clear_by_fill(g, pl, C, v) ? 1 : 0;
    }
  }
  auto enqueue = [&]() {
    if (!split) {
      enqueue_batch(g, b, G, C, st);
      return;
    }
    const int ntiles = (G + C - 1) / C;
    SplitWs *cw[2] = {&b.sw, &b.sw2};
    uint64_t *tm[2] = {b.tmask.as<uint64_t>(), b.tmask2.as<uint64_t>()};
    const int64_t *offs = b.offsets.as<const int64_t>();
    const int *mem = b.members.as<const int>(), *mc = b.mcol.as<const int>();
    auto push = [&](int t) {
      const int g0 = t * C, nc = std::min(C, G - g0);
      split_tile_push(g, *cw[t & 1], pl, C, offs, mem, mc, g0, nc, hoff[g0 + nc] - hoff[g0],
                      tm[t & 1], b.side);
      GED_HIP(hipEventRecord(b.ev_push[t & 1], b.side));
    };
    // side stream: push(0), push(1), clear(0), push(2), clear(1), ...  A tile's
    // buffers are cleared (side, in order) before the tile two later pushes.
    GED_HIP(hipEventRecord(b.ev_fork, st));
    GED_HIP(hipStreamWaitEvent(b.side, b.ev_fork, 0));
    push(0);
    for (int t = 0; t < ntiles; ++t) {
      const int g0 = t * C, nc = std::min(C, G - g0), p = t & 1;
      if (t + 1 < ntiles) push(t + 1);
      GED_HIP(hipStreamWaitEvent(st, b.ev_push[p], 0));
      split_dense(g, b.sw, pl, C, tm[p], st, true, cw[p]);
      // scores of this tile's columns (the buffer has C entries of slack)
      split_tile_reduce(g, b.sw, pl, C, b.scores.as<double>() + g0, st);
      GED_HIP(hipEventRecord(b.ev_dense[p], st));
      GED_HIP(hipStreamWaitEvent(b.side, b.ev_dense[p], 0));
      split_tile_clear(g, *cw[p], pl, C, offs, mem, mc, g0, nc, hoff[g0 + nc] - hoff[g0], tm[p],
                       b.side, fill[t] != 0);
    }
    GED_HIP(hipEventRecord(b.ev_join, b.side));
    GED_HIP(hipStreamWaitEvent(st, b.ev_join, 0));
  };
  double abits_d = alpha;
  const void *abits;
  std::memcpy(&abits, &abits_d, sizeof(abits));
  std::vector<const void *> sig = {b.tmask.p,      b.X.p,       b.Y.p,
                                   b.offsets.p,    b.members.p, b.mcol.p,   b.scores.p,
                                   b.ws.blk.p,     b.ws.seg.p,  b.ws.lng.p, b.ws.red2.p,
                                   b.sw.cnt1.p,    b.sw.cnt2.p, b.sw.lv.p,  b.sw.wl.p,
                                   b.sw.wl_n.p,    b.sw.ws.blk.p, b.sw.ws.seg.p, b.sw.ws.lng.p,
                                   b.sw2.cnt1.p,   b.sw2.cnt2.p, b.sw2.wl.p,   b.sw2.wl_n.p,
                                   b.tmask2.p,     (const void *)b.side,
                                   b.sw.ws.red2.p, g->omega2.p, g->omega_lv.p, g->prep.tr.p,
                                   g->prep.t_levels.p, (const void *)st, abits,
                                   (const void *)(uintptr_t)b.sw.wl_cap,
                                   (const void *)(uintptr_t)b.sw2.wl_cap,
                                   (const void *)(intptr_t)b.sw.wl_blocks,
                                   (const void *)(intptr_t)split,
                                   (const void *)(intptr_t)g->prep.ell, (const void *)(intptr_t)G,
                                   (const void *)(intptr_t)C,
                                   (const void *)(intptr_t)g->batch_cut_div,
                                   (const void *)(intptr_t)pl.c16_hub};

  if (g->prof.on) {
    // profiling times every step launch with events: run the batch eagerly
    enqueue();
  } else {
    if (b.exec && sig != b.sig) {
      (void)hipGraphExecDestroy(b.exec);
      (void)hipGraphDestroy(b.graph);
      b.exec = nullptr;
      b.graph = nullptr;
    }
    if (!b.exec) {
      GED_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        enqueue();
      } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(st, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
      }
      GED_HIP(hipStreamEndCapture(st, &b.graph));
      GED_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
      b.sig = sig;
    }
    GED_HIP(hipGraphLaunch(b.exec, st));
  }
  double *hs = b.h_scores.as<double>();
  GED_HIP(hipMemcpyAsync(hs, b.scores.p, sizeof(double) * (size_t)G, hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  if (split) b.sw.zero = b.sw2.zero = true;
  std::memcpy(out, hs, sizeof(double) * (size_t)G);
  return GED_OK;
}

}  // namespace ged

using namespace ged;

extern "C" int ged_score_batch(ged_graph *g, const int64_t *offsets, const int32_t *members,
                               int32_t n_groups, double alpha, double eps, double *out_scores) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() { return score_batch(g, offsets, members, n_groups, alpha, eps, out_scores); });
}

extern "C" int32_t ged_batch_tile(const ged_graph *g) { return g ? g->batch_tile : 0; }

extern "C" int ged_set_batch_tile(ged_graph *g, int32_t tile) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  if (tile != 0 && (tile < 1 || tile > 64 || (tile & (tile - 1)) != 0))
    return fail(GED_ERR_ARG, "tile must be 0 (autotune) or a power of two <= 64");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  g->batch_tile = tile;
  if (tile == 0) g->batch_cut_div = 0;
  return GED_OK;
}

extern "C" int32_t ged_batch_row_cut(const ged_graph *g) { return g ? g->batch_cut_div : 0; }

extern "C" int ged_set_count16(ged_graph *g, int32_t hub) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  if (hub < -1 || hub >= g->n) return fail(GED_ERR_ARG, "hub must be -1, 0 or a cut below n");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() -> int {
    if (hub > 0 && !g->weighted && split_ok(g) && hub < least_c16_hub(g, g->stream))
      return fail(GED_ERR_ARG, "hub cut below the last vertex whose omega_2 exceeds 2^16 - 2");
    g->count16 = hub;
    return GED_OK;
  });
}

extern "C" int32_t ged_count16_hub(const ged_graph *g) { return g ? g->c16_used : -1; }

extern "C" int ged_set_batch_row_cut(ged_graph *g, int32_t cut_div) {
  if (!g) return fail(GED_ERR_ARG, "graph is null");
  if (cut_div != 0 && cut_div != 1 && cut_div != 2 && cut_div != 4)
    return fail(GED_ERR_ARG, "cut_div must be 0 (autotune), 1, 2 or 4");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  g->batch_cut_div = cut_div;
  return GED_OK;
}
