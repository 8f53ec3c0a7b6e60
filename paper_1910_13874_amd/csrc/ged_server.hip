// Continuous-batching request server.
//
// Every score query on a graph runs the same number of walk-count levels
// (ell*, fixed per graph), so queries on one graph batch as SpMM columns.
// Undirected graphs run them as split tiles (the scoring of ged_split.hip:
// integer pushes, two or so dense levels, a combining level): each launch
// takes up to C waiting requests of the graph, at the narrowest power-of-two
// width that holds them, and requests that arrive while a tile is on the
// device join the next one.  Directed graphs keep a pool of
// SpMM columns ("slots"): one launch advances every occupied column by one
// level, each column at its own level (the injection reads t_{level(c)}), and
// a column whose request has run ell* levels is harvested and refilled with
// the next waiting request before the following step.  Either way requests
// join and leave while others are mid-flight, and the lanes of different
// graphs run on their own streams, so their work overlaps on the device.
//
// Greedy requests run whole (ged_greedy) on worker threads.  Admission,
// queue limits, deadlines and cancellation follow server_policy.h: a greedy
// request's working memory is estimated from the allocations the greedy makes
// at the largest walk length its k can reach (the first power of two whose
// tail bound is below eps/k, from a table built when the graph is added), it
// starts when that fits the HBM budget beside the lanes, the memory the
// graphs already hold and the running requests, and the memory its graph
// holds afterwards stays counted.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "ged_internal.h"
#include "server_policy.h"

namespace ged {

int greedy_run(ged_graph *g, int32_t k, double alpha, double eps, double eta, uint64_t seed,
               bool stochastic, int32_t *out_group, double *out_score, ged_greedy_trace *tr,
               const std::atomic<int> *stop);
void split_fit_width(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C);

static double now_us() {
  using namespace std::chrono;
  return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

// (vertex, column) pairs: set (value=1) or clear bit `column` of tmask[vertex].
__global__ void k_tmask_pairs(unsigned long long *tmask, const int2 *pairs, int count, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int2 p = pairs[i];
  const unsigned long long bit = 1ull << p.y;
  if (value)
    atomicOr(&tmask[p.x], bit);
  else
    atomicAnd(&tmask[p.x], ~bit);
}

// acc[c] = 0 for columns that start this step.
__global__ void k_pool_start(double *acc, const int *fresh, int C) {
  const int c = threadIdx.x;
  if (c < C && fresh[c]) acc[c] = 0.0;
}

struct Req {
  uint64_t id = 0;
  int kind = 0;  // 0 score, 1 greedy
  int graph = 0;
  std::vector<int> S;  // internal ids (score)
  int k = 0;
  double t_submit = 0;
  size_t footprint = 0;
};

struct Done {
  ged_result r;
  std::vector<int> group;
};

struct Lane {
  ged_graph *g = nullptr;
  int gid = 0;
  double alpha = 0, eps = 0;
  int ell = 0;
  int C = 0;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  bool inflight = false;
  DBuf X, Y, tmask, acc, state, pairs;
  HBuf h_state, h_acc, h_pairs;
  StepWs ws;
  std::vector<int> step;     // level the column computes next (0 = idle)
  std::vector<int> fresh;
  std::vector<int> launched; // level computed by the step in flight
  std::vector<Req> slot;     // request in each column
  std::vector<int> done_cols;  // columns finished by the previous step (bits to clear)
  std::deque<Req> pending;
  // greedy admission: walk lengths 1, 2, 4, ... with their tail bounds B_ell,
  // up to the first one below eps / n, and the greedy footprint at each
  std::vector<std::pair<int, double>> sep;
  std::vector<size_t> fp;
  int cur = 0;
  size_t bytes = 0;
  // split tiles (undirected graphs)
  bool split = false;
  SplitPlan pl;
  SplitWs sw;
  DBuf tin;                  // tile input: int64 offsets[C+1], int members[m], int columns[m]
  HBuf h_tin;
  std::vector<Req> tile;     // requests of the tile in flight
  std::vector<double> om2;   // omega_2 per vertex (undirected unweighted lanes; push volumes)
};

}  // namespace ged

struct ged_server {
  ged_server_config cfg{};
  std::vector<std::unique_ptr<ged::Lane>> lanes;
  std::mutex mu;  // guards inbox, results, the policy, the greedy queue, stop flags
  std::condition_variable cv_work, cv_done, cv_greedy;
  std::deque<ged::Req> inbox;
  std::deque<ged::Req> greedy_q;
  std::deque<ged::Done> results;
  std::unordered_map<uint64_t, std::vector<int>> groups;
  // stop flags of the running greedy requests (polled between their rounds)
  std::unordered_map<uint64_t, std::shared_ptr<std::atomic<int>>> running_stop;
  std::unique_ptr<ged::ServePolicy> pol;
  uint64_t next_id = 1;
  int64_t steps = 0, peak_cols = 0;
  double last_expire_us = 0;
  bool stop = false;
  std::thread sched;
  std::vector<std::thread> workers;
  bool started = false;
};

namespace ged {

static void lane_setup(Lane &L, int C) {
  ged_graph *g = L.g;
  const int64_t n = g->n;
  L.C = C;
  Partition &p = partition(g, C);
  L.ws.fit(p);
  // everything the greedy path may need, so no partition is built while the
  // lane runs on another thread
  partition(g, 1);
  partition(g, 8);
  if (g->flags == GED_DIRECTED) partition(g, 1, true);
  if (split_ok(g)) partition_narrow(g, 8);  // 32-bit gain levels
  if (split_ok(g)) {
    L.split = true;
    L.pl = split_plan(g, g->prep.ell);
    GED_HIP(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
    GED_HIP(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
    split_tables(g, L.pl, L.st);  // per-graph tables now, not while greedy runs
    if (L.pl.s >= 2) L.om2 = omega2_host(g, L.st);
    // worklist: a tile holds requests while their needs (<= n + nnz/512 + 1
    // each) fit C * (nnz/512 + 1) + 2n entries; one larger group grows it
    const size_t cap = (size_t)C * split_wl_need(g, 0) + 2 * (size_t)n;
    split_fit(g, L.sw, L.pl, C, cap, L.st);
    // a tile runs at the narrowest power-of-two width that holds its requests
    for (int w = 1; w < C; w *= 2) split_fit_width(g, L.sw, L.pl, w);
    L.tmask.ensure(sizeof(uint64_t) * (size_t)n);
    L.acc.ensure(sizeof(double) * 64);
    L.h_acc.ensure(sizeof(double) * 64);
    launch_fill_i32(L.tmask.as<int>(), 0, (size_t)n * 2, L.st);
    GED_HIP(hipStreamSynchronize(L.st));
    L.sw.zero = true;
    L.bytes = L.tmask.bytes + L.sw.cnt1.bytes + L.sw.cnt2.bytes + L.sw.lv.bytes +
              L.sw.wl.bytes + L.sw.ws.blk.bytes + L.sw.ws.seg.bytes + L.sw.ws.lng.bytes;
    return;
  }
  L.X.ensure(sizeof(double) * (size_t)n * C);
  L.Y.ensure(sizeof(double) * (size_t)n * C);
  L.tmask.ensure(sizeof(uint64_t) * (size_t)n);
  L.acc.ensure(sizeof(double) * 64);
  L.state.ensure(sizeof(int) * 128);
  L.h_state.ensure(sizeof(int) * 128);
  L.h_acc.ensure(sizeof(double) * 64);
  GED_HIP(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
  GED_HIP(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
  launch_fill_f64(L.X.as<double>(), 0.0, (size_t)n * C, L.st);
  launch_fill_f64(L.Y.as<double>(), 0.0, (size_t)n * C, L.st);
  launch_fill_i32(L.tmask.as<int>(), 0, (size_t)n * 2, L.st);
  GED_HIP(hipStreamSynchronize(L.st));
  L.step.assign(C, 0);
  L.fresh.assign(C, 0);
  L.launched.assign(C, 0);
  L.slot.assign(C, Req());
  L.bytes = L.X.bytes + L.Y.bytes + L.tmask.bytes + L.ws.blk.bytes + L.ws.seg.bytes +
            L.ws.lng.bytes;
}

// Complete request q (held_after: for a greedy request that ran, the bytes
// its graph's greedy workspace holds now).
static void emit(ged_server *s, const Req &q, int status, double score, std::vector<int> group,
                 double t_done, size_t held_after = 0) {
  Done d;
  d.r.id = q.id;
  d.r.kind = q.kind;
  d.r.status = status;
  d.r.score = score;
  d.r.k = q.k;
  d.r.graph = q.graph;
  d.r.t_submit_us = q.t_submit;
  d.r.t_done_us = t_done;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->pol->finish(q.id, held_after);
    if (q.kind == 1 && status == GED_OK) s->groups[q.id] = group;
    d.group = std::move(group);
    s->results.push_back(std::move(d));
  }
  s->cv_done.notify_all();
  s->cv_greedy.notify_all();  // a greedy reservation may have been released
}

// Move requests from the front of a lane's queue onto the device (up to
// `max`, and while take(q) accepts them); requests asked to stop meanwhile
// are completed with their stop status instead.
template <class Take>
static std::vector<Req> take_pending(ged_server *s, Lane &L, size_t max, Take &&take) {
  std::vector<Req> got, stopped;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!L.pending.empty() && got.size() < max) {
      Req &q = L.pending.front();
      if (s->pol->stop_status(q.id)) {
        stopped.push_back(std::move(q));
        L.pending.pop_front();
        continue;
      }
      if (!take(q, got.size())) break;
      s->pol->start(q.id);
      got.push_back(std::move(q));
      L.pending.pop_front();
    }
  }
  for (auto &q : stopped) {
    int st;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      st = s->pol->stop_status(q.id);
    }
    emit(s, q, st, 0.0, {}, now_us());
  }
  return got;
}

// Harvest the step that just finished: columns that ran level ell* are done
// (split lanes: every request of the tile).
static void lane_harvest(ged_server *s, Lane &L) {
  const double t = now_us();
  const double *acc = L.h_acc.as<double>();
  if (L.split) {
    for (size_t j = 0; j < L.tile.size(); ++j) emit(s, L.tile[j], GED_OK, acc[j], {}, t);
    L.tile.clear();
    L.sw.zero = true;
    return;
  }
  for (int c = 0; c < L.C; ++c) {
    if (L.launched[c] == 0) continue;
    if (L.launched[c] == L.ell) {
      emit(s, L.slot[c], GED_OK, acc[c], {}, t);
      L.done_cols.push_back(c);
      L.step[c] = 0;
    } else {
      L.step[c] = L.launched[c] + 1;
    }
    L.fresh[c] = 0;
  }
}

// Split lane: the next tile of up to C waiting requests.
static bool lane_launch_split(ged_server *s, Lane &L) {
  if (L.pending.empty()) return false;
  ged_graph *g = L.g;
  const int C = L.C;
  if (!L.sw.zero) split_fit(g, L.sw, L.pl, C, L.sw.wl_cap, L.st);  // after a failed tile
  std::vector<int64_t> offs(1, 0);
  std::vector<int> mem, col;
  size_t need = 0;
  int64_t ds_tile = 0;  // members' degree sum: about the tile's worklist entries
  double om2 = 0.0;     // members' omega_2 sum: the level-2 push volume
  const std::vector<double> &h_om2 = L.om2;
  L.tile = take_pending(s, L, (size_t)C, [&](const Req &q, size_t have) {
    int64_t ds = 0;
    for (int v : q.S) ds += g->h_rp[v + 1] - g->h_rp[v];
    if (!h_om2.empty())
      for (int v : q.S) om2 += h_om2[v];
    const size_t nq = split_wl_need(g, ds);
    if (have > 0 && need + nq > L.sw.wl_cap) return false;
    need += nq;
    ds_tile += ds;
    const int c = (int)have;
    for (int v : q.S) {
      mem.push_back(v);
      col.push_back(c);
    }
    offs.push_back((int64_t)mem.size());
    return true;
  });
  const int nc = (int)L.tile.size();
  if (nc == 0) return false;
  if (need > L.sw.wl_cap) split_fit(g, L.sw, L.pl, C, need, L.st);
  // worklist kernels loop over their grid: size it for this tile
  L.sw.wl_blocks = split_wl_blocks(ds_tile);
  const size_t m = mem.size();
  const size_t ob = sizeof(int64_t) * (size_t)(nc + 1);
  const size_t bytes = ob + 2 * sizeof(int) * std::max<size_t>(m, 1);
  L.tin.ensure(bytes);
  L.h_tin.ensure(bytes);
  char *h = L.h_tin.as<char>();
  std::memcpy(h, offs.data(), ob);
  if (m) {
    std::memcpy(h + ob, mem.data(), sizeof(int) * m);
    std::memcpy(h + ob + sizeof(int) * m, col.data(), sizeof(int) * m);
  }
  GED_HIP(hipMemcpyAsync(L.tin.p, h, bytes, hipMemcpyHostToDevice, L.st));
  const int64_t *d_offs = L.tin.as<const int64_t>();
  const int *d_mem = reinterpret_cast<const int *>(L.tin.as<char>() + ob);
  const int *d_col = d_mem + m;
  L.sw.zero = false;
  // the narrowest width that holds the tile: a step's cost grows with its
  // width, so a tile of one request on a large graph runs as one column
  int W = 1;
  while (W < nc) W *= 2;
  enqueue_split_tile(g, L.sw, L.pl, W, d_offs, d_mem, d_col, 0, nc, (int64_t)m,
                     L.tmask.as<uint64_t>(), L.acc.as<double>(), L.st, false,
                     split_clear_by_fill(g, L.pl, W, om2));
  GED_HIP(hipMemcpyAsync(L.h_acc.p, L.acc.p, sizeof(double) * nc, hipMemcpyDeviceToHost, L.st));
  GED_HIP(hipEventRecord(L.ev, L.st));
  L.inflight = true;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->steps++;
    s->peak_cols = std::max<int64_t>(s->peak_cols, nc);
  }
  return true;
}

// Admit waiting requests into free columns and launch one step.
static bool lane_launch(ged_server *s, Lane &L) {
  if (L.split) return lane_launch_split(s, L);
  ged_graph *g = L.g;
  const int C = L.C;
  // bit updates: clear finished columns' members, set new members
  std::vector<int2> clr, set;
  for (int c : L.done_cols)
    for (int v : L.slot[c].S) clr.push_back(make_int2(v, c));
  L.done_cols.clear();
  size_t free_cols = 0;
  for (int c = 0; c < C; ++c) free_cols += L.step[c] == 0;
  std::vector<Req> fresh_reqs =
      take_pending(s, L, free_cols, [](const Req &, size_t) { return true; });
  size_t next = 0;
  for (int c = 0; c < C && next < fresh_reqs.size(); ++c) {
    if (L.step[c] != 0) continue;
    L.slot[c] = std::move(fresh_reqs[next++]);
    L.step[c] = 1;
    L.fresh[c] = 1;
    for (int v : L.slot[c].S) set.push_back(make_int2(v, c));
  }
  int active = 0;
  for (int c = 0; c < C; ++c) active += L.step[c] > 0;
  if (active == 0) {
    if (!clr.empty()) {
      const size_t need = clr.size();
      L.pairs.ensure(sizeof(int2) * need);
      L.h_pairs.ensure(sizeof(int2) * need);
      std::memcpy(L.h_pairs.p, clr.data(), sizeof(int2) * need);
      GED_HIP(hipMemcpyAsync(L.pairs.p, L.h_pairs.p, sizeof(int2) * need,
                             hipMemcpyHostToDevice, L.st));
      hipLaunchKernelGGL(k_tmask_pairs, dim3(((int)need + 255) / 256), dim3(256), 0, L.st,
                         L.tmask.as<unsigned long long>(), L.pairs.as<const int2>(), (int)need, 0);
      GED_HIP(hipStreamSynchronize(L.st));
    }
    return false;
  }
  const size_t np = clr.size() + set.size();
  if (np > 0) {
    L.pairs.ensure(sizeof(int2) * np);
    L.h_pairs.ensure(sizeof(int2) * np);
    std::memcpy(L.h_pairs.p, clr.data(), sizeof(int2) * clr.size());
    std::memcpy(L.h_pairs.as<int2>() + clr.size(), set.data(), sizeof(int2) * set.size());
    GED_HIP(hipMemcpyAsync(L.pairs.p, L.h_pairs.p, sizeof(int2) * np, hipMemcpyHostToDevice,
                           L.st));
    if (!clr.empty())
      hipLaunchKernelGGL(k_tmask_pairs, dim3(((int)clr.size() + 255) / 256), dim3(256), 0, L.st,
                         L.tmask.as<unsigned long long>(), L.pairs.as<const int2>(),
                         (int)clr.size(), 0);
    if (!set.empty())
      hipLaunchKernelGGL(k_tmask_pairs, dim3(((int)set.size() + 255) / 256), dim3(256), 0, L.st,
                         L.tmask.as<unsigned long long>(),
                         L.pairs.as<const int2>() + clr.size(), (int)set.size(), 1);
  }
  int *hs = L.h_state.as<int>();
  for (int c = 0; c < C; ++c) {
    hs[c] = L.step[c];
    hs[64 + c] = L.fresh[c];
    L.launched[c] = L.step[c];
  }
  GED_HIP(hipMemcpyAsync(L.state.p, hs, sizeof(int) * 128, hipMemcpyHostToDevice, L.st));
  const int *d_step = L.state.as<const int>();
  const int *d_fresh = d_step + 64;
  hipLaunchKernelGGL(k_pool_start, dim3(1), dim3(64), 0, L.st, L.acc.as<double>(), d_fresh, C);
  Partition &p = partition(g, C);
  StepArgs a = base_args(g);
  L.ws.into(a);
  a.C = C;
  a.alpha = L.alpha;
  a.tmask = L.tmask.as<const uint64_t>();
  a.col_step = d_step;
  a.fresh = d_fresh;
  a.inj = g->prep.t_levels.as<const double>();
  a.X = (L.cur ? L.Y : L.X).as<const double>();
  a.Y = (L.cur ? L.X : L.Y).as<double>();
  launch_step(p, a, IN_FRESH, OUT_POOL, L.st);
  launch_reduce(p, a, nullptr, L.acc.as<double>(), d_step, L.st, L.ws.scratch());
  GED_HIP(hipMemcpyAsync(L.h_acc.p, L.acc.p, sizeof(double) * C, hipMemcpyDeviceToHost, L.st));
  GED_HIP(hipEventRecord(L.ev, L.st));
  L.cur ^= 1;
  L.inflight = true;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->steps++;
    s->peak_cols = std::max<int64_t>(s->peak_cols, active);
  }
  return true;
}

static void sched_loop(ged_server *s) {
  for (;;) {
    std::vector<Req> incoming, dropped;
    std::vector<uint64_t> drop_ids;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      bool busy = false;
      for (auto &L : s->lanes) busy = busy || L->inflight || !L->pending.empty();
      if (!busy && s->inbox.empty() && !s->stop)
        s->cv_work.wait_for(lk, std::chrono::microseconds(200));
      if (s->stop) break;
      const double now = now_us();
      if (now - s->last_expire_us >= 500.0) {
        s->pol->expire(now);
        s->last_expire_us = now;
      }
      for (auto &kv : s->running_stop) {
        const int st = s->pol->stop_status(kv.first);
        if (st) kv.second->store(st, std::memory_order_relaxed);
      }
      drop_ids = s->pol->take_dropped();
      auto is_dropped = [&](const Req &q) {
        return std::find(drop_ids.begin(), drop_ids.end(), q.id) != drop_ids.end();
      };
      for (auto *dq : {&s->inbox, &s->greedy_q})
        for (auto it = dq->begin(); it != dq->end();) {
          if (!drop_ids.empty() && is_dropped(*it)) {
            dropped.push_back(std::move(*it));
            it = dq->erase(it);
          } else {
            ++it;
          }
        }
      while (!s->inbox.empty()) {
        incoming.push_back(std::move(s->inbox.front()));
        s->inbox.pop_front();
      }
    }
    for (auto &q : incoming) s->lanes[q.graph]->pending.push_back(std::move(q));
    if (!drop_ids.empty())
      for (auto &Lp : s->lanes)
        for (auto it = Lp->pending.begin(); it != Lp->pending.end();) {
          if (std::find(drop_ids.begin(), drop_ids.end(), it->id) != drop_ids.end()) {
            dropped.push_back(std::move(*it));
            it = Lp->pending.erase(it);
          } else {
            ++it;
          }
        }
    for (auto &q : dropped) {
      int st;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        st = s->pol->stop_status(q.id);
      }
      emit(s, q, st ? st : GED_ERR_CANCELLED, 0.0, {}, now_us());
    }
    bool progressed = false;
    for (auto &Lp : s->lanes) {
      Lane &L = *Lp;
      try {
        if (L.inflight) {
          const hipError_t e = hipEventQuery(L.ev);
          if (e == hipErrorNotReady) continue;
          GED_HIP(e);
          L.inflight = false;
          lane_harvest(s, L);
          progressed = true;
        }
        if (lane_launch(s, L)) progressed = true;
      } catch (const HipError &err) {
        // fail every request of this lane and drop it from service
        const double t = now_us();
        if (L.split) {
          for (auto &q : L.tile) emit(s, q, err.code, 0.0, {}, t);
          L.tile.clear();
          L.sw.zero = false;
        } else {
          for (int c = 0; c < L.C; ++c)
            if (L.step[c] > 0) emit(s, L.slot[c], err.code, 0.0, {}, t);
        }
        for (auto &q : L.pending) emit(s, q, err.code, 0.0, {}, t);
        L.pending.clear();
        std::fill(L.step.begin(), L.step.end(), 0);
        L.inflight = false;
      }
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

static void greedy_worker(ged_server *s) {
  for (;;) {
    Req q;
    std::shared_ptr<std::atomic<int>> flag;
    int stopped = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // admission: the head of the queue starts once its working memory
      // fits (or leaves at once if it was asked to stop)
      s->cv_greedy.wait(lk, [&] {
        if (s->stop) return true;
        if (s->greedy_q.empty()) return false;
        const uint64_t id = s->greedy_q.front().id;
        return s->pol->stop_status(id) != 0 || s->pol->greedy_fits(id);
      });
      if (s->stop) return;
      q = std::move(s->greedy_q.front());
      s->greedy_q.pop_front();
      stopped = s->pol->stop_status(q.id);
      if (!stopped) {
        s->pol->start(q.id);
        flag = std::make_shared<std::atomic<int>>(0);
        s->running_stop[q.id] = flag;
      }
    }
    if (stopped) {
      emit(s, q, stopped, 0.0, {}, now_us());
      continue;
    }
    Lane &L = *s->lanes[q.graph];
    std::vector<int> grp(q.k);
    double score = 0.0;
    int rc;
    size_t held = 0;
    {
      std::lock_guard<std::recursive_mutex> lk(L.g->mu);
      rc = guarded([&]() {
        return greedy_run(L.g, q.k, L.alpha, L.eps, 0.0, 0, false, grp.data(), &score, nullptr,
                          flag.get());
      });
      held = greedy_bytes_held(L.g);
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->running_stop.erase(q.id);
    }
    emit(s, q, rc, score, rc == GED_OK ? grp : std::vector<int>(), now_us(), held);
  }
}

static void start(ged_server *s) {
  if (s->started) return;
  s->started = true;
  s->sched = std::thread(sched_loop, s);
  for (int i = 0; i < std::max(1, s->cfg.greedy_workers); ++i)
    s->workers.emplace_back(greedy_worker, s);
}

}  // namespace ged

using namespace ged;

extern "C" int ged_server_create(const ged_server_config *cfg, ged_server **out) {
  if (!cfg || !out) return fail(GED_ERR_ARG, "null argument");
  if (cfg->hbm_budget_bytes <= 0 || cfg->max_queue <= 0 || cfg->score_slots < 0 ||
      cfg->score_slots > 64 || (cfg->score_slots & (cfg->score_slots - 1)) != 0)
    return fail(GED_ERR_ARG, "bad server config (score_slots must be 0 or a power of two <= 64)");
  auto s = std::make_unique<ged_server>();
  s->cfg = *cfg;
  s->pol = std::make_unique<ServePolicy>(cfg->hbm_budget_bytes, cfg->max_queue);
  *out = s.release();
  return GED_OK;
}

extern "C" int ged_server_add_graph(ged_server *s, ged_graph *g, double alpha, double eps,
                                    int32_t *graph_id) {
  if (!s || !g || !graph_id) return fail(GED_ERR_ARG, "null argument");
  if (s->started) return fail(GED_ERR_ARG, "graphs must be added before the first request");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  if (g->served) return fail(GED_ERR_BUSY, "the graph is registered with a server already");
  return guarded([&]() -> int {
    int rc = prepare(g, alpha, eps);
    if (rc) return rc;
    auto L = std::make_unique<Lane>();
    L->g = g;
    L->gid = (int)s->lanes.size();
    L->alpha = alpha;
    L->eps = eps;
    L->ell = g->prep.ell;
    int C = s->cfg.score_slots;
    if (C == 0) {
      // split tiles run no wider than their requests need, so a wide limit
      // costs memory only; a column pool steps all its columns every time
      const int64_t n = g->n;
      if (split_ok(g))
        C = n <= 1000000 ? 64 : 32;
      else
        C = n <= 200000 ? 64 : n <= 1000000 ? 32 : n <= 2000000 ? 16 : 8;
    }
    lane_setup(*L, C);
    // the handle's single-group score workspace (a greedy's final score uses
    // it): materialised now and counted with the lane
    double tmp = 0.0;
    const int32_t v0 = 0;
    rc = score_group(g, &v0, 1, alpha, eps, &tmp, nullptr);
    if (rc) return rc;
    // walk lengths a greedy can reach: ell doubles until the tail bound drops
    // below eps / k, after which every round separates
    for (int ell = 1;; ell *= 2) {
      const double B = comb_bound(g, alpha, walk_total(g, ell));
      L->sep.push_back({ell, B});
      L->fp.push_back(greedy_footprint(g, ell, 0));
      if (B < eps / (double)g->n || ell >= 65536) break;
    }
    GED_HIP(hipStreamSynchronize(g->stream));
    {
      std::lock_guard<std::mutex> lk2(s->mu);
      if (s->pol->add_lane(L->bytes + score_bytes_held(g)) != GED_OK)
        return fail(GED_ERR_NOMEM, "graph pool exceeds the HBM budget");
      s->pol->set_held(L->gid, greedy_bytes_held(g));
    }
    g->served = true;
    g->served_alpha = alpha;
    g->served_eps = eps;
    *graph_id = L->gid;
    s->lanes.push_back(std::move(L));
    return GED_OK;
  });
}

static int submit(ged_server *s, Req &&q, uint64_t *req_id) {
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t id = s->next_id;
  const int rc = s->pol->submit(id, q.kind, q.graph, q.footprint, 0.0);
  if (rc == GED_ERR_BUSY) return fail(rc, "request queue full");
  if (rc == GED_ERR_NOMEM) return fail(rc, "greedy request exceeds the HBM budget");
  s->next_id++;
  q.id = id;
  q.t_submit = now_us();
  if (req_id) *req_id = q.id;
  if (q.kind == 0) {
    s->inbox.push_back(std::move(q));
    s->cv_work.notify_one();
  } else {
    s->greedy_q.push_back(std::move(q));
    s->cv_greedy.notify_all();
  }
  return GED_OK;
}

extern "C" int ged_server_submit_score(ged_server *s, int32_t graph_id, const int32_t *S,
                                       int32_t s_len, uint64_t *req_id) {
  if (!s || graph_id < 0 || graph_id >= (int)s->lanes.size() || s_len < 0 || (s_len > 0 && !S))
    return fail(GED_ERR_ARG, "bad score request");
  ged_graph *g = s->lanes[graph_id]->g;
  Req q;
  q.kind = 0;
  q.graph = graph_id;
  q.S.reserve(s_len);
  for (int i = 0; i < s_len; ++i) {
    if (S[i] < 0 || S[i] >= g->n) return fail(GED_ERR_VERTEX, "group member out of range");
    q.S.push_back(g->new_id[S[i]]);
  }
  std::sort(q.S.begin(), q.S.end());
  q.S.erase(std::unique(q.S.begin(), q.S.end()), q.S.end());
  start(s);
  return submit(s, std::move(q), req_id);
}

extern "C" int ged_server_submit_greedy(ged_server *s, int32_t graph_id, int32_t k,
                                        uint64_t *req_id) {
  if (!s || graph_id < 0 || graph_id >= (int)s->lanes.size())
    return fail(GED_ERR_ARG, "bad greedy request");
  ged_graph *g = s->lanes[graph_id]->g;
  if (k < 1 || k > g->n) return fail(GED_ERR_ARG, "k must be in [1, n]");
  Req q;
  q.kind = 1;
  q.graph = graph_id;
  q.k = k;
  // working memory at the largest walk length this k can reach: the first
  // tabulated length whose tail bound is below eps / k (the last one, where
  // the table ends, bounds every k)
  const Lane &L = *s->lanes[graph_id];
  size_t fp = L.fp.back();
  for (size_t j = 0; j < L.sep.size(); ++j)
    if (L.sep[j].second < L.eps / (double)k) {
      fp = L.fp[j];
      break;
    }
  q.footprint = fp + 16 * (size_t)k + 4096;
  start(s);
  return submit(s, std::move(q), req_id);
}

extern "C" int ged_server_poll(ged_server *s, ged_result *out, int32_t max, int32_t *n_out,
                               int64_t timeout_us) {
  if (!s || !n_out || max < 0 || (max > 0 && !out)) return fail(GED_ERR_ARG, "bad poll");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->results.empty() && timeout_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                        [&] { return !s->results.empty(); });
  int m = 0;
  while (m < max && !s->results.empty()) {
    out[m++] = s->results.front().r;
    s->results.pop_front();
  }
  *n_out = m;
  return GED_OK;
}

extern "C" int ged_server_group(ged_server *s, uint64_t req_id, int32_t *out, int32_t k) {
  if (!s || !out) return fail(GED_ERR_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->groups.find(req_id);
  if (it == s->groups.end()) return fail(GED_ERR_ARG, "no greedy result with this id");
  if ((int)it->second.size() != k) return fail(GED_ERR_ARG, "k does not match the request");
  std::memcpy(out, it->second.data(), sizeof(int) * k);
  return GED_OK;
}

extern "C" int ged_server_stats(ged_server *s, int64_t *out6) {
  if (!s || !out6) return fail(GED_ERR_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  out6[0] = s->pol->admitted();
  out6[1] = s->pol->completed();
  out6[2] = s->steps;
  out6[3] = (int64_t)s->pol->peak_bytes();
  out6[4] = s->peak_cols;
  out6[5] = s->pol->rejected();
  return GED_OK;
}

extern "C" int ged_server_cancel(ged_server *s, uint64_t req_id) {
  if (!s) return fail(GED_ERR_ARG, "null argument");
  int rc;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rc = s->pol->request_stop(req_id, GED_ERR_CANCELLED);
    auto it = s->running_stop.find(req_id);
    if (rc == GED_OK && it != s->running_stop.end())
      it->second->store(s->pol->stop_status(req_id), std::memory_order_relaxed);
  }
  s->cv_work.notify_all();
  s->cv_greedy.notify_all();
  if (rc == GED_ERR_ARG) return fail(rc, "no waiting or running request with this id");
  if (rc == GED_ERR_BUSY) return fail(rc, "the score is already on the device");
  return rc;
}

extern "C" int ged_server_set_deadline(ged_server *s, uint64_t req_id, double deadline_us) {
  if (!s || !(deadline_us >= 0.0)) return fail(GED_ERR_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const int rc = s->pol->set_deadline(req_id, deadline_us);
  if (rc) return fail(rc, "no waiting or running request with this id");
  return GED_OK;
}

extern "C" int ged_server_destroy(ged_server *s) {
  if (!s) return GED_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_greedy.notify_all();
  if (s->sched.joinable()) s->sched.join();
  for (auto &w : s->workers)
    if (w.joinable()) w.join();
  for (auto &L : s->lanes) {
    if (L->st) {
      (void)hipStreamSynchronize(L->st);
      (void)hipStreamDestroy(L->st);
    }
    if (L->ev) (void)hipEventDestroy(L->ev);
    std::lock_guard<std::recursive_mutex> lk(L->g->mu);
    L->g->served = false;
  }
  delete s;
  return GED_OK;
}
