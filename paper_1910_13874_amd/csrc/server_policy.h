// Admission, queue limits, deadlines and cancellation of the request server
// (ged_server_*), kept free of device code: the server calls it from its
// threads under its own lock, and the CPU tests drive it with a fake executor
// (a loop that starts and finishes requests on a simulated clock).
//
// Memory model.  A lane (one resident graph) holds its score pool for the
// server's lifetime, and each graph keeps the greedy working memory its
// largest request grew, since device memory is not returned between requests.
// Both count against the budget permanently (lane_bytes, held per graph).  A
// greedy request is admitted at submission only if its estimated peak
// footprint could ever fit beside them; it starts when the bytes it may add
// beyond what its graph already holds -- its reservation -- fit beside the
// reservations of the greedy requests running; when it finishes, its
// reservation is released and the graph's held bytes become what the request
// measured.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <map>
#include <memory>
#include <vector>

#include "ged.h"

namespace ged {

enum class ReqState : int { Waiting = 0, Running = 1 };

struct Ticket {
  int kind = 0;      // 0 score, 1 greedy
  int graph = 0;
  size_t footprint = 0;   // greedy: estimated peak bytes of its working memory
  size_t reserved = 0;    // greedy, while running: bytes beyond what the graph held
  double deadline_us = 0; // absolute (the server's clock); 0: none
  ReqState state = ReqState::Waiting;
  int stop = 0;           // 0, or GED_ERR_CANCELLED / GED_ERR_DEADLINE once asked to stop
};

class ServePolicy {
 public:
  ServePolicy(int64_t budget, int64_t max_queue) : budget_(budget), max_queue_(max_queue) {}

  // A lane's pool joins the budget (GED_ERR_NOMEM if it does not fit).
  int add_lane(size_t bytes) {
    if (committed() + bytes > (size_t)budget_) return GED_ERR_NOMEM;
    lane_bytes_ += bytes;
    note_peak();
    return GED_OK;
  }

  // Bytes graph `graph`'s greedy working memory holds when it joins.
  void set_held(int graph, size_t bytes) {
    held_[graph] = bytes;
    note_peak();
  }

  // A new request: GED_ERR_BUSY if max_queue requests are waiting; for a
  // greedy request GED_ERR_NOMEM (counted as rejected) if its footprint
  // could never fit beside the lanes and every graph's held memory.
  int submit(uint64_t id, int kind, int graph, size_t footprint, double deadline_us) {
    if (waiting_ >= max_queue_) return GED_ERR_BUSY;
    if (kind == 1 && committed() + extra_for(graph, footprint) > (size_t)budget_) {
      ++rejected_;
      return GED_ERR_NOMEM;
    }
    Ticket t;
    t.kind = kind;
    t.graph = graph;
    t.footprint = footprint;
    t.deadline_us = deadline_us;
    tickets_[id] = t;
    ++waiting_;
    ++admitted_;
    return GED_OK;
  }

  // Can greedy request `id` start now (its reservation fits)?
  bool greedy_fits(uint64_t id) const {
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return false;
    return committed() + reserved_ + extra_for(it->second.graph, it->second.footprint) <=
           (size_t)budget_;
  }

  // Request `id` leaves the queue for the device (greedy: reserve).
  void start(uint64_t id) {
    Ticket &t = tickets_.at(id);
    t.state = ReqState::Running;
    --waiting_;
    if (t.kind == 1) {
      t.reserved = extra_for(t.graph, t.footprint);
      reserved_ += t.reserved;
      note_peak();
    }
  }

  // Request `id` is done (any status).  held_after: for a greedy request that
  // ran, the bytes its graph's greedy workspace holds now (it keeps them);
  // ignored otherwise.  Returns the status a stop request asked for, or 0.
  int finish(uint64_t id, size_t held_after = 0) {
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return 0;
    Ticket &t = it->second;
    if (t.state == ReqState::Waiting) --waiting_;
    if (t.kind == 1 && t.state == ReqState::Running) {
      reserved_ -= t.reserved;
      size_t &h = held_[t.graph];
      h = std::max(h, held_after);
      note_peak();
    }
    const int stop = t.stop;
    tickets_.erase(it);
    ++completed_;
    return stop;
  }

  // Ask request `id` to stop: GED_OK if it will complete with `why`
  // (GED_ERR_CANCELLED or GED_ERR_DEADLINE) -- a waiting request is dropped
  // by the next scheduler pass, a running greedy stops at its next pick --
  // GED_ERR_BUSY for a score already on the device (it completes normally),
  // GED_ERR_ARG for an unknown or finished id.
  int request_stop(uint64_t id, int why) {
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return GED_ERR_ARG;
    Ticket &t = it->second;
    if (t.state == ReqState::Running && t.kind == 0) return GED_ERR_BUSY;
    if (!t.stop) t.stop = why;
    if (t.state == ReqState::Waiting) drop_.push_back(id);
    return GED_OK;
  }

  int set_deadline(uint64_t id, double deadline_us) {
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return GED_ERR_ARG;
    it->second.deadline_us = deadline_us;
    return GED_OK;
  }

  // Every request whose deadline has passed is asked to stop (scores already
  // on the device excepted).
  void expire(double now_us) {
    for (auto &kv : tickets_) {
      const Ticket &t = kv.second;
      if (t.deadline_us > 0 && now_us >= t.deadline_us && !t.stop &&
          !(t.state == ReqState::Running && t.kind == 0))
        request_stop(kv.first, GED_ERR_DEADLINE);
    }
  }

  // Waiting requests asked to stop since the last call: the scheduler removes
  // them from its queues and completes them with stop_status().
  std::vector<uint64_t> take_dropped() {
    std::vector<uint64_t> d;
    d.swap(drop_);
    return d;
  }

  int stop_status(uint64_t id) const {
    auto it = tickets_.find(id);
    return it == tickets_.end() ? 0 : it->second.stop;
  }

  bool known(uint64_t id) const { return tickets_.count(id) != 0; }
  int64_t waiting() const { return waiting_; }
  int64_t admitted() const { return admitted_; }
  int64_t completed() const { return completed_; }
  int64_t rejected() const { return rejected_; }
  size_t peak_bytes() const { return peak_; }
  size_t in_use() const { return committed() + reserved_; }
  size_t held(int graph) const {
    auto it = held_.find(graph);
    return it == held_.end() ? 0 : it->second;
  }

 private:
  size_t committed() const {
    size_t h = 0;
    for (const auto &kv : held_) h += kv.second;
    return lane_bytes_ + h;
  }
  size_t extra_for(int graph, size_t footprint) const {
    const size_t h = held(graph);
    return footprint > h ? footprint - h : 0;
  }
  void note_peak() { peak_ = std::max(peak_, committed() + reserved_); }

  int64_t budget_, max_queue_;
  size_t lane_bytes_ = 0, reserved_ = 0, peak_ = 0;
  std::map<int, size_t> held_;
  std::map<uint64_t, Ticket> tickets_;
  std::vector<uint64_t> drop_;
  int64_t waiting_ = 0, admitted_ = 0, completed_ = 0, rejected_ = 0;
};

}  // namespace ged
