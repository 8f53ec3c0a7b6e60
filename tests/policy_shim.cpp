// C entry points over the request server's admission policy
// (paper_1910_13874_amd/csrc/server_policy.h) for the CPU tests, which build
// this file with g++ and drive the policy with a fake executor.  No device
// code is involved.
#include "server_policy.h"

using ged::ServePolicy;

extern "C" {
void *pol_new(int64_t budget, int64_t max_queue) { return new ServePolicy(budget, max_queue); }
void pol_free(void *p) { delete static_cast<ServePolicy *>(p); }
int pol_add_lane(void *p, uint64_t bytes) { return static_cast<ServePolicy *>(p)->add_lane(bytes); }
void pol_set_held(void *p, int graph, uint64_t bytes) {
  static_cast<ServePolicy *>(p)->set_held(graph, bytes);
}
int pol_submit(void *p, uint64_t id, int kind, int graph, uint64_t footprint, double deadline) {
  return static_cast<ServePolicy *>(p)->submit(id, kind, graph, footprint, deadline);
}
int pol_greedy_fits(void *p, uint64_t id) { return static_cast<ServePolicy *>(p)->greedy_fits(id); }
void pol_start(void *p, uint64_t id) { static_cast<ServePolicy *>(p)->start(id); }
int pol_finish(void *p, uint64_t id, uint64_t held) {
  return static_cast<ServePolicy *>(p)->finish(id, held);
}
int pol_request_stop(void *p, uint64_t id, int why) {
  return static_cast<ServePolicy *>(p)->request_stop(id, why);
}
int pol_set_deadline(void *p, uint64_t id, double d) {
  return static_cast<ServePolicy *>(p)->set_deadline(id, d);
}
void pol_expire(void *p, double now) { static_cast<ServePolicy *>(p)->expire(now); }
int pol_take_dropped(void *p, uint64_t *out, int max) {
  std::vector<uint64_t> d = static_cast<ServePolicy *>(p)->take_dropped();
  int m = 0;
  for (uint64_t x : d)
    if (m < max) out[m++] = x;
  return m;
}
int pol_stop_status(void *p, uint64_t id) { return static_cast<ServePolicy *>(p)->stop_status(id); }
int64_t pol_stat(void *p, int which) {
  const ServePolicy &q = *static_cast<ServePolicy *>(p);
  switch (which) {
    case 0: return q.waiting();
    case 1: return q.admitted();
    case 2: return q.completed();
    case 3: return q.rejected();
    case 4: return (int64_t)q.peak_bytes();
    case 5: return (int64_t)q.in_use();
    default: return -1;
  }
}
uint64_t pol_held(void *p, int graph) { return static_cast<ServePolicy *>(p)->held(graph); }
}
