// C entry point over the host-side graph construction
// (paper_1910_13874_amd/csrc/graph_build.h) for the CPU tests, which build
// this file with g++ and compare the result with a direct construction.  No
// device code is involved.  The caller sizes the outputs: n for the id maps,
// n + 1 for the row pointers, max(1, nnz) for the entries (weights only when
// w is given).  Returns null, or the construction's error message.
#include "graph_build.h"

extern "C" const char *gb_build(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *ci,
                                const double *w, int undirected, int keep_order, int threads,
                                int *new_id, int *old_id, int *irp, int *ici, double *iw, int *orp,
                                int *oci, double *ow, int *max_deg, double *max_wdeg,
                                int *simple) {
  ged::HostCsr h;
  const char *m = ged::build_host_csr(n, nnz, rp, ci, w, undirected != 0, keep_order != 0,
                                      threads, h);
  if (m) return m;
  std::copy(h.new_id.begin(), h.new_id.end(), new_id);
  std::copy(h.old_id.begin(), h.old_id.end(), old_id);
  std::copy(h.irp.begin(), h.irp.end(), irp);
  std::copy(h.ici.begin(), h.ici.end(), ici);
  std::copy(h.orp.begin(), h.orp.end(), orp);
  std::copy(h.oci.begin(), h.oci.end(), oci);
  if (w) {
    std::copy(h.iw.begin(), h.iw.end(), iw);
    std::copy(h.ow.begin(), h.ow.end(), ow);
  }
  *max_deg = h.max_deg;
  *max_wdeg = h.max_wdeg;
  *simple = h.simple ? 1 : 0;
  return nullptr;
}

extern "C" int gb_threads(int64_t n, int64_t nnz) { return ged::build_threads(n, nnz); }

// run_threads with part `bad` throwing: 1 if the exception reaches the caller
// after every other part ran, else 0.
extern "C" int gb_threads_rethrow(int T, int bad) {
  std::vector<int> ran((size_t)T, 0);
  try {
    ged::build_detail::run_threads(T, [&](int t) {
      if (t == bad) throw std::bad_alloc();
      ran[(size_t)t] = 1;
    });
  } catch (const std::bad_alloc &) {
    for (int t = 0; t < T; ++t)
      if (t != bad && !ran[(size_t)t]) return 0;
    return 1;
  }
  return 0;
}
