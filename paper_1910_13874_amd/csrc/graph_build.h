// Host-side construction of a graph's internal CSR: validation of the
// caller's CSR, the internal vertex order (decreasing out-degree, stable) and
// the in- and out-row arrays in internal ids with sorted rows.  No device
// code: the library uploads the result, and the CPU tests build this header
// alone (tests/build_shim.cpp) and compare it with a direct construction.
//
// The arc passes run on up to kBuildThreads threads over contiguous row
// ranges.  An undirected graph's rows are built in place: each internal row
// is the caller's row relabelled and sorted.  A directed graph takes two
// scatters (to the out-rows, then back to the in-rows), each stable: thread t
// writes its arcs of bucket b from the offset of b plus the arcs of b held by
// threads 0 .. t-1 (per-thread histograms), and threads hold rows in
// increasing order.  Either way every row lists its entries in increasing
// order, equal entries in arc order: the same arrays whatever the thread
// count.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <exception>
#include <system_error>
#include <thread>
#include <vector>

namespace ged {

constexpr int kBuildThreads = 16;

struct HostCsr {
  std::vector<int> new_id, old_id;  // caller id -> internal id, and back
  std::vector<int> irp, ici;        // in-rows: row v lists u for every arc u -> v
  std::vector<double> iw;           // their weights (weighted graphs)
  std::vector<int> orp, oci;        // out-rows (the reverse graph; oci and ow
  std::vector<double> ow;           // directed graphs only: undirected ones equal irp/ici)
  int32_t max_deg = 0;              // maximum out-degree
  double max_wdeg = 0.0;            // maximum weighted out-degree
  bool simple = true;               // no arc listed twice
};

namespace build_detail {

inline uint64_t mix64(uint64_t z) {  // splitmix64 finaliser (Steele et al.)
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Run f(t) for t in [0, T): on T - 1 new threads and the caller's.  Parts
// whose thread cannot be started run on the caller's; an exception thrown by
// any part (a failed allocation) is rethrown here once every thread has
// joined.
template <class F>
void run_threads(int T, F &&f) {
  if (T <= 1) {
    f(0);
    return;
  }
  std::vector<std::exception_ptr> err((size_t)T);
  auto part = [&f, &err](int t) {
    try {
      f(t);
    } catch (...) {
      err[(size_t)t] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  std::vector<int> here{0};
  th.reserve((size_t)T - 1);
  for (int t = 1; t < T; ++t) {
    try {
      th.emplace_back(part, t);
    } catch (const std::system_error &) {
      here.push_back(t);
    }
  }
  for (int t : here) part(t);
  for (auto &x : th) x.join();
  for (const auto &e : err)
    if (e) std::rethrow_exception(e);
}

// Row range bounds [b[t], b[t+1]) splitting rows 0..N-1 of the monotone
// prefix array p (p[N] entries in all) into T parts of about equal entries.
inline std::vector<int64_t> split_rows(const int64_t *p, int64_t N, int T) {
  std::vector<int64_t> b((size_t)T + 1, N);
  b[0] = 0;
  for (int t = 1; t < T; ++t) {
    const int64_t goal = p[N] / T * t;
    b[t] = std::max(b[t - 1], (int64_t)(std::lower_bound(p, p + N, goal) - p));
  }
  return b;
}

// Stable scatter of T row ranges into buckets.  rows [b[t], b[t+1]) of the
// source are taken in order; key(r, j) is the bucket of entry j of row r, and
// emit(pos, r, j) writes it at position pos.  bp[k] is the first position of
// bucket k (nb buckets); cnt is scratch of T * nb counters.
template <class RowArcs, class Key, class Emit>
void stable_scatter(int T, const std::vector<int64_t> &b, int64_t nb, const int *bp,
                    std::vector<int> &cnt, RowArcs &&arcs, Key &&key, Emit &&emit) {
  cnt.assign((size_t)T * (size_t)nb, 0);
  run_threads(T, [&](int t) {
    int *c = cnt.data() + (size_t)t * nb;
    for (int64_t r = b[t]; r < b[t + 1]; ++r) {
      int64_t j0, j1;
      arcs(r, j0, j1);
      for (int64_t j = j0; j < j1; ++j) c[key(r, j)]++;
    }
  });
  // counts -> start offsets, bucket by bucket (ranges of buckets in parallel)
  run_threads(T, [&](int t) {
    const int64_t k0 = nb * t / T, k1 = nb * (t + 1) / T;
    for (int64_t k = k0; k < k1; ++k) {
      int s = bp[k];
      for (int u = 0; u < T; ++u) {
        int &x = cnt[(size_t)u * nb + k];
        const int n = x;
        x = s;
        s += n;
      }
    }
  });
  run_threads(T, [&](int t) {
    int *c = cnt.data() + (size_t)t * nb;
    for (int64_t r = b[t]; r < b[t + 1]; ++r) {
      int64_t j0, j1;
      arcs(r, j0, j1);
      for (int64_t j = j0; j < j1; ++j) emit(c[key(r, j)]++, r, j);
    }
  });
}

}  // namespace build_detail

// Threads for a graph: one below 2^20 arcs; otherwise up to kBuildThreads
// and the host's hardware threads, with at most nnz/n (the per-thread
// counters then take no more memory than the arcs themselves).
inline int build_threads(int64_t n, int64_t nnz) {
  if (nnz < (1 << 20)) return 1;
  const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
  return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kBuildThreads, hw, nnz / n}));
}

// Validates the caller's CSR (row v lists the sources u of the arcs u -> v)
// and fills `out`.  Returns nullptr, or the message of the first error by
// row: a decreasing row_ptr, then -- row by row, arc by arc -- a source out of
// range, a self-loop or a weight outside (0, 1]; then, for undirected graphs,
// asymmetry.  The caller has checked n, nnz, the arrays and row_ptr's ends.
// threads <= 0: build_threads(n, nnz).
inline const char *build_host_csr(int64_t n, int64_t nnz, const int64_t *row_ptr,
                                  const int32_t *col_idx, const double *weights, bool undirected,
                                  bool keep_order, int threads, HostCsr &out) {
  using namespace build_detail;
  const int N = (int)n;
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return "row_ptr decreases";
  const int T = threads > 0 ? threads : build_threads(n, nnz);
  std::vector<int> cnt;  // per-thread counters, reused by every pass
  // ---- arcs: validity, out-degrees (per-thread counts), symmetry hashes
  std::vector<int64_t> outdeg((size_t)n, 0);
  {
    const std::vector<int64_t> b = split_rows(row_ptr, n, T);
    struct Part {
      int64_t bad_row = -1;
      const char *msg = nullptr;
      uint64_t hf = 0, hb = 0;
    };
    std::vector<Part> part((size_t)T);
    cnt.assign((size_t)T * (size_t)n, 0);
    run_threads(T, [&](int t) {
      Part &P = part[(size_t)t];
      int *c = cnt.data() + (size_t)t * n;
      for (int64_t v = b[t]; v < b[t + 1] && !P.msg; ++v)
        for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
          const int32_t u = col_idx[j];
          const char *m = nullptr;
          if (u < 0 || u >= n)
            m = "col_idx out of range";
          else if (u == v)
            m = "self-loop";
          else if (weights && !(weights[j] > 0.0 && weights[j] <= 1.0))
            m = "weights must be in (0, 1]";
          if (m) {
            P.msg = m;
            P.bad_row = v;
            break;
          }
          c[u]++;
          if (undirected) {
            P.hf += mix64(((uint64_t)u << 32) | (uint64_t)v);
            P.hb += mix64(((uint64_t)v << 32) | (uint64_t)u);
            if (weights) {
              uint64_t wb;
              std::memcpy(&wb, &weights[j], sizeof(wb));
              P.hf += mix64((((uint64_t)u << 32) | (uint64_t)v) ^ mix64(wb));
              P.hb += mix64((((uint64_t)v << 32) | (uint64_t)u) ^ mix64(wb));
            }
          }
        }
    });
    uint64_t hf = 0, hb = 0;
    for (const Part &P : part) {  // threads hold increasing rows: the first error is the first
      if (P.msg) return P.msg;
      hf += P.hf;
      hb += P.hb;
    }
    run_threads(T, [&](int t) {
      const int64_t v0 = n * t / T, v1 = n * (t + 1) / T;
      for (int u = 0; u < T; ++u) {
        const int *c = cnt.data() + (size_t)u * n;
        for (int64_t v = v0; v < v1; ++v) outdeg[(size_t)v] += c[v];
      }
    });
    if (undirected) {
      for (int64_t v = 0; v < n; ++v)
        if (outdeg[(size_t)v] != row_ptr[v + 1] - row_ptr[v])
          return "GED_UNDIRECTED graph is not symmetric";
      if (hf != hb) return "GED_UNDIRECTED graph is not symmetric";
    }
  }
  int64_t md = 0;
  for (int64_t v = 0; v < n; ++v) md = std::max(md, outdeg[(size_t)v]);
  out.max_deg = (int32_t)md;
  out.max_wdeg = 0.0;
  if (weights) {
    // sum of the weights of the arcs leaving v, added in arc order
    std::vector<double> wout((size_t)n, 0.0);
    for (int64_t v = 0; v < n; ++v)
      for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) wout[(size_t)col_idx[j]] += weights[j];
    for (double x : wout) out.max_wdeg = std::max(out.max_wdeg, x);
  }
  // ---- internal vertex order: stable counting sort by decreasing out-degree
  out.new_id.assign((size_t)N, 0);
  out.old_id.assign((size_t)N, 0);
  if (keep_order) {
    for (int v = 0; v < N; ++v) out.new_id[(size_t)v] = out.old_id[(size_t)v] = v;
  } else {
    std::vector<int64_t> c((size_t)md + 2, 0);
    for (int v = 0; v < N; ++v) c[(size_t)(md - outdeg[(size_t)v]) + 1]++;
    for (size_t d = 1; d < c.size(); ++d) c[d] += c[d - 1];
    for (int v = 0; v < N; ++v) {
      const int pos = (int)c[(size_t)(md - outdeg[(size_t)v])]++;
      out.new_id[(size_t)v] = pos;
      out.old_id[(size_t)pos] = v;
    }
  }
  const int *nid = out.new_id.data();
  const int *oid = out.old_id.data();
  const size_t ne = (size_t)std::max<int64_t>(1, nnz);
  // ---- row pointers in internal ids: in-rows keep the caller's row lengths,
  // out-rows take the out-degrees
  out.irp.assign((size_t)N + 1, 0);
  out.orp.assign((size_t)N + 1, 0);
  for (int nv = 0; nv < N; ++nv) {
    const int v = oid[nv];
    out.irp[(size_t)nv + 1] = (int)(row_ptr[v + 1] - row_ptr[v]);
    out.orp[(size_t)nv + 1] = (int)outdeg[(size_t)v];
  }
  for (int v = 0; v < N; ++v) {
    out.irp[(size_t)v + 1] += out.irp[(size_t)v];
    out.orp[(size_t)v + 1] += out.orp[(size_t)v];
  }
  if (undirected) {
    // in-rows directly: internal row nv is the caller's row old_id[nv],
    // relabelled and sorted (equal sources in arc order); the out-rows of an
    // undirected graph are the same rows and are not built
    out.ici.assign(ne, 0);
    out.iw.assign(weights ? ne : 0, 0.0);
    std::vector<int64_t> ip(out.irp.begin(), out.irp.end());
    const std::vector<int64_t> b = split_rows(ip.data(), n, T);
    run_threads(T, [&](int t) {
      std::vector<uint64_t> key;
      for (int64_t nv = b[t]; nv < b[t + 1]; ++nv) {
        const int v = oid[nv];
        const int64_t j0 = row_ptr[v], len = row_ptr[v + 1] - j0;
        int *dst = out.ici.data() + out.irp[(size_t)nv];
        if (!weights) {
          for (int64_t k = 0; k < len; ++k) dst[k] = nid[col_idx[j0 + k]];
          std::sort(dst, dst + len);
        } else {
          key.resize((size_t)len);
          for (int64_t k = 0; k < len; ++k)
            key[(size_t)k] = ((uint64_t)nid[col_idx[j0 + k]] << 32) | (uint64_t)k;
          std::sort(key.begin(), key.end());
          double *dw = out.iw.data() + out.irp[(size_t)nv];
          for (int64_t k = 0; k < len; ++k) {
            dst[k] = (int)(key[(size_t)k] >> 32);
            dw[k] = weights[j0 + (int64_t)(key[(size_t)k] & 0xffffffffu)];
          }
        }
      }
    });
  } else {
    // ---- out-rows: row nu lists nv for every arc u -> v, the caller's rows
    // taken in internal order
    out.oci.assign(ne, 0);
    out.ow.assign(weights ? ne : 0, 0.0);
    {
      std::vector<int64_t> ip(out.irp.begin(), out.irp.end());
      const std::vector<int64_t> b = split_rows(ip.data(), n, T);
      int *oci = out.oci.data();
      double *ow = out.ow.data();
      stable_scatter(
          T, b, n, out.orp.data(), cnt,
          [&](int64_t nv, int64_t &j0, int64_t &j1) {
            const int v = oid[nv];
            j0 = row_ptr[v];
            j1 = row_ptr[v + 1];
          },
          [&](int64_t, int64_t j) { return nid[col_idx[j]]; },
          [&](int q, int64_t nv, int64_t j) {
            oci[q] = (int)nv;
            if (weights) ow[q] = weights[j];
          });
    }
    // ---- in-rows: scatter the out-rows back (row nv lists nu for u -> v)
    out.ici.assign(ne, 0);
    out.iw.assign(weights ? ne : 0, 0.0);
    {
      std::vector<int64_t> op(out.orp.begin(), out.orp.end());
      const std::vector<int64_t> b = split_rows(op.data(), n, T);
      const int *orp = out.orp.data();
      const int *oci = out.oci.data();
      const double *ow = out.ow.data();
      int *ici = out.ici.data();
      double *iw = out.iw.data();
      stable_scatter(
          T, b, n, out.irp.data(), cnt,
          [&](int64_t nu, int64_t &j0, int64_t &j1) {
            j0 = orp[nu];
            j1 = orp[nu + 1];
          },
          [&](int64_t, int64_t q) { return oci[q]; },
          [&](int r, int64_t nu, int64_t q) {
            ici[r] = (int)nu;
            if (weights) iw[r] = ow[q];
          });
    }
  }
  std::vector<int>().swap(cnt);
  // ---- simple: no row lists a source twice (rows are sorted)
  {
    std::vector<char> dup((size_t)T, 0);
    run_threads(T, [&](int t) {
      const int64_t v0 = n * t / T, v1 = n * (t + 1) / T;
      for (int64_t v = v0; v < v1 && !dup[(size_t)t]; ++v)
        for (int r = out.irp[(size_t)v] + 1; r < out.irp[(size_t)v + 1]; ++r)
          if (out.ici[(size_t)r] == out.ici[(size_t)r - 1]) {
            dup[(size_t)t] = 1;
            break;
          }
    });
    out.simple = std::find(dup.begin(), dup.end(), 1) == dup.end();
  }
  return nullptr;
}

}  // namespace ged
