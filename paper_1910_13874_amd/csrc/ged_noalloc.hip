// GED_{<=ell*}(S) for one group without any device allocation in the call
// (ged_score_noalloc): the per-call working memory -- membership bitmaps, the
// two hit-chain vectors, block and segment partial sums, the reduction
// scratch, the score and the group itself -- lives in one file-scope device
// array.  The per-graph state the chain reads (device CSR, row partition,
// decayed total-walk levels t_i) is built beforehand by ged_prepare.
//
// The chain is the paper's phi^hit recurrence in its single-vector form
// (Section 3.1.1, Eq. phisum): h_0 = 1_S, h_i(v) = t_i(v) for v in S (every
// walk ending in S meets S) and alpha * sum_{u->v} h_{i-1}(u) otherwise, and
// the score is sum_{i=1}^{ell*} sum_v h_i(v) (Algorithm "GED-Walk
// Computation"), the same level-by-level chain ged_score runs on directed
// graphs, here for every graph kind.
#include <algorithm>
#include <mutex>

#include "ged_internal.h"

namespace ged {

// Working memory of ged_score_noalloc.  Each device the library runs on holds
// its own copy until the process ends.  Host code never uses this name as an
// address: it takes the device address once per device from
// hipGetSymbolAddress and passes that.
constexpr size_t kNoallocScratchBytes = size_t(80) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;                 // one call at a time (the array is shared)
static unsigned char *g_scratch_ptr[kMaxDevices];  // device address per device, null until set

// Device address of the scratch array on the current device (looked up once).
static unsigned char *scratch_ptr() {
  int dev = 0;
  GED_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw HipError{GED_ERR_DEVICE, "device index out of range"};
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw HipError{GED_ERR_DEVICE,
                     std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
  }
  return g_scratch_ptr[dev];
}

// Layout of one call's working memory inside the scratch array.
struct NoallocLayout {
  size_t cmask, mask, vec0, vec1, blk, seg, lng, red2, acc, members, total;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static NoallocLayout noalloc_layout(int64_t n, const Partition &p, int64_t s_len) {
  NoallocLayout L;
  const size_t words = sizeof(uint32_t) * (size_t)((n + 31) / 32 + 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(std::max<size_t>(bytes, 1));
    return at;
  };
  L.cmask = take(words);  // bitmap over caller ids
  L.mask = take(words);   // bitmap over internal ids (what the step kernels read)
  L.vec0 = take(sizeof(double) * (size_t)n);
  L.vec1 = take(sizeof(double) * (size_t)n);
  L.blk = take(sizeof(double) * (size_t)std::max(1, p.n_blocks));
  L.seg = take(sizeof(double) * (size_t)std::max(1, p.n_segs));
  L.lng = take(sizeof(double) * (size_t)std::max(1, p.n_long));
  L.red2 = take(sizeof(double) * (size_t)kReduceBlocks);
  L.acc = take(sizeof(double) * 64);
  L.members = take(sizeof(int32_t) * (size_t)s_len);
  L.total = o;
  return L;
}

// Bits of the caller ids in S (duplicates set the same bit).
__global__ void k_noalloc_caller_bits(uint32_t *cmask, const int32_t *S, int s_len) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < s_len; q += gridDim.x * blockDim.x) {
    const int v = S[q];
    atomicOr(&cmask[v >> 5], 1u << (v & 31));
  }
}

// Internal bitmap word w from the caller bitmap: internal vertex i is in S
// iff its caller id old_id[i] is.
__global__ void k_noalloc_internal_bits(const uint32_t *__restrict__ cmask,
                                       const int *__restrict__ old_id, int n, uint32_t *mask) {
  const int words = (n + 31) / 32;
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x) {
    uint32_t bits = 0;
    const int i1 = min(n, 32 * w + 32);
    for (int i = 32 * w; i < i1; ++i) {
      const int v = old_id[i];
      bits |= ((cmask[v >> 5] >> (v & 31)) & 1u) << (i & 31);
    }
    mask[w] = bits;
  }
}

static int score_noalloc(ged_graph *g, const int32_t *S, int32_t s_len, double alpha, double eps,
                         double *out_score, ged_score_info *info) {
  if (s_len < 0 || (s_len > 0 && !S)) return fail(GED_ERR_ARG, "bad group");
  int rc = check_alpha_eps(g, alpha, eps);
  if (rc) return rc;
  const PrepCache &pc = g->prep;
  const Partition *part = partition_if_built(g, 1);
  if (!pc.valid || pc.alpha != alpha || pc.eps != eps || !part)
    return fail(GED_ERR_ARG,
                "graph not prepared for this alpha and eps: call ged_prepare(g, alpha, eps) "
                "first (ged_score_noalloc allocates nothing, so it cannot precompute)");
  for (int32_t q = 0; q < s_len; ++q)
    if (S[q] < 0 || S[q] >= g->n) return fail(GED_ERR_VERTEX, "group member out of range");
  const int64_t n = g->n;
  const Partition &p = *part;
  const NoallocLayout L = noalloc_layout(n, p, s_len);
  if (L.total > kNoallocScratchBytes)
    return fail(GED_ERR_NOMEM, "ged_score_noalloc needs " + std::to_string(L.total) +
                                   " bytes of working memory for this graph and group; its "
                                   "fixed maximum is " +
                                   std::to_string(kNoallocScratchBytes) + " bytes");
  if (info) {
    info->ell = pc.ell;
    info->bound = pc.bound;
    info->walk_total = pc.W[pc.ell];
  }
  if (s_len == 0) {
    *out_score = 0.0;
    return GED_OK;
  }
  unsigned char *base = scratch_ptr();
  hipStream_t st = g->stream;
  uint32_t *cmask = reinterpret_cast<uint32_t *>(base + L.cmask);
  uint32_t *mask = reinterpret_cast<uint32_t *>(base + L.mask);
  int32_t *members = reinterpret_cast<int32_t *>(base + L.members);
  double *acc = reinterpret_cast<double *>(base + L.acc);
  const size_t words = (size_t)((n + 31) / 32 + 1);
  // the array keeps the previous call's contents: the caller bitmap must
  // start at zero (the internal bitmap and every other buffer is written in
  // full before it is read)
  launch_fill_i32(reinterpret_cast<int *>(cmask), 0, words, st);
  GED_HIP(hipMemcpyAsync(members, S, sizeof(int32_t) * (size_t)s_len, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_noalloc_caller_bits, dim3(std::min(1024, (s_len + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, st, cmask, members, s_len);
  const int nw = (int)((n + 31) / 32);
  hipLaunchKernelGGL(k_noalloc_internal_bits, dim3(std::max(1, std::min(4096, (nw + kBlock - 1) / kBlock))),
                     dim3(kBlock), 0, st, cmask, g->d_old_id.as<const int>(), (int)n, mask);
  GED_HIP(hipGetLastError());
  // the trailing bitmap word past n is read by nothing but is kept zero
  launch_fill_i32(reinterpret_cast<int *>(mask) + nw, 0, words - (size_t)nw, st);
  StepArgs a = base_args(g);
  a.blk_part = reinterpret_cast<double *>(base + L.blk);
  a.seg_out = reinterpret_cast<double *>(base + L.seg);
  a.long_part = reinterpret_cast<double *>(base + L.lng);
  double *vec[2] = {reinterpret_cast<double *>(base + L.vec0),
                    reinterpret_cast<double *>(base + L.vec1)};
  const double *T = pc.t_levels.as<const double>();
  for (int i = 1; i <= pc.ell; ++i) {
    a.C = 1;
    a.alpha = pc.alpha;
    a.accum = i > 1;  // block partials of all levels add up to the score
    a.smask = mask;
    a.X = vec[(i - 1) & 1];
    a.Y = vec[i & 1];
    a.inj = T + (size_t)i * n;
    launch_step(p, a, i == 1 ? IN_MASK : IN_VEC, OUT_INJ, st);
  }
  launch_reduce(p, a, acc, nullptr, nullptr, st, reinterpret_cast<double *>(base + L.red2));
  GED_HIP(hipMemcpyAsync(out_score, acc, sizeof(double), hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  return GED_OK;
}

}  // namespace ged

using namespace ged;

extern "C" int ged_score_noalloc(ged_graph *g, const int32_t *S, int32_t s_len, double alpha,
                                 double eps, double *out_score, ged_score_info *info) {
  if (!g || !out_score) return fail(GED_ERR_ARG, "bad argument to ged_score_noalloc");
  std::lock_guard<std::mutex> lk0(g_noalloc_mu);
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() { return score_noalloc(g, S, s_len, alpha, eps, out_score, info); });
}
