// Greedy GED-Walk maximisation on the GPU (Section 3.2, Algorithm "lazy
// greedy", with the priorities of Lemma "initialize").
//
// Per separation attempt at (S, ell):
//   1. miss chain m_i(v) = [v not in S] alpha * sum_{u->v} m_{i-1}(u), m_0 = 1_{V\S}
//      (the paper's phi^miss, decayed), all levels 0..ell kept; for directed
//      graphs the same chain on the reverse graph gives psi^miss (b_i).
//   2. upper bounds I(x) = sum_{1 <= a+c <= ell} m_a(x) b_c(x) on L_ell(S, x)
//      (Lemma "initialize"), tightened by exact values already computed at this
//      ell for a smaller S (L_ell is non-increasing in S, Section 3.2.1).
//   3. candidates in decreasing bound order, C at a time: their exact gains
//      L_ell(S, x) come from one SpMM whose column c runs the chain
//         d_0 = e_x, d_i(v) = 0 (v in S), m_i(x) (v = x), alpha*sum d_{i-1} (else)
//      -- the walks that avoid S and contain x, counted by end vertex -- and
//      L = sum_{i=1}^{ell} sum_v d_i(v).  Batches continue until every
//      unevaluated bound is below the runner-up's exact gain, so the exact
//      top two of L_ell over V \ S are known (the heaps of the paper's
//      algorithm find the same pair).
//   4. accept u iff L(u) > L(v) + B_ell - eps/k ((eps/k)-separation), else
//      ell <- 2 ell.  Ties order by larger value, then smaller id.
//
// Undirected graphs split the walks as split scoring does: a walk of length
// a + c that avoids S and contains x, cut after a arcs at v, has either a
// first part that contains x (d_a(v) of them, each continued by the m_c(v)
// S-avoiding walks leaving v) or one that does not (m_a(v) - d_a(v)) followed
// by a last part that contains x (d_c(v), by reversal), so
//   L_{a+c}(S, x) = sum_v d_a(v) m_c(v) + (m_a(v) - d_a(v)) d_c(v)
// and both chains are needed only up to a = ceil(ell/2).  The bound of step 2
// then takes t_j(x) >= m_j(x) for the levels j > a it no longer has.
#include <math.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "ged_internal.h"

namespace ged {

// Relative slack added to upper bounds before they are compared with exact
// gains: both sides are rounded sums, and exact equality (e.g. ell = 1, where
// the bound is tight) must not prune a candidate by one ulp.
constexpr double kBoundSlack = 1e-12;

// ---------------------------------------------------------------- kernels --

__global__ void k_mask_bit(uint32_t *mask, int v, int value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const uint32_t bit = 1u << (v & 31);
    if (value)
      mask[v >> 5] |= bit;
    else
      mask[v >> 5] &= ~bit;
  }
}

// A vertex u joined S: one more arc from S into each v in N(u) (undirected,
// so the row of u lists them; repeated arcs count each time), and u's bit in
// the S bitmap.
__global__ void k_sdeg_add(const int *__restrict__ rp, const int *__restrict__ ci, int u,
                           int *sdeg, uint32_t *smask) {
  if (blockIdx.x == 0 && threadIdx.x == 0) smask[u >> 5] |= 1u << (u & 31);
  for (int k = rp[u] + blockIdx.x * blockDim.x + threadIdx.x; k < rp[u + 1];
       k += gridDim.x * blockDim.x)
    atomicAdd(&sdeg[ci[k]], 1);
}

// Miss level 1 (unweighted, undirected): m_1(v) = alpha * (deg(v) - arcs from
// S into v) outside S, 0 on S -- the same integer times alpha as the dense
// step from the complement mask computes, at O(n).
// m1c (nullable) receives the count itself.
__global__ void k_miss1(const int *__restrict__ rp, const int *__restrict__ sdeg,
                        const uint32_t *__restrict__ smask, double alpha, int n, double *m1,
                        uint32_t *m1c) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const bool inS = (smask[v >> 5] >> (v & 31)) & 1u;
    const int cnt = inS ? 0 : rp[v + 1] - rp[v] - sdeg[v];
    m1[v] = alpha * (double)cnt;
    if (m1c) m1c[v] = (uint32_t)cnt;
  }
}

// Miss levels 2 .. top of S + {x} from those of S (undirected, 32-bit
// counts): the walks that avoid S + {x} are the walks that avoid S minus
// those that also contain x, whose counts x's gain chain has just stored
// (column col of the 32-bit gain levels dl32, level i at (i-1)*n*C, the top
// one by the combining step; at x itself they equal x's miss counts, so x's
// rows become 0).  M_i = fl(alpha^i)
// * count on both sides, the counts are exact integers (M_i / alpha^i rounds
// back to the count), so the result equals the recomputed chain bit for bit.
// mc_top receives the level-top counts for the next dense level.  Level 1
// is written as k_miss1 writes it (from the arcs-from-S counts).
__global__ void k_miss_sub(const int *__restrict__ rp, const int *__restrict__ sdeg,
                           const uint32_t *__restrict__ smask, double *__restrict__ M, int n,
                           const uint32_t *__restrict__ dl32, int C, int col, int top,
                           double alpha, uint32_t *__restrict__ mc_top) {
  const size_t nC = (size_t)n * C;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const bool inS = (smask[v >> 5] >> (v & 31)) & 1u;
    M[(size_t)n + v] = alpha * (double)(inS ? 0 : rp[v + 1] - rp[v] - sdeg[v]);
    double ai = alpha;
    for (int i = 2; i <= top; ++i) {
      ai *= alpha;
      const double m = M[(size_t)i * n + v];
      const double cnt = rint(m / ai) - (double)dl32[(size_t)(i - 1) * nC + (size_t)v * C + col];
      M[(size_t)i * n + v] = ai * cnt;
      if (i == top) mc_top[v] = (uint32_t)cnt;
    }
  }
}

// Speculative miss columns (gain batches on FP64 levels, undirected graphs
// without repeated arcs, unweighted): column W + j of a batch of width C
// carries the miss chain of S + {x_j} beside x_j's gain chain, so that after
// x_j wins the next pick's miss levels are already computed.  Their first
// level is the count of arcs into v from outside S + {x_j}: deg(v) - sdeg(v)
// - [v in N(x_j)] outside S + {x_j}, 0 on it -- the integer k_miss1 writes
// for that group, with alpha times it as FP64.  k_spec_miss1 writes deg -
// sdeg (0 on S and at x_j) for every vertex; k_spec_miss1_fix takes one off
// at x_j's neighbours outside S (each once: no repeated arcs).
__global__ void k_spec_miss1(const int *__restrict__ rp, const int *__restrict__ sdeg,
                             const uint32_t *__restrict__ smask, const int *__restrict__ cand,
                             int nc, int W, int C, int n, double alpha, uint32_t *__restrict__ c1,
                             double *__restrict__ d1) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const bool inS = (smask[v >> 5] >> (v & 31)) & 1u;
    const int base = inS ? 0 : rp[v + 1] - rp[v] - sdeg[v];
    for (int j = 0; j < nc; ++j) {
      const int cnt = v == cand[j] ? 0 : base;
      c1[(size_t)v * C + W + j] = (uint32_t)cnt;
      d1[(size_t)v * C + W + j] = alpha * (double)cnt;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_spec_miss1_fix(const int *__restrict__ rp,
                                                           const int *__restrict__ ci,
                                                           const uint32_t *__restrict__ smask,
                                                           const int *__restrict__ cand, int W,
                                                           int C, double alpha,
                                                           uint32_t *__restrict__ c1,
                                                           double *__restrict__ d1) {
  const int j = blockIdx.y;
  const int x = cand[j];
  for (int k = rp[x] + blockIdx.x * kBlock + (int)threadIdx.x; k < rp[x + 1];
       k += gridDim.x * kBlock) {
    const int v = ci[k];
    if (v != x && !((smask[v >> 5] >> (v & 31)) & 1u)) {
      const size_t o = (size_t)v * C + W + j;
      const uint32_t cnt = c1[o] - 1u;
      c1[o] = cnt;
      d1[o] = alpha * (double)cnt;
    }
  }
}

// The miss levels 1 .. la of S + {x_j}, taken from column col of a
// speculative batch's stored levels (level i at src + (i-1) * n * C).
__global__ void k_spec_take(const double *__restrict__ src, int la, int n, int C, int col,
                            double *__restrict__ M) {
  const size_t nC = (size_t)n * C;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    for (int i = 1; i <= la; ++i) M[(size_t)i * n + v] = src[(size_t)(i - 1) * nC + (size_t)v * C + col];
}

// I(x) = b_0 * sum_{a=1}^{ell} m_a + sum_{c=1}^{ell} b_c * sum_{a=0}^{ell-c} m_a with
// m_0 = b_0 = 1 for x outside S: every term of Lemma "initialize" once, no
// subtraction.  ub[x] = -1 marks members of S.
// Levels j <= ma come from the miss chain M, higher ones from the total-walk
// levels (an upper bound: walks that avoid S are walks), held in T for
// j <= tb and in Te (level tb + 1 first) above.  Bl (reverse chain, directed
// graphs) null means b = m.
__global__ __launch_bounds__(kBlock) void k_pbound(const double *__restrict__ M,
                                                   const double *__restrict__ T,
                                                   const double *__restrict__ Te, int tb, int ma,
                                                   const double *__restrict__ Bl, int n, int ell,
                                                   const uint32_t *__restrict__ smask,
                                                   const double *__restrict__ stale,
                                                   double *__restrict__ ub, double slack) {
  const int x = blockIdx.x * kBlock + threadIdx.x;
  if (x >= n) return;
  if ((smask[x >> 5] >> (x & 31)) & 1u) {
    ub[x] = -1.0;
    return;
  }
  auto mv = [&](int j) {
    if (j <= ma) return M[(size_t)j * n + x];
    return j <= tb ? T[(size_t)j * n + x] : Te[(size_t)(j - tb - 1) * n + x];
  };
  double pre = 1.0, tail = 0.0, acc = 0.0;
  for (int s = 0; s < ell; ++s) {
    if (s > 0) {
      const double ms = mv(s);
      pre += ms;
      tail += ms;
    }
    acc += (Bl ? Bl[(size_t)(ell - s) * n + x] : mv(ell - s)) * pre;
  }
  tail += mv(ell);
  acc += tail;
  const double st = stale[x];
  if (st >= 0.0 && st < acc) acc = st;
  ub[x] = acc * (1.0 + slack);
}

__device__ __forceinline__ bool kv_better(double ka, int ia, double kb, int ib) {
  return ka > kb || (ka == kb && ia < ib);
}

// K rounds of block-wide argmax over E register-resident (key, id) pairs per
// thread; writes the block's top K (key descending, id ascending).
template <int E>
__device__ void block_topk(double (&kv)[E], int (&iv)[E], int K, double *ok, int *oi) {
  __shared__ double sk[kBlock / 64];
  __shared__ int si[kBlock / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int r = 0; r < K; ++r) {
    double bk = -INFINITY;
    int bi = INT_MAX;
#pragma unroll
    for (int q = 0; q < E; ++q)
      if (kv_better(kv[q], iv[q], bk, bi)) {
        bk = kv[q];
        bi = iv[q];
      }
    for (int off = 32; off > 0; off >>= 1) {
      const double k2 = __shfl_xor(bk, off, 64);
      const int i2 = __shfl_xor(bi, off, 64);
      if (kv_better(k2, i2, bk, bi)) {
        bk = k2;
        bi = i2;
      }
    }
    if (lane == 0) {
      sk[wave] = bk;
      si[wave] = bi;
    }
    __syncthreads();
    double wk = sk[0];
    int wi = si[0];
    for (int w = 1; w < kBlock / 64; ++w)
      if (kv_better(sk[w], si[w], wk, wi)) {
        wk = sk[w];
        wi = si[w];
      }
    __syncthreads();
    if (wi != INT_MAX) {
#pragma unroll
      for (int q = 0; q < E; ++q)
        if (iv[q] == wi) {
          kv[q] = -INFINITY;
          iv[q] = INT_MAX;
        }
    }
    if (t == 0) {
      ok[r] = wk;
      oi[r] = wi;
    }
  }
}

constexpr int kTopE = 16;  // elements per thread in the selection kernels

// Eligible: bound >= 0 (not in S), not evaluated in this round, and (for the
// stochastic variant) in the current sample.
// Keys carry the caller's vertex id, so ties break by it whatever the
// internal vertex order is.
__global__ __launch_bounds__(kBlock) void k_topk_ub(const double *__restrict__ ub,
                                                    const int *__restrict__ done, int round,
                                                    const int *__restrict__ sampled, int pick,
                                                    const int *__restrict__ orig, int n, int K,
                                                    double *ok, int *oi) {
  double kv[kTopE];
  int iv[kTopE];
  const int base = blockIdx.x * kBlock * kTopE + threadIdx.x;
#pragma unroll
  for (int q = 0; q < kTopE; ++q) {
    const int x = base + q * kBlock;
    kv[q] = -INFINITY;
    iv[q] = INT_MAX;
    if (x < n) {
      const double u = ub[x];
      if (u >= 0.0 && done[x] != round && (!sampled || sampled[x] == pick)) {
        kv[q] = u;
        iv[q] = orig[x];
      }
    }
  }
  block_topk<kTopE>(kv, iv, K, ok + (size_t)blockIdx.x * K, oi + (size_t)blockIdx.x * K);
}

__global__ __launch_bounds__(kBlock) void k_topk_pairs(const double *__restrict__ ik,
                                                       const int *__restrict__ ii, int count,
                                                       int K, double *ok, int *oi) {
  double kv[kTopE];
  int iv[kTopE];
  const int base = blockIdx.x * kBlock * kTopE + threadIdx.x;
#pragma unroll
  for (int q = 0; q < kTopE; ++q) {
    const int x = base + q * kBlock;
    kv[q] = -INFINITY;
    iv[q] = INT_MAX;
    if (x < count) {
      kv[q] = ik[x];
      iv[q] = ii[x];
    }
  }
  block_topk<kTopE>(kv, iv, K, ok + (size_t)blockIdx.x * K, oi + (size_t)blockIdx.x * K);
}

// Candidates of a batch: cand_col[x_c] = c (value=1) or -1 (value=0).

// A batch's candidates, passed by value (no host-to-device copy).
struct CandList {
  int v[64];
};

// cand[c] = the batch's c-th candidate, cand_col[candidate] = c; a non-null
// wl_n (the batch's level-2 worklist) starts empty.  With injc, the
// candidates' unscaled miss counts injc[i*C + c] = m_i(x_c) / alpha^i rounded
// to the nearest integer, 2 <= i <= inj_top: exact when the count is below
// 2^32 and i*(deg_max + 3) < 2^19, since every miss level is a sum of
// nonnegative terms with relative error at most about i*(deg_max + 2)*2^-53,
// under 1/4 of a unit at 2^32.
__global__ void k_cand_put(int *cand_col, int *cand, CandList cl, int nc, unsigned *wl_n,
                           const double *__restrict__ M, int n, int C, double alpha, int inj_top,
                           double *injc) {
  const int c = threadIdx.x;
  if (c < nc) {
    const int x = cl.v[c];
    cand[c] = x;
    cand_col[x] = c;
    if (injc) {
      double ap = alpha;
      for (int i = 2; i <= inj_top; ++i) {
        ap *= alpha;
        injc[i * C + c] = rint(M[(size_t)i * n + x] / ap);
      }
    }
  }
  if (wl_n && c == 0) *wl_n = 0;
}

// After a batch: remember the exact gains (valid upper bounds for any larger
// S at this ell) and mark the candidates as evaluated in this round.
// The gains also go to host_gains (coherent host memory, read by the host
// after it waits for the stream).
__global__ void k_after_batch(const int *cand, const double *gains, int nc, double *stale,
                              double *ub, int *done, int round, double *host_gains,
                              int *cand_col) {
  const int c = threadIdx.x;
  if (c < nc) {
    const int x = cand[c];
    cand_col[x] = -1;  // no longer a candidate column
    host_gains[c] = gains[c];
    stale[x] = gains[c];
    ub[x] = gains[c];
    done[x] = round;
  }
}

// ------------------------------------------------------------- host side --

// Mr[v] = sum_{c=1..r} M[c][v]
__global__ void k_sum_range(const double *__restrict__ M, int n, int r, double *__restrict__ Mr) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 1; c <= r; ++c) s += M[(size_t)c * n + v];
    Mr[v] = s;
  }
}

// Level 1 of the gain chains of a candidate batch (undirected graph, no arc
// listed twice, unweighted): d_1(v, c) = alpha for each v in N(x_c) outside S
// and v != x_c (one walk x_c -> v), m_1(x_c) at the candidate, 0 elsewhere --
// what a dense step from the one-hot columns would write, at O(deg(x_c)).
// The buffer is zero between batches; clear = 1 stores the zeros back.
__global__ __launch_bounds__(kBlock) void k_gain_level1(const int *__restrict__ rp,
                                                        const int *__restrict__ ci,
                                                        const uint32_t *__restrict__ smask,
                                                        const int *cand, int C, double alpha,
                                                        const double *__restrict__ m1, double *d1,
                                                        int clear) {
  const int c = blockIdx.y;
  const int x = cand[c];
  const int k1 = rp[x + 1];
  for (int k = rp[x] + blockIdx.x * kBlock + (int)threadIdx.x; k < k1; k += gridDim.x * kBlock) {
    const int v = ci[k];
    if (v != x && !((smask[v >> 5] >> (v & 31)) & 1u)) d1[(size_t)v * C + c] = clear ? 0.0 : alpha;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) d1[(size_t)x * C + c] = clear ? 0.0 : m1[x];
}

// The same level as unscaled 32-bit counts: 1 on N(x_c) outside S, and at the
// candidate the number of its arcs from outside S, deg(x_c) - sdeg(x_c).
// With wl (level 2 pushed), every vertex written here, the candidate
// included, appends its chunks: they are the sources of level 2.
__global__ __launch_bounds__(kBlock) void k_gain_level1_32(const int *__restrict__ rp,
                                                           const int *__restrict__ ci,
                                                           const uint32_t *__restrict__ smask,
                                                           const int *cand, int C,
                                                           const int *__restrict__ sdeg,
                                                           uint32_t *d1, int clear, uint64_t *wl,
                                                           unsigned *wl_n, unsigned wl_cap) {
  const int c = blockIdx.y;
  const int x = cand[c];
  const int k0 = rp[x], k1 = rp[x + 1];
  for (int kb = k0 + blockIdx.x * kBlock; kb < k1; kb += gridDim.x * kBlock) {  // uniform trips
    const int k = kb + (int)threadIdx.x;
    unsigned nch = 0;
    int v = 0;
    if (k < k1) {
      v = ci[k];
      if (v != x && !((smask[v >> 5] >> (v & 31)) & 1u)) {
        d1[(size_t)v * C + c] = clear ? 0u : 1u;
        if (wl) nch = wl_chunks(rp, v);
      }
    }
    if (wl) wl_append(wl, wl_n, wl_cap, v, c, nch);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d1[(size_t)x * C + c] = clear ? 0u : (uint32_t)(k1 - k0 - sdeg[x]);
    if (wl && k1 > k0) {
      const unsigned nch = wl_chunks(rp, x);
      const unsigned base = atomicAdd(wl_n, nch);
      for (unsigned q = 0; q < nch; ++q)
        if (base + q < wl_cap) wl[base + q] = wl_entry(x, c, q);
    }
  }
}

// Level 2 of a batch's gain chains as 32-bit counts by a push: each listed
// source u (a level-1 vertex of column c) adds its level-1 count to its
// neighbours outside S other than the candidate x_c, whose own entry is its
// miss count (injc2[c]); the level is zero before.  The same integers the
// dense step gathers.  A wave issues all loads of a chunk before their uses;
// the adds return nothing.
__global__ __launch_bounds__(kBlock) void k_gain_push2(const int *__restrict__ rp,
                                                       const int *__restrict__ ci,
                                                       const uint32_t *__restrict__ smask,
                                                       const int *cand, int nc, int C,
                                                       const uint32_t *d1, uint32_t *d2,
                                                       const uint64_t *wl, const unsigned *wl_n,
                                                       unsigned wl_cap,
                                                       const double *__restrict__ injc2) {
  if (blockIdx.x == 0 && (int)threadIdx.x < nc)
    d2[(size_t)cand[threadIdx.x] * C + threadIdx.x] = (uint32_t)injc2[threadIdx.x];
  constexpr int U = kWlChunk / 64;
  const unsigned count = min(*wl_n, wl_cap);
  const int lane = threadIdx.x & 63;
  const unsigned nwaves = (gridDim.x * kBlock) >> 6;
  for (unsigned i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < count; i += nwaves) {
    const uint64_t e = wl[i];
    const int u = (int)(e >> 32);
    const int c = (int)((e >> 24) & 0xffu);
    const int q = (int)(e & 0xffffffu);
    const int x = cand[c];
    const int j0 = rp[u] + q * kWlChunk + lane, j1 = min(rp[u] + (q + 1) * kWlChunk, rp[u + 1]);
    int w[U];
#pragma unroll
    for (int k = 0; k < U; ++k) w[k] = j0 + 64 * k < j1 ? ci[j0 + 64 * k] : -1;
    bool ok[U];
#pragma unroll
    for (int k = 0; k < U; ++k)
      ok[k] = w[k] >= 0 && w[k] != x && !((smask[w[k] >> 5] >> (w[k] & 31)) & 1u);
    const uint32_t val = d1[(size_t)u * C + c];
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (ok[k]) atomicAdd(&d2[(size_t)w[k] * C + c], val);
  }
}

// Zero what k_gain_push2 wrote for a batch (cand, nc, its worklist): the
// candidates' entries and every neighbour of every listed source.
__global__ __launch_bounds__(kBlock) void k_gain_clear2(const int *__restrict__ rp,
                                                        const int *__restrict__ ci,
                                                        const int *cand, int nc, int C,
                                                        uint32_t *d2, const uint64_t *wl,
                                                        const unsigned *wl_n, unsigned wl_cap) {
  if (blockIdx.x == 0 && (int)threadIdx.x < nc)
    d2[(size_t)cand[threadIdx.x] * C + threadIdx.x] = 0u;
  constexpr int U = kWlChunk / 64;
  const unsigned count = min(*wl_n, wl_cap);
  const int lane = threadIdx.x & 63;
  const unsigned nwaves = (gridDim.x * kBlock) >> 6;
  for (unsigned i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < count; i += nwaves) {
    const uint64_t e = wl[i];
    const int u = (int)(e >> 32);
    const int c = (int)((e >> 24) & 0xffu);
    const int q = (int)(e & 0xffffffu);
    const int j0 = rp[u] + q * kWlChunk + lane, j1 = min(rp[u] + (q + 1) * kWlChunk, rp[u + 1]);
    int w[U];
#pragma unroll
    for (int k = 0; k < U; ++k) w[k] = j0 + 64 * k < j1 ? ci[j0 + 64 * k] : -1;
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (w[k] >= 0) d2[(size_t)w[k] * C + c] = 0u;
  }
}

struct GreedyCtx {
  ged_graph *g;
  hipStream_t st;
  int n;
  int C;      // widest candidate batch of this run (buffers are sized for it)
  int fixed;  // every batch this wide, or 0: batches of a round widen 2, 4, 8, 16
  int Lcap = 0;
  bool split = false;  // undirected: chains to ceil(ell/2) (walk split)
  DBuf smask, m_levels, b_levels, ub, stale, done, cand_col, sampled;
  DBuf sdeg;            // split, unweighted: int32 [n] arcs from S into each vertex
  DBuf mc32;            // 2 x uint32 [n]: miss counts of the last two levels (32-bit chain)
  DBuf dlv, Mr;        // split: stored gain levels [(a-1)*n*C], sum of miss levels [n]
  void *d1_zeroed = nullptr;  // dlv allocation whose level 1 is known to be all zero
  int d1_bytes = 0;           // ... in this element size (8 = FP64 levels, 4 = 32-bit)
  DBuf injc;                  // [(a)*C] candidate injections of the 32-bit gain levels
  DBuf dc32;                  // 2 x uint32 [n*C]: gain levels 1, 2 as counts (FP64 chains)
  void *dc1_zeroed = nullptr; // dc32 allocation whose level 1 is known to be all zero
  int g32_ell = -1;           // walk length g32_ok was decided for
  bool g32_ok = false;        // gain levels as 32-bit counts at g32_ell
  // gain level 2 by a push: worklist of its sources, and the state of the
  // level-2 region of dlv (d2_buf): all zero, or holding the last batch's
  // pushed level (kept until the next batch: a pick reads it) with that
  // batch's size last_nc2
  DBuf wl2, wl2_n;
  unsigned wl2_cap = 0;
  void *d2_buf = nullptr;
  bool d2_zero = false, d2_pending = false;
  int last_nc2 = 0;
  // the last gain batch's candidates when it left gain levels 2 ..
  // last_levels as 32-bit counts at last_src (level i at (i-1)*n*C) for walk
  // length last_ell (-1: none), and the column of the vertex just added to S
  // if it is one of them (-1: recompute the chain)
  std::vector<int> last_cand;
  int last_ell = -1;
  int last_levels = 0;
  const uint32_t *last_src = nullptr;
  int last_C = 0;  // width of the batch that left them (their layout [n][last_C])
  int sub_col = -1;
  // the last batch, if it carried speculative miss columns and was the last
  // batch of its round: its candidates, walk length, layout and stored levels
  // (level i at spec_src + (i-1)*n*spec_C, miss column of candidate j at
  // spec_W + j); spec_col: the column to take after a pick (-1: none)
  std::vector<int> spec_cand;
  int spec_ell = -1, spec_C = 0, spec_W = 0, spec_la = 0, spec_col = -1;
  const double *spec_src = nullptr;
  bool spec_dirty = false;  // miss columns left dense data in the level-1 regions
  DBuf X, Y, cand_dev, gains, topk_k[2], topk_i[2];
  HBuf h_small;
  int layout_C = 0;  // batch width the zero-state flags above were established for
  StepWs ws1, ws1r, wsC;
  int64_t evals = 0;
  int rounds = 0;
};

// The working buffers stay allocated on the graph between calls (a serving
// process runs many greedy requests; freeing device memory can stall the
// device for every stream).
static std::mutex g_greedy_mu;
static std::map<const ged_graph *, std::unique_ptr<GreedyCtx>> g_greedy;

static GreedyCtx &greedy_ctx(const ged_graph *g) {
  std::lock_guard<std::mutex> lk(g_greedy_mu);
  auto &p = g_greedy[g];
  if (!p) p = std::make_unique<GreedyCtx>();
  return *p;
}

void greedy_forget(const ged_graph *g) {
  std::lock_guard<std::mutex> lk(g_greedy_mu);
  g_greedy.erase(g);
}

// The library's choice (greedy_width 0) starts each separation round with a
// batch of 2 and widens the round's later batches to 4, 8, 16.  Measured with
// fixed widths on R-MAT scale 22, k = 100: 214 gain evaluations in about 105
// rounds at width 2 (the two best bounds are nearly always the exact top
// two), 0.97 s, against 1.10 s at 4, 1.35 s at 8 and 1.79 s at 16; on BA
// n = 1e6, k = 10: 4.0 ms at 2 against 6.2 ms at 8.  On graphs of at most
// 2^20 arcs a step is launch-bound whatever its width, so rounds start at 8
// there (Erdos-Renyi n = 1000, k = 5: 2.4 ms at 8 against 4.2 ms at 2).
constexpr int kWidthFirst = 2, kWidthSmall = 8, kWidthMax = 16;
constexpr int64_t kSmallArcs = int64_t(1) << 20;

int greedy_width_for(const ged_graph *g) {
  if (g->greedy_width > 0) return g->greedy_width;
  return g->nnz <= kSmallArcs ? kWidthSmall : kWidthFirst;
}

static size_t step_ws_bytes(const StepWs &w) {
  return w.blk.bytes + w.seg.bytes + w.lng.bytes + w.red2.bytes;
}

size_t greedy_bytes_held(const ged_graph *g) {
  size_t b = g->prep.t_ext.bytes + g->prep.t_tail[0].bytes + g->prep.t_tail[1].bytes;
  std::lock_guard<std::mutex> lk(g_greedy_mu);
  auto it = g_greedy.find(g);
  if (it == g_greedy.end() || !it->second) return b;
  const GreedyCtx &c = *it->second;
  for (const DBuf *d : {&c.smask, &c.m_levels, &c.b_levels, &c.ub, &c.stale, &c.done,
                        &c.cand_col, &c.sampled, &c.sdeg, &c.mc32, &c.dlv, &c.Mr, &c.injc,
                        &c.dc32, &c.wl2, &c.wl2_n, &c.X, &c.Y, &c.cand_dev, &c.gains,
                        &c.topk_k[0], &c.topk_k[1], &c.topk_i[0], &c.topk_i[1]})
    b += d->bytes;
  return b + step_ws_bytes(c.ws1) + step_ws_bytes(c.ws1r) + step_ws_bytes(c.wsC);
}

// Upper bound of the device bytes a greedy run of k picks whose walk length
// stays at most ell_max can leave allocated on g (its workspace, grown to the
// largest walk length and batch width, and the total-walk levels beyond ell*
// with their transient copy), counted from nothing; the single-group score
// of the final group reuses the handle's score workspace, which the caller
// accounts separately.  Mirrors every allocation of this file.  Builds the
// partitions of the batch widths if they are missing (host-side descriptors).
size_t greedy_footprint(ged_graph *g, int ell_max, int k) {
  const size_t n = (size_t)g->n, nnz = (size_t)g->nnz;
  const size_t Cm = (size_t)std::max(kWidthMax, (int)g->greedy_width);
  const bool split = split_ok(g), directed = g->flags == GED_DIRECTED;
  size_t b = 4 * (n / 32 + 2);           // smask
  b += 2 * 8 * n + 4 * 4 * n;            // ub, stale; done, cand_col, sampled, sdeg
  int cap = 16;
  while (cap < ell_max) cap *= 2;
  b += 8 * n * (size_t)(cap + 1) * (directed ? 2 : 1);  // miss levels (both chains)
  b += 2 * 4 * n;                        // mc32
  const size_t nb0 = (n + kBlock * kTopE - 1) / (kBlock * kTopE), K = Cm + 1;
  b += 2 * nb0 * K * (8 + 4);            // top-K pairs
  b += 64 * 12 + 4;                      // cand_dev, gains, wl2_n
  if (split) {
    const size_t la = (size_t)(ell_max + 1) / 2;
    b += 8 * n;                          // Mr
    b += 8 * n * Cm * la;                // dlv: la levels of FP64 at the widest batch
    b += 2 * 4 * n * Cm;                 // dc32
    b += 8 * (la + 2) * Cm;              // injc
    b += 8 * 2 * (nnz / 8 + nnz / kWlChunk + Cm + 2);  // wl2: twice its largest need
  } else {
    b += 2 * 8 * n * Cm;                 // X, Y
  }
  // step partials: C = 1 in each direction, and the widest need of each
  // partial buffer over the batch partitions (StepWs grows field by field);
  // the partitions themselves (descriptors, and the copied col_idx of
  // source-bucketed ones)
  size_t parts = 0;
  auto fields = [&parts](const Partition &p, size_t *f) {
    parts += p.device_bytes();
    f[0] = std::max(f[0], 8 * (size_t)std::max(1, p.n_blocks) * p.C);
    f[1] = std::max(f[1], 8 * (size_t)std::max(1, p.n_segs) * p.C);
    f[2] = std::max(f[2], 8 * (size_t)std::max(1, p.n_long) * p.C);
    f[3] = std::max(f[3], 8 * (size_t)kReduceBlocks * p.C);
  };
  size_t f1[4] = {0, 0, 0, 0}, fr[4] = {0, 0, 0, 0}, fc[4] = {0, 0, 0, 0};
  fields(partition(g, 1), f1);
  if (directed) fields(partition(g, 1, true), fr);
  for (int C = 2; C <= (int)Cm; C *= 2) {
    fields(partition(g, C), fc);
    if (split && !g->weighted) fields(partition_narrow(g, C), fc);
  }
  for (int i = 0; i < 4; ++i) b += f1[i] + fr[i] + fc[i];
  b += parts;
  // total-walk levels beyond ell* (the bounds read them up to ell on
  // undirected graphs): the buffer doubles, and the old one is copied
  // before it is freed; the two chain vectors of the level sums
  const int pe = g->prep.valid ? g->prep.ell : 0;
  if (split && ell_max > pe) b += 3 * 8 * n * (size_t)(ell_max - pe);
  b += 2 * 8 * n;
  return b + 16 * (size_t)k + 4096;
}

static int batch_width(const GreedyCtx &c, int batch_in_round) {
  if (c.fixed) return c.fixed;
  int w = greedy_width_for(c.g);
  for (int b = 0; b < batch_in_round && w < kWidthMax; ++b) w *= 2;
  return w;
}

static void ensure_levels_cap(GreedyCtx &c, int ell) {
  if (ell <= c.Lcap) return;
  int cap = std::max(16, c.Lcap);
  while (cap < ell) cap *= 2;
  c.m_levels.ensure(sizeof(double) * (size_t)c.n * (cap + 1));
  if (c.g->flags == GED_DIRECTED) c.b_levels.ensure(sizeof(double) * (size_t)c.n * (cap + 1));
  c.Lcap = cap;
}

// Miss chain(s) for the current S at walk length ell.
// Last miss level (<= L) kept as exact 32-bit counts: the counts are at most
// omega_i, so on undirected unweighted graphs with 32-bit level-2 counts (no
// repeated arcs, or max degree below 2^16) levels 1, 2 always fit and level i
// fits when max omega_j < 2^32 for j <= i.  1 = no 32-bit chain.
static int miss32_top(GreedyCtx &c, int L) {
  ged_graph *g = c.g;
  if (L < 2 || !c.split || g->weighted || !(g->simple || g->max_deg < 65536)) return 1;
  return omega_fit_level(g, L, c.st);
}

static void miss_chains(GreedyCtx &c, int ell) {
  ged_graph *g = c.g;
  const int n = c.n;
  // levels 2 .. top32 gather the previous level's counts (half the bytes of
  // FP64) and store the count and alpha^i times it; level top32 + 1 gathers
  // counts and stores FP64; later levels continue the FP64 chain
  const int top32 = miss32_top(c, ell);
  const bool m32 = top32 >= 2;
  // right after a pick from the last gain batch: levels 2 .. sub_top by
  // subtracting the new member's stored gain counts (levels whose miss
  // values are counts too); the rest gather from the level-sub_top counts
  const int sub = c.sub_col;
  c.sub_col = -1;
  const int sub_top = std::min({ell, c.last_levels, top32});
  const bool by_sub = sub >= 0 && m32 && sub_top >= 2 && g->flags != GED_DIRECTED && c.split &&
                      !g->weighted;
  if (m32) c.mc32.ensure(2 * sizeof(uint32_t) * (size_t)n);
  uint32_t *mc = c.mc32.as<uint32_t>();
  for (int dir = 0; dir < (g->flags == GED_DIRECTED ? 2 : 1); ++dir) {
    const bool rev = dir == 1;
    Partition &p = partition(g, 1, rev);
    StepWs &ws = rev ? c.ws1r : c.ws1;
    ws.fit(p);
    double *L = (rev ? c.b_levels : c.m_levels).as<double>();
    int i0 = 1;
    if (c.split && !g->weighted) {  // level 1 from the S-arc counts
      if (by_sub) {  // ... with levels 2 .. sub_top by subtraction, one pass
        hipLaunchKernelGGL(k_miss_sub, dim3(std::min(8192, (n + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, c.st, g->rp.as<const int>(), c.sdeg.as<const int>(),
                           c.smask.as<const uint32_t>(), L, n, c.last_src, c.last_C, sub, sub_top,
                           g->prep.alpha, mc + (size_t)(sub_top & 1) * n);
        i0 = sub_top + 1;
      } else {
        hipLaunchKernelGGL(k_miss1, dim3(std::min(8192, (n + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, c.st, g->rp.as<const int>(), c.sdeg.as<const int>(),
                           c.smask.as<const uint32_t>(), g->prep.alpha, n, L + (size_t)n,
                           m32 ? mc + (size_t)n : nullptr);
        i0 = 2;
      }
      GED_HIP(hipGetLastError());
    }
    double ai = g->prep.alpha;  // alpha^i
    for (int i = 2; i < i0; ++i) ai *= g->prep.alpha;
    for (int i = i0; i <= ell; ++i) {
      StepArgs a = base_args(g, rev);
      ws.into(a);
      a.C = 1;
      a.alpha = g->prep.alpha;
      a.smask = c.smask.as<const uint32_t>();
      a.X = L + (size_t)(i - 1) * n;
      a.Y = L + (size_t)i * n;
      ai *= g->prep.alpha;
      if (m32 && !rev && i <= top32 + 1) {
        a.alpha = ai;
        a.Xc32 = mc + (size_t)((i - 1) & 1) * n;
        if (i <= top32) {
          a.Y32 = mc + (size_t)(i & 1) * n;
          run_step(g, p, a, IN_CNT32, OUT_ZERO32, c.st);
        } else {
          run_step(g, p, a, IN_CNT32, OUT_ZERO, c.st);
        }
      } else {
        run_step(g, p, a, i == 1 ? IN_NOTMASK : IN_VEC, OUT_ZERO, c.st);
      }
    }
  }
}

static void compute_bounds(GreedyCtx &c, int ell) {
  const double *M = c.m_levels.as<const double>();
  const double *B = c.g->flags == GED_DIRECTED ? c.b_levels.as<const double>() : nullptr;
  const int ma = c.split ? (ell + 1) / 2 : ell;
  if (c.split) t_levels_to(c.g, ell);
  const PrepCache &pc = c.g->prep;
  const double *T = pc.t_levels.as<const double>();
  const double *Te = pc.t_ext_count > 0 ? pc.t_ext.as<const double>() : T;
  hipLaunchKernelGGL(k_pbound, dim3((c.n + kBlock - 1) / kBlock), dim3(kBlock), 0, c.st, M, T, Te,
                     pc.ell, ma, B, c.n, ell, c.smask.as<const uint32_t>(),
                     c.stale.as<const double>(), c.ub.as<double>(), kBoundSlack);
  GED_HIP(hipGetLastError());
}

// Miss levels 1..a of the current S and, for the split gain, their sum to r.
// After a pick whose candidate carried a speculative miss column, the levels
// are copied from it instead of recomputed.
static void chains_for(GreedyCtx &c, int ell) {
  if (!c.split) {
    miss_chains(c, ell);
    return;
  }
  const int a = (ell + 1) / 2, r = ell - a;
  if (c.spec_col >= 0 && c.spec_ell == ell && c.spec_la == a) {
    hipLaunchKernelGGL(k_spec_take, dim3(std::min(8192, (c.n + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, c.st, c.spec_src, a, c.n, c.spec_C,
                       c.spec_W + c.spec_col, c.m_levels.as<double>());
    GED_HIP(hipGetLastError());
    c.sub_col = -1;
  } else {
    miss_chains(c, a);
  }
  c.spec_col = -1;
  c.Mr.ensure(sizeof(double) * c.n);
  hipLaunchKernelGGL(k_sum_range, dim3(std::min(8192, (c.n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, c.st, c.m_levels.as<const double>(), c.n, r, c.Mr.as<double>());
  GED_HIP(hipGetLastError());
}

// Top-K eligible (bound, caller id) pairs, best first, into host arrays.
static int select_topk(GreedyCtx &c, int K, int round, const int *sampled, int pick, double *hk,
                       int *hi) {
  const int chunk = kBlock * kTopE;
  // the launch that leaves one block writes its K pairs straight into the
  // coherent host buffer
  double *sk = c.h_small.as<double>();
  int *si = reinterpret_cast<int *>(sk + 64);
  int nb = (c.n + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_topk_ub, dim3(nb), dim3(kBlock), 0, c.st, c.ub.as<const double>(),
                     c.done.as<const int>(), round, sampled, pick, c.g->d_old_id.as<const int>(),
                     c.n, K, nb == 1 ? sk : c.topk_k[0].as<double>(),
                     nb == 1 ? si : c.topk_i[0].as<int>());
  GED_HIP(hipGetLastError());
  int cur = 0, count = nb * K;
  while (nb > 1) {
    nb = (count + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_topk_pairs, dim3(nb), dim3(kBlock), 0, c.st,
                       c.topk_k[cur].as<const double>(), c.topk_i[cur].as<const int>(), count, K,
                       nb == 1 ? sk : c.topk_k[cur ^ 1].as<double>(),
                       nb == 1 ? si : c.topk_i[cur ^ 1].as<int>());
    GED_HIP(hipGetLastError());
    cur ^= 1;
    count = nb * K;
  }
  GED_HIP(hipStreamSynchronize(c.st));
  int m = 0;
  for (int q = 0; q < K; ++q) {
    if (si[q] == INT_MAX || !(sk[q] >= 0.0)) break;
    hk[m] = sk[q];
    hi[m] = si[q];
    ++m;
  }
  return m;
}

// Gain levels as unscaled 32-bit counts at walk length ell (undirected,
// unweighted, no repeated arcs): d_i(v) / alpha^i counts walks that avoid S
// and contain x, at most omega_i(v), so levels 1 .. ceil(ell/2)-1 fit when
// max omega_i < 2^32; the candidates' injected miss counts are recovered
// exactly by rounding when i*(deg_max + 3) < 2^19 (k_cand_put).
static bool gains32(GreedyCtx &c, int ell) {
  if (c.g32_ell == ell) return c.g32_ok;
  ged_graph *g = c.g;
  const int top = (ell + 1) / 2 - 1;
  bool ok = c.split && g->simple && !g->weighted && top >= 1 &&
            (int64_t)top * ((int64_t)g->max_deg + 3) + 2 < (int64_t(1) << 19);
  if (ok) ok = omega_fit_level(g, top, c.st) >= top;
  c.g32_ell = ell;
  c.g32_ok = ok;
  return ok;
}

// Exact L_ell(S, x) for up to Cb candidates (one SpMM column each; Cb a
// power of two, at most c.C).  want_spec: the first batch of a round, which
// on FP64 gain levels also carries a speculative miss column per candidate
// (the step then runs 2 Cb columns).
static void eval_batch(GreedyCtx &c, const int *cand, int nc, int Cb, int ell, int round,
                       double *out, bool want_spec) {
  ged_graph *g = c.g;
  const int n = c.n;
  c.last_ell = -1;  // set below when the batch stores its levels as counts
  c.spec_ell = -1;  // set below when this batch carries miss columns
  const int la0 = (ell + 1) / 2;
  const bool spec = want_spec && c.split && la0 >= 3 && g->simple && !g->weighted &&
                    2 * Cb <= c.C && !gains32(c, ell);
  const int C = spec ? 2 * Cb : Cb;
  if (c.spec_dirty) {  // dense miss columns sit in the level-1 regions
    c.d1_zeroed = nullptr;
    c.dc1_zeroed = nullptr;
    c.spec_dirty = false;
  }
  if (C != c.layout_C) {
    // the stored levels' layout [n][C] changes with the width: regions that
    // must be zero (the pushed first and second gain levels) are zeroed
    // again in the new layout before their next push
    c.d1_zeroed = nullptr;
    c.dc1_zeroed = nullptr;
    c.d2_zero = c.d2_pending = false;
    c.layout_C = C;
  }
  Partition &p = partition(g, C);
  c.wsC.fit(p);
  if (nc > 64) throw HipError{GED_ERR_ARG, "candidate batch larger than 64"};
  // Level 2 of 32-bit gain chains by a push from the level-1 vertices when
  // the arcs it adds along are few: at most sum_x (omega_2(x) + deg(x)) <=
  // nnz/8 (the dense step gathers every arc; the push's adds are scattered
  // and contend at hubs: on BA-1M a push at that size takes a third of the
  // gather).  Its sources are N(x) outside S and x, so the
  // worklist needs at most sum (deg(x) + 1) + that sum / 512 + 1 entries.
  bool push2 = false;
  size_t wl2_need = 0;
  if (c.split && (ell + 1) / 2 >= 3 && g->simple && !g->weighted && gains32(c, ell)) {
    const std::vector<double> &om2 = omega2_host(g, c.st);
    double vol = 0.0;
    size_t src = 0;
    for (int q = 0; q < nc; ++q) {
      const int d = g->h_rp[cand[q] + 1] - g->h_rp[cand[q]];
      vol += om2[(size_t)cand[q]] + d;
      src += (size_t)d + 1;
    }
    push2 = vol <= (double)(g->nnz / 8);
    wl2_need = src + (size_t)(vol / kWlChunk) + 1;
  }
  if (c.d2_buf != c.dlv.p) c.d2_zero = c.d2_pending = false;
  if (c.d2_pending && push2) {  // zero what the last batch pushed (its candidates are in cand_dev)
    hipLaunchKernelGGL(k_gain_clear2, dim3(std::min(4096, std::max(64, (int)(c.wl2_cap / 4)))),
                       dim3(kBlock), 0, c.st, g->rp.as<const int>(), g->ci.as<const int>(),
                       c.cand_dev.as<const int>(), c.last_nc2, C, c.dlv.as<uint32_t>() + (size_t)n * C,
                       c.wl2.as<const uint64_t>(), c.wl2_n.as<const unsigned>(), c.wl2_cap);
    GED_HIP(hipGetLastError());
    c.d2_zero = true;
  }
  c.d2_pending = false;
  if (push2) {
    if (wl2_need > c.wl2_cap || !c.wl2.p) {
      const size_t cap = std::min<size_t>(std::max<size_t>(wl2_need, 2 * (size_t)c.wl2_cap),
                                          0xffffffffu);
      c.wl2.ensure(sizeof(uint64_t) * cap);
      c.wl2_cap = (unsigned)cap;
    }
    c.wl2_n.ensure(sizeof(unsigned));
  }
  const double *M = c.m_levels.as<const double>();
  // the candidates' miss counts the 32-bit gain levels inject (levels 2 ..
  // a-1, or 2 on FP64 chains that keep levels 1-2 as counts)
  int inj_top = 0;
  if (c.split) {
    const int la = (ell + 1) / 2;
    const bool push1 = la > 1 && g->simple && !g->weighted;
    if (la > 2 && gains32(c, ell))
      inj_top = la - 1;
    else if (push1 && la >= 3)
      inj_top = 2;
    if (inj_top > 0) c.injc.ensure(sizeof(double) * (size_t)(la + 1) * C);
  }
  CandList cl;
  for (int q = 0; q < nc; ++q) cl.v[q] = cand[q];
  hipLaunchKernelGGL(k_cand_put, dim3(1), dim3(64), 0, c.st, c.cand_col.as<int>(),
                     c.cand_dev.as<int>(), cl, nc, push2 ? c.wl2_n.as<unsigned>() : nullptr, M,
                     n, C, g->prep.alpha, inj_top, inj_top > 0 ? c.injc.as<double>() : nullptr);
  StepArgs a = base_args(g);
  c.wsC.into(a);
  a.C = C;
  a.alpha = g->prep.alpha;
  a.smask = c.smask.as<const uint32_t>();
  a.cand_col = c.cand_col.as<const int>();
  Partition *pr = &p;  // partition of the last step (its partials are reduced)
  if (c.split) {
    // gain levels 1..a-1 stored, level a combined (walk split)
    const int la = (ell + 1) / 2, r = ell - la;
    const size_t nC = (size_t)n * C;
    const bool g32 = la > 1 && gains32(c, ell);
    const int eb = g32 ? 4 : 8;  // bytes per stored value
    // the combining level's counts too, when they fit 32 bits: after a pick
    // from this batch the whole miss chain follows by subtraction
    const bool top_a = g32 && la > 2 && omega_fit_level(g, la, c.st) >= la;
    // miss columns keep their level la too
    if (la > 1) c.dlv.ensure((size_t)eb * nC * (size_t)(la - 1 + (top_a || spec ? 1 : 0)));
    double *dl = c.dlv.as<double>();
    uint32_t *dl32 = c.dlv.as<uint32_t>();
    if (c.dlv.p != c.d2_buf) {
      c.d2_buf = c.dlv.p;
      c.d2_zero = false;
    }
    if (push2 && !c.d2_zero) launch_fill_i32(c.dlv.as<int>() + nC, 0, nC, c.st);
    const double *any = c.Mr.as<const double>();
    // level 1 by a push from the candidates when each neighbour is one walk
    const bool push1 = la > 1 && g->simple && !g->weighted;
    int gx = 1;
    if (push1) {
      if (c.d1_zeroed != c.dlv.p || c.d1_bytes != eb)
        launch_fill_i32(c.dlv.as<int>(), 0, nC * eb / sizeof(int), c.st);
      c.d1_zeroed = nullptr;  // dirty until the clear below has been enqueued
      int dmax = 0;
      for (int q = 0; q < nc; ++q) dmax = std::max(dmax, g->h_rp[cand[q] + 1] - g->h_rp[cand[q]]);
      gx = std::max(1, std::min(64, (dmax + kBlock - 1) / kBlock));
      if (g32)
        hipLaunchKernelGGL(k_gain_level1_32, dim3(gx, nc), dim3(kBlock), 0, c.st, a.rp, a.ci,
                           a.smask, c.cand_dev.as<const int>(), C, c.sdeg.as<const int>(), dl32,
                           0, push2 ? c.wl2.as<uint64_t>() : nullptr,
                           push2 ? c.wl2_n.as<unsigned>() : nullptr, c.wl2_cap);
      else
        hipLaunchKernelGGL(k_gain_level1, dim3(gx, nc), dim3(kBlock), 0, c.st, a.rp, a.ci,
                           a.smask, c.cand_dev.as<const int>(), C, a.alpha, M + (size_t)n, dl, 0);
      GED_HIP(hipGetLastError());
    }
    a.accum = 0;
    if (g32) {
      Partition &pn = partition_narrow(g, C);
      c.wsC.fit(pn);
      c.wsC.into(a);
      pr = &pn;
      // the candidates' injected miss counts were written by k_cand_put
      if (push2) {  // injc (level 2) is ready
        hipLaunchKernelGGL(k_gain_push2, dim3(std::min(4096, std::max(64, (int)(wl2_need / 4)))),
                           dim3(kBlock), 0, c.st, a.rp, a.ci, a.smask, c.cand_dev.as<const int>(),
                           nc, C, dl32, dl32 + nC, c.wl2.as<const uint64_t>(),
                           c.wl2_n.as<const unsigned>(), c.wl2_cap,
                           c.injc.as<const double>() + (size_t)2 * C);
        GED_HIP(hipGetLastError());
        c.d2_pending = true;
        c.last_nc2 = nc;
      }
      c.d2_zero = false;  // pushed (cleared by the next batch) or gathered
      if (la > 2) {
        c.last_cand.assign(cand, cand + nc);
        c.last_ell = ell;
        c.last_src = dl32;
        c.last_C = C;
        c.last_levels = top_a ? la : la - 1;
      }
      double alpha_a = g->prep.alpha;
      for (int i = 1; i < la; ++i) alpha_a *= g->prep.alpha;
      for (int i = 2; i <= la; ++i) {
        a.Xc32 = dl32 + (size_t)(i - 2) * nC;
        if (i == 2 && push2) continue;
        if (i < la) {
          a.alpha = 1.0;
          a.injc = c.injc.as<const double>() + (size_t)i * C;
          a.Y32 = dl32 + (size_t)(i - 1) * nC;
          run_step(g, pn, a, IN_CNT32, OUT_GAIN32, c.st);
        } else {
          a.alpha = alpha_a;
          a.inj = M + (size_t)i * n;
          a.Y = nullptr;
          a.Y32 = nullptr;
          a.tr = c.Mr.as<const double>();
          a.q_cnt1 = any;
          a.q_cnt2 = any;
          a.q_m1 = a.q_m2 = 0;
          a.q_s1 = a.q_s2 = 0.0;
          a.q_lv = dl32;
          a.q_mlv = ~0ull;
          a.q_slv = g->prep.alpha;
          a.q_alpha = g->prep.alpha;
          a.q_nlv = la - 1;
          a.q_even = r == la ? 1 : 0;
          a.Y32 = top_a ? dl32 + (size_t)(la - 1) * nC : nullptr;
          run_step(g, pn, a, IN_CNT32, top_a ? OUT_GAINCOMB32S : OUT_GAINCOMB32L, c.st,
                   0.5 * (la - 1));
        }
      }
    } else {
      // FP64 levels.  With the first level pushed and a >= 3, levels 1 and 2
      // are also kept as 32-bit counts (they fit: level 2 <= omega_2 <= nnz on
      // a graph without repeated arcs), so levels 2 and 3 gather counts; the
      // candidate's level-2 miss count is exact (the miss chain stores level
      // 2 as fl(alpha^2) times its count).
      const bool p32 = push1 && la >= 3;
      Partition &pn = partition_narrow(g, C);
      uint32_t *dc = nullptr;
      const double al = g->prep.alpha;
      if (p32) {
        c.wsC.fit(pn);
        c.wsC.into(a);
        c.dc32.ensure(2 * sizeof(uint32_t) * nC);
        dc = c.dc32.as<uint32_t>();
        if (c.dc1_zeroed != c.dc32.p) launch_fill_i32(c.dc32.as<int>(), 0, nC, c.st);
        c.dc1_zeroed = nullptr;
        hipLaunchKernelGGL(k_gain_level1_32, dim3(gx, nc), dim3(kBlock), 0, c.st, a.rp, a.ci,
                           a.smask, c.cand_dev.as<const int>(), C, c.sdeg.as<const int>(), dc, 0,
                           (uint64_t *)nullptr, (unsigned *)nullptr, 0u);
        GED_HIP(hipGetLastError());
      }
      if (spec) {  // level 1 of the miss columns (counts and FP64), dense
        hipLaunchKernelGGL(k_spec_miss1, dim3(std::min(8192, (n + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, c.st, a.rp, c.sdeg.as<const int>(), a.smask,
                           c.cand_dev.as<const int>(), nc, Cb, C, n, al, dc, dl);
        hipLaunchKernelGGL(k_spec_miss1_fix, dim3(gx, nc), dim3(kBlock), 0, c.st, a.rp, a.ci,
                           a.smask, c.cand_dev.as<const int>(), Cb, C, al, dc, dl);
        GED_HIP(hipGetLastError());
        a.spec_from = Cb;
      }
      double ai = al;  // alpha^i
      for (int i = push1 ? 2 : 1; i <= la; ++i) {
        ai *= al;
        const bool from32 = p32 && i <= 3;  // gathers the counts of level i - 1
        Partition &ps = from32 ? pn : p;
        const int in = from32 ? IN_CNT32 : (i == 1 ? IN_ONEHOT : IN_VEC);
        a.X = i == 1 ? nullptr : dl + (size_t)(i - 2) * nC;
        a.Xc32 = from32 ? dc + (size_t)(i - 2) * nC : nullptr;
        a.alpha = from32 ? ai : al;
        a.inj = M + (size_t)i * n;
        if (i < la) {
          a.Y = dl + (size_t)(i - 1) * nC;
          if (p32 && i == 2) {  // counts for level 3's gather, FP64 for the combination
            a.Y32 = dc + nC;
            a.injc = c.injc.as<const double>() + (size_t)2 * C;
            run_step(g, ps, a, IN_CNT32, OUT_GAIN32D, c.st);
          } else {
            run_step(g, ps, a, in, OUT_GAIN, c.st);
          }
        } else {
          // miss columns store their level la after the stored levels
          a.Y = spec ? dl + (size_t)(la - 1) * nC : nullptr;
          a.tr = c.Mr.as<const double>();
          a.q_cnt1 = any;
          a.q_cnt2 = any;
          a.q_m1 = a.q_m2 = 0;
          a.q_s1 = a.q_s2 = 0.0;
          a.q_lv = la > 1 ? dl : any;
          a.q_mlv = la > 1 ? ~0ull : 0ull;
          a.q_slv = la > 1 ? 1.0 : 0.0;
          a.q_nlv = la - 1;
          a.q_even = r == la ? 1 : 0;
          run_step(g, ps, a, in, OUT_GAINCOMB, c.st, la - 1);
          pr = &ps;
        }
      }
      if (spec) {
        c.spec_cand.assign(cand, cand + nc);
        c.spec_ell = ell;
        c.spec_C = C;
        c.spec_W = Cb;
        c.spec_la = la;
        c.spec_src = dl;
        c.spec_dirty = true;
      }
      if (p32) {
        hipLaunchKernelGGL(k_gain_level1_32, dim3(gx, nc), dim3(kBlock), 0, c.st, a.rp, a.ci,
                           a.smask, c.cand_dev.as<const int>(), C, c.sdeg.as<const int>(), dc, 1,
                           (uint64_t *)nullptr, (unsigned *)nullptr, 0u);
        GED_HIP(hipGetLastError());
        c.dc1_zeroed = c.dc32.p;
        // level 2 stays as counts until the next batch: a pick from this
        // batch subtracts it from the miss chain
        c.last_cand.assign(cand, cand + nc);
        c.last_ell = ell;
        c.last_src = dc;
        c.last_C = C;
        c.last_levels = 2;
      }
    }
    if (push1) {
      if (g32)
        hipLaunchKernelGGL(k_gain_level1_32, dim3(gx, nc), dim3(kBlock), 0, c.st, a.rp, a.ci,
                           a.smask, c.cand_dev.as<const int>(), C, c.sdeg.as<const int>(), dl32,
                           1, (uint64_t *)nullptr, (unsigned *)nullptr, 0u);
      else
        hipLaunchKernelGGL(k_gain_level1, dim3(gx, nc), dim3(kBlock), 0, c.st, a.rp, a.ci,
                           a.smask, c.cand_dev.as<const int>(), C, a.alpha, M + (size_t)n, dl, 1);
      GED_HIP(hipGetLastError());
      c.d1_zeroed = c.dlv.p;
      c.d1_bytes = eb;
    }
  } else {
    for (int i = 1; i <= ell; ++i) {
      a.accum = i > 1;  // L = sum over all levels of the column sums
      a.X = ((i & 1) ? c.X : c.Y).as<const double>();
      a.Y = ((i & 1) ? c.Y : c.X).as<double>();
      a.inj = M + (size_t)i * n;
      run_step(g, p, a, i == 1 ? IN_ONEHOT : IN_VEC, OUT_GAIN, c.st);
    }
  }
  launch_reduce(*pr, a, c.gains.as<double>(), nullptr, nullptr, c.st, c.wsC.scratch());
  double *hg = c.h_small.as<double>() + 256;
  hipLaunchKernelGGL(k_after_batch, dim3(1), dim3(64), 0, c.st, c.cand_dev.as<const int>(),
                     c.gains.as<const double>(), nc, c.stale.as<double>(), c.ub.as<double>(),
                     c.done.as<int>(), round, hg, c.cand_col.as<int>());
  GED_HIP(hipGetLastError());
  GED_HIP(hipStreamSynchronize(c.st));
  for (int q = 0; q < nc; ++q) out[q] = hg[q];
  c.evals += nc;
}

struct Top2 {
  double L1 = -1, L2 = -1;
  int u = -1, v = -1;
  void add(double L, int x) {
    if (u < 0 || kv_less(L1, u, L, x)) {
      L2 = L1;
      v = u;
      L1 = L;
      u = x;
    } else if (v < 0 || kv_less(L2, v, L, x)) {
      L2 = L;
      v = x;
    }
  }
  static bool kv_less(double ka, int ia, double kb, int ib) {  // is (kb, ib) better?
    return kb > ka || (kb == ka && ib < ia);
  }
};

// Sampling for the stochastic variant: splitmix64 at counter (pick, j).
static uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

int greedy_run(ged_graph *g, int32_t k, double alpha, double eps, double eta, uint64_t seed,
               bool stochastic, int32_t *out_group, double *out_score, ged_greedy_trace *tr,
               const std::atomic<int> *stop) {
  const int64_t n64 = g->n;
  if (k < 1 || k > n64) return fail(GED_ERR_ARG, "k must be in [1, n]");
  if (stochastic && !(eta > 0.0 && eta < 1.0)) return fail(GED_ERR_ARG, "eta must be in (0,1)");
  int rc = prepare(g, alpha, eps);
  if (rc) return rc;
  const int n = (int)n64;
  GreedyCtx &c = greedy_ctx(g);
  c.g = g;
  c.st = g->stream;
  c.n = n;
  c.fixed = g->greedy_width;
  c.C = c.fixed ? c.fixed : kWidthMax;
  c.split = split_ok(g);
  c.evals = 0;
  c.rounds = 0;
  c.last_ell = -1;  // nothing of an earlier call is reused
  c.sub_col = -1;
  c.spec_ell = -1;
  c.spec_col = -1;
  c.d2_zero = c.d2_pending = false;
  const int K = c.C + 1;  // the most pairs one selection returns
  c.smask.ensure(sizeof(uint32_t) * (size_t)((n + 31) / 32 + 1));
  c.ub.ensure(sizeof(double) * n);
  c.stale.ensure(sizeof(double) * n);
  c.done.ensure(sizeof(int) * n);
  c.cand_col.ensure(sizeof(int) * n);
  if (!c.split) {  // ping-pong gain levels (split gains store theirs in dlv)
    c.X.ensure(sizeof(double) * (size_t)n * c.C);
    c.Y.ensure(sizeof(double) * (size_t)n * c.C);
  }
  c.cand_dev.ensure(sizeof(int) * 64);
  c.gains.ensure(sizeof(double) * 64);
  const int nb0 = (n + kBlock * kTopE - 1) / (kBlock * kTopE);
  c.topk_k[0].ensure(sizeof(double) * (size_t)nb0 * K);
  c.topk_i[0].ensure(sizeof(int) * (size_t)nb0 * K);
  c.topk_k[1].ensure(sizeof(double) * (size_t)nb0 * K);
  c.topk_i[1].ensure(sizeof(int) * (size_t)nb0 * K);
  c.h_small.ensure(4096, hipHostMallocCoherent);
  launch_fill_i32(c.smask.as<int>(), 0, c.smask.bytes / sizeof(int), c.st);
  const bool track_sdeg = c.split && !g->weighted;
  if (track_sdeg) {
    c.sdeg.ensure(sizeof(int) * (size_t)n);
    launch_fill_i32(c.sdeg.as<int>(), 0, (size_t)n, c.st);
  }
  auto join = [&](int u) {
    if (track_sdeg) {  // S-arc counts and u's S bit in one launch
      const int d = g->h_rp[u + 1] - g->h_rp[u];
      hipLaunchKernelGGL(k_sdeg_add, dim3(std::max(1, std::min(256, (d + kBlock - 1) / kBlock))),
                         dim3(kBlock), 0, c.st, g->rp.as<const int>(), g->ci.as<const int>(), u,
                         c.sdeg.as<int>(), c.smask.as<uint32_t>());
    } else {
      hipLaunchKernelGGL(k_mask_bit, dim3(1), dim3(64), 0, c.st, c.smask.as<uint32_t>(), u, 1);
    }
    GED_HIP(hipGetLastError());
  };
  launch_fill_i32(c.done.as<int>(), -1, (size_t)n, c.st);
  launch_fill_i32(c.cand_col.as<int>(), -1, (size_t)n, c.st);
  std::vector<int> sample_host;
  if (stochastic) {
    c.sampled.ensure(sizeof(int) * n);
    launch_fill_i32(c.sampled.as<int>(), -1, (size_t)n, c.st);
  }

  std::vector<uint8_t> inS((size_t)n, 0);
  int s_size = 0;
  int ell = 1;
  if (tr && tr->n_forced > 0) {
    if (tr->n_forced > k || !tr->forced) return fail(GED_ERR_ARG, "bad forced prefix");
    for (int q = 0; q < tr->n_forced; ++q) {
      const int f = tr->forced[q];
      if (f < 0 || f >= n) return fail(GED_ERR_VERTEX, "bad forced vertex");
      const int u = g->new_id[f];
      if (inS[u]) return fail(GED_ERR_VERTEX, "repeated forced vertex");
      inS[u] = 1;
      out_group[s_size] = f;
      if (tr->ell) tr->ell[s_size] = -1;
      if (tr->L1) tr->L1[s_size] = NAN;
      if (tr->U2) tr->U2[s_size] = NAN;
      if (tr->L2) tr->L2[s_size] = NAN;
      if (tr->B) tr->B[s_size] = NAN;
      if (tr->evals) tr->evals[s_size] = 0;
      s_size++;
      join(u);
    }
    ell = tr->forced_ell >= 1 ? tr->forced_ell : 1;
  }
  int round = 0;
  int sample_pick = -1;
  std::vector<double> hk(K);
  std::vector<int> hi(K);
  std::vector<double> gains(c.C);
  std::vector<int> internal(c.C);
  while (s_size < k) {
    if (ell > 65536) return fail(GED_ERR_ELL, "walk length limit reached in greedy");
    ensure_levels_cap(c, ell);
    const double B = comb_bound(g, alpha, walk_total(g, ell));
    launch_fill_f64(c.stale.as<double>(), -1.0, (size_t)n, c.st);
    bool need_chain = true;
    while (s_size < k) {
      if (stop) {  // a server asked this request to stop (between rounds only)
        const int why = stop->load(std::memory_order_relaxed);
        if (why)
          return fail(why, why == GED_ERR_DEADLINE ? "greedy request passed its deadline"
                                                  : "greedy request cancelled");
      }
      if (stochastic && sample_pick != s_size) {
        // one sample of ceil((n/k) ln(1/eta)) vertices of V \ S per addition
        const int64_t want = (int64_t)ceil((double)n / k * log(1.0 / eta));
        const int rest = n - s_size;
        const int m = (int)std::min<int64_t>(want, rest);
        std::vector<int> pool;  // caller ids outside S, increasing
        pool.reserve(rest);
        for (int x = 0; x < n; ++x)
          if (!inS[g->new_id[x]]) pool.push_back(x);
        // partial Fisher-Yates with splitmix64 at counter (addition, j)
        for (int j = 0; j < m; ++j) {
          const uint64_t r =
              sm_mix(seed + 0x9E3779B97F4A7C15ULL * ((uint64_t)s_size * 0x100000000ULL + j + 1));
          const int q = j + (int)(((__uint128_t)r * (uint64_t)(rest - j)) >> 64);
          std::swap(pool[j], pool[q]);
        }
        sample_host.assign((size_t)n, -1);
        for (int j = 0; j < m; ++j) sample_host[g->new_id[pool[j]]] = s_size;
        GED_HIP(hipMemcpyAsync(c.sampled.p, sample_host.data(), sizeof(int) * n,
                               hipMemcpyHostToDevice, c.st));
        GED_HIP(hipStreamSynchronize(c.st));
        sample_pick = s_size;
      }
      if (need_chain) {
        chains_for(c, ell);
        need_chain = false;
      }
      compute_bounds(c, ell);
      ++round;
      ++c.rounds;
      Top2 top;
      int batch_in_round = 0;
      for (;;) {
        const int Cb = batch_width(c, batch_in_round++);
        const int m = select_topk(c, Cb + 1, round,
                                  stochastic ? c.sampled.as<const int>() : nullptr, s_size,
                                  hk.data(), hi.data());
        if (m == 0) break;
        if (top.v >= 0 && hk[0] < top.L2) break;  // no bound reaches the runner-up
        const int nc = std::min(m, Cb);
        for (int q = 0; q < nc; ++q) internal[q] = g->new_id[hi[q]];
        eval_batch(c, internal.data(), nc, Cb, ell, round, gains.data(), batch_in_round == 1);
        for (int q = 0; q < nc; ++q) top.add(gains[q], hi[q]);
        if (m <= Cb) break;  // nothing else eligible
        // the (Cb+1)-th bound is the best among the candidates not evaluated
        // (their bounds do not change within a round): the next selection
        // would stop on it
        if (top.v >= 0 && hk[Cb] < top.L2) break;
      }
      if (top.u < 0) return fail(GED_ERR_ARG, "no candidate left");
      if (top.v >= 0 && top.L1 <= (top.L2 + B) - eps / (double)k) break;  // not separated
      const int u = g->new_id[top.u];
      inS[u] = 1;
      out_group[s_size] = top.u;
      if (tr) {
        if (tr->ell) tr->ell[s_size] = ell;
        if (tr->L1) tr->L1[s_size] = top.L1;
        if (tr->U2) tr->U2[s_size] = top.v >= 0 ? top.L2 + B : NAN;
        if (tr->L2) tr->L2[s_size] = top.v >= 0 ? top.L2 : NAN;
        if (tr->B) tr->B[s_size] = B;
        if (tr->evals) tr->evals[s_size] = c.evals;
      }
      s_size++;
      join(u);
      need_chain = true;
      c.sub_col = -1;
      c.spec_col = -1;
      if (c.last_ell == ell)
        for (size_t q = 0; q < c.last_cand.size(); ++q)
          if (c.last_cand[q] == u) c.sub_col = (int)q;
      if (c.spec_ell == ell)
        for (size_t q = 0; q < c.spec_cand.size(); ++q)
          if (c.spec_cand[q] == u) c.spec_col = (int)q;
    }
    if (s_size < k) ell *= 2;
  }
  GED_HIP(hipStreamSynchronize(c.st));
  if (tr) tr->n_rounds = c.rounds;
  if (out_score) {
    ged_score_info info;
    rc = score_group(g, out_group, k, alpha, eps, out_score, &info);
    if (rc) return rc;
    if (tr) tr->score_ell = info.ell;
  }
  return GED_OK;
}

}  // namespace ged

using namespace ged;

extern "C" int ged_greedy(ged_graph *g, int32_t k, double alpha, double eps, int32_t *out_group,
                          double *out_score, ged_greedy_trace *trace) {
  if (!g || !out_group) return fail(GED_ERR_ARG, "bad argument to ged_greedy");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() {
    return greedy_run(g, k, alpha, eps, 0.0, 0, false, out_group, out_score, trace, nullptr);
  });
}

extern "C" int ged_greedy_footprint(ged_graph *g, int32_t k, double alpha, double eps,
                                    int64_t *estimate, int64_t *held) {
  if (!g || !estimate) return fail(GED_ERR_ARG, "bad argument to ged_greedy_footprint");
  if (k < 1 || k > g->n) return fail(GED_ERR_ARG, "k must be in [1, n]");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() -> int {
    int rc = prepare(g, alpha, eps);
    if (rc) return rc;
    // ell doubles from 1 until the tail bound is below eps / k, where every
    // round separates (L1 >= L2 > L2 + B - eps/k)
    int ell = 1;
    while (ell < 65536 && !(comb_bound(g, alpha, walk_total(g, ell)) < eps / (double)k)) ell *= 2;
    *estimate = (int64_t)greedy_footprint(g, ell, k);
    if (held) *held = (int64_t)greedy_bytes_held(g);
    return GED_OK;
  });
}

extern "C" int ged_set_greedy_width(ged_graph *g, int32_t width) {
  if (!g) return fail(GED_ERR_ARG, "null graph");
  if (width != 0 && width != 2 && width != 4 && width != 8 && width != 16)
    return fail(GED_ERR_ARG, "greedy width must be 0, 2, 4, 8 or 16");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  g->greedy_width = width;
  return GED_OK;
}

extern "C" int32_t ged_greedy_width(const ged_graph *g) { return g ? greedy_width_for(g) : 0; }

extern "C" int ged_greedy_stochastic(ged_graph *g, int32_t k, double alpha, double eps,
                                     double eta, uint64_t seed, int32_t *out_group,
                                     double *out_score, ged_greedy_trace *trace) {
  if (!g || !out_group) return fail(GED_ERR_ARG, "bad argument to ged_greedy_stochastic");
  std::lock_guard<std::recursive_mutex> lk(g->mu);
  return guarded([&]() {
    return greedy_run(g, k, alpha, eps, eta, seed, true, out_group, out_score, trace, nullptr);
  });
}
