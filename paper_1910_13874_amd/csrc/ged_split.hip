// Split scoring for undirected graphs: the truncated score of a group from
// the hit chain up to level a = ceil(ell*/2) instead of ell*.
//
// A walk of length a + c, cut after its first a arcs at vertex v, meets S iff
// its first a + 1 vertices do or its last c vertices do.  On an undirected
// graph the walks of length c leaving v are the reversals of those ending at
// v, so both halves are counted by chains the scoring path already has: the
// hit chain h (walks ending at v that meet S, the phi^hit recurrence of
// Section 3.1.1) and the total chain t (Eq. phisum's omega, decayed):
//   phi_{a+c}(S) = sum_v h_a(v) t_c(v) + sum_{v not in S} (t_a(v) - h_a(v)) h_c(v).
// t_a - h_a is the miss count phi^miss of walks ending at v outside S; its
// rounding error is bounded by the first term.  Every level up to 2a follows
// from levels <= a, so ell* levels cost ceil(ell*/2) chain levels; the last
// dense step applies the combination in its epilogue (OUT_COMBINE).
//
// On unweighted graphs the first two levels are integer walk counts
// (h_i = alpha^i * count_i), pushed from the group's members with integer
// atomics (exact and order-free, so the result stays deterministic), 32-bit
// when count_2 <= omega_2 is known to fit (maximum degree below 2^16, or no
// duplicate arcs: then omega_2 <= nnz < 2^31), else 64-bit:
//   count_1(y) = |N(y) ∩ S| outside S,        deg(y) on S
//   count_2(x) = sum_{y in N(x)} count_1(y) outside S,   omega_2(x) on S
// Members push deg(s) to their neighbours (level-2 paths through a member)
// and every non-member y adjacent to S pushes count_1(y) to N(y) once, from a
// worklist of (y, column, chunk) entries that splits long rows.  Everything a
// tile touched is cleared by replaying the same traversal with stores of 0.
//
// The dense levels i = 3 .. a-1 that the combining step reads back are the
// same integer counts scaled by alpha^i, and count_i(v) <= omega_i(v), the
// number of all walks of length i ending at v.  When max_v omega_i(v) < 2^32
// for each of them they are stored unscaled as 32-bit integers (half the
// bytes of FP64, so a 32-column tile gathers one 128-byte line per vertex):
// members take the exact omega_i(v), computed once per graph by an integer
// chain, and alpha^a is applied once in the combining step.
#include <algorithm>
#include <cstring>

#include "ged_internal.h"

namespace ged {

constexpr int kPushGrid = 2048; // blocks of the member kernels (grid-stride)
// Blocks of the worklist kernels (4 waves each, grid-stride over the entries):
// about one wave per expected entry, between kWlGridMin and kWlGridMax.
constexpr int kWlGridMin = 64;
constexpr int kWlGridMax = 16384;
// Grid of the pushed level 3 and its clearing: one wave per entry up to
// 4096 entries (waves without an entry end at once).
constexpr int kWl3Grid = 1024;
// Largest single group whose members the score's first kernel reads from
// host memory instead of a copy.
constexpr int kStageMembers = 1024;
int split_wl_blocks(int64_t expected_entries) {
  return (int)std::max<int64_t>(kWlGridMin,
                                std::min<int64_t>(kWlGridMax, (expected_entries + 3) / 4));
}

bool split_ok(const ged_graph *g) { return g->flags == GED_UNDIRECTED; }

SplitPlan split_plan(const ged_graph *g, int ell) {
  SplitPlan p;
  p.a = (ell + 1) / 2;
  p.r = ell - p.a;
  p.even = p.r == p.a;
  p.s = g->weighted ? 0 : std::min(2, p.a - 1);
  p.nlv = p.a - 1 - p.s;
  // count_2(x) <= omega_2(x) = sum_{y in N(x)} deg(y), which is at most
  // (max degree)^2, and at most nnz < 2^31 when no arc is listed twice
  p.c32 = g->max_deg < 65536 || g->simple;
  return p;
}

size_t split_wl_need(const ged_graph *g, int64_t deg_sum) {
  // distinct non-members y adjacent to the group (at most min(n, deg_sum)),
  // each split into ceil(deg(y)/chunk) <= 1 + deg(y)/chunk entries, and the
  // degrees of distinct vertices add up to at most nnz
  return (size_t)std::min<int64_t>(g->n, deg_sum) + (size_t)(g->nnz / kWlChunk) + 1;
}

// --------------------------------------------------------------- kernels --

// The level-2 count array in either layout: plain CT[n*C] (h16 < 0), or the
// 16-bit layout with hub cut h16 (32-bit counts only; c16_pk_offset).  In the
// packed part a column's count is one half of a 32-bit word, so it is added
// to, read from and set through that word.
template <class CT>
__device__ __forceinline__ void c16_word(CT *p, int h16, int C, int v, int c, uint32_t *&w,
                                         int &sh) {
  uint16_t *pk = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(p) + c16_pk_offset(h16, C));
  const size_t o = (size_t)v * C + c;  // C is even: o is odd iff c is
  w = reinterpret_cast<uint32_t *>(pk + (o & ~(size_t)1));
  sh = (int)(o & 1) << 4;
}

// Add val at (v, c); returns the count before the add.
template <class CT>
__device__ __forceinline__ CT cnt2_add(CT *p, int h16, int C, int v, int c, CT val) {
  if constexpr (sizeof(CT) == 4) {
    if (h16 >= 0 && v >= h16) {
      uint32_t *w;
      int sh;
      c16_word(p, h16, C, v, c, w, sh);
      return (CT)((atomicAdd(w, (uint32_t)val << sh) >> sh) & 0xffffu);
    }
  }
  return atomicAdd(&p[(size_t)v * C + c], val);
}

// Store 0 at (v, c) (a 16-bit store in the packed part: the other half of
// its word is left as it is).
template <class CT>
__device__ __forceinline__ void cnt2_zero(CT *p, int h16, int C, int v, int c) {
  if constexpr (sizeof(CT) == 4) {
    if (h16 >= 0 && v >= h16) {
      uint16_t *pk =
          reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(p) + c16_pk_offset(h16, C));
      pk[(size_t)v * C + c] = 0;
      return;
    }
  }
  p[(size_t)v * C + c] = 0;
}

// Set (v, c) to val >= its current count while other threads may add to the
// other half of its word (member rows are fixed inside the level-2 push,
// whose adds skip the row's own column): read the half, add the difference.
template <class CT>
__device__ __forceinline__ void cnt2_raise(CT *p, int h16, int C, int v, int c, CT val) {
  if constexpr (sizeof(CT) == 4) {
    if (h16 >= 0 && v >= h16) {
      uint32_t *w;
      int sh;
      c16_word(p, h16, C, v, c, w, sh);
      const uint32_t cur =
          (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> sh) & 0xffffu;
      atomicAdd(w, ((uint32_t)val - cur) << sh);
      return;
    }
  }
  p[(size_t)v * C + c] = val;
}

// Members of groups g0 .. g0+nc-1, one block per member: level-1 counts, the
// level-2 contributions of paths through the member, and worklist entries for
// the non-members they reach first.  With wl3 (single group, pushed level 3)
// also the entries of every vertex holding a level-2 count so far: the
// member itself (its count is omega_2) and each non-member neighbour the
// first time its level-2 count is touched.
template <class CT>
__global__ __launch_bounds__(kBlock) void k_push(const int *__restrict__ rp,
                                                 const int *__restrict__ ci,
                                                 const uint64_t *__restrict__ tmask,
                                                 const int64_t *offsets, const int *members,
                                                 const int *mcol, int g0, int nc, int C, CT *cnt1,
                                                 CT *cnt2, uint64_t *wl, unsigned *wl_n,
                                                 unsigned wl_cap, uint64_t *wl3, unsigned *wl3_n,
                                                 unsigned wl3_cap, int h16) {
  const int64_t jb = offsets[g0], je = offsets[g0 + nc];
  for (int64_t j = jb + blockIdx.x; j < je; j += gridDim.x) {
    const int s = members[j];
    const int c = mcol[j] - g0;
    const int k0 = rp[s], k1 = rp[s + 1];
    const CT ds = (CT)(k1 - k0);
    if (wl3 && threadIdx.x == 0 && k1 > k0) {
      const unsigned nch = wl_chunks(rp, s);
      const unsigned base = atomicAdd(wl3_n, nch);
      for (unsigned q = 0; q < nch; ++q)
        if (base + q < wl3_cap) wl3[base + q] = wl_entry(s, c, q);
    }
    for (int kb = k0; kb < k1; kb += kBlock) {  // same trip count for the whole block
      const int k = kb + (int)threadIdx.x;
      unsigned nch = 0, nch3 = 0;
      int y = 0;
      if (k < k1) {
        y = ci[k];
        const size_t o = (size_t)y * C + c;
        const CT old = atomicAdd(&cnt1[o], (CT)1);
        if (cnt2) {
          const CT old2 = cnt2_add(cnt2, h16, C, y, c, ds);
          if (!((tmask[y] >> c) & 1ull)) {
            const unsigned ch = wl_chunks(rp, y);
            if (old == 0) nch = ch;
            if (old2 == 0) nch3 = ch;
          }
        }
      }
      if (cnt2) wl_append(wl, wl_n, wl_cap, y, c, nch);
      if (wl3) wl_append(wl3, wl3_n, wl3_cap, y, c, nch3);
    }
  }
}

// Member rows hold the unrestricted counts: deg(s), omega_2(s) and, for a
// pushed level 3, omega_3(s) (om3, exact integers as doubles).  members ==
// nullptr: nothing to do.
template <class CT>
struct MemberFix {
  const int *rp = nullptr;
  const unsigned long long *omega2 = nullptr;
  const int64_t *offsets = nullptr;
  const int *members = nullptr, *mcol = nullptr;
  int g0 = 0, nc = 0, C = 1;
  CT *cnt1 = nullptr, *cnt2 = nullptr, *lv3 = nullptr;
  const double *om3 = nullptr;
  int h16 = -1;  // cnt2 layout
};

// All threads of the launch, grid-stride over the members.
template <class CT>
__device__ __forceinline__ void fix_members(const MemberFix<CT> &f) {
  if (!f.members) return;
  const int64_t jb = f.offsets[f.g0], je = f.offsets[f.g0 + f.nc];
  for (int64_t j = jb + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < je;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int s = f.members[j];
    const size_t o = (size_t)s * f.C + (f.mcol[j] - f.g0);
    f.cnt1[o] = (CT)(f.rp[s + 1] - f.rp[s]);
    if (f.cnt2) cnt2_raise(f.cnt2, f.h16, f.C, s, f.mcol[j] - f.g0, (CT)f.omega2[s]);
    if (f.lv3) f.lv3[o] = (CT)f.om3[s];
  }
}

// Zero dst at the targets of one worklist entry (one wavefront, all loads
// of the chunk issued first).
template <class CT>
__device__ __forceinline__ void clear_entry(const int *__restrict__ rp,
                                            const int *__restrict__ ci, int C, CT *dst,
                                            uint64_t e, int h16 = -1) {
  constexpr int U = kWlChunk / 64;
  const int lane = threadIdx.x & 63;
  const int y = (int)(e >> 32);
  const int c = (int)((e >> 24) & 0xffu);
  const int q = (int)(e & 0xffffffu);
  const int j0 = rp[y] + q * kWlChunk + lane, j1 = min(rp[y] + (q + 1) * kWlChunk, rp[y + 1]);
  int x[U];
#pragma unroll
  for (int k = 0; k < U; ++k) x[k] = j0 + 64 * k < j1 ? ci[j0 + 64 * k] : -1;
#pragma unroll
  for (int k = 0; k < U; ++k)
    if (x[k] >= 0) cnt2_zero(dst, h16, C, x[k], c);
}

// Worklist entries, one wavefront each: src(y) (the next lower level's
// count) goes to dst at every x in one chunk of N(y) outside the group
// (member rows are overwritten with the unrestricted counts afterwards, and a
// member hub would take one contended atomic per neighbour); with wl_next,
// each x whose dst count is first touched appends its entries there.  CLEAR
// stores zeros instead.  NEXT: wl_next is used (the adds return the old
// count); otherwise the adds return nothing and the wave does not wait.  The
// level-2 push also fixes the member rows (fx): it neither reads nor writes
// them, and the member pushes before it have finished.
template <class CT, bool CLEAR, bool NEXT>
__global__ __launch_bounds__(kBlock) void k_push_wl(const int *__restrict__ rp,
                                                    const int *__restrict__ ci, int C,
                                                    const CT *src, CT *dst, const uint64_t *wl,
                                                    const unsigned *wl_n, unsigned wl_cap,
                                                    const uint64_t *__restrict__ tmask,
                                                    uint64_t *wl_next, unsigned *wl_next_n,
                                                    unsigned wl_next_cap, MemberFix<CT> fx,
                                                    int h16) {
  fix_members(fx);
  const unsigned count = min(*wl_n, wl_cap);  // capacities are sized to never overflow
  // A chunk is at most U arcs per lane: every col_idx load of the chunk is
  // issued before the first use, then every tmask load, then every add, so a
  // wave waits for one round trip of each instead of U.
  constexpr int U = kWlChunk / 64;
  const int lane = threadIdx.x & 63;
  const unsigned nwaves = (gridDim.x * kBlock) >> 6;
  for (unsigned i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < count; i += nwaves) {
    const uint64_t e = wl[i];
    const int y = (int)(e >> 32);
    const int c = (int)((e >> 24) & 0xffu);
    const int q = (int)(e & 0xffffffu);
    if (CLEAR) {
      clear_entry(rp, ci, C, dst, e, h16);
      continue;
    }
    const int j0 = rp[y] + q * kWlChunk + lane, j1 = min(rp[y] + (q + 1) * kWlChunk, rp[y + 1]);
    int x[U];
#pragma unroll
    for (int k = 0; k < U; ++k) x[k] = j0 + 64 * k < j1 ? ci[j0 + 64 * k] : -1;
    bool out[U];
#pragma unroll
    for (int k = 0; k < U; ++k) out[k] = x[k] >= 0 && !((tmask[x[k]] >> c) & 1ull);
    const CT v = src[(size_t)y * C + c];
    if (!NEXT) {
#pragma unroll
      for (int k = 0; k < U; ++k)
        if (out[k]) cnt2_add(dst, h16, C, x[k], c, v);
      continue;
    }
    bool first[U];
#pragma unroll
    for (int k = 0; k < U; ++k)
      first[k] = out[k] && cnt2_add(dst, h16, C, x[k], c, v) == 0;
    unsigned nch[U], tot = 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      nch[k] = first[k] ? wl_chunks(rp, x[k]) : 0u;
      tot += nch[k];
    }
    // one append for the lane's vertices (in k order)
    unsigned total;
    const unsigned ex = wave_excl_scan(tot, &total);
    unsigned base = 0;
    if (lane == 63 && total) base = atomicAdd(wl_next_n, total);
    base = __shfl(base, 63, 64) + ex;
#pragma unroll
    for (int k = 0; k < U; ++k)
      for (unsigned r = 0; r < nch[k]; ++r, ++base)
        if (base < wl_next_cap) wl_next[base] = wl_entry(x[k], c, r);
  }
}

// The member rows alone (tiles without a level-2 push).
template <class CT>
__global__ void k_fix_members(MemberFix<CT> fx) {
  fix_members(fx);
}

// Zero dst_a at every target of list a's entries and dst_b at every target
// of list b's (a single score's pushed levels 2 and 3): one launch.
template <class CT>
__global__ __launch_bounds__(kBlock) void k_clear_two(const int *__restrict__ rp,
                                                      const int *__restrict__ ci, int C,
                                                      CT *dst_a, const uint64_t *wl_a,
                                                      const unsigned *n_a, unsigned cap_a,
                                                      CT *dst_b, const uint64_t *wl_b,
                                                      const unsigned *n_b, unsigned cap_b) {
  const unsigned ca = min(*n_a, cap_a), cb = min(*n_b, cap_b);
  const unsigned nwaves = (gridDim.x * kBlock) >> 6;
  for (unsigned i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < ca + cb; i += nwaves) {
    if (i < ca)
      clear_entry(rp, ci, C, dst_a, wl_a[i]);
    else
      clear_entry(rp, ci, C, dst_b, wl_b[i - ca]);
  }
}

// Zero every count entry k_push / k_fix_members wrote for these members, and
// the members' column bits in tmask; reset the worklist lengths (the worklist
// replays that read them have finished).
template <class CT>
__global__ __launch_bounds__(kBlock) void k_clear_members(const int *__restrict__ rp,
                                                          const int *__restrict__ ci,
                                                          const int64_t *offsets,
                                                          const int *members, const int *mcol,
                                                          int g0, int nc, int C, CT *cnt1,
                                                          CT *cnt2, CT *lv3,
                                                          unsigned long long *tmask,
                                                          unsigned *wl_n, unsigned *wl3_n,
                                                          int h16) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (wl_n) *wl_n = 0;
    if (wl3_n) *wl3_n = 0;
  }
  const int64_t jb = offsets[g0], je = offsets[g0 + nc];
  for (int64_t j = jb + blockIdx.x; j < je; j += gridDim.x) {
    const int s = members[j];
    const int c = mcol[j] - g0;
    if (threadIdx.x == 0) {
      cnt1[(size_t)s * C + c] = 0;
      if (cnt2) cnt2_zero(cnt2, h16, C, s, c);
      if (lv3) lv3[(size_t)s * C + c] = 0;
      atomicAnd(&tmask[s], ~(1ull << c));
    }
    for (int k = rp[s] + (int)threadIdx.x; k < rp[s + 1]; k += kBlock) {
      const int y = ci[k];
      cnt1[(size_t)y * C + c] = 0;
      if (cnt2) cnt2_zero(cnt2, h16, C, y, c);
    }
  }
}

// omega_2(v) = sum_{u in N(v)} deg(u): walks of length 2 ending at v.  One
// wavefront per row (lanes over its arcs, integer sum), so hub rows do not
// serialise on one lane.
// Block-wide max and saturating sum of the wave leaders' values (lane 0 of
// each wave holds one); thread 0 returns them.  Keeps the same-address
// atomics that follow at one per block.
__device__ __forceinline__ void block_max_sum(unsigned long long &m, unsigned long long &acc) {
  __shared__ unsigned long long sm[kBlock / 64], sa[kBlock / 64];
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[wid] = m;
    sa[wid] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      m = sm[w] > m ? sm[w] : m;
      acc += sa[w];
    }
  }
}

// *sum (zeroed by the caller) receives sum_v omega_2(v).
__global__ __launch_bounds__(kBlock) void k_omega2(const int *__restrict__ rp,
                                                   const int *__restrict__ ci, int n,
                                                   unsigned long long *out,
                                                   unsigned long long *sum) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
  unsigned long long acc = 0, m = 0;
  for (int64_t v = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6; v < n; v += nw) {
    unsigned long long s = 0;
    for (int k = rp[v] + lane; k < rp[v + 1]; k += 64) {
      const int u = ci[k];
      s += (unsigned long long)(rp[u + 1] - rp[u]);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) out[v] = s;
    acc += s;
  }
  block_max_sum(m, acc);
  if (threadIdx.x == 0 && acc > 0) atomicAdd(sum, acc);
}

// omega_i(v) = sum_{u in N(v)} omega_{i-1}(u), saturating at 2^64 - 1, also
// written as a double (exact below 2^53, the only range it is used in); the
// wave's largest value goes to *maxv and its sum to *sumv (exact while the
// level fits 2^32).  One wavefront per row, as k_omega2.
__device__ __forceinline__ unsigned long long sat_add(unsigned long long x, unsigned long long y) {
  const unsigned long long z = x + y;
  return z < x ? ~0ull : z;
}

__global__ __launch_bounds__(kBlock) void k_omega_next(const int *__restrict__ rp,
                                                       const int *__restrict__ ci, int n,
                                                       const unsigned long long *__restrict__ prev,
                                                       unsigned long long *out, double *out_d,
                                                       unsigned long long *maxv,
                                                       unsigned long long *sumv) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (kBlock / 64);
  unsigned long long m = 0, acc = 0;
  for (int64_t v = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6; v < n; v += nw) {
    unsigned long long s = 0;
    for (int k = rp[v] + lane; k < rp[v + 1]; k += 64) s = sat_add(s, prev[ci[k]]);
    for (int o = 32; o > 0; o >>= 1) s = sat_add(s, __shfl_xor(s, o, 64));
    if (lane == 0) {
      out[v] = s;
      if (out_d) out_d[v] = (double)s;
      m = s > m ? s : m;
      acc = sat_add(acc, s);
    }
  }
  block_max_sum(m, acc);
  if (threadIdx.x == 0 && m > 0) {
    atomicMax(maxv, m);
    atomicAdd(sumv, acc);
  }
}

// tr(v) = sum_{c=1..r} t_c(v), added in level order.
__global__ void k_sum_t(const double *__restrict__ T, int64_t n, int r, double *out) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 1; c <= r; ++c) s += T[(size_t)c * n + v];
    out[v] = s;
  }
}

// A single group staged from coherent host memory by the first kernel of a
// score: offsets {0, len} and members copied to the device buffer every later
// kernel reads (the deferred clean-up included, so the host may reuse its
// buffer once the score is done), and the members' column bit set in tmask.
__global__ void k_stage_group(const int64_t *h_offs, const int *h_mem, int64_t *d_offs,
                              int *d_mem, unsigned long long *tmask) {
  const int64_t len = h_offs[1];
  if (blockIdx.x == 0 && threadIdx.x < 2) d_offs[threadIdx.x] = h_offs[threadIdx.x];
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < len;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int v = h_mem[j];
    d_mem[j] = v;
    atomicOr(&tmask[v], 1ull);
  }
}

// t_i(v) = apow.a[i] * omega_i(v) for i = 1 .. P (omega_1 = degree): the
// walk-count levels of the precomputation from the integer counts.
struct TPow {
  double a[kTPrefixMax + 1];
};

__global__ void k_t_from_omega(const int *__restrict__ rp,
                               const unsigned long long *__restrict__ om2,
                               const double *__restrict__ omlv, int64_t n, int P, TPow apow,
                               double *__restrict__ T) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    T[(size_t)n + v] = apow.a[1] * (double)(rp[v + 1] - rp[v]);
    if (P >= 2) T[2 * (size_t)n + v] = apow.a[2] * (double)om2[v];
    for (int i = 3; i <= P; ++i)
      T[(size_t)i * n + v] = apow.a[i] * omlv[(size_t)(i - 3) * n + v];
  }
}

// ------------------------------------------------------------------ host --

static int grid_for(int64_t items, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(items, cap));
}

// Per-graph omega tables are built under this lock (greedy workers and lanes
// of a server may ask for them from several threads).
static std::mutex g_omega_mu;

static void ensure_omega2(ged_graph *g, hipStream_t st) {
  if (g->omega2_ready) return;
  const int64_t n = g->n;
  g->omega2.ensure(sizeof(uint64_t) * (size_t)n);
  DBuf sum;
  sum.ensure(sizeof(unsigned long long));
  launch_fill_i32(sum.as<int>(), 0, 2, st);
  const int og = (int)std::max<int64_t>(
      1, std::min<int64_t>(2048, (n + kBlock / 64 - 1) / (kBlock / 64)));
  hipLaunchKernelGGL(k_omega2, dim3(og), dim3(kBlock), 0, st, g->rp.as<const int>(),
                     g->ci.as<const int>(), (int)n, g->omega2.as<unsigned long long>(),
                     sum.as<unsigned long long>());
  GED_HIP(hipGetLastError());
  unsigned long long hs = 0;
  GED_HIP(hipMemcpyAsync(&hs, sum.p, sizeof(hs), hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  g->omega_sum.assign(3, 0.0);
  g->omega_sum[1] = (double)g->nnz;
  g->omega_sum[2] = (double)hs;
  g->omega2_ready = true;
}

// The integer chain omega_3 .. omega_top from omega_2, written as doubles to
// out[(i-3)*n ..] if out is non-null (then their sums go to omega_sum).
// Returns the largest i <= top such that max_v omega_j(v) < 2^32 for
// 3 <= j <= i (2 if omega_3 does not fit); *exact (if non-null) gets the
// largest level no value of which can have wrapped around 2^64: level i is
// safe when the one below is and max_deg times its maximum stays below 2^64
// (omega_2 <= max_deg^2, and <= nnz without repeated arcs).  Synchronizes
// the stream.
static int omega_chain(ged_graph *g, int top, double *out, hipStream_t st, int *exact = nullptr) {
  const int64_t n = g->n;
  const int L = top - 2;
  DBuf tmp, mx;
  tmp.ensure(2 * sizeof(unsigned long long) * (size_t)n);
  mx.ensure(2 * sizeof(unsigned long long) * L);  // maxima, then sums
  launch_fill_i32(mx.as<int>(), 0, (size_t)L * 4, st);
  const int og = (int)std::max<int64_t>(
      1, std::min<int64_t>(2048, (n + kBlock / 64 - 1) / (kBlock / 64)));
  unsigned long long *t2 = tmp.as<unsigned long long>();
  for (int i = 3; i <= top; ++i) {
    const unsigned long long *prev = i == 3 ? g->omega2.as<const unsigned long long>()
                                            : t2 + (size_t)((i - 1) & 1) * n;
    hipLaunchKernelGGL(k_omega_next, dim3(og), dim3(kBlock), 0, st, g->rp.as<const int>(),
                       g->ci.as<const int>(), (int)n, prev, t2 + (size_t)(i & 1) * n,
                       out ? out + (size_t)(i - 3) * n : nullptr,
                       mx.as<unsigned long long>() + (i - 3),
                       mx.as<unsigned long long>() + L + (i - 3));
    GED_HIP(hipGetLastError());
  }
  std::vector<unsigned long long> hm(2 * (size_t)L);
  GED_HIP(hipMemcpyAsync(hm.data(), mx.p, 2 * sizeof(unsigned long long) * L,
                         hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  int fit = 2;
  while (fit < top && hm[(size_t)(fit - 2)] < (1ull << 32)) ++fit;
  if (exact) {
    const double md = (double)g->max_deg;
    double m = md * md;  // bound on max omega_2
    if (g->simple) m = std::min(m, (double)g->nnz);
    int e = 2;
    while (e < top && md * m < 0.99 * 18446744073709551616.0) {
      ++e;
      m = (double)hm[(size_t)(e - 3)];  // exact: no value of level e wrapped
    }
    *exact = e;
  }
  if (out) {  // sums of levels past fit may have wrapped: not kept
    g->omega_sum.resize((size_t)fit + 1);
    for (int i = 3; i <= fit; ++i) g->omega_sum[(size_t)i] = (double)hm[(size_t)L + (i - 3)];
  }
  if (top > g->omax_top) {
    g->omax_top = top;
    g->omax_fit = fit;
  }
  return fit;
}

// omega_3 .. omega_top as doubles (levels past the first one whose maximum
// reaches 2^32 are not used).  Built in fresh buffers and published after
// the stream has finished them; a replaced buffer is kept until the graph is
// destroyed, since captured work may still name it.
static void omega_levels(ged_graph *g, int top, hipStream_t st) {
  DBuf lv;
  lv.ensure(sizeof(double) * (size_t)g->n * (top - 2));
  int exact = 2;
  const int fit = omega_chain(g, top, lv.as<double>(), st, &exact);
  if (g->omega_lv.p) {
    g->omega_old.emplace_back();
    std::swap(g->omega_old.back().p, g->omega_lv.p);
    std::swap(g->omega_old.back().bytes, g->omega_lv.bytes);
  }
  std::swap(g->omega_lv.p, lv.p);
  std::swap(g->omega_lv.bytes, lv.bytes);
  g->omega_top = top;
  g->omega_fit = fit;
  g->omega_exact = exact;
}

int omega_fit_level(ged_graph *g, int L, hipStream_t st) {
  if (L <= 2) return L;
  std::lock_guard<std::mutex> lk(g_omega_mu);
  if (L > g->omax_top && g->omax_fit == g->omax_top) {
    ensure_omega2(g, st);
    omega_chain(g, std::max(L, 4), nullptr, st);
  }
  return std::min(L, g->omax_fit);
}

int omega_prefix_levels(ged_graph *g) {
  if (g->weighted) return 0;
  std::lock_guard<std::mutex> lk(g_omega_mu);
  const int P = !g->omega2_ready ? 1 : g->omega_lv.p ? g->omega_fit : 2;
  return std::min(P, kTPrefixMax);
}

int t_levels_from_omega(ged_graph *g, double alpha, double eps, int levels_cap, double *T,
                        std::vector<double> &W, hipStream_t st) {
  if (g->weighted || levels_cap < 1) return 0;
  // the tables only grow, so they still hold the levels_cap levels counted
  std::lock_guard<std::mutex> lk(g_omega_mu);
  TPow apow;
  apow.a[0] = 1.0;
  int L = 0;
  while (L < levels_cap) {
    ++L;
    apow.a[L] = apow.a[L - 1] * alpha;
    W.push_back(apow.a[L] * (L == 1 ? (double)g->nnz : g->omega_sum[(size_t)L]));
    if (comb_bound(g, alpha, W.back()) < eps) break;
  }
  const int64_t n = g->n;
  hipLaunchKernelGGL(k_t_from_omega, dim3(grid_for((n + kBlock - 1) / kBlock, 8192)),
                     dim3(kBlock), 0, st, g->rp.as<const int>(),
                     L >= 2 ? g->omega2.as<const unsigned long long>() : nullptr,
                     L >= 3 ? g->omega_lv.as<const double>() : nullptr, n, L, apow, T);
  GED_HIP(hipGetLastError());
  return L;
}

void split_tables(ged_graph *g, SplitPlan &pl, hipStream_t st) {
  const int64_t n = g->n;
  const int eg = (int)std::min<int64_t>(8192, (n + kBlock - 1) / kBlock);
  std::unique_lock<std::mutex> lk(g_omega_mu);
  if (pl.s >= 2) ensure_omega2(g, st);
  // 32-bit stored levels: 3 .. a-1 must all fit (levels only grow past a
  // level that does not, so none is computed beyond the first that fails)
  pl.lv32 = false;
  if (pl.nlv > 0 && pl.c32 && pl.s == 2) {
    const int need = pl.a - 1;
    if (need > g->omega_top && g->omega_fit == g->omega_top)
      omega_levels(g, std::max(need, 4), st);
    pl.lv32 = g->omega_fit >= need;
  }
  lk.unlock();
  PrepCache &pc = g->prep;
  if (pc.tr_r != pl.r) {
    pc.tr.ensure(sizeof(double) * (size_t)n);
    hipLaunchKernelGGL(k_sum_t, dim3(eg), dim3(kBlock), 0, st, pc.t_levels.as<const double>(),
                       n, pl.r, pc.tr.as<double>());
    GED_HIP(hipGetLastError());
    pc.tr_r = pl.r;
  }
}

// Gather of the last (combining) dense level of a tile.
static int final_in(const SplitPlan &pl) {
  if (pl.c16_hub >= 0) return IN_CNT16;  // level 2, or the 16-bit copy of level a-1
  if (pl.lv32) return IN_CNT32;
  if (pl.a == 1) return IN_TILEMASK;
  if (pl.a == pl.s + 1) return pl.c32 ? IN_CNT32 : IN_CNT;
  return IN_VEC;
}

// Partition of a step gathering `in` at C columns (row-split threshold of pl).
static Partition &step_partition(ged_graph *g, const SplitPlan &pl, int C, int in) {
  if (in == IN_CNT16) return partition_quad(g, C, pl.cut_div);
  return narrow_gather(C, in, g->weighted) ? partition_narrow(g, C, pl.cut_div)
                                           : partition(g, C, false, pl.cut_div);
}

// The level-3 push adds each level-2 source's count to all its neighbours:
// as many adds as the sources' degrees sum to, scattered and contended at
// hubs, so it is taken only for groups whose bound on that sum (below) is at
// most nnz/32; the dense step gathers every arc.
static int64_t push3_max_arcs(const ged_graph *g) { return g->nnz / 32; }

// Worklist entries the push can need: each source has an arc, so at most one
// per arc plus one per further 512 arcs.
static size_t push3_cap(const ged_graph *g) {
  const int64_t v = push3_max_arcs(g);
  return (size_t)std::min<int64_t>(v + v / kWlChunk + 2, 0xffffffffll);
}

const std::vector<double> &omega2_host(ged_graph *g, hipStream_t st) {
  if (g->h_omega2.size() == (size_t)g->n) return g->h_omega2;
  const size_t n = (size_t)g->n;
  {
    std::lock_guard<std::mutex> lk(g_omega_mu);
    ensure_omega2(g, st);
  }
  std::vector<unsigned long long> om2(n);
  GED_HIP(hipMemcpyAsync(om2.data(), g->omega2.p, sizeof(unsigned long long) * n,
                         hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  std::vector<double> h(n);
  for (size_t v = 0; v < n; ++v) h[v] = (double)om2[v];
  g->h_omega2.swap(h);
  return g->h_omega2;
}

int least_c16_hub(ged_graph *g, hipStream_t st) {
  if (g->c16_least_hub >= 0) return g->c16_least_hub;
  const std::vector<double> &om2 = omega2_host(g, st);
  int64_t last = -1;
  for (int64_t v = 0; v < g->n; ++v)
    if (om2[(size_t)v] > (double)kC16Max) last = v;
  g->c16_least_hub = (int)(last + 1);
  return g->c16_least_hub;
}

int split_c16_hub(ged_graph *g, const SplitPlan &pl, int C, hipStream_t st) {
  if (g->count16 < 0 || g->weighted || !split_ok(g) || C < 4) return -1;
  if (!pl.c32 || pl.s != 2 || pl.push3 || !(pl.lv32 || pl.nlv == 0)) return -1;
  const int least = least_c16_hub(g, st);
  if (g->count16 > 0) return g->count16;  // checked against least when set
  return (int64_t)least * 8 <= g->n && least < g->n ? least : -1;
}

// Host table of deg(v) + omega_2(v) + omega_3(v), which bounds the degrees
// added by the sources v contributes: its neighbours (2-walks from v) and the
// ends of its 2-walks (3-walks); members count themselves (deg).
static void ensure_push_bound(ged_graph *g, hipStream_t st) {
  if (g->push_bound.size() == (size_t)g->n) return;
  const size_t n = (size_t)g->n;
  const std::vector<double> &om2 = omega2_host(g, st);
  std::vector<double> om3(n);
  const void *lv;
  {
    std::lock_guard<std::mutex> lk(g_omega_mu);
    lv = g->omega_lv.p;  // a replaced table stays allocated with the graph
  }
  GED_HIP(hipMemcpyAsync(om3.data(), lv, sizeof(double) * n, hipMemcpyDeviceToHost,
                         st));  // omega_3 is level 0 of the table
  GED_HIP(hipStreamSynchronize(st));
  std::vector<double> b(n);
  for (size_t v = 0; v < n; ++v)
    b[v] = (double)(g->h_rp[v + 1] - g->h_rp[v]) + om2[v] + om3[v];
  g->push_bound.swap(b);
}

// omega_i(v) on the host, for a level i >= 3 that the graph's integer chain
// holds (level i - 3 of omega_lv); copied once.
static const std::vector<double> &omega_level_host(ged_graph *g, int i, hipStream_t st) {
  auto it = g->h_omega_lv.find(i);
  if (it != g->h_omega_lv.end()) return it->second;
  const size_t n = (size_t)g->n;
  std::vector<double> h(n);
  const void *lv;
  {
    std::lock_guard<std::mutex> lk(g_omega_mu);
    lv = g->omega_lv.p;  // a replaced table stays allocated with the graph
  }
  GED_HIP(hipMemcpyAsync(h.data(), static_cast<const double *>(lv) + (size_t)(i - 3) * n,
                         sizeof(double) * n, hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  return g->h_omega_lv[i] = std::move(h);
}

// Per-group 32-bit stored levels (single scores on graphs whose omega maxima
// do not fit 32 bits).  A walk of length i that ends at v and meets S can be
// cut after its last member s, at position j < i (v itself is a member only
// on the member rows, which hold omega_i(v), the j = 0 term): a walk of
// length j ending at s followed by one of length i - j leaving s, so the
// level-i count at any row is at most
//   sum_{s in S} sum_{j=0}^{i-1} omega_j(s) omega_{i-j}(s)
// (omega_0 = 1; walks leaving s are walks ending at s reversed).  When that
// is below 2^32 for every stored level (and the graph holds omega up to the
// top stored level, for the member rows), the levels are stored as exact
// 32-bit counts as for graphs whose maxima fit.
static bool group_levels_fit32(ged_graph *g, const SplitPlan &pl, const std::vector<int> &mem,
                               hipStream_t st) {
  const int top = pl.a - 1;
  if (pl.nlv <= 0 || pl.s != 2 || !pl.c32 || g->weighted || top < 3) return false;
  {
    std::lock_guard<std::mutex> lk(g_omega_mu);
    if (g->omega_top < top || g->omega_exact < top) return false;
  }
  const std::vector<double> &om2 = omega2_host(g, st);
  std::vector<const std::vector<double> *> om((size_t)top + 1, nullptr);
  for (int i = 3; i <= top; ++i) om[i] = &omega_level_host(g, i, st);
  auto w = [&](int j, int v) -> double {
    if (j == 0) return 1.0;
    if (j == 1) return (double)(g->h_rp[v + 1] - g->h_rp[v]);
    return j == 2 ? om2[(size_t)v] : (*om[j])[(size_t)v];
  };
  for (int i = pl.s + 1; i <= top; ++i) {
    double b = 0.0;
    for (int v : mem)
      for (int j = 0; j < i; ++j) b += w(j, v) * w(i - j, v);
    if (!(b < 0.999 * 4294967296.0)) return false;
  }
  return true;
}

void split_fit(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, size_t wl_need,
               hipStream_t st, bool counts_only) {
  const size_t nC = (size_t)g->n * C;
  const bool dirty = !w.zero;
  if (!counts_only) {
    w.ws.fit(partition(g, C, false, pl.cut_div));
    if (pl.s >= 1 && pl.c32) w.ws.fit(step_partition(g, pl, C, IN_CNT32));
    if (pl.c16_hub >= 0) w.ws.fit(step_partition(g, pl, C, IN_CNT16));
  }
  if (pl.s >= 1) {
    const size_t cb = (pl.c32 ? sizeof(uint32_t) : sizeof(uint64_t)) * nC;
    // the 16-bit layout's packed part starts on a 256-byte boundary, which on
    // a tiny graph can reach past 4nC bytes
    const size_t cb2 = pl.c16_hub >= 0 ? std::max(cb, c16_bytes(g->n, pl.c16_hub, C)) : cb;
    if (w.cnt1.bytes < cb || w.cnt2.bytes < cb2) {
      w.cnt1.ensure(cb);
      w.cnt2.ensure(cb2);
      w.zero = false;
    }
    if (!w.zero || w.cnt_bytes != cb) {
      launch_fill_i32(w.cnt1.as<int>(), 0, w.cnt1.bytes / sizeof(int), st);
      launch_fill_i32(w.cnt2.as<int>(), 0, w.cnt2.bytes / sizeof(int), st);
      w.wl_n.ensure(sizeof(unsigned));
      launch_fill_i32(w.wl_n.as<int>(), 0, 1, st);
      w.cnt_bytes = cb;
      w.zero = true;
    }
    if (pl.s >= 2 && (wl_need > w.wl_cap || !w.wl.p)) {
      size_t cap = std::max<size_t>(wl_need, 2 * (size_t)w.wl_cap);
      cap = std::min<size_t>(cap, 0xffffffffu);
      w.wl.ensure(sizeof(uint64_t) * cap);
      w.wl_cap = (unsigned)cap;
    }
  }
  if (pl.nlv > 0 && !counts_only) {
    const void *old = w.lv.p;
    w.lv.ensure((pl.lv32 ? sizeof(uint32_t) : sizeof(double)) * nC * (size_t)pl.nlv);
    if (w.lv.p != old) w.lv_zero = false;
    if (pl.c16_hub >= 0) w.lv16.ensure(sizeof(uint16_t) * nC);
  }
  if (pl.push3) {
    const size_t cap = push3_cap(g);
    if (w.wl3_cap < cap || !w.wl3.p) {
      w.wl3.ensure(sizeof(uint64_t) * cap);
      w.wl3_cap = (unsigned)cap;
    }
    if (!w.wl3_n.p) {
      w.wl3_n.ensure(sizeof(unsigned));
      w.lv_zero = false;
    }
    if (dirty || !w.lv_zero) {
      launch_fill_i32(w.lv.as<int>(), 0, nC, st);  // the first stored level (uint32)
      launch_fill_i32(w.wl3_n.as<int>(), 0, 1, st);
      w.lv_zero = true;
    }
  }
}

// Partitions and partial buffers for tiles of width C in a workspace whose
// counts were fitted for a wider tile: the counts, levels and worklists of a
// narrower tile use the first n * C entries of the same buffers.
void split_fit_width(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C) {
  w.ws.fit(partition(g, C, false, pl.cut_div));
  if (pl.s >= 1 && pl.c32) w.ws.fit(step_partition(g, pl, C, IN_CNT32));
  if (pl.c16_hub >= 0) w.ws.fit(step_partition(g, pl, C, IN_CNT16));
  w.ws.fit(step_partition(g, pl, C, final_in(pl)));
}

template <class CT>
static void push_phase(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, const int64_t *offs,
                       const int *mem, const int *mcol, int g0, int nc, int mgrid,
                       int64_t tile_members, const uint64_t *tmask, hipStream_t st) {
  const int *rp = g->rp.as<const int>(), *ci = g->ci.as<const int>();
  CT *c1 = w.cnt1.as<CT>();
  CT *c2 = pl.s >= 2 ? w.cnt2.as<CT>() : nullptr;
  // pushed level 3: 32-bit counts only (push3 implies lv32, hence CT = uint32)
  CT *l3 = pl.push3 ? w.lv.as<CT>() : nullptr;
  uint64_t *wl3 = l3 ? w.wl3.as<uint64_t>() : nullptr;
  unsigned *wl3_n = l3 ? w.wl3_n.as<unsigned>() : nullptr;
  const int h16 = sizeof(CT) == 4 ? pl.c16_hub : -1;
  hipLaunchKernelGGL(k_push<CT>, dim3(mgrid), dim3(kBlock), 0, st, rp, ci, tmask, offs, mem,
                     mcol, g0, nc, C, c1, c2, w.wl.as<uint64_t>(), w.wl_n.as<unsigned>(),
                     w.wl_cap, wl3, wl3_n, w.wl3_cap, h16);
  GED_HIP(hipGetLastError());
  MemberFix<CT> fx;
  fx.rp = rp;
  fx.omega2 = g->omega2.as<const unsigned long long>();
  fx.offsets = offs;
  fx.members = mem;
  fx.mcol = mcol;
  fx.g0 = g0;
  fx.nc = nc;
  fx.C = C;
  fx.cnt1 = c1;
  fx.cnt2 = c2;
  fx.lv3 = l3;
  fx.om3 = l3 ? g->omega_lv.as<const double>() : nullptr;  // omega_3 is level 0
  fx.h16 = h16;
  if (c2) {  // level 2, with the member rows
    if (wl3)
      hipLaunchKernelGGL((k_push_wl<CT, false, true>), dim3(w.wl_blocks), dim3(kBlock), 0, st, rp,
                         ci, C, c1, c2, w.wl.as<const uint64_t>(), w.wl_n.as<const unsigned>(),
                         w.wl_cap, tmask, wl3, wl3_n, w.wl3_cap, fx, h16);
    else
      hipLaunchKernelGGL((k_push_wl<CT, false, false>), dim3(w.wl_blocks), dim3(kBlock), 0, st,
                         rp, ci, C, c1, c2, w.wl.as<const uint64_t>(),
                         w.wl_n.as<const unsigned>(), w.wl_cap, tmask, (uint64_t *)nullptr,
                         (unsigned *)nullptr, 0u, fx, h16);
  } else {
    hipLaunchKernelGGL(k_fix_members<CT>, dim3(grid_for((tile_members + kBlock - 1) / kBlock, 256)),
                       dim3(kBlock), 0, st, fx);
  }
  GED_HIP(hipGetLastError());
  if (l3) {  // level 3 from every vertex holding a level-2 count
    hipLaunchKernelGGL((k_push_wl<CT, false, false>), dim3(kWl3Grid), dim3(kBlock), 0, st, rp, ci, C,
                       static_cast<const CT *>(c2), l3, w.wl3.as<const uint64_t>(),
                       w.wl3_n.as<const unsigned>(), w.wl3_cap, tmask, (uint64_t *)nullptr,
                       (unsigned *)nullptr, 0u, MemberFix<CT>(), -1);
    GED_HIP(hipGetLastError());
  }
}

template <class CT>
static void clear_phase(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C,
                        const int64_t *offs, const int *mem, const int *mcol, int g0, int nc,
                        int mgrid, uint64_t *tmask, hipStream_t st) {
  const int *rp = g->rp.as<const int>(), *ci = g->ci.as<const int>();
  CT *c1 = w.cnt1.as<CT>();
  CT *c2 = pl.s >= 2 ? w.cnt2.as<CT>() : nullptr;
  CT *l3 = pl.push3 ? w.lv.as<CT>() : nullptr;
  const int h16 = sizeof(CT) == 4 ? pl.c16_hub : -1;
  if (l3) {  // level-2 and pushed level-3 targets in one launch
    hipLaunchKernelGGL(k_clear_two<CT>, dim3(kWl3Grid), dim3(kBlock), 0, st, rp, ci, C, c2,
                       w.wl.as<const uint64_t>(), w.wl_n.as<const unsigned>(), w.wl_cap, l3,
                       w.wl3.as<const uint64_t>(), w.wl3_n.as<const unsigned>(), w.wl3_cap);
    GED_HIP(hipGetLastError());
  } else if (c2) {
    hipLaunchKernelGGL((k_push_wl<CT, true, false>), dim3(w.wl_blocks), dim3(kBlock), 0, st, rp, ci, C,
                       c1, c2, w.wl.as<const uint64_t>(), w.wl_n.as<const unsigned>(), w.wl_cap,
                       tmask, (uint64_t *)nullptr, (unsigned *)nullptr, 0u, MemberFix<CT>(),
                       h16);
    GED_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_clear_members<CT>, dim3(mgrid), dim3(kBlock), 0, st, rp, ci, offs, mem,
                     mcol, g0, nc, C, c1, c2, l3, reinterpret_cast<unsigned long long *>(tmask),
                     c2 ? w.wl_n.as<unsigned>() : nullptr, l3 ? w.wl3_n.as<unsigned>() : nullptr,
                     h16);
  GED_HIP(hipGetLastError());
}

void split_dense(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, const uint64_t *tmask,
                 hipStream_t st, bool profile, const SplitWs *counts) {
  const int64_t n = g->n;
  const size_t nC = (size_t)n * C;
  const PrepCache &pc = g->prep;
  const double alpha = pc.alpha;
  Partition &p = partition(g, C, false, pl.cut_div);
  Partition &pn = step_partition(g, pl, C, IN_CNT32);  // 32-bit gathers (count levels)
  const double *T = pc.t_levels.as<const double>();
  const SplitWs &cw = counts ? *counts : w;
  const void *c1 = pl.s >= 1 ? cw.cnt1.p : nullptr;
  const void *c2 = pl.s >= 2 ? cw.cnt2.p : nullptr;
  double lv_scale = alpha;  // alpha^(s+1) for the first dense level after the counts
  for (int i = 0; i < pl.s; ++i) lv_scale *= alpha;
  double *lv = w.lv.as<double>();
  uint32_t *lv32 = w.lv.as<uint32_t>();
  StepArgs a = base_args(g);
  w.ws.into(a);
  a.C = C;
  a.tmask = tmask;
  a.accum = 0;
  // 16-bit level-2 counts: the level-3 gather reads them (IN_CNT16), the
  // combining step reads their rows (OUT_COMBINE16), and the last stored
  // level gets a 16-bit copy (OUT_TILE32H) that the combining step gathers
  const bool c16 = pl.c16_hub >= 0;
  const uint16_t *pk2 = nullptr;
  if (c16) {
    pk2 = reinterpret_cast<const uint16_t *>(static_cast<const char *>(c2) +
                                             c16_pk_offset(pl.c16_hub, C));
    a.q_pk2 = pk2;
    a.q_hub2 = pl.c16_hub;
    a.hub = pl.c16_hub;
    a.Xc16 = pk2;
  }
  if (pl.lv32) {
    // unscaled 32-bit counts for levels s+1 .. a-1 (members: omega_i), then
    // h_a = alpha^a * (sum of level a-1 counts) in the combining step
    const double *om = g->omega_lv.as<const double>();
    double alpha_a = lv_scale;  // alpha^(s+1)
    for (int i = pl.s + 1; i < pl.a; ++i) alpha_a *= alpha;
    for (int i = pl.s + 1; i <= pl.a; ++i) {
      a.Xc32 = i == pl.s + 1 ? static_cast<const uint32_t *>(c2) : lv32 + (size_t)(i - 2 - pl.s) * nC;
      // level s+1 gathers the 16-bit level 2 (cut pl.c16_hub), the combining
      // step the 16-bit copy of level a-1 (cut 0, marked values from lv32)
      const bool g16 = c16 && (i == pl.s + 1 || i == pl.a);
      if (c16 && i == pl.a && i > pl.s + 1) {
        a.Xc16 = w.lv16.as<const uint16_t>();
        a.hub = 0;
      }
      const int in = g16 ? IN_CNT16 : IN_CNT32;
      Partition &pi = in == IN_CNT16 ? step_partition(g, pl, C, IN_CNT16) : pn;
      if (i < pl.a) {
        a.alpha = 1.0;
        a.inj = om + (size_t)(i - 3) * n;
        a.Y32 = lv32 + (size_t)(i - 1 - pl.s) * nC;
        const int out = c16 && i == pl.a - 1 ? OUT_TILE32H : OUT_TILE32;
        a.Y16 = w.lv16.as<uint16_t>();
        // the only stored level: the combining step reads it through the copy
        a.y32_marked = out == OUT_TILE32H && pl.nlv == 1 ? 1 : 0;
        if (pl.push3 && i == pl.s + 1) continue;  // pushed with the first levels
        if (profile)
          run_step(g, pi, a, in, out, st);
        else
          launch_step(pi, a, in, out, st);
      } else {
        a.alpha = alpha_a;
        a.inj = T + (size_t)i * n;
        a.Y = nullptr;
        a.Y32 = nullptr;
        a.tr = pc.tr.as<const double>();
        a.q_cnt1 = c1;
        a.q_cnt2 = c2;
        a.q_m1 = ~0ull;
        a.q_m2 = ~0ull;
        a.q_s1 = alpha;
        a.q_s2 = alpha * alpha;
        a.q_lv = lv32;
        a.q_mlv = ~0ull;
        a.q_slv = lv_scale;
        a.q_alpha = alpha;
        a.q_nlv = pl.nlv;
        a.q_even = pl.even ? 1 : 0;
        a.Y16 = nullptr;
        a.y32_marked = 0;
        const int out = c16 ? OUT_COMBINE16 : OUT_COMBINE32L;
        if (profile)
          run_step(g, pi, a, in, out, st,
                   c16 ? 0.75 + (pl.nlv == 1 ? 0.25 : 0.5 * pl.nlv) : 0.5 * (pl.s + pl.nlv));
        else
          launch_step(pi, a, in, out, st);
      }
    }
    return;
  }
  for (int i = pl.s + 1; i <= pl.a; ++i) {
    int in;
    if (i == 1) {
      in = IN_TILEMASK;
      a.alpha = alpha;
    } else if (i == pl.s + 1) {
      const void *src = pl.s == 1 ? c1 : c2;
      if (c16) {  // a = 3: the combining step gathers the 16-bit level 2
        in = IN_CNT16;
        a.Xc32 = static_cast<const uint32_t *>(src);
      } else if (pl.c32) {
        in = IN_CNT32;
        a.Xc32 = static_cast<const uint32_t *>(src);
      } else {
        in = IN_CNT;
        a.Xc = static_cast<const uint64_t *>(src);
      }
      a.alpha = lv_scale;
    } else {
      in = IN_VEC;
      a.X = lv + (size_t)(i - 2 - pl.s) * nC;
      a.alpha = alpha;
    }
    a.inj = T + (size_t)i * n;
    Partition &ps = in == IN_CNT16 ? step_partition(g, pl, C, IN_CNT16) : in == IN_CNT32 ? pn : p;
    if (i < pl.a) {
      a.Y = lv + (size_t)(i - 1 - pl.s) * nC;
      if (profile)
        run_step(g, ps, a, in, OUT_TILE, st);
      else
        launch_step(ps, a, in, OUT_TILE, st);
    } else {
      // absent inputs: index mask 0 into a valid buffer, weight 0
      const double *any = pc.tr.as<const double>();
      a.Y = nullptr;
      a.tr = pc.tr.as<const double>();
      a.q_cnt1 = c1 ? c1 : any;
      a.q_cnt2 = c2 ? c2 : any;
      a.q_m1 = c1 ? ~0ull : 0ull;
      a.q_m2 = c2 ? ~0ull : 0ull;
      a.q_s1 = c1 ? alpha : 0.0;
      a.q_s2 = c2 ? alpha * alpha : 0.0;
      a.q_lv = pl.nlv > 0 ? lv : any;
      a.q_mlv = pl.nlv > 0 ? ~0ull : 0ull;
      a.q_slv = pl.nlv > 0 ? 1.0 : 0.0;
      a.q_nlv = pl.nlv;
      a.q_even = pl.even ? 1 : 0;
      const int out = c16 ? OUT_COMBINE16 : (pl.c32 && pl.s >= 1) ? OUT_COMBINE32 : OUT_COMBINE;
      if (profile)
        run_step(g, ps, a, in, out, st, c16 ? 0.75 : pl.s * (pl.c32 ? 0.5 : 1.0) + pl.nlv);
      else
        launch_step(ps, a, in, out, st);
    }
  }
}

void split_tile_push(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, const int64_t *offs,
                     const int *mem, const int *mcol, int g0, int nc, int64_t tile_members,
                     uint64_t *tmask, hipStream_t st, bool set_tmask) {
  const int mgrid = grid_for(tile_members, kPushGrid);
  if (set_tmask) launch_tmask_set(tmask, offs, mem, g0, nc, 1, st);
  if (pl.s >= 1) {
    if (pl.c32)
      push_phase<unsigned>(g, w, pl, C, offs, mem, mcol, g0, nc, mgrid, tile_members, tmask, st);
    else
      push_phase<unsigned long long>(g, w, pl, C, offs, mem, mcol, g0, nc, mgrid, tile_members,
                                     tmask, st);
  }
}

// Replaying a push stores one zero per arc it wrote along, each to its own
// cache line (about 64 bytes of traffic); a fill writes the count levels of
// the tile's width once.  Replay while that is cheaper.
bool split_clear_by_fill(const ged_graph *g, const SplitPlan &pl, int C, double push2_arcs) {
  if (pl.s < 2 || pl.push3) return false;
  const double cb = pl.c32 ? 4.0 : 8.0;
  const double cb2 = pl.c16_hub >= 0 ? 2.0 : cb;  // level 2 in the 16-bit layout
  return push2_arcs * 64.0 > (double)g->n * C * (cb + cb2);
}

void split_tile_clear(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, const int64_t *offs,
                      const int *mem, const int *mcol, int g0, int nc, int64_t tile_members,
                      uint64_t *tmask, hipStream_t st, bool fill) {
  const int mgrid = grid_for(tile_members, kPushGrid);
  if (fill && pl.s >= 2 && !pl.push3) {
    // the two count levels of this width, the members' column bits and the
    // worklist length: everything the pushes wrote
    const size_t words = (size_t)g->n * C * (pl.c32 ? 1 : 2);
    launch_fill_i32(w.cnt1.as<int>(), 0, words, st);
    launch_fill_i32(w.cnt2.as<int>(), 0,
                    pl.c16_hub >= 0 ? (c16_bytes(g->n, pl.c16_hub, C) + 3) / 4 : words, st);
    launch_fill_i32(w.wl_n.as<int>(), 0, 1, st);
    launch_tmask_set(tmask, offs, mem, g0, nc, 0, st);
  } else if (pl.s >= 1) {  // clears the members' tmask bits too
    if (pl.c32)
      clear_phase<unsigned>(g, w, pl, C, offs, mem, mcol, g0, nc, mgrid, tmask, st);
    else
      clear_phase<unsigned long long>(g, w, pl, C, offs, mem, mcol, g0, nc, mgrid, tmask, st);
  } else {
    launch_tmask_set(tmask, offs, mem, g0, nc, 0, st);
  }
}

void split_tile_reduce(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, double *out,
                       hipStream_t st) {
  StepArgs a = base_args(g);
  w.ws.into(a);
  a.C = C;
  // the partials are laid out by the partition of the combining step
  launch_reduce(step_partition(g, pl, C, final_in(pl)), a, out, nullptr, nullptr, st,
                w.ws.scratch());
}

void enqueue_split_tile(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C,
                        const int64_t *offs, const int *mem, const int *mcol, int g0, int nc,
                        int64_t tile_members, uint64_t *tmask, double *out, hipStream_t st,
                        bool profile, bool fill_clear) {
  split_tile_push(g, w, pl, C, offs, mem, mcol, g0, nc, tile_members, tmask, st);
  split_dense(g, w, pl, C, tmask, st, profile);
  split_tile_reduce(g, w, pl, C, out, st);
  split_tile_clear(g, w, pl, C, offs, mem, mcol, g0, nc, tile_members, tmask, st, fill_clear);
}

int64_t map_group(ged_graph *g, const int32_t *S, int64_t len, std::vector<int> &out) {
  if (g->stamp.size() != (size_t)g->n) {
    g->stamp.assign((size_t)g->n, 0u);
    g->stamp_gen = 0;
  }
  if (++g->stamp_gen == 0) {
    std::fill(g->stamp.begin(), g->stamp.end(), 0u);
    g->stamp_gen = 1;
  }
  const uint32_t gen = g->stamp_gen;
  int64_t deg_sum = 0;
  for (int64_t q = 0; q < len; ++q) {
    const int v = g->new_id[S[q]];
    if (g->stamp[v] == gen) continue;
    g->stamp[v] = gen;
    out.push_back(v);
    deg_sum += g->h_rp[v + 1] - g->h_rp[v];
  }
  return deg_sum;
}

// ------------------------------------------------------- single group --

void SplitExec::drop() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (clear_exec) (void)hipGraphExecDestroy(clear_exec);
  if (clear_graph) (void)hipGraphDestroy(clear_graph);
  exec = clear_exec = nullptr;
  graph = clear_graph = nullptr;
  sig.clear();
}

template <class F>
static void capture(hipStream_t st, F &&enqueue, hipGraph_t *graph, hipGraphExec_t *exec) {
  GED_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    enqueue();
  } catch (...) {
    hipGraph_t dummy = nullptr;
    (void)hipStreamEndCapture(st, &dummy);
    if (dummy) (void)hipGraphDestroy(dummy);
    throw;
  }
  GED_HIP(hipStreamEndCapture(st, graph));
  GED_HIP(hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0));
}

int split_score(ged_graph *g, const int32_t *S, int32_t s_len, double *out) {
  hipStream_t st = g->stream;
  const int64_t n = g->n;
  SplitPlan pl = split_plan(g, g->prep.ell);
  std::vector<int> mem;
  mem.reserve((size_t)s_len);
  const int64_t deg_sum = map_group(g, S, s_len, mem);
  const int len = (int)mem.size();
  if (len > g->split_cap) {
    int cap = std::max(256, g->split_cap);
    while (cap < len) cap *= 2;
    const size_t bytes = 2 * sizeof(int64_t) + 2 * sizeof(int) * (size_t)cap;
    g->split_in.ensure(bytes);
    g->split_in_host.ensure(bytes, hipHostMallocCoherent);
    // mcol: every member is in column 0
    launch_fill_i32(reinterpret_cast<int *>(g->split_in.as<char>() + 2 * sizeof(int64_t)) + cap,
                    0, (size_t)cap, st);
    g->split_cap = cap;
  }
  if (!g->split_tmask.p || g->split_tmask.bytes < sizeof(uint64_t) * (size_t)n) {
    g->split_tmask.ensure(sizeof(uint64_t) * (size_t)n);
    g->split_tmask_ready = false;
  }
  if (!g->split_tmask_ready) {
    launch_fill_i32(g->split_tmask.as<int>(), 0, (size_t)n * 2, st);
    g->split_tmask_ready = true;
  }
  split_tables(g, pl, st);
  if (!pl.lv32 && group_levels_fit32(g, pl, mem, st)) pl.lv32 = true;
  if (pl.lv32 && pl.s == 2 && pl.nlv >= 1) {
    ensure_push_bound(g, st);
    double b = 0.0;
    for (int v : mem) b += g->push_bound[(size_t)v];
    pl.push3 = b <= (double)push3_max_arcs(g);
  }
  split_fit(g, g->split_ws, pl, 1, split_wl_need(g, deg_sum), st);
  // a fixed worklist grid, so the captured graph serves every group
  g->split_ws.wl_blocks = 256;
  // the score is reduced straight into coherent host memory (no copy)
  g->out_host.ensure(64, hipHostMallocCoherent);
  double *ho = g->out_host.as<double>();
  const int cap = g->split_cap;
  char *hb = g->split_in_host.as<char>();
  int64_t offs[2] = {0, len};
  std::memcpy(hb, offs, sizeof(offs));
  std::memcpy(hb + sizeof(offs), mem.data(), sizeof(int) * (size_t)len);
  // small groups are staged by the graph's first kernel (no copy launch);
  // larger ones are copied (a kernel reading thousands of members over the
  // host link would take longer)
  const bool staged = len <= kStageMembers;
  if (!staged)
    GED_HIP(hipMemcpyAsync(g->split_in.p, hb, sizeof(offs) + sizeof(int) * (size_t)len,
                           hipMemcpyHostToDevice, st));
  const int64_t *d_offs = g->split_in.as<const int64_t>();
  const int *d_mem = reinterpret_cast<const int *>(g->split_in.as<char>() + sizeof(offs));
  const int *d_mcol = d_mem + cap;
  SplitWs &w = g->split_ws;
  uint64_t *tm = g->split_tmask.as<uint64_t>();
  // The tile's clean-up (zeroing the counts and member bits) is enqueued after
  // the result copy and not waited for: any later work on this stream runs
  // after it, and ged_set_stream / ged_graph_destroy synchronize the stream.
  auto enqueue_main = [&]() {
    if (staged) {
      hipLaunchKernelGGL(k_stage_group, dim3(grid_for((len + kBlock - 1) / kBlock, 16)),
                         dim3(kBlock), 0, st, reinterpret_cast<const int64_t *>(hb),
                         reinterpret_cast<const int *>(hb + sizeof(offs)),
                         g->split_in.as<int64_t>(), const_cast<int *>(d_mem),
                         reinterpret_cast<unsigned long long *>(tm));
      GED_HIP(hipGetLastError());
    }
    split_tile_push(g, w, pl, 1, d_offs, d_mem, d_mcol, 0, 1, cap, tm, st, !staged);
    split_dense(g, w, pl, 1, tm, st);
    split_tile_reduce(g, w, pl, 1, ho, st);
  };
  auto enqueue_clear = [&]() {
    split_tile_clear(g, w, pl, 1, d_offs, d_mem, d_mcol, 0, 1, cap, tm, st);
  };
  if (!g->score_done) GED_HIP(hipEventCreateWithFlags(&g->score_done, hipEventDisableTiming));
  w.zero = false;
  try {
    if (g->prof.on) {
      enqueue_main();
      GED_HIP(hipEventRecord(g->score_done, st));
      enqueue_clear();
    } else {
      double ab = g->prep.alpha;
      const void *abits;
      std::memcpy(&abits, &ab, sizeof(ab));
      std::vector<const void *> sig = {
          g->split_tmask.p, w.cnt1.p, w.cnt2.p, w.lv.p, w.wl.p, w.wl_n.p, w.wl3.p, w.wl3_n.p,
          (const void *)(uintptr_t)w.wl3_cap, (const void *)(intptr_t)pl.push3, w.ws.blk.p, w.ws.seg.p,
          w.ws.lng.p, w.ws.red2.p, g->split_in.p, g->split_in_host.p, (const void *)(intptr_t)staged,
          g->prep.t_levels.p, g->prep.tr.p, g->omega2.p,
          g->omega_lv.p, g->out_host.p, (const void *)st, abits, (const void *)(intptr_t)g->prep.ell,
          (const void *)(intptr_t)cap, (const void *)(uintptr_t)w.wl_cap,
          (const void *)(intptr_t)1 /* split */, (const void *)(intptr_t)pl.lv32};
      SplitExec &x = g->split_exec[(pl.push3 ? 1 : 0) + (staged ? 2 : 0) + (pl.lv32 ? 4 : 0)];
      if (x.exec && sig != x.sig) x.drop();
      if (!x.exec) {
        capture(st, enqueue_main, &x.graph, &x.exec);
        capture(st, enqueue_clear, &x.clear_graph, &x.clear_exec);
        x.sig = sig;
      }
      GED_HIP(hipGraphLaunch(x.exec, st));
      GED_HIP(hipEventRecord(g->score_done, st));
      GED_HIP(hipGraphLaunch(x.clear_exec, st));
    }
  } catch (...) {
    g->split_tmask_ready = false;  // member bits may be left set
    throw;
  }
  w.zero = true;  // the clean-up is queued ahead of any later work on the stream
  // a dense first stored level leaves its values; the pushed one is cleared
  if (pl.nlv > 0) w.lv_zero = pl.push3;
  GED_HIP(hipEventSynchronize(g->score_done));
  *out = ho[0];
  return GED_OK;
}

}  // namespace ged
