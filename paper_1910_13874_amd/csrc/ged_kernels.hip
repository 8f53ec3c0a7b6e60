// Walk-count step kernels for gfx950 (wave64, FP64).
//
// Every recurrence of the method is one "step": for each vertex v and each of
// C columns, y(v, c) = alpha * sum_{u in N_in(v)} w(u,v) x(u, c), followed by a
// per-row epilogue that masks group members or injects values (Section 3.1.1
// recurrences; the hit, miss and gain chains differ only in the epilogue), and
// a column sum (Eq. phisum).  The step is HBM-bound: per launch it streams
// row_ptr and col_idx once and reads/writes the C-column dense vectors.
//
// Layout of one launch:
//   * row blocks: consecutive rows with at most kLdsDoubles/C arcs.  The block
//     streams its slice of col_idx coalesced, gathers x(u, 0..C-1) into LDS,
//     then sums each row from LDS with 1..64 lanes per (row, column) chosen
//     from the block's row count, reduces lanes with DPP/bpermute shuffles and
//     writes the masked output coalesced.  Column partial sums of the block go
//     to blk_part in a fixed tree order.
//   * long rows (more arcs than a row block holds, the power-law hubs): split
//     into fixed segments, one block each, whose raw sums go to seg_out; a
//     fix-up kernel adds the segments of each row in order.
//   * a reduction kernel sums the block and long-row partials of each column
//     in a fixed order.
// No floating-point atomics anywhere, so results are bitwise reproducible.
#include <algorithm>

#include "ged_internal.h"

namespace ged {

__device__ __forceinline__ bool bit_of(const uint32_t *m, int v) {
  return (m[v >> 5] >> (v & 31)) & 1u;
}

template <int C, int IN>
__device__ __forceinline__ double load_in(const StepArgs &a, int u, int c) {
  if constexpr (IN == IN_VEC) {
    return a.X[(size_t)u * C + c];
  } else if constexpr (IN == IN_ONES) {
    return 1.0;
  } else if constexpr (IN == IN_NOTMASK) {
    return bit_of(a.smask, u) ? 0.0 : 1.0;
  } else if constexpr (IN == IN_MASK) {
    return bit_of(a.smask, u) ? 1.0 : 0.0;
  } else if constexpr (IN == IN_TILEMASK) {
    return ((a.tmask[u] >> c) & 1ull) ? 1.0 : 0.0;
  } else if constexpr (IN == IN_ONEHOT) {
    return (a.cand_col[u] == c) ? 1.0 : 0.0;
  } else {  // IN_FRESH
    return a.fresh[c] ? (((a.tmask[u] >> c) & 1ull) ? 1.0 : 0.0) : a.X[(size_t)u * C + c];
  }
}

template <int C, int OUT>
__device__ __forceinline__ double epilogue(const StepArgs &a, int v, int c, double sum) {
  const double y = a.alpha * sum;
  if constexpr (OUT == OUT_PLAIN) {
    return y;
  } else if constexpr (OUT == OUT_INJ) {
    return bit_of(a.smask, v) ? a.inj[v] : y;
  } else if constexpr (OUT == OUT_ZERO) {
    return bit_of(a.smask, v) ? 0.0 : y;
  } else if constexpr (OUT == OUT_TILE) {
    return ((a.tmask[v] >> c) & 1ull) ? a.inj[v] : y;
  } else if constexpr (OUT == OUT_GAIN) {
    return bit_of(a.smask, v) ? 0.0 : (a.cand_col[v] == c ? a.inj[v] : y);
  } else {  // OUT_POOL
    const int s = a.col_step[c];
    if (s <= 0) return 0.0;
    return ((a.tmask[v] >> c) & 1ull) ? a.inj[(size_t)s * a.n + v] : y;
  }
}

template <int C, int IN, int OUT, bool WGT>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a, const int2 *__restrict__ blocks,
                                                 const int4 *__restrict__ segs, int n_blocks) {
  __shared__ double vals[kLdsDoubles];
  __shared__ double red[kBlock];
  constexpr int LPC = kBlock / C;  // lanes per column in reductions
  const int t = threadIdx.x;
  const int b = blockIdx.x;
  if (b < n_blocks) {
    const int2 rr = blocks[b];
    const int r0 = rr.x, r1 = rr.y;
    const int p0 = a.rp[r0];
    const int tot = (a.rp[r1] - p0) * C;
    // Phase 1: coalesced col_idx stream, gather x(u, c) into LDS.  Four
    // independent gathers per thread are kept in flight.
    int f = t;
    for (; f + 3 * kBlock < tot; f += 4 * kBlock) {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ff = f + q * kBlock;
        const int j = p0 + ff / C;
        v[q] = load_in<C, IN>(a, a.ci[j], ff & (C - 1));
        if constexpr (WGT) v[q] *= a.w[j];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) vals[f + q * kBlock] = v[q];
    }
    for (; f < tot; f += kBlock) {
      const int j = p0 + f / C;
      double v = load_in<C, IN>(a, a.ci[j], f & (C - 1));
      if constexpr (WGT) v *= a.w[j];
      vals[f] = v;
    }
    __syncthreads();
    // Phase 2: tpr lanes per (row, column).
    const int nrows = r1 - r0;
    int tpr = (LPC < 64) ? LPC : 64;
    while (tpr > 1 && nrows * C * tpr > kBlock) tpr >>= 1;
    const int s = t & (tpr - 1);
    const int pair = t / tpr;
    const int c = pair & (C - 1);
    const int rstep = (kBlock / tpr) / C;
    double colsum = 0.0;
    for (int rl = pair / C; rl < nrows; rl += rstep) {
      const int r = r0 + rl;
      const int j0 = a.rp[r] - p0, j1 = a.rp[r + 1] - p0;
      double acc = 0.0;
      for (int j = j0 + s; j < j1; j += tpr) acc += vals[j * C + c];
      for (int off = tpr >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (s == 0) {
        const double y = epilogue<C, OUT>(a, r, c, acc);
        a.Y[(size_t)r * C + c] = y;
        colsum += y;
      }
    }
    // Column partials: each column's 256/C lanes reduced in a fixed tree.
    const int k = (pair / C) * tpr + s;
    red[c * LPC + k] = colsum;
    __syncthreads();
    for (int st = LPC >> 1; st > 0; st >>= 1) {
      if (k < st) red[c * LPC + k] += red[c * LPC + k + st];
      __syncthreads();
    }
    if (k == 0) a.blk_part[(size_t)b * C + c] = red[c * LPC];
  } else {
    // One segment of a long row: LPC lanes per column stride over its arcs.
    const int4 sd = segs[b - n_blocks];
    const int c = t & (C - 1);
    const int s = t / C;
    double acc0 = 0.0, acc1 = 0.0;
    int j = sd.y + s;
    for (; j + LPC < sd.z; j += 2 * LPC) {
      double v0 = load_in<C, IN>(a, a.ci[j], c);
      double v1 = load_in<C, IN>(a, a.ci[j + LPC], c);
      if constexpr (WGT) {
        v0 *= a.w[j];
        v1 *= a.w[j + LPC];
      }
      acc0 += v0;
      acc1 += v1;
    }
    if (j < sd.z) {
      double v0 = load_in<C, IN>(a, a.ci[j], c);
      if constexpr (WGT) v0 *= a.w[j];
      acc0 += v0;
    }
    red[c * LPC + s] = acc0 + acc1;
    __syncthreads();
    for (int st = LPC >> 1; st > 0; st >>= 1) {
      if (s < st) red[c * LPC + s] += red[c * LPC + s + st];
      __syncthreads();
    }
    if (s == 0) a.seg_out[(size_t)(b - n_blocks) * C + c] = red[c * LPC];
  }
}

// Long rows: add the segment sums of each row in segment order, apply the
// epilogue, and keep the output for the column sums.
template <int C, int OUT>
__global__ __launch_bounds__(kBlock) void k_fixup(StepArgs a, const int *__restrict__ long_rows,
                                                  const int *__restrict__ long_first, int n_long) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int l = gid / C, c = gid & (C - 1);
  if (l >= n_long) return;
  const int r = long_rows[l];
  double acc = 0.0;
  for (int q = long_first[l]; q < long_first[l + 1]; ++q) acc += a.seg_out[(size_t)q * C + c];
  const double y = epilogue<C, OUT>(a, r, c, acc);
  a.Y[(size_t)r * C + c] = y;
  a.long_part[(size_t)l * C + c] = y;
}

// One block per column: fixed-order sum of block and long-row partials.
__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ blk_part, int nb,
                                                   const double *__restrict__ long_part, int nl,
                                                   int C, double *level, double *acc,
                                                   const int *active) {
  __shared__ double red[kBlock];
  const int c = blockIdx.x;
  if (active && active[c] == 0) return;
  const int t = threadIdx.x;
  double s = 0.0;
  for (int i = t; i < nb; i += kBlock) s += blk_part[(size_t)i * C + c];
  double s2 = 0.0;
  for (int i = t; i < nl; i += kBlock) s2 += long_part[(size_t)i * C + c];
  red[t] = s + s2;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  if (t == 0) {
    const double tot = red[0];
    if (level) level[c] = tot;
    if (acc) acc[c] += tot;
  }
}

// ------------------------------------------------------------ dispatch --

template <int C, int IN, int OUT, bool WGT>
static void launch_t(const Partition &p, const StepArgs &a, hipStream_t st) {
  const int grid = p.n_blocks + p.n_segs;
  if (grid > 0)
    hipLaunchKernelGGL((k_step<C, IN, OUT, WGT>), dim3(grid), dim3(kBlock), 0, st, a,
                       p.blocks.as<const int2>(), p.segs.as<const int4>(), p.n_blocks);
  if (p.n_long > 0) {
    const int thr = p.n_long * C;
    hipLaunchKernelGGL((k_fixup<C, OUT>), dim3((thr + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       a, p.long_rows.as<const int>(), p.long_first.as<const int>(), p.n_long);
  }
}

template <int C, bool WGT>
static bool dispatch_multi(int in, int out, const Partition &p, const StepArgs &a,
                           hipStream_t st) {
#define GED_CASE(I, O)                  \
  if (in == I && out == O) {            \
    launch_t<C, I, O, WGT>(p, a, st);   \
    return true;                        \
  }
  GED_CASE(IN_TILEMASK, OUT_TILE)
  GED_CASE(IN_VEC, OUT_TILE)
  GED_CASE(IN_ONEHOT, OUT_GAIN)
  GED_CASE(IN_VEC, OUT_GAIN)
  GED_CASE(IN_FRESH, OUT_POOL)
  if constexpr (C == 1) {
    GED_CASE(IN_ONES, OUT_PLAIN)
    GED_CASE(IN_VEC, OUT_PLAIN)
    GED_CASE(IN_MASK, OUT_INJ)
    GED_CASE(IN_VEC, OUT_INJ)
    GED_CASE(IN_NOTMASK, OUT_ZERO)
    GED_CASE(IN_VEC, OUT_ZERO)
  }
#undef GED_CASE
  return false;
}

template <bool WGT>
static bool dispatch_c(int C, int in, int out, const Partition &p, const StepArgs &a,
                       hipStream_t st) {
  switch (C) {
    case 1: return dispatch_multi<1, WGT>(in, out, p, a, st);
    case 2: return dispatch_multi<2, WGT>(in, out, p, a, st);
    case 4: return dispatch_multi<4, WGT>(in, out, p, a, st);
    case 8: return dispatch_multi<8, WGT>(in, out, p, a, st);
    case 16: return dispatch_multi<16, WGT>(in, out, p, a, st);
    case 32: return dispatch_multi<32, WGT>(in, out, p, a, st);
    case 64: return dispatch_multi<64, WGT>(in, out, p, a, st);
    default: return false;
  }
}

void launch_step(const Partition &p, const StepArgs &a, int in_mode, int out_mode,
                 hipStream_t st) {
  if (a.C != p.C) throw HipError{GED_ERR_ARG, "step column count does not match partition"};
  const bool ok = a.w ? dispatch_c<true>(a.C, in_mode, out_mode, p, a, st)
                      : dispatch_c<false>(a.C, in_mode, out_mode, p, a, st);
  if (!ok)
    throw HipError{GED_ERR_ARG, "no step kernel for C=" + std::to_string(a.C) + " in=" +
                                    std::to_string(in_mode) + " out=" + std::to_string(out_mode)};
  GED_HIP(hipGetLastError());
}

void launch_reduce(const Partition &p, const StepArgs &a, double *level, double *acc,
                   const int *active, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(a.C), dim3(kBlock), 0, st, a.blk_part, p.n_blocks,
                     a.long_part, p.n_long, a.C, level, acc, active);
  GED_HIP(hipGetLastError());
}

// ----------------------------------------------------------- partition --

void build_partition(Partition &p, const std::vector<int> &rp, int C) {
  const int n = (int)rp.size() - 1;
  const int nnz_blk = kLdsDoubles / C;
  const int seg_len = std::max(1, kSegDoubles / C);
  std::vector<int2> blocks;
  std::vector<int4> segs;
  std::vector<int> lrows, lfirst;
  int r = 0;
  while (r < n) {
    const int deg = rp[r + 1] - rp[r];
    if (deg > nnz_blk) {
      const int l = (int)lrows.size();
      lrows.push_back(r);
      lfirst.push_back((int)segs.size());
      for (int j = rp[r]; j < rp[r + 1]; j += seg_len)
        segs.push_back(make_int4(r, j, std::min(j + seg_len, rp[r + 1]), l));
      ++r;
      continue;
    }
    const int r0 = r;
    int acc = 0;
    while (r < n && r - r0 < kRowsPerBlock) {
      const int d = rp[r + 1] - rp[r];
      if (d > nnz_blk || acc + d > nnz_blk) break;
      acc += d;
      ++r;
    }
    blocks.push_back(make_int2(r0, r));
  }
  lfirst.push_back((int)segs.size());
  p.C = C;
  p.n_blocks = (int)blocks.size();
  p.n_segs = (int)segs.size();
  p.n_long = (int)lrows.size();
  p.blocks.ensure(sizeof(int2) * std::max<size_t>(1, blocks.size()));
  p.segs.ensure(sizeof(int4) * std::max<size_t>(1, segs.size()));
  p.long_rows.ensure(sizeof(int) * std::max<size_t>(1, lrows.size()));
  p.long_first.ensure(sizeof(int) * lfirst.size());
  if (!blocks.empty())
    GED_HIP(hipMemcpy(p.blocks.p, blocks.data(), sizeof(int2) * blocks.size(),
                      hipMemcpyHostToDevice));
  if (!segs.empty())
    GED_HIP(hipMemcpy(p.segs.p, segs.data(), sizeof(int4) * segs.size(), hipMemcpyHostToDevice));
  if (!lrows.empty())
    GED_HIP(hipMemcpy(p.long_rows.p, lrows.data(), sizeof(int) * lrows.size(),
                      hipMemcpyHostToDevice));
  GED_HIP(hipMemcpy(p.long_first.p, lfirst.data(), sizeof(int) * lfirst.size(),
                    hipMemcpyHostToDevice));
}

// -------------------------------------------------------- small kernels --

__global__ void k_fill_f64(double *p, double v, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i32(int *p, int v, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_copy_f64(double *dst, const double *src, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

static int fill_grid(size_t count) {
  size_t g = (count + kBlock - 1) / kBlock;
  return (int)std::max<size_t>(1, std::min<size_t>(g, 8192));
}

void launch_fill_f64(double *p, double v, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f64, dim3(fill_grid(count)), dim3(kBlock), 0, st, p, v, count);
  GED_HIP(hipGetLastError());
}

void launch_fill_i32(int *p, int v, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(count)), dim3(kBlock), 0, st, p, v, count);
  GED_HIP(hipGetLastError());
}

void launch_copy_f64(double *dst, const double *src, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f64, dim3(fill_grid(count)), dim3(kBlock), 0, st, dst, src, count);
  GED_HIP(hipGetLastError());
}

// S given as a device list whose length is read from device memory, so a
// captured graph can be replayed for any group up to `cap` members.
__global__ void k_mask_set(uint32_t *mask, const int *S, const int *s_len, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *s_len) return;
  const int v = S[i];
  const uint32_t bit = 1u << (v & 31);
  if (value)
    atomicOr(&mask[v >> 5], bit);
  else
    atomicAnd(&mask[v >> 5], ~bit);
}

void launch_mask_set(uint32_t *mask, const int *S, const int *s_len, int cap, int value,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_mask_set, dim3((std::max(cap, 1) + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     st, mask, S, s_len, value);
  GED_HIP(hipGetLastError());
}

// Column c of a tile holds group g0 + c: set (value=1) or clear bit c of
// tmask[v] for each member v.
__global__ void k_tmask_set(unsigned long long *tmask, const int64_t *offsets, const int *members,
                            int g0, int ncols, int value) {
  const int c = blockIdx.x;
  if (c >= ncols) return;
  const int64_t b = offsets[g0 + c], e = offsets[g0 + c + 1];
  const unsigned long long bit = 1ull << c;
  for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) {
    const int v = members[j];
    if (value)
      atomicOr(&tmask[v], bit);
    else
      atomicAnd(&tmask[v], ~bit);
  }
}

void launch_tmask_set(uint64_t *tmask, const int64_t *offsets, const int *members, int g0,
                      int ncols, int value, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_tmask_set, dim3(ncols), dim3(kBlock), 0, st,
                     reinterpret_cast<unsigned long long *>(tmask), offsets, members, g0, ncols,
                     value);
  GED_HIP(hipGetLastError());
}

__global__ void k_sum_levels(const double *levels, int count, double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < count; ++i) s += levels[i];
    *out = s;
  }
}

void launch_sum_levels(const double *levels, int count, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_levels, dim3(1), dim3(64), 0, st, levels, count, out);
  GED_HIP(hipGetLastError());
}

}  // namespace ged
