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
//     32-bit inputs at C >= 2 (integer walk counts) are gathered as pairs of
//     adjacent columns, 8 bytes per lane like an FP64 value, into blocks of
//     twice the arcs, so each wavefront keeps as many cache lines in flight;
//     16-bit level-2 counts (batch tiles, C >= 4) as units of four columns
//     into blocks of four times the arcs.  A block's LDS (16 KiB of staged
//     values plus a few words per row) is sized so that eight blocks fit a
//     CU: the random gathers are latency-bound, and more resident blocks
//     keep more of them in flight.
//   * long rows (more arcs than a row block holds, the power-law hubs): split
//     into fixed segments, one block each, whose raw sums go to seg_out; a
//     fix-up kernel adds the segments of each row in order.
//   * a reduction kernel sums the block and long-row partials of each column
//     in a fixed order.
// Combining epilogues (split scoring and split gains, undirected graphs) do not
// store y; they add, per (row, column), the combination of y with the lower
// levels of the chain to the column sums (combine_fin below).
// No floating-point atomics anywhere, so results are bitwise reproducible.
#include <algorithm>
#include <type_traits>

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
  } else if constexpr (IN == IN_FRESH) {
    return a.fresh[c] ? (((a.tmask[u] >> c) & 1ull) ? 1.0 : 0.0) : a.X[(size_t)u * C + c];
  } else if constexpr (IN == IN_CNT) {
    return (double)a.Xc[(size_t)u * C + c];
  } else if constexpr (IN == IN_CNT16) {
    return u < a.hub ? (double)a.Xc32[(size_t)u * C + c] : (double)a.Xc16[(size_t)u * C + c];
  } else {  // IN_CNT32
    return (double)a.Xc32[(size_t)u * C + c];
  }
}

// Columns 4k .. 4k+3 of row u of a 16-bit level (IN_CNT16), as 32-bit values:
// the packed row's 8 bytes, with -- rows below the hub cut, or the marked
// values of a unit holding any -- the counts from 16 bytes of the 32-bit level
// (long-row segments, which sum in registers).
template <int C>
__device__ __forceinline__ uint4 load_quad16(const StepArgs &a, int u, int k) {
  const uint2 p = *reinterpret_cast<const uint2 *>(a.Xc16 + (size_t)u * C + 4 * k);
  uint4 r = make_uint4(p.x & 0xffffu, p.x >> 16, p.y & 0xffffu, p.y >> 16);
  const bool marked = r.x == kC16Hub || r.y == kC16Hub || r.z == kC16Hub || r.w == kC16Hub;
  if (u < a.hub || marked) {
    // rows below the cut: every count; otherwise only the marked ones (the
    // 32-bit level may hold nothing else, see y32_marked)
    const uint4 h = *reinterpret_cast<const uint4 *>(a.Xc32 + (size_t)u * C + 4 * k);
    const bool all = u < a.hub;
    r.x = all || r.x == kC16Hub ? h.x : r.x;
    r.y = all || r.y == kC16Hub ? h.y : r.y;
    r.z = all || r.z == kC16Hub ? h.z : r.z;
    r.w = all || r.w == kC16Hub ? h.w : r.w;
  }
  return r;
}

// The packed 8 bytes of columns 4k .. 4k+3 of row u as staged in LDS: the
// row's four 16-bit counts; for a row below the hub cut its 32-bit counts,
// loaded with the other gathers, each staged as itself when it fits 16 bits
// (most do: the cut is a bound) and as kC16Hub when it does not.
template <int C>
__device__ __forceinline__ uint2 load_pk16(const StepArgs &a, int u, int k) {
  uint2 p = *reinterpret_cast<const uint2 *>(a.Xc16 + (size_t)u * C + 4 * k);
  if (u < a.hub) {
    const uint4 h = *reinterpret_cast<const uint4 *>(a.Xc32 + (size_t)u * C + 4 * k);
    auto m = [](uint32_t x) -> uint32_t { return x > kC16Max ? kC16Hub : x; };
    p = make_uint2(m(h.x) | (m(h.y) << 16), m(h.z) | (m(h.w) << 16));
  }
  return p;
}

// Row epilogue given the row's membership bit (S), column bits (tile/pool
// masks) and candidate column, which the caller has already fetched.
template <int C, int OUT>
__device__ __forceinline__ double epilogue_v(const StepArgs &a, int v, int c, double sum,
                                             bool inS, uint64_t tbits, int cand) {
  const double y = a.alpha * sum;
  if constexpr (OUT == OUT_PLAIN) {
    return y;
  } else if constexpr (OUT == OUT_INJ) {
    return inS ? a.inj[v] : y;
  } else if constexpr (OUT == OUT_ZERO) {
    return inS ? 0.0 : y;
  } else if constexpr (OUT == OUT_ZERO32) {
    return inS ? 0.0 : sum;  // the count; the caller also stores alpha * it
  } else if constexpr (OUT == OUT_TILE || OUT == OUT_COMBINE || OUT == OUT_COMBINE32 ||
                       OUT == OUT_TILE32 || OUT == OUT_COMBINE32L || OUT == OUT_COMBINE16 ||
                       OUT == OUT_TILE32H) {
    return ((tbits >> c) & 1ull) ? a.inj[v] : y;
  } else if constexpr (OUT == OUT_GAIN || OUT == OUT_GAINCOMB) {
    if (c >= a.spec_from) return (inS || cand == c - a.spec_from) ? 0.0 : y;  // miss column
    return inS ? 0.0 : (cand == c ? a.inj[v] : y);
  } else if constexpr (OUT == OUT_GAINCOMB32L || OUT == OUT_GAINCOMB32S) {
    return inS ? 0.0 : (cand == c ? a.inj[v] : y);
  } else if constexpr (OUT == OUT_GAIN32D) {
    if (c >= a.spec_from) return (inS || cand == c - a.spec_from) ? 0.0 : sum;  // miss column
    return inS ? 0.0 : (cand == c ? a.injc[c] : sum);  // the count
  } else if constexpr (OUT == OUT_GAIN32) {
    return inS ? 0.0 : (cand == c ? a.injc[c] : sum);  // the count
  } else {  // OUT_POOL
    const int s = a.col_step[c];
    if (s <= 0) return 0.0;
    return ((tbits >> c) & 1ull) ? a.inj[(size_t)s * a.n + v] : y;
  }
}

// Split scoring, last dense level a (undirected graphs).  Cutting a walk of
// length a + c after its first a arcs at vertex v: it meets S iff its first
// part does (h_a(v) of them, each continued by any of the t_c(v) walks of
// length c leaving v -- by symmetry the walks of length c ending at v), or
// its first part misses S (t_a(v) - h_a(v), zero for v in S) and its last c
// vertices meet S (again by reversal, h_c(v) for v outside S).  Summed over
// c = 1..r and added to levels 1..a, the row's share of the truncated score
// (Alg. "GED-Walk Computation") is
//   sum_{i<a} h_i + h_a + h_a * sum_{c<=r} t_c + [v not in S](t_a - h_a) * sum_{c<=r} h_c.
// Raw inputs of the combination for row v, column c: the two count levels,
// the first stored dense level, sum_{c<=r} t_c(v) and t_a(v).  Loads only, so
// they can be issued early and consumed later.  C32: the count levels are
// 32-bit.  LV32: the stored levels are unscaled 32-bit counts too, level l
// weighted by q_slv * q_alpha^l; otherwise they hold h_i itself (weight 1).
// C16: the level-2 counts are in the 16-bit layout (q_cnt2 is the hub table,
// q_pk2 the packed rows); both loads are issued, the one not needed at index 0.
template <int C, bool C32, bool LV32, bool C16 = false>
struct CombineIn {
  using CT = typename std::conditional<C32, uint32_t, uint64_t>::type;
  using LT = typename std::conditional<LV32, uint32_t, double>::type;
  CT c1 = 0, c2 = 0;
  LT lv0 = 0;
  uint16_t h0 = 0;  // C16 with one stored level: that level's 16-bit copy
  double trv = 0.0, ta = 0.0;
  // Wide tiles stream these rows once: nontemporal loads keep them from
  // displacing the gathered vector in the caches.
  __device__ __forceinline__ void load(const StepArgs &a, int v, int c) {
    const uint64_t o = (uint64_t)v * C + c;
    c1 = ld(static_cast<const CT *>(a.q_cnt1) + (o & a.q_m1));
    if constexpr (C16) {
      const bool hb = v < a.q_hub2;
      const CT h = ld(static_cast<const CT *>(a.q_cnt2) + (hb ? o : 0));
      const uint16_t pk = ld(a.q_pk2 + (hb ? 0 : o));
      c2 = hb ? h : (CT)pk;
    } else {
      c2 = ld(static_cast<const CT *>(a.q_cnt2) + (o & a.q_m2));
    }
    if constexpr (C16) {
      // one stored level: its 16-bit copy (the gathered Xc16) stands in for it,
      // and only its marked values are read from the 32-bit level (in q)
      const bool cp = a.q_nlv == 1;
      h0 = ld(a.Xc16 + (cp ? o : 0));
      lv0 = ld(static_cast<const LT *>(a.q_lv) + (cp ? 0 : (o & a.q_mlv)));
    } else {
      lv0 = ld(static_cast<const LT *>(a.q_lv) + (o & a.q_mlv));
    }
    trv = a.tr[v];
    ta = a.inj[v];
  }
  template <class T>
  static __device__ __forceinline__ T ld(const T *p) {
    if constexpr (C >= 8)
      return __builtin_nontemporal_load(p);
    else
      return *p;
  }
  // sum_{i<a} h_i(v) for column c (levels beyond the first stored one are
  // loaded here; there are none unless ell > 8)
  __device__ __forceinline__ double q(const StepArgs &a, int v, int c) const {
    const LT *lv = static_cast<const LT *>(a.q_lv);
    const size_t o = (size_t)v * C + c, ls = (size_t)a.n * C;
    LT l0 = lv0;
    if constexpr (C16)
      if (a.q_nlv == 1) l0 = h0 != kC16Hub ? (LT)h0 : lv[o];
    double s = (a.q_s1 * (double)c1 + a.q_s2 * (double)c2) + a.q_slv * (double)l0;
    double w = a.q_slv;
    int l = 1;
    for (; l + 3 < a.q_nlv; l += 4) {  // four loads in flight, added in level order
      const LT x0 = lv[l * ls + o], x1 = lv[(l + 1) * ls + o];
      const LT x2 = lv[(l + 2) * ls + o], x3 = lv[(l + 3) * ls + o];
      if constexpr (LV32) {
        w *= a.q_alpha;
        s += w * (double)x0;
        w *= a.q_alpha;
        s += w * (double)x1;
        w *= a.q_alpha;
        s += w * (double)x2;
        w *= a.q_alpha;
        s += w * (double)x3;
      } else {
        s += x0;
        s += x1;
        s += x2;
        s += x3;
      }
    }
    for (; l < a.q_nlv; ++l) {
      if constexpr (LV32) {
        w *= a.q_alpha;
        s += w * (double)lv[l * ls + o];
      } else {
        s += lv[l * ls + o];
      }
    }
    return s;
  }
};

template <int C, int OUT>
using CombineFor = CombineIn<C, OUT == OUT_COMBINE32 || OUT == OUT_COMBINE32L || OUT == OUT_COMBINE16,
                             OUT == OUT_COMBINE32L || OUT == OUT_GAINCOMB32L ||
                                 OUT == OUT_GAINCOMB32S || OUT == OUT_COMBINE16,
                             OUT == OUT_COMBINE16>;

// Output modes by property.
template <int OUT>
struct OutTraits {
  static constexpr bool gain = OUT == OUT_GAIN || OUT == OUT_GAINCOMB || OUT == OUT_GAIN32 ||
                               OUT == OUT_GAINCOMB32L || OUT == OUT_GAIN32D ||
                               OUT == OUT_GAINCOMB32S;  // S bits, candidates
  static constexpr bool gaincomb =
      OUT == OUT_GAINCOMB || OUT == OUT_GAINCOMB32L || OUT == OUT_GAINCOMB32S;
  // the combination's level count is stored as well (gain levels by counts)
  static constexpr bool cstore = OUT == OUT_GAINCOMB32S;
  static constexpr bool combine = OUT == OUT_COMBINE || OUT == OUT_COMBINE32 ||
                                  OUT == OUT_COMBINE32L || OUT == OUT_COMBINE16 ||
                                  gaincomb;  // y not stored
  static constexpr bool store32 = OUT == OUT_TILE32 || OUT == OUT_GAIN32 || OUT == OUT_TILE32H;
  static constexpr bool tile = OUT == OUT_TILE || OUT == OUT_POOL || OUT == OUT_COMBINE ||
                               OUT == OUT_COMBINE32 || OUT == OUT_TILE32 ||
                               OUT == OUT_COMBINE32L || OUT == OUT_COMBINE16 ||
                               OUT == OUT_TILE32H;  // per-vertex column bits (tmask)
};

// The count behind a gain combination's level value y (OUT_GAINCOMB32S): 0 on
// S (y = 0), the candidate's miss count at it (y = m_a = alpha^a times that
// count, exactly: it rounds back), else the gathered sum itself.
__device__ __forceinline__ uint32_t gain_count(const StepArgs &a, double y, double sum,
                                               bool cand) {
  return (uint32_t)(y == 0.0 ? 0.0 : (cand ? rint(y / a.alpha) : sum));
}

// y is h_a(v) (t_a(v) for v in S), q = sum_{i<a} h_i(v), trv = sum_{c<=r} t_c(v),
// ta = t_a(v).
__device__ __forceinline__ double combine_fin(const StepArgs &a, double q, double y, double trv,
                                              double ta, bool inS) {
  const double rs = a.q_even ? q + y : q;
  const double miss = inS ? 0.0 : (ta - y) * rs;
  return ((q + y) + y * trv) + miss;
}

template <int C, int OUT>
__device__ __forceinline__ double epilogue(const StepArgs &a, int v, int c, double sum) {
  constexpr bool M1 = OUT == OUT_INJ || OUT == OUT_ZERO || OUT == OUT_ZERO32 ||
                      OutTraits<OUT>::gain;
  constexpr bool TM = OutTraits<OUT>::tile;
  constexpr bool CA = OutTraits<OUT>::gain;
  return epilogue_v<C, OUT>(a, v, c, sum, M1 ? bit_of(a.smask, v) : false,
                            TM ? a.tmask[v] : 0ull, CA ? a.cand_col[v] : -1);
}

// Column sums of a block: lanes holding the same column are combined with
// butterfly shuffles inside each wavefront, then the four wavefront partials
// are added in a fixed order.  The thread -> column map is
// c = (t / tpr) & (C - 1) with tpr lanes per (row, column) pair; only lanes
// with s = t % tpr == 0 carry values.  red (4*C doubles) may hold anything:
// each wavefront first zeroes its own row, since its lanes may cover only
// part of the columns (a wavefront's LDS writes take effect in order).
template <int C>
__device__ __forceinline__ void block_colsum(double v, int tpr, double *red, double *out,
                                             int accum) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int o = 1; o < tpr; o <<= 1) v += __shfl_xor(v, o, 64);
  const int G = tpr * C;
  for (int o = G; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  if (lane < C) red[w * C + lane] = 0.0;
  if ((lane & (tpr - 1)) == 0 && lane < G) red[w * C + ((t / tpr) & (C - 1))] = v;
  __syncthreads();
  if (t < C) {
    const double bs = (red[t] + red[C + t]) + (red[2 * C + t] + red[3 * C + t]);
    out[t] = accum ? out[t] + bs : bs;
  }
}

// The same for lanes holding a pair of columns (2k, 2k+1), k = t % (C/2), one
// value each; every lane carries values (tpr = 1).
template <int C>
__device__ __forceinline__ void block_colsum_pairs(double v0, double v1, double *red,
                                                   double *out) {
  constexpr int CU = C / 2;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int o = CU; o < 64; o <<= 1) {
    v0 += __shfl_xor(v0, o, 64);
    v1 += __shfl_xor(v1, o, 64);
  }
  if (lane < CU) {
    red[w * C + 2 * lane] = v0;
    red[w * C + 2 * lane + 1] = v1;
  }
  __syncthreads();
  if (t < C) out[t] = (red[t] + red[C + t]) + (red[2 * C + t] + red[3 * C + t]);
}

// Per-row sum of staged integer counts (32-bit pairs or 16-bit units) over
// arcs j0 + s, j0 + s + tpr, .. < j1 of column c: four independent partials
// keep four LDS reads in flight, and integer sums are exact in any order, so
// the result is the exact count (converted once; exact below 2^53).  Q4: the
// partials are 32-bit (a block stages at most 2048 arcs of 16-bit values); a
// staged kC16Hub counts as 0 in the branch-free main loop, which only
// counts them, and a row that met any adds their 32-bit counts from Xc32 at
// the arc's source src[j].  With a cut (a.hub > 0) they can only be arcs
// from rows below it, which -- rows list their sources in increasing order,
// and those rows have the smallest ids -- come first in the row (and in
// every lane's share of it), so only that prefix is walked; marked values
// of a 16-bit copy (cut 0) may sit anywhere, so the row is scanned again.
template <int C, bool Q4, class SV>
__device__ __forceinline__ double sum_staged_counts(const StepArgs &a, const SV *vals, int j0,
                                                   int j1, int s, int tpr, int c,
                                                   const int *src) {
  using AT = typename std::conditional<Q4, uint32_t, uint64_t>::type;
  AT q0 = 0, q1 = 0, q2 = 0, q3 = 0;
  uint32_t nh = 0;
  auto keep = [](uint32_t x) -> uint32_t { return (Q4 && x == kC16Hub) ? 0u : x; };
  int j = j0 + s;
  for (; j + 3 * tpr < j1; j += 4 * tpr) {
    const uint32_t x0 = vals[j * C + c], x1 = vals[(j + tpr) * C + c];
    const uint32_t x2 = vals[(j + 2 * tpr) * C + c], x3 = vals[(j + 3 * tpr) * C + c];
    if constexpr (Q4)
      nh += (uint32_t)(x0 == kC16Hub) + (uint32_t)(x1 == kC16Hub) + (uint32_t)(x2 == kC16Hub) +
            (uint32_t)(x3 == kC16Hub);
    q0 += keep(x0);
    q1 += keep(x1);
    q2 += keep(x2);
    q3 += keep(x3);
  }
  for (; j < j1; j += tpr) {
    const uint32_t x = vals[j * C + c];
    if constexpr (Q4) nh += (uint32_t)(x == kC16Hub);
    q0 += keep(x);
  }
  uint64_t sum = (uint64_t)((q0 + q1) + (q2 + q3));
  if constexpr (Q4) {
    if (nh != 0) {
      if (a.hub > 0) {
        for (j = j0 + s; j < j1; j += tpr) {
          const int u = src[j];
          if (u >= a.hub) break;
          if (vals[j * C + c] == kC16Hub) sum += a.Xc32[(size_t)u * C + c];
        }
      } else {
        for (j = j0 + s; j < j1; j += tpr)
          if (vals[j * C + c] == kC16Hub) sum += a.Xc32[(size_t)src[j] * C + c];
      }
    }
  }
  return (double)sum;
}

// The same for lanes holding four columns (4k .. 4k+3), k = t % (C/4).
template <int C>
__device__ __forceinline__ void block_colsum_quads(const double (&v)[4], double *red, double *out) {
  constexpr int CQ = C / 4;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double x[4] = {v[0], v[1], v[2], v[3]};
  for (int o = CQ; o < 64; o <<= 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] += __shfl_xor(x[j], o, 64);
  }
  if (lane < CQ) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[w * C + 4 * lane + j] = x[j];
  }
  __syncthreads();
  if (t < C) out[t] = (red[t] + red[C + t]) + (red[2 * C + t] + red[3 * C + t]);
}

// Waves per SIMD the register allocation must allow (1: the compiler's
// choice).  The combining steps over 16-bit counts would take 68-70 VGPRs,
// i.e. seven waves; held to eight (64 VGPRs, no spill) they ran the 4,096-group
// BA-2M batch 7 % faster, the LDS of eight resident blocks of four waves
// fitting a CU.  The bound is not set on the other steps: those within 64
// VGPRs already are scheduled differently under it (the FP64 gain step lost
// 2 %), and the larger ones would spill.
template <int C, int IN, int OUT, bool WGT>
constexpr int step_waves() {
  return !WGT && IN == IN_CNT16 && OUT == OUT_COMBINE16 ? 8 : 1;
}

template <int C, int IN, int OUT, bool WGT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(step_waves<C, IN, OUT, WGT>())))
void k_step(StepArgs a, const int4 *__restrict__ blocks,
                                                 const int4 *__restrict__ segs, int n_blocks) {
  constexpr bool M1 = OUT == OUT_INJ || OUT == OUT_ZERO || OUT == OUT_ZERO32 ||
                      OutTraits<OUT>::gain;
  constexpr bool CB = OutTraits<OUT>::combine;
  constexpr bool TM = OutTraits<OUT>::tile;
  constexpr bool CA = OutTraits<OUT>::gain;
  // NP: 32-bit input gathered as column pairs; a gather unit is 8 bytes
  // either way (one FP64 value or two 32-bit values), CU units per arc
  constexpr bool NP = narrow_gather(C, IN, WGT);
  // Q4: 16-bit inputs (IN_CNT16) gathered as 8-byte units of four columns
  // and staged as 16-bit values (partition_quad: kLdsDoubles / (C/4) arcs)
  constexpr bool Q4 = IN == IN_CNT16 && C >= 4 && !WGT;
  constexpr int CU = NP ? C / 2 : C;
  constexpr int LV = lds_values(C);          // gather units staged per block
  constexpr int PT = LV / kBlock;            // gather units per thread
  constexpr int GU = Q4 ? C / 4 : CU;        // gather units per arc
  constexpr int RT = (kRowsPerBlock + kBlock) / kBlock;  // row_ptr entries per thread
  constexpr int RB = (kRowsPerBlock + kBlock - 1) / kBlock;  // rows per thread (masks)
  // HC: a single column of 32-bit counts; rows below hc_rows are read from
  // an LDS copy filled once per row block, and values are staged as 32 bits
  constexpr bool HC = C == 1 && IN == IN_CNT32 && !WGT;
  using SV = typename std::conditional<
      Q4, uint16_t, typename std::conditional<NP || HC, uint32_t, double>::type>::type;
  // per-row column bits: the columns of a tile of C <= 32 fit 32 bits
  using TW = typename std::conditional<(C <= 32), uint32_t, uint64_t>::type;
  // LDS is what bounds the resident blocks (latency-bound gathers want as
  // many as fit): 16 KiB of staged values, the column-sum scratch sharing
  // their storage once phase 2 has read them, and one or two words per row.
  __shared__ alignas(16) SV vals[(Q4 ? 4 : NP ? 2 : 1) * LV];
  double *const red = reinterpret_cast<double *>(vals);  // (kBlock / 64) * C doubles
  __shared__ int rps[kRowsPerBlock + 1];
  __shared__ uint32_t hubv[HC ? kHubRows : 1];
  __shared__ uint32_t mw[M1 ? kRowsPerBlock / 32 + 2 : 1];
  __shared__ TW tmw[TM ? kRowsPerBlock : 1];
  __shared__ int cw[CA ? kRowsPerBlock : 1];
  constexpr int LPC = kBlock / C;  // lanes per column in a segment
  const int t = threadIdx.x;
  const int b = blockIdx.x;
  if (b < n_blocks) {
    // descriptor: rows [r0, r0 + nrows), arcs [p0, p1)
    const int4 d = blocks[b];
    const int r0 = d.x, nrows = d.y - d.x, p0 = d.z;
    const int tot = (d.w - d.z) * GU;  // gather units of the block
    // Phase 1.  Load order matters: the col_idx stream first, then the row
    // pointers and epilogue masks of the block, then the gathers (which wait
    // only for col_idx), so a block pays two dependent memory round trips.
    // Every index is clamped into range and every load is unconditional.
    // A block whose rows have no arcs may start at p0 == nnz: its loads are
    // redirected to entry 0 (always allocated) and its gathers to vertex 0.
    const int jlo = tot > 0 ? p0 : 0;
    const int jmax = tot > 0 ? d.w - 1 : 0;
    int u[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      u[q] = __builtin_nontemporal_load(a.ci + min(jlo + (t + q * kBlock) / GU, jmax));
      if (tot == 0) u[q] = 0;
    }
    // HC: the first rows' counts, requested right behind the col_idx stream
    // (unconditional loads of clamped rows; unused when hc_rows is 0)
    uint32_t hv[HC ? kHubRows / kBlock : 1];
    if constexpr (HC) {
#pragma unroll
      for (int q = 0; q < kHubRows / kBlock; ++q)
        hv[q] = a.Xc32[min(t + q * kBlock, max(a.hc_rows - 1, 0))];
    }
    int rv[RT];
#pragma unroll
    for (int k = 0; k < RT; ++k) rv[k] = a.rp[r0 + min(t + k * kBlock, nrows)];
    const int nw = ((r0 + nrows - 1) >> 5) - (r0 >> 5) + 1;
    uint32_t mv = 0;
    if constexpr (M1) mv = a.smask[(r0 >> 5) + min(t, nw - 1)];
    TW tv[RB];
    int cv[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int rr = r0 + min(t + k * kBlock, nrows - 1);
      tv[k] = 0;
      cv[k] = -1;
      if constexpr (TM) tv[k] = (TW)a.tmask[rr];
      if constexpr (CA) cv[k] = a.cand_col[rr];
    }
    // The combining epilogue's row data for this thread's first (row, column)
    // pair of phase 2, loaded now so it arrives with the gathers.
    int tpr = (kBlock / C < 64) ? kBlock / C : 64;
    while (tpr > 1 && nrows * C * tpr > kBlock) tpr >>= 1;
    const int rl0 = (t / tpr) / C;
    CombineFor<C, OUT> pf;
    if constexpr (CB) pf.load(a, r0 + min(rl0, nrows - 1), (t / tpr) & (C - 1));
    if constexpr (HC) {
      if (a.hc_rows > 0) {  // uniform: the copy of the first rows is in place
#pragma unroll
        for (int q = 0; q < kHubRows / kBlock; ++q) hubv[t + q * kBlock] = hv[q];
        __syncthreads();
      }
    }
    double v[NP || Q4 ? 1 : PT];
    uint2 v2[NP || Q4 ? PT : 1];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      if constexpr (Q4) {
        v2[q] = load_pk16<C>(a, u[q], (t + q * kBlock) & (GU - 1));
      } else if constexpr (NP) {
        v2[q] = *reinterpret_cast<const uint2 *>(a.Xc32 + (size_t)u[q] * C +
                                                 2 * ((t + q * kBlock) & (CU - 1)));
      } else if constexpr (HC) {
        // separate registers for the two sources: a shared one would make
        // the LDS read wait for every gather in flight
        uint32_t g = 0;
        if (u[q] >= a.hc_rows) g = a.Xc32[u[q]];
        const uint32_t h = hubv[min(u[q], kHubRows - 1)];
        v[q] = (double)(u[q] < a.hc_rows ? h : g);
      } else {
        v[q] = load_in<C, IN>(a, u[q], (t + q * kBlock) & (C - 1));
        if constexpr (WGT) v[q] *= a.w[min(jlo + (t + q * kBlock) / C, jmax)];
      }
    }
#pragma unroll
    for (int k = 0; k < RT; ++k)
      if (t + k * kBlock <= nrows) rps[t + k * kBlock] = rv[k] - p0;
    if constexpr (M1)
      if (t < nw) mw[t] = mv;
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (t + k * kBlock < nrows) {
        if constexpr (TM) tmw[t + k * kBlock] = tv[k];
        if constexpr (CA) cw[t + k * kBlock] = cv[k];
      }
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int f = t + q * kBlock;
      if (f < tot) {
        if constexpr (NP || Q4)
          reinterpret_cast<uint2 *>(vals)[f] = v2[q];
        else
          vals[f] = (SV)v[q];
      }
    }
    __syncthreads();
    // Phase 2: tpr lanes per (row, column), as many as the row count allows.
    const int s = t & (tpr - 1);
    const int pair = t / tpr;
    const int c = pair & (C - 1);
    const int rstep = (kBlock / tpr) / C;
    double colsum = 0.0;
    for (int rl = pair / C; rl < nrows; rl += rstep) {
      const int j0 = rps[rl], j1 = rps[rl + 1];
      double acc = 0.0;
      if constexpr (NP || Q4)
        acc = sum_staged_counts<C, Q4>(a, vals, j0, j1, s, tpr, c, a.ci + p0);
      else
        for (int j = j0 + s; j < j1; j += tpr) acc += (double)vals[j * C + c];
      for (int off = tpr >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (s == 0) {
        const int r = r0 + rl;
        bool inS = false;
        if constexpr (M1) inS = (mw[(r >> 5) - (r0 >> 5)] >> (r & 31)) & 1u;
        if constexpr (CB) {
          CombineFor<C, OUT> in = pf;
          if (rl != rl0) in.load(a, r, c);
          double y;
          bool member = false;
          if constexpr (OutTraits<OUT>::gaincomb) {
            if constexpr (OUT == OUT_GAINCOMB) {
              if (c >= a.spec_from) {  // miss column: its level is stored, not combined
                a.Y[(size_t)r * C + c] =
                    (inS || cw[rl] == c - a.spec_from) ? 0.0 : a.alpha * acc;
                continue;
              }
            }
            // gain chains: 0 on S (where m_a = 0 too), m_a(x) at the candidate
            y = inS ? 0.0 : (cw[rl] == c ? in.ta : a.alpha * acc);
            if constexpr (OutTraits<OUT>::cstore)
              __builtin_nontemporal_store(gain_count(a, y, acc, cw[rl] == c),
                                          a.Y32 + (size_t)r * C + c);
          } else {
            member = (tmw[rl] >> c) & 1ull;
            y = member ? in.ta : a.alpha * acc;
          }
          colsum += combine_fin(a, in.q(a, r, c), y, in.trv, in.ta, member);
        } else {
          const double y = epilogue_v<C, OUT>(a, r, c, acc, inS, TM ? tmw[rl] : 0ull,
                                              CA ? cw[rl] : -1);
          // wide tiles: the output is not read again before the next
          // launch, which gathers it from beyond the L2 anyway
          if constexpr (OUT == OUT_ZERO32 || OUT == OUT_GAIN32D) {
            a.Y32[(size_t)r * C + c] = (uint32_t)y;
            a.Y[(size_t)r * C + c] = a.alpha * y;
          } else if constexpr (OutTraits<OUT>::store32) {
            if (OUT != OUT_TILE32H || !a.y32_marked || y > (double)kC16Max) {
              if constexpr (C >= 8)
                __builtin_nontemporal_store((uint32_t)y, a.Y32 + (size_t)r * C + c);
              else
                a.Y32[(size_t)r * C + c] = (uint32_t)y;
            }
            if constexpr (OUT == OUT_TILE32H)
              __builtin_nontemporal_store((uint16_t)(y > (double)kC16Max ? kC16Hub : (uint32_t)y),
                                          a.Y16 + (size_t)r * C + c);
          } else {
            if constexpr (C >= 8)
              __builtin_nontemporal_store(y, a.Y + (size_t)r * C + c);
            else
              a.Y[(size_t)r * C + c] = y;
          }
          colsum += y;
        }
      }
    }
    __syncthreads();  // red shares the staged values' storage
    block_colsum<C>(colsum, tpr, red, a.blk_part + (size_t)b * C, a.accum);
  } else if (a.bk_ci != nullptr) {
    // Bucket block: pieces [s0, s0 + np) of long rows, all of whose sources
    // lie in one or two adjacent buckets; the same two phases as a row block
    // over the pieces' copied col_idx, writing each piece's raw sum (the
    // fix-up applies the epilogue).  Weighted graphs are never bucketed.
    if constexpr (!WGT) {
      const int4 d = segs[b - n_blocks];
      const int s0 = d.x, np = d.y - d.x, p0 = d.z;
      const int tot = (d.w - d.z) * GU;  // >= GU: every piece has an arc
      const int jmax = d.w - 1;
      int u[PT];
#pragma unroll
      for (int q = 0; q < PT; ++q)
        u[q] = __builtin_nontemporal_load(a.bk_ci + min(p0 + (t + q * kBlock) / GU, jmax));
      int rv[RT];
#pragma unroll
      for (int k = 0; k < RT; ++k) rv[k] = a.bk_ptr[s0 + min(t + k * kBlock, np)];
      double v[NP || Q4 ? 1 : PT];
      uint2 v2[NP || Q4 ? PT : 1];
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        if constexpr (Q4)
          v2[q] = load_pk16<C>(a, u[q], (t + q * kBlock) & (GU - 1));
        else if constexpr (NP)
          v2[q] = *reinterpret_cast<const uint2 *>(a.Xc32 + (size_t)u[q] * C +
                                                   2 * ((t + q * kBlock) & (CU - 1)));
        else
          v[q] = load_in<C, IN>(a, u[q], (t + q * kBlock) & (C - 1));
      }
#pragma unroll
      for (int k = 0; k < RT; ++k)
        if (t + k * kBlock <= np) rps[t + k * kBlock] = rv[k] - p0;
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const int f = t + q * kBlock;
        if (f < tot) {  // vals holds exactly LV units
          if constexpr (NP || Q4)
            reinterpret_cast<uint2 *>(vals)[f] = v2[q];
          else
            vals[f] = (SV)v[q];
        }
      }
      __syncthreads();
      int tpr = (kBlock / C < 64) ? kBlock / C : 64;
      while (tpr > 1 && np * C * tpr > kBlock) tpr >>= 1;
      const int s = t & (tpr - 1);
      const int pair = t / tpr;
      const int c = pair & (C - 1);
      const int rstep = (kBlock / tpr) / C;
      for (int rl = pair / C; rl < np; rl += rstep) {
        const int j0 = rps[rl], j1 = rps[rl + 1];
        double acc = 0.0;
        if constexpr (NP || Q4)
          acc = sum_staged_counts<C, Q4>(a, vals, j0, j1, s, tpr, c, a.bk_ci + p0);
        else
          for (int j = j0 + s; j < j1; j += tpr) acc += (double)vals[j * C + c];
        for (int off = tpr >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (s == 0) a.seg_out[(size_t)(s0 + rl) * C + c] = acc;
      }
    }
  } else if constexpr (Q4) {
    // One segment of a long row, four columns per lane: kBlock / GU lanes per
    // 4-column unit.
    const int4 sd = segs[b - n_blocks];
    const int k = t & (GU - 1);
    const int s = t / GU;
    constexpr int LPU = kBlock / GU;
    constexpr int U = 8;  // arcs in flight per lane
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j0 = sd.y + s; j0 < sd.z; j0 += U * LPU) {
      int u[U];
#pragma unroll
      for (int q = 0; q < U; ++q) u[q] = __builtin_nontemporal_load(a.ci + min(j0 + q * LPU, sd.z - 1));
      uint4 v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) v[q] = load_quad16<C>(a, u[q], k);
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const bool ok = j0 + q * LPU < sd.z;
        acc[0] += ok ? (double)v[q].x : 0.0;
        acc[1] += ok ? (double)v[q].y : 0.0;
        acc[2] += ok ? (double)v[q].z : 0.0;
        acc[3] += ok ? (double)v[q].w : 0.0;
      }
    }
    block_colsum_quads<C>(acc, red, a.seg_out + (size_t)(b - n_blocks) * C);
  } else if constexpr (NP) {
    // One segment of a long row, column pairs: kBlock / CU lanes per pair.
    const int4 sd = segs[b - n_blocks];
    const int k = t & (CU - 1);
    const int s = t / CU;
    constexpr int LPU = kBlock / CU;
    constexpr int U = 8;  // arcs in flight per lane
    double acc0 = 0.0, acc1 = 0.0;
    for (int j0 = sd.y + s; j0 < sd.z; j0 += U * LPU) {
      int u[U];
#pragma unroll
      for (int q = 0; q < U; ++q) u[q] = __builtin_nontemporal_load(a.ci + min(j0 + q * LPU, sd.z - 1));
      uint2 v[U];
#pragma unroll
      for (int q = 0; q < U; ++q)
        v[q] = *reinterpret_cast<const uint2 *>(a.Xc32 + (size_t)u[q] * C + 2 * k);
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const bool ok = j0 + q * LPU < sd.z;
        acc0 += ok ? (double)v[q].x : 0.0;
        acc1 += ok ? (double)v[q].y : 0.0;
      }
    }
    block_colsum_pairs<C>(acc0, acc1, red, a.seg_out + (size_t)(b - n_blocks) * C);
  } else {
    // One segment of a long row: LPC lanes per column stride over its arcs.
    const int4 sd = segs[b - n_blocks];
    const int c = t & (C - 1);
    const int s = t / C;
    constexpr int U = 8;  // arcs in flight per lane
    double acc = 0.0;
    for (int j0 = sd.y + s; j0 < sd.z; j0 += U * LPC) {
      int u[U];
#pragma unroll
      for (int q = 0; q < U; ++q) u[q] = __builtin_nontemporal_load(a.ci + min(j0 + q * LPC, sd.z - 1));
      double v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        v[q] = load_in<C, IN>(a, u[q], c);
        if constexpr (WGT) v[q] *= a.w[min(j0 + q * LPC, sd.z - 1)];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) acc += (j0 + q * LPC < sd.z) ? v[q] : 0.0;
    }
    block_colsum<C>(acc, 1, red, a.seg_out + (size_t)(b - n_blocks) * C, 0);
  }
}

// Long row l (row r), column c, given the sum of its segments or pieces:
// apply the epilogue and keep the output for the column sums.
template <int C, int OUT>
__device__ __forceinline__ void fixup_tail(const StepArgs &a, int l, int r, int c, double acc) {
  double y = epilogue<C, OUT>(a, r, c, acc);
  if constexpr (OUT == OUT_GAINCOMB) {
    if (c >= a.spec_from) {  // miss column: its level is stored, not combined
      a.Y[(size_t)r * C + c] = y;
      a.long_part[(size_t)l * C + c] = 0.0;
      return;
    }
  }
  if constexpr (OutTraits<OUT>::cstore)
    a.Y32[(size_t)r * C + c] = gain_count(a, y, acc, a.cand_col[r] == c);
  if constexpr (OutTraits<OUT>::combine) {
    CombineFor<C, OUT> in;
    in.load(a, r, c);
    const bool member = OutTraits<OUT>::gaincomb ? false : ((a.tmask[r] >> c) & 1ull);
    y = combine_fin(a, in.q(a, r, c), y, in.trv, in.ta, member);
  } else if constexpr (OUT == OUT_ZERO32 || OUT == OUT_GAIN32D) {
    a.Y32[(size_t)r * C + c] = (uint32_t)y;
    a.Y[(size_t)r * C + c] = a.alpha * y;
  } else if constexpr (OutTraits<OUT>::store32) {
    if (OUT != OUT_TILE32H || !a.y32_marked || y > (double)kC16Max)
      a.Y32[(size_t)r * C + c] = (uint32_t)y;
    if constexpr (OUT == OUT_TILE32H)
      a.Y16[(size_t)r * C + c] = (uint16_t)(y > (double)kC16Max ? kC16Hub : (uint32_t)y);
  } else {
    a.Y[(size_t)r * C + c] = y;
  }
  double *lp = a.long_part + (size_t)l * C + c;
  *lp = a.accum ? *lp + y : y;
}

// Long rows cut into segments: one thread per (row, column) adds the row's
// segment sums in segment order.
template <int C, int OUT>
__global__ __launch_bounds__(kBlock) void k_fixup(StepArgs a, const int *__restrict__ long_rows,
                                                  const int *__restrict__ long_first, int n_long) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int l = gid / C, c = gid & (C - 1);
  if (l >= n_long) return;
  const int q0 = long_first[l], q1 = long_first[l + 1];
  // four independent partial sums keep four loads in flight; combined in a
  // fixed order
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  int q = q0;
  for (; q + 3 < q1; q += 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s4[k] += a.seg_out[(size_t)(q + k) * C + c];
  }
  for (; q < q1; ++q) s4[0] += a.seg_out[(size_t)q * C + c];
  fixup_tail<C, OUT>(a, l, long_rows[l], c, (s4[0] + s4[1]) + (s4[2] + s4[3]));
}

// Long rows in source-bucket pieces (scattered over seg_out, listed per row
// by lsub; a hub row has hundreds): one wavefront per row, lanes striding
// over its pieces with all columns, then a butterfly sum (fixed order, so
// deterministic); lane c finishes column c.  Bucketed partitions gather at
// most 4 units per arc, so C <= 8 here.
template <int C, int OUT>
__global__ __launch_bounds__(kBlock) void k_fixup_pieces(StepArgs a,
                                                         const int *__restrict__ long_rows,
                                                         const int *__restrict__ long_first,
                                                         const int *__restrict__ lsub,
                                                         int n_long) {
  if constexpr (C <= 8) {
    const int l = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= n_long) return;  // the whole wavefront
    const int q0 = long_first[l], q1 = long_first[l + 1];
    double s[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = 0.0;
    for (int q = q0 + lane; q < q1; q += 64) {
      const double *p = a.seg_out + (size_t)lsub[q] * C;
#pragma unroll
      for (int c = 0; c < C; ++c) s[c] += p[c];
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
      for (int off = 32; off > 0; off >>= 1) s[c] += __shfl_xor(s[c], off, 64);
    double acc = s[0];
#pragma unroll
    for (int c = 1; c < C; ++c)
      if (lane == c) acc = s[c];
    if (lane < C) fixup_tail<C, OUT>(a, l, long_rows[l], lane, acc);
  }
}

// Pass 1: block g sums rows [g*R, (g+1)*R) of the concatenation of blk_part
// (nb rows) and long_part (nl rows), all C columns, lanes mapped as
// (row offset t / C, column t % C) so every load is coalesced.  Columns are
// combined across lanes with butterflies (offsets C .. 32) and across the
// four wavefronts in a fixed order.  Pass 2: one block per column adds the
// kReduceBlocks pass-1 values in order.
template <int C>
__global__ __launch_bounds__(kBlock) void k_reduce1(const double *__restrict__ blk_part, int nb,
                                                    const double *__restrict__ long_part, int nl,
                                                    int R, double *out2) {
  __shared__ double red[(kBlock / 64) * C];
  const int t = threadIdx.x, c = t & (C - 1), q = t / C;
  constexpr int RPP = kBlock / C;  // rows per pass
  const int r0 = blockIdx.x * R, r1 = min(r0 + R, nb + nl);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int r = r0 + q;
  for (; r + 3 * RPP < r1; r += 4 * RPP) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rr = r + k * RPP;
      s[k] += rr < nb ? blk_part[(size_t)rr * C + c] : long_part[(size_t)(rr - nb) * C + c];
    }
  }
  for (; r < r1; r += RPP) s[0] += r < nb ? blk_part[(size_t)r * C + c] : long_part[(size_t)(r - nb) * C + c];
  block_colsum<C>((s[0] + s[1]) + (s[2] + s[3]), 1, red, out2 + (size_t)blockIdx.x * C, 0);
}

__global__ __launch_bounds__(kBlock) void k_reduce2(const double *__restrict__ in2, int C,
                                                    double *level, double *acc,
                                                    const int *active) {
  __shared__ double red[kBlock];
  const int c = blockIdx.x;
  if (active && active[c] == 0) return;
  const int t = threadIdx.x;
  red[t] = t < kReduceBlocks ? in2[(size_t)t * C + c] : 0.0;
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
static void launch_t(const Partition &p, const StepArgs &a, hipStream_t st, hipEvent_t ev) {
  const int grid = p.n_blocks + p.n_grid2;
  StepArgs b = a;
  const bool bk = p.bucket_rows > 0 && p.n_grid2 > 0;
  if (bk && C > 8) throw HipError{GED_ERR_ARG, "source buckets at more than 8 columns"};
  b.bk_ci = bk ? p.bk_ci.as<const int>() : nullptr;
  b.bk_ptr = bk ? p.bk_ptr.as<const int>() : nullptr;
  if (grid > 0)
    hipLaunchKernelGGL((k_step<C, IN, OUT, WGT>), dim3(grid), dim3(kBlock), 0, st, b,
                       p.blocks.as<const int4>(), p.segs.as<const int4>(), p.n_blocks);
  if (ev) GED_HIP(hipEventRecord(ev, st));
  if (p.n_long > 0 && bk) {
    const int rows_per_block = kBlock / 64;
    hipLaunchKernelGGL((k_fixup_pieces<C, OUT>),
                       dim3((p.n_long + rows_per_block - 1) / rows_per_block), dim3(kBlock), 0, st,
                       b, p.long_rows.as<const int>(), p.long_first.as<const int>(),
                       p.bk_lsub.as<const int>(), p.n_long);
  } else if (p.n_long > 0) {
    const int thr = p.n_long * C;
    hipLaunchKernelGGL((k_fixup<C, OUT>), dim3((thr + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       b, p.long_rows.as<const int>(), p.long_first.as<const int>(), p.n_long);
  }
}

template <int C, bool WGT>
static bool dispatch_multi(int in, int out, const Partition &p, const StepArgs &a,
                           hipStream_t st, hipEvent_t ev) {
#define GED_CASE(I, O)                      \
  if (in == I && out == O) {                \
    launch_t<C, I, O, WGT>(p, a, st, ev);   \
    return true;                            \
  }
  GED_CASE(IN_TILEMASK, OUT_TILE)
  GED_CASE(IN_VEC, OUT_TILE)
  GED_CASE(IN_ONEHOT, OUT_GAIN)
  GED_CASE(IN_VEC, OUT_GAIN)
  GED_CASE(IN_FRESH, OUT_POOL)
  GED_CASE(IN_TILEMASK, OUT_COMBINE)
  GED_CASE(IN_VEC, OUT_COMBINE)
  if constexpr (!WGT) {  // integer walk counts exist for unweighted graphs only
    GED_CASE(IN_CNT, OUT_TILE)
    GED_CASE(IN_CNT, OUT_COMBINE)
    GED_CASE(IN_CNT32, OUT_TILE)
    GED_CASE(IN_CNT32, OUT_COMBINE32)
    GED_CASE(IN_VEC, OUT_COMBINE32)
    GED_CASE(IN_CNT32, OUT_TILE32)
    GED_CASE(IN_CNT32, OUT_COMBINE32L)
    if constexpr (C >= 4) {  // 16-bit level-2 counts of batch tiles
      GED_CASE(IN_CNT16, OUT_TILE32)
      GED_CASE(IN_CNT16, OUT_TILE32H)
      GED_CASE(IN_CNT32, OUT_TILE32H)
      GED_CASE(IN_CNT16, OUT_COMBINE16)
      GED_CASE(IN_CNT32, OUT_COMBINE16)
    }
  }
  if constexpr (C == 2 || C == 4 || C == 8 || C == 16) {  // the greedy's candidate batches
    GED_CASE(IN_ONEHOT, OUT_GAINCOMB)
    GED_CASE(IN_VEC, OUT_GAINCOMB)
    if constexpr (!WGT) {
      GED_CASE(IN_CNT32, OUT_GAIN32)
      GED_CASE(IN_CNT32, OUT_GAINCOMB32L)
      GED_CASE(IN_CNT32, OUT_GAINCOMB32S)
      GED_CASE(IN_CNT32, OUT_GAIN32D)
      GED_CASE(IN_CNT32, OUT_GAIN)
      GED_CASE(IN_CNT32, OUT_GAINCOMB)
    }
  }
  if constexpr (C == 1) {
    GED_CASE(IN_ONES, OUT_PLAIN)
    GED_CASE(IN_VEC, OUT_PLAIN)
    GED_CASE(IN_MASK, OUT_INJ)
    GED_CASE(IN_VEC, OUT_INJ)
    GED_CASE(IN_NOTMASK, OUT_ZERO)
    GED_CASE(IN_VEC, OUT_ZERO)
    if constexpr (!WGT) {
      GED_CASE(IN_CNT32, OUT_ZERO32)
      GED_CASE(IN_CNT32, OUT_ZERO)
    }
  }
#undef GED_CASE
  return false;
}

template <bool WGT>
static bool dispatch_c(int C, int in, int out, const Partition &p, const StepArgs &a,
                       hipStream_t st, hipEvent_t ev) {
  switch (C) {
    case 1: return dispatch_multi<1, WGT>(in, out, p, a, st, ev);
    case 2: return dispatch_multi<2, WGT>(in, out, p, a, st, ev);
    case 4: return dispatch_multi<4, WGT>(in, out, p, a, st, ev);
    case 8: return dispatch_multi<8, WGT>(in, out, p, a, st, ev);
    case 16: return dispatch_multi<16, WGT>(in, out, p, a, st, ev);
    case 32: return dispatch_multi<32, WGT>(in, out, p, a, st, ev);
    case 64: return dispatch_multi<64, WGT>(in, out, p, a, st, ev);
    default: return false;
  }
}

void launch_step(const Partition &p, const StepArgs &a, int in_mode, int out_mode,
                 hipStream_t st, hipEvent_t after_main) {
  if (a.C != p.C) throw HipError{GED_ERR_ARG, "step column count does not match partition"};
  if (in_mode == IN_CNT16 && (a.C < 4 || a.w || !a.Xc16 || a.hub < 0 || a.hub >= a.n))
    throw HipError{GED_ERR_ARG, "16-bit counts need C >= 4, an unweighted graph and a cut below n"};
  if (out_mode == OUT_COMBINE16 && (a.C < 4 || !a.q_pk2 || a.q_hub2 < 0 || a.q_hub2 >= a.n))
    throw HipError{GED_ERR_ARG, "16-bit level-2 rows need C >= 4 and a cut below n"};
  if (out_mode == OUT_TILE32H && !a.Y16)
    throw HipError{GED_ERR_ARG, "no 16-bit output buffer"};
  const int units = gather_units(a.C, in_mode, a.w != nullptr);
  if (p.units != units)
    throw HipError{GED_ERR_ARG, "step gather width does not match partition"};
  const bool ok = a.w ? dispatch_c<true>(a.C, in_mode, out_mode, p, a, st, after_main)
                      : dispatch_c<false>(a.C, in_mode, out_mode, p, a, st, after_main);
  if (!ok)
    throw HipError{GED_ERR_ARG, "no step kernel for C=" + std::to_string(a.C) + " in=" +
                                    std::to_string(in_mode) + " out=" + std::to_string(out_mode)};
  GED_HIP(hipGetLastError());
}

template <int C>
static void launch_reduce1(const Partition &p, const StepArgs &a, hipStream_t st, double *ws2) {
  const int rows = p.n_blocks + p.n_long;
  const int R = (rows + kReduceBlocks - 1) / kReduceBlocks;
  hipLaunchKernelGGL((k_reduce1<C>), dim3(kReduceBlocks), dim3(kBlock), 0, st, a.blk_part,
                     p.n_blocks, a.long_part, p.n_long, R > 0 ? R : 1, ws2);
}

void launch_reduce(const Partition &p, const StepArgs &a, double *level, double *acc,
                   const int *active, hipStream_t st, double *ws2) {
  switch (a.C) {
    case 1: launch_reduce1<1>(p, a, st, ws2); break;
    case 2: launch_reduce1<2>(p, a, st, ws2); break;
    case 4: launch_reduce1<4>(p, a, st, ws2); break;
    case 8: launch_reduce1<8>(p, a, st, ws2); break;
    case 16: launch_reduce1<16>(p, a, st, ws2); break;
    case 32: launch_reduce1<32>(p, a, st, ws2); break;
    case 64: launch_reduce1<64>(p, a, st, ws2); break;
    default: throw HipError{GED_ERR_ARG, "bad column count"};
  }
  GED_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce2, dim3(a.C), dim3(kBlock), 0, st, ws2, a.C, level, acc, active);
  GED_HIP(hipGetLastError());
}

// ----------------------------------------------------------- partition --

// Source buckets of the long rows (see Partition): pieces of at most cut
// arcs, each inside one bucket, numbered bucket by bucket (rows in order,
// arcs in order); bk_lsub lists each row's pieces in its arc order; bucket
// blocks pack consecutive pieces (at most cut arcs, kRowsPerBlock pieces)
// and are dealt to the XCDs in eight contiguous runs.
static void plan_buckets(PartitionPlan &pl, const int *rp, const int *ci, int nnz_blk,
                         int64_t n) {
  const int64_t BR = pl.bucket_rows;
  const int64_t nbk = (n + BR - 1) / BR;
  const int nl = (int)pl.long_rows.size();
  std::vector<int64_t> pcnt((size_t)nbk + 1, 0), acnt((size_t)nbk + 1, 0);
  auto runs = [&](int r, auto &&f) {  // f(bucket, j0, j1) for each piece of row r
    int j = rp[r];
    const int e = rp[r + 1];
    while (j < e) {
      const int64_t b = ci[j] / BR;
      int k = j + 1;
      while (k < e && k - j < nnz_blk && ci[k] / BR == b) ++k;
      f(b, j, k);
      j = k;
    }
  };
  for (int l = 0; l < nl; ++l)
    runs(pl.long_rows[l], [&](int64_t b, int j0, int j1) {
      pcnt[(size_t)b + 1] += 1;
      acnt[(size_t)b + 1] += j1 - j0;
    });
  for (int64_t b = 0; b < nbk; ++b) {
    pcnt[(size_t)b + 1] += pcnt[(size_t)b];
    acnt[(size_t)b + 1] += acnt[(size_t)b];
  }
  const int npieces = (int)pcnt[(size_t)nbk];
  const int64_t narcs = acnt[(size_t)nbk];
  pl.bk_ptr.assign((size_t)npieces + 1, 0);
  pl.bk_ci.assign((size_t)std::max<int64_t>(1, narcs), 0);
  pl.bk_lsub.assign((size_t)std::max(1, npieces), 0);
  pl.long_first.assign((size_t)nl + 1, 0);
  std::vector<int64_t> pc(pcnt.begin(), pcnt.end() - 1), ac(acnt.begin(), acnt.end() - 1);
  int q = 0;
  for (int l = 0; l < nl; ++l) {
    pl.long_first[(size_t)l] = q;
    runs(pl.long_rows[l], [&](int64_t b, int j0, int j1) {
      const int id = (int)pc[(size_t)b]++;
      const int64_t at = ac[(size_t)b];
      ac[(size_t)b] += j1 - j0;
      pl.bk_ptr[(size_t)id] = (int)at;
      std::copy(ci + j0, ci + j1, pl.bk_ci.begin() + at);
      pl.bk_lsub[(size_t)q++] = id;
    });
  }
  pl.long_first[(size_t)nl] = q;
  pl.bk_ptr[(size_t)npieces] = (int)narcs;
  // bucket blocks in piece order
  std::vector<int> bb;
  for (int s0 = 0; s0 < npieces;) {
    int s1 = s0, arcs = 0;
    while (s1 < npieces && s1 - s0 < kRowsPerBlock) {
      const int len = pl.bk_ptr[(size_t)s1 + 1] - pl.bk_ptr[(size_t)s1];
      if (arcs + len > nnz_blk) break;
      arcs += len;
      ++s1;
    }
    bb.insert(bb.end(), {s0, s1, pl.bk_ptr[(size_t)s0], pl.bk_ptr[(size_t)s1]});
    s0 = s1;
  }
  const int nb = (int)bb.size() / 4;
  // grid position n_blocks + i runs on XCD (n_blocks + i) mod kXcds: XCD x
  // takes the x-th contiguous run of the blocks, as long as its positions
  int start[kXcds + 1] = {0}, take[kXcds] = {0};
  for (int i = 0; i < nb; ++i) ++start[(pl.n_blocks + i) % kXcds + 1];
  for (int x = 0; x < kXcds; ++x) start[x + 1] += start[x];
  pl.grid2.resize((size_t)nb * 4);
  for (int i = 0; i < nb; ++i) {
    const int x = (pl.n_blocks + i) % kXcds;
    const int src = start[x] + take[x]++;
    std::copy(bb.begin() + (size_t)src * 4, bb.begin() + (size_t)src * 4 + 4,
              pl.grid2.begin() + (size_t)i * 4);
  }
  pl.n_segs = npieces;
  pl.n_grid2 = nb;
}

void plan_partition(PartitionPlan &pl, const int *rp, const int *ci, int n, int units,
                    int cut_div, int64_t bucket_rows) {
  pl = PartitionPlan();
  const int nnz_blk = std::max(1, lds_values(0) / units / std::max(1, cut_div));
  const int seg_len = std::max(1, kSegDoubles / units);
  pl.cut = nnz_blk;
  std::vector<int> &segs = pl.grid2;
  int r = 0;
  while (r < n) {
    const int deg = rp[r + 1] - rp[r];
    if (deg > nnz_blk) {
      const int l = (int)pl.long_rows.size();
      pl.long_rows.push_back(r);
      if (bucket_rows <= 0) {
        pl.long_first.push_back((int)segs.size() / 4);
        for (int j = rp[r]; j < rp[r + 1]; j += seg_len)
          segs.insert(segs.end(), {r, j, std::min(j + seg_len, rp[r + 1]), l});
      }
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
    pl.blocks.insert(pl.blocks.end(), {r0, r, rp[r0], rp[r]});
  }
  pl.n_blocks = (int)pl.blocks.size() / 4;
  pl.n_long = (int)pl.long_rows.size();
  if (bucket_rows > 0 && pl.n_long > 0) {
    pl.bucket_rows = bucket_rows;
    plan_buckets(pl, rp, ci, nnz_blk, n);
  } else {
    pl.long_first.push_back((int)segs.size() / 4);
    pl.n_segs = (int)segs.size() / 4;
    pl.n_grid2 = pl.n_segs;
  }
}

void build_partition(Partition &p, const std::vector<int> &rp, int C, int units, int cut_div,
                     const int *ci, int64_t bucket_rows) {
  PartitionPlan pl;
  plan_partition(pl, rp.data(), ci, (int)rp.size() - 1, units, cut_div, ci ? bucket_rows : 0);
  p.C = C;
  p.units = units;
  p.cut = pl.cut;
  p.n_blocks = pl.n_blocks;
  p.n_segs = pl.n_segs;
  p.n_grid2 = pl.n_grid2;
  p.n_long = pl.n_long;
  p.bucket_rows = pl.bucket_rows;
  auto up = [](DBuf &d, const std::vector<int> &v) {
    d.ensure(sizeof(int) * std::max<size_t>(4, v.size()));
    if (!v.empty())
      GED_HIP(hipMemcpy(d.p, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice));
  };
  up(p.blocks, pl.blocks);
  up(p.segs, pl.grid2);
  up(p.long_rows, pl.long_rows);
  up(p.long_first, pl.long_first);
  if (p.bucket_rows > 0) {
    up(p.bk_ci, pl.bk_ci);
    up(p.bk_ptr, pl.bk_ptr);
    up(p.bk_lsub, pl.bk_lsub);
  }
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
