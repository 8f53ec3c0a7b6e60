// Internal declarations shared by the HIP translation units of libged_hip.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ged.h"

namespace ged {

// ----------------------------------------------------------------- errors --

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

struct HipError {
  int code;
  std::string msg;
};

#define GED_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::ged::HipError{GED_ERR_DEVICE, std::string(#expr) + ": " +                \
                                                hipGetErrorString(e_)};                \
  } while (0)

// --------------------------------------------------------- device memory --

// Owning device buffer (hipMalloc); throws HipError{GED_ERR_NOMEM} on failure.
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grow to at least `nbytes` (contents are not preserved)
  void ensure(size_t nbytes) {
    if (nbytes <= bytes && p) return;
    release();
    if (nbytes == 0) nbytes = 256;
    if (hipMalloc(&p, nbytes) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw HipError{GED_ERR_NOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed"};
    }
    bytes = nbytes;
  }
  template <class T>
  T *as() const {
    return reinterpret_cast<T *>(p);
  }
};

// Pinned host buffer (hipHostMalloc).  With hipHostMallocCoherent kernels
// may store results into it directly (uncached on the device side), so the
// host reads them after waiting for the stream, without a copy.
struct HBuf {
  void *p = nullptr;
  size_t bytes = 0;
  unsigned flags = hipHostMallocDefault;
  HBuf() = default;
  HBuf(const HBuf &) = delete;
  HBuf &operator=(const HBuf &) = delete;
  ~HBuf() {
    if (p) (void)hipHostFree(p);
  }
  void ensure(size_t nbytes, unsigned fl = hipHostMallocDefault) {
    if (nbytes <= bytes && p && fl == flags) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, nbytes ? nbytes : 256, fl) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw HipError{GED_ERR_NOMEM, "hipHostMalloc failed"};
    }
    bytes = nbytes ? nbytes : 256;
    flags = fl;
  }
  template <class T>
  T *as() const {
    return reinterpret_cast<T *>(p);
  }
};

// ------------------------------------------------------------ worklists --
// Push kernels walk lists of (vertex, column, chunk) entries, one wavefront
// per chunk of at most kWlChunk arcs.

constexpr int kWlChunk = 512;  // arcs per worklist entry (one wavefront)

// Exclusive prefix sum over the 64 lanes of a wavefront (all lanes active).
__device__ __forceinline__ unsigned wave_excl_scan(unsigned v, unsigned *total) {
  const int lane = threadIdx.x & 63;
  unsigned x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

// Worklist entry: chunk q of vertex y's arcs, column c.
__device__ __forceinline__ uint64_t wl_entry(int y, int c, unsigned q) {
  return ((uint64_t)(unsigned)y << 32) | ((uint64_t)c << 24) | q;
}

__device__ __forceinline__ unsigned wl_chunks(const int *rp, int y) {
  return (unsigned)((rp[y + 1] - rp[y] + kWlChunk - 1) / kWlChunk);
}

// Each lane appends its nch entries for vertex y (all lanes of the wave
// call this together): one atomic per wave.  Entries past cap are dropped;
// every caller sizes cap so that none is.
__device__ __forceinline__ void wl_append(uint64_t *wl, unsigned *wl_n, unsigned cap, int y, int c,
                                          unsigned nch) {
  unsigned total;
  const unsigned ex = wave_excl_scan(nch, &total);
  unsigned base = 0;
  if ((threadIdx.x & 63) == 63 && total) base = atomicAdd(wl_n, total);
  base = __shfl(base, 63, 64);
  for (unsigned q = 0; q < nch; ++q) {
    const unsigned at = base + ex + q;
    if (at < cap) wl[at] = wl_entry(y, c, q);
  }
}

// ------------------------------------------------------ work partitioning --

// Launch geometry shared by every walk-count step kernel.
constexpr int kBlock = 256;            // threads per block (4 wavefronts of 64)
constexpr int kLdsDoubles = 2048;      // LDS staging per block (16 KiB)
// Values a block stages in LDS for a C-column step, whatever C is.  (64 KiB
// blocks for wide steps were measured slower on BA n=2e6: 816 vs 764 us at
// C = 16.)
__host__ __device__ constexpr int lds_values(int) { return kLdsDoubles; }
constexpr int kRowsPerBlock = 255;     // max rows of one row block (row_ptr slice: 1 load per thread)
// Single-column steps over 32-bit counts keep the counts of the first
// kHubRows vertices (the highest degrees under the library's order) in LDS,
// loaded once per row block, when those rows are the sources of at least
// 1/kHubShareDiv of the arcs (StepArgs::hc_rows).
constexpr int kHubRows = 2048;
constexpr int kHubShareDiv = 10;
constexpr int kSegDoubles = 8192;      // nnz*C handled by one long-row segment

// Row partition for a step with C columns: row blocks of consecutive short
// rows staged through LDS, and rows longer than the row-split threshold
// split into fixed segments whose partial sums a fix-up pass combines.
// units = 8-byte gather units per arc: C, or C/2 for 32-bit inputs gathered
// as column pairs (narrow_gather).  The threshold -- also the most arcs a
// block takes -- is the LDS capacity lds_values(C) / units divided by
// cut_div (1, 2 or 4; the batch autotuner chooses it per graph).
//
// Source buckets.  On graphs whose gathered vector is many times the L2 of
// an XCD, the arcs of the long rows are instead grouped by source: the
// vertex range is cut into buckets of bucket_rows vertices (about 3 MiB of
// gathered vector each), every long row's arcs in one bucket form pieces of
// at most the threshold's arcs, and the pieces -- bucket by bucket -- are
// packed into bucket blocks that write each piece's raw sum; the fix-up
// adds a row's pieces in (bucket, offset) order.  Workgroup i of a launch
// runs on XCD i mod 8, so the bucket blocks are cut into eight contiguous
// runs, one per XCD, interleaved in the grid: each XCD walks its own range
// of buckets, and the slice of the vector it gathers from stays in its L2
// (the short rows gather mostly the low-id, high-degree vertices, which
// stay cached anyway).  The pieces copy the long rows' col_idx entries; a
// fix-up wavefront per long row adds its pieces.  Measured on R-MAT scale 22
// (4 FP64 columns): the step takes 924 instead of 1009 us; single-column
// steps were slower, so by default only gathers of 2 to 4 units are bucketed.
constexpr int kMaxCutDiv = 4;
constexpr int kXcds = 8;                       // XCDs of the device (dispatch round-robin)
constexpr int64_t kBucketBytes = 3 << 20;      // gathered bytes per source bucket
constexpr int64_t kBucketAutoBytes = 24 << 20; // bucket long rows above this gathered size
constexpr int kBucketMinUnits = 2;             // narrowest gather (8-byte units per arc) and
constexpr int kBucketMaxUnits = 4;             // widest, bucketed by default
struct Partition {
  int C = 0;
  int units = 0;
  int cut = 0;       // row-split threshold in arcs
  int n_blocks = 0;  // row blocks
  int n_segs = 0;    // long-row segments, or pieces (the slots of seg_out)
  int n_grid2 = 0;   // blocks after the row blocks: segments, or bucket blocks
  int n_long = 0;    // long rows
  int64_t bucket_rows = 0;  // 0: long rows cut into segments, else source buckets
  DBuf blocks;       // int4 [n_blocks]: (row0, row1, nnz0, nnz1)
  DBuf segs;         // int4 [n_grid2]: segments (row, nnz0, nnz1, long index), or
                     // bucket blocks (piece0, piece1, arc0, arc1) in launch order
  DBuf long_rows;    // int  [n_long]:   row id
  DBuf long_first;   // int  [n_long+1]: first segment (or entry of bk_lsub) of each long row
  DBuf bk_ci;        // int [arcs of long rows]: sources, piece by piece
  DBuf bk_ptr;       // int [n_segs+1]: first arc of each piece in bk_ci
  DBuf bk_lsub;      // int [n_segs]: the pieces of each long row in (bucket, offset) order
  size_t device_bytes() const {
    return blocks.bytes + segs.bytes + long_rows.bytes + long_first.bytes + bk_ci.bytes +
           bk_ptr.bytes + bk_lsub.bytes;
  }
};

// Host plan of a partition (what build_partition uploads).
struct PartitionPlan {
  int n_blocks = 0, n_segs = 0, n_grid2 = 0, n_long = 0, cut = 0;
  int64_t bucket_rows = 0;
  std::vector<int> blocks, grid2, long_rows, long_first, bk_ci, bk_ptr, bk_lsub;  // int4 as 4 ints
};
// ci: the CSR's col_idx on the host (read only when bucket_rows > 0).
void plan_partition(PartitionPlan &pl, const int *rp, const int *ci, int n, int units,
                    int cut_div, int64_t bucket_rows);

// Gather source of a step (what x(u) means).
enum InMode : int {
  IN_VEC = 0,      // X[u*C + c]
  IN_ONES = 1,     // 1
  IN_NOTMASK = 2,  // 1 - [u in S]          (miss chain, level 0)
  IN_MASK = 3,     // [u in S]              (hit chain, level 0)
  IN_TILEMASK = 4, // bit c of tmask[u]     (batched hit chains, level 0)
  IN_ONEHOT = 5,   // [cand_col[u] == c]    (gain chains, level 0)
  IN_FRESH = 6,    // fresh[c] ? bit c of tmask[u] : X[u*C+c]   (serving pool)
  IN_CNT = 7,      // Xc[u*C + c] (integer walk counts, exact in FP64 below 2^53)
  IN_CNT32 = 8,    // Xc32[u*C + c] (the same counts, 32-bit)
  IN_CNT16 = 9     // level-2 counts in the 16-bit layout (below): u < hub ? Xc32[u*C + c]
                   // : Xc16[u*C + c]; C >= 4, gathered as 4-column units
};

// Row epilogue of a step (what y(v) becomes).
enum OutMode : int {
  OUT_PLAIN = 0, // alpha * sum
  OUT_INJ = 1,   // v in S ? inj[v] : alpha * sum                   (hit chain)
  OUT_ZERO = 2,  // v in S ? 0 : alpha * sum                        (miss chain)
  OUT_TILE = 3,  // bit c of tmask[v] ? inj[v] : alpha * sum        (batched hit chains)
  OUT_GAIN = 4,  // v in S ? 0 : (cand_col[v] == c ? inj[v] : alpha * sum)  (gain chains)
  OUT_POOL = 5,  // bit c of tmask[v] ? inj[step[c]*n + v] : alpha * sum   (serving pool)
  OUT_COMBINE = 6, // y as OUT_TILE, not stored; the column sum takes the split
                   // combination of y with the stored lower levels (split scoring)
  OUT_COMBINE32 = 7, // the same with 32-bit count levels
  OUT_GAINCOMB = 8,  // y as OUT_GAIN, not stored; the column sum takes the split
                     // combination of a gain chain (undirected greedy)
  OUT_TILE32 = 9,    // y as OUT_TILE, stored to Y32 as an exact 32-bit integer
                     // (unscaled walk counts: alpha = 1, inj = integer omega level)
  OUT_COMBINE32L = 10, // OUT_COMBINE32 whose stored levels are 32-bit counts too
  OUT_GAIN32 = 11,     // y as OUT_GAIN (inj at the candidate from injc[c]), stored to Y32
                       // as an exact 32-bit integer (unscaled gain-chain counts)
  OUT_GAINCOMB32L = 12, // OUT_GAINCOMB whose stored levels are 32-bit counts
  OUT_ZERO32 = 13,      // miss-chain count: y = v in S ? 0 : sum (exact integer), stored
                        // to Y32, and alpha * y to Y (alpha = alpha^i: the FP64 level)
  OUT_GAIN32D = 14,     // OUT_GAIN32 that also stores alpha * y to Y (the FP64 level)
  OUT_GAINCOMB32S = 15, // OUT_GAINCOMB32L that also stores y's count to Y32: 0 on S, the
                        // candidate's miss count (inj / alpha) at it, else the sum
  OUT_COMBINE16 = 16,   // OUT_COMBINE32L (32-bit stored levels, or none) whose level-2
                        // counts q_cnt2 are in the 16-bit layout (hub table q_cnt2, q_pk2)
  OUT_TILE32H = 17      // OUT_TILE32 that also stores a 16-bit copy of the count to Y16,
                        // kC16Hub where the count exceeds kC16Max
};
// Profile records and kernel names encode a (gather, epilogue) pair as
// in * kKindBase + out.
constexpr int kKindBase = 32;

struct StepArgs {
  const int *rp = nullptr;       // row_ptr int32 [n+1]
  const int *ci = nullptr;       // col_idx int32 [nnz]
  const double *w = nullptr;     // arc weights [nnz] or null
  int n = 0;
  int C = 1;
  const double *X = nullptr;     // [n*C]
  double *Y = nullptr;           // [n*C]
  uint32_t *Y32 = nullptr;       // [n*C] (OUT_TILE32)
  const uint32_t *smask = nullptr;  // S bitmap [ceil(n/32)]
  const uint64_t *tmask = nullptr;  // per-vertex column bits [n]
  const int *cand_col = nullptr;    // [n], -1 = not a candidate
  const double *inj = nullptr;      // injection vector [n] (or level array for OUT_POOL)
  const int *col_step = nullptr;    // [C] per-column level (OUT_POOL), 0 = idle
  const int *fresh = nullptr;       // [C] first-step flags (IN_FRESH)
  const double *injc = nullptr;     // [C] value at column c's candidate (OUT_GAIN32)
  double alpha = 0;
  int accum = 0;                 // 1: add this step's column sums to blk_part/long_part
  double *blk_part = nullptr;    // [n_blocks*C] block column sums
  double *seg_out = nullptr;     // [n_segs*C] raw segment (or piece) sums
  double *long_part = nullptr;   // [n_long*C] long-row outputs (for column sums)
  // IN_CNT / IN_CNT32 source
  const uint64_t *Xc = nullptr;    // [n*C]
  const uint32_t *Xc32 = nullptr;  // [n*C]
  // IN_CNT16: the 16-bit copy of the gathered level ([n*C]; rows below hub, and
  // values marked kC16Hub, are read from Xc32)
  const uint16_t *Xc16 = nullptr;
  int hub = 0;
  uint16_t *Y16 = nullptr;         // [n*C] (OUT_TILE32H)
  // OUT_TILE32H: 1 = Y32 receives only the counts above kC16Max (those its
  // 16-bit copy marks); set when the level is the only stored one, which the
  // combining step then reads through the copy (OUT_COMBINE16, q_nlv == 1)
  int y32_marked = 0;
  // C = 1 steps over 32-bit counts (IN_CNT32): rows [0, hc_rows) of Xc32 are
  // read from an LDS copy (0: none)
  int hc_rows = 0;
  // OUT_COMBINE16: the level-2 rows in the 16-bit layout (table q_cnt2, packed
  // rows q_pk2, cut q_hub2)
  const uint16_t *q_pk2 = nullptr;
  int q_hub2 = 0;
  // OUT_COMBINE(32): per row v and column c the column sum takes
  //   q + y + y*tr[v] + [v not in S](inj[v] - y) * (q_even ? q + y : q),
  // q = q_s1*q_cnt1[v,c] + q_s2*q_cnt2[v,c] + sum_l q_lv[l][v,c]
  // (OUT_COMBINE32L: sum_l q_slv * q_alpha^l * q_lv[l][v,c], 32-bit counts).
  // Every pointer is valid: an absent input is read at index (o & mask) = 0
  // of some valid buffer and weighted by 0, so the loads are unconditional.
  const double *tr = nullptr;       // [n]
  const void *q_cnt1 = nullptr;     // [n*C] uint64 (uint32 for OUT_COMBINE32)
  const void *q_cnt2 = nullptr;
  uint64_t q_m1 = 0, q_m2 = 0, q_mlv = 0;  // index masks: ~0 present, 0 absent
  double q_s1 = 0, q_s2 = 0, q_slv = 0;    // weights (q_slv = 1 if q_nlv > 0)
  const void *q_lv = nullptr;       // [q_nlv * n * C] double (uint32 for OUT_COMBINE32L)
  double q_alpha = 0;               // weight ratio of consecutive stored levels (OUT_COMBINE32L)
  int q_nlv = 0;
  int q_even = 0;
  // Gain batches with speculative miss columns (OUT_GAIN, OUT_GAIN32D,
  // OUT_GAINCOMB): column c >= spec_from carries the miss chain of S plus the
  // candidate of column c - spec_from -- 0 on S and at that candidate, the
  // plain level elsewhere (alpha * sum; the count for OUT_GAIN32D) -- and a
  // combining step stores it to Y instead of combining it.
  int spec_from = 1 << 30;
  // source-bucketed partitions (set by the launch from the partition)
  const int *bk_ci = nullptr;   // sources of the pieces
  const int *bk_ptr = nullptr;  // [pieces+1] first arc of each piece
};

// Walk-count step: Y = epilogue(alpha * A X) with column sums.  Three
// launches: row blocks + segments, long-row fix-up, column reduction.
// If `after_main` is non-null it is recorded right after the main step kernel
// (before the fix-up), so profiling brackets exactly that kernel.
void launch_step(const Partition &p, const StepArgs &a, int in_mode, int out_mode,
                 hipStream_t st, hipEvent_t after_main = nullptr);
// Column sums of the partials in a (one step, or a chain of steps launched
// with accum = 1): level[c] = the sum; if acc is non-null acc[c] += level[c].
// level may be null.  active (nullable, [C]) skips columns whose flag is 0.
// Two passes of fixed order, so the result is deterministic.  ws2 is a
// scratch buffer of at least kReduceBlocks * C doubles.
constexpr int kReduceBlocks = 256;
void launch_reduce(const Partition &p, const StepArgs &a, double *level, double *acc,
                   const int *active, hipStream_t st, double *ws2);

// bucket_rows > 0 groups the long rows by source (ci: host col_idx).
void build_partition(Partition &p, const std::vector<int> &row_ptr, int C, int units,
                     int cut_div = 1, const int *ci = nullptr, int64_t bucket_rows = 0);

// 32-bit inputs at C >= 2 are gathered as pairs of adjacent columns (8 bytes
// per lane), so a wavefront's load covers as many cache lines as an FP64
// gather and keeps as many in flight; such steps take the partition of
// partition_narrow (blocks of kLdsDoubles / (C/2) arcs).
__host__ __device__ constexpr bool narrow_gather(int C, int in_mode, bool weighted) {
  return in_mode == IN_CNT32 && C >= 2 && !weighted;
}

// 16-bit layout of the level-2 counts (split tiles of C >= 4 columns).  On an
// unweighted graph count_2(v) <= omega_2(v), the number of length-2 walks
// ending at v, and the partial sums the pushes build never exceed it.  With
// the vertices in decreasing-degree order, those of omega_2 >= 2^16 - 1 sit
// at the front; `hub` is a cut below which all of them lie.  Rows v < hub
// keep 32-bit counts at v*C + c of the buffer; rows v >= hub hold 16-bit
// counts, at most 2^16 - 2, at v*C + c of the packed array that starts at
// c16_pk_offset bytes (its rows below the cut stay zero).  Two adjacent
// columns share a 32-bit word, so the pushes add (value << 16*(c & 1)) to
// that word: no carry crosses between the halves.  A 32-column row is 64
// bytes instead of 128.  The gather (IN_CNT16) stages the packed values in
// LDS, with the value 2^16 - 1 -- which no packed count takes -- standing for
// rows below the cut, whose 32-bit counts the per-row sums fetch instead.
// The last stored dense level (a walk-count level the step computes exactly)
// gets a 16-bit copy with the same marker where its count exceeds kC16Max
// (cut 0: any row may carry it), so the combining step gathers it the same
// way, reading marked values from the 32-bit level.
constexpr uint32_t kC16Max = 0xfffe;    // largest count the packed rows hold
constexpr uint32_t kC16Hub = 0xffff;    // staged in place of a hub row's value
__host__ __device__ constexpr size_t c16_pk_offset(int hub, int C) {
  return ((size_t)hub * C * 4 + 255) & ~(size_t)255;
}
inline size_t c16_bytes(int64_t n, int hub, int C) {
  return c16_pk_offset(hub, C) + 2 * (size_t)n * C;
}

// 8-byte gather units per arc of a step: C values, C/2 column pairs of 32-bit
// inputs, C/4 four-column units of 16-bit inputs.
__host__ __device__ constexpr int gather_units(int C, int in_mode, bool weighted) {
  return in_mode == IN_CNT16 && C >= 4 && !weighted ? C / 4
                                                    : narrow_gather(C, in_mode, weighted) ? C / 2
                                                                                           : C;
}

// Partial-sum buffers of one step stream (each path owns its own, so captured
// graphs never see a buffer another path reallocated).
struct StepWs {
  DBuf blk, seg, lng, red2;
  void fit(const Partition &p) {
    blk.ensure(sizeof(double) * (size_t)(p.n_blocks > 0 ? p.n_blocks : 1) * p.C);
    seg.ensure(sizeof(double) * (size_t)(p.n_segs > 0 ? p.n_segs : 1) * p.C);
    lng.ensure(sizeof(double) * (size_t)(p.n_long > 0 ? p.n_long : 1) * p.C);
    red2.ensure(sizeof(double) * (size_t)kReduceBlocks * p.C);
  }
  double *scratch() const { return red2.as<double>(); }
  void into(StepArgs &a) const {
    a.blk_part = blk.as<double>();
    a.seg_out = seg.as<double>();
    a.long_part = lng.as<double>();
  }
};

// --------------------------------------------------------- small kernels --
void launch_fill_f64(double *p, double v, size_t count, hipStream_t st);
void launch_fill_i32(int *p, int v, size_t count, hipStream_t st);
void launch_mask_set(uint32_t *mask, const int *S, const int *s_len, int cap, int value,
                     hipStream_t st);
void launch_tmask_set(uint64_t *tmask, const int64_t *offsets, const int *members, int g0,
                      int ncols, int value, hipStream_t st);
void launch_sum_levels(const double *levels, int count, double *out, hipStream_t st);
void launch_copy_f64(double *dst, const double *src, size_t count, hipStream_t st);

// ------------------------------------------------------------ graph handle --

struct PrepCache {
  bool valid = false;
  double alpha = 0, eps = 0;
  int ell = 0;                 // ell*
  double bound = 0;            // B_{ell*}
  std::vector<double> W;       // W[i] = sum t_i, i = 0..computed
  DBuf t_levels;               // [(ell*+1) * n] decayed total walk counts t_0..t_ell*
  DBuf t_tail[2];              // ping-pong vectors to extend W beyond ell*
  int tail_level = -1;         // level held in t_tail[tail_cur]
  int tail_cur = 0;
  DBuf tr;                     // [n] sum_{c=1..tr_r} t_c (split scoring)
  int tr_r = -1;               // -1: not built for this (alpha, eps)
  // Levels beyond ell* (the greedy's walk length may exceed ell*) live in a
  // buffer of their own, so t_levels never moves after prepare (a server's
  // score pool may be reading it on another stream).
  DBuf t_ext;                  // [t_ext_count * n] levels ell*+1 ..
  int t_ext_count = 0;
};

// ------------------------------------------------------- split scoring --
//
// Undirected graphs only.  ell* levels are obtained from the hit chain up to
// a = ceil(ell/2): levels 1..s by integer pushes from the group's members,
// levels s+1..a by dense steps, the last of which combines (OUT_COMBINE).
struct SplitPlan {
  int a = 0, r = 0, s = 0, nlv = 0;  // nlv = dense levels stored (s+1 .. a-1)
  bool even = false;                 // r == a
  bool c32 = false;                  // counts fit 32 bits (max degree < 2^16)
  // stored levels are unscaled 32-bit counts: count_i(v) <= omega_i(v), the
  // number of all walks of length i ending at v, and max omega_i < 2^32 for
  // every stored level (set by split_tables)
  bool lv32 = false;
  // single group with 32-bit stored levels whose level-3 push is small: the
  // first stored level (3) is pushed from the vertices holding level-2
  // counts instead of gathered
  bool push3 = false;
  int cut_div = 1;  // row-split threshold divisor of the dense steps' partitions
  // level-2 counts in the 16-bit layout with this hub cut (c16_pk_offset),
  // -1: plain 32-bit counts.  Batch tiles of C >= 4 columns only (c32, s = 2,
  // no pushed level 3, stored levels 32-bit or none).
  int c16_hub = -1;
};

struct SplitWs {
  DBuf cnt1, cnt2;       // [n*C] walk counts of levels 1, 2 (uint32 or uint64); zero
                         // between tiles
  DBuf lv;               // [nlv*n*C] stored dense levels (double, or uint32 counts)
  DBuf lv16;             // [n*C] 16-bit copy of the last stored level (16-bit layout)
  DBuf wl, wl_n;         // uint64 worklist [wl_cap], uint32 length
  unsigned wl_cap = 0;
  DBuf wl3, wl3_n;       // sources of the pushed level 3 (push3)
  unsigned wl3_cap = 0;
  bool lv_zero = false;  // first stored level all zero, as the push needs
  int wl_blocks = 64;    // grid of the worklist kernels (any value is correct)
  size_t cnt_bytes = 0;  // bytes of the count layout the arrays were zeroed for
  bool zero = false;
  StepWs ws;
};


// A single-group split score captured as two graphs: the main work up to the
// result, and its clean-up (left running after the result is on the host;
// the next call is on the same stream).
struct SplitExec {
  hipGraph_t graph = nullptr, clear_graph = nullptr;
  hipGraphExec_t exec = nullptr, clear_exec = nullptr;
  std::vector<const void *> sig;  // pointers/values the captured graphs depend on
  void drop();
};

struct Profiler {
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    int C;
    double bytes, edges;
    int kind;  // in_mode * kKindBase + out_mode: one kernel instantiation per (C, kind)
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};

}  // namespace ged

struct ged_graph {
  int64_t n = 0, nnz = 0;
  uint32_t flags = 0;
  int32_t max_deg = 0;          // maximum out-degree (structural)
  int32_t bound_kind = 0;       // GED_BOUND_COMBINATORIAL or GED_BOUND_SPECTRAL
  double sigma = -1.0;          // upper estimate of sigma_max, -1 until computed
  double max_wdeg = 0;          // maximum weighted out-degree (weighted graphs)
  bool weighted = false;
  bool simple = false;          // no arc listed twice (rows are sorted internally)
  std::vector<int> h_rp;        // host copy of row_ptr (int32) for partitioning
  // Vertices are stored in degree-descending order (stable by id) unless
  // GED_KEEP_ORDER is given: internal id = new_id[caller id],
  // caller id = old_id[internal id].
  std::vector<int> new_id, old_id;
  ged::DBuf d_old_id;           // int [n] caller ids, for tie-breaking on the device
  ged::DBuf rp, ci, w;          // device CSR (in-neighbour rows)
  ged::DBuf rp_r, ci_r, w_r;    // reverse graph (directed only)
  std::vector<int> h_rp_r;
  // host col_idx (and of the reverse graph), copied when a source-bucketed
  // partition is first built
  std::vector<int> h_ci, h_ci_r;
  // gathered bytes per source bucket of new partitions: 0 = kBucketBytes
  // where the gathered vector exceeds kBucketAutoBytes, < 0 = never, > 0 =
  // always, with this size
  int64_t bucket_bytes = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  std::recursive_mutex mu;
  // partitions are looked up by server lanes on their own thread while calls
  // holding mu may add new ones: the maps have a lock of their own (entries
  // are never removed, so a returned reference stays valid)
  std::mutex parts_mu;
  std::map<int, std::unique_ptr<ged::Partition>> parts, parts_r;
  ged::PrepCache prep;
  // precomputation workspace (C = 1 steps)
  ged::StepWs pws;
  // plain-score workspace
  ged::StepWs sws;
  ged::DBuf mask;               // uint32 [ceil(n/32)+1], all zero between calls
  ged::DBuf vec[2];             // double [n]
  ged::DBuf s_levels;           // double [ell*+1] per-level hit sums
  ged::DBuf acc;                // double [64]
  ged::DBuf s_dev;              // int [1 + cap]: length, then members
  ged::HBuf s_host;             // pinned staging of S
  ged::HBuf out_host;
  int s_cap = 0;
  bool mask_ready = false;
  hipGraphExec_t score_exec = nullptr;
  hipGraph_t score_graph = nullptr;
  std::vector<const void *> score_sig;  // pointers/values the captured graph depends on
  // split scoring: one captured pair per variant (third level gathered or
  // pushed; group copied to the device or staged by the first kernel), so
  // groups that alternate between them keep each
  ged::SplitExec split_exec[8];
  hipEvent_t score_done = nullptr;  // recorded after the result copy
  // batched scoring: tile width and row-split threshold divisor (0 = autotune)
  int32_t batch_tile = 0;
  int32_t batch_cut_div = 0;
  // greedy candidate batch width (0 = the library's choice)
  int32_t greedy_width = 0;
  // 16-bit level-2 counts in batch tiles: 0 the library's choice, -1 off,
  // > 0 this hub cut (at least c16_least_hub)
  int32_t count16 = 0;
  int c16_least_hub = -1;       // 1 + the last vertex with omega_2 > kC16Max (-1: not known)
  int c16_used = -1;            // hub cut of the last batch's tiles (-1: 32-bit counts)
  int hc_rows = 0;              // rows of the LDS copy in C = 1 count steps (kHubRows or 0)
  // registered with a server at (served_alpha, served_eps): other values,
  // invalidation and a change of tail bound are refused until it is destroyed
  bool served = false;
  double served_alpha = 0, served_eps = 0;
  // split scoring
  ged::DBuf omega2;             // uint64 [n] walks of length 2 ending at v (unweighted)
  bool omega2_ready = false;
  // omega_i(v) for i = 3 .. omega_top, exact integers as doubles [(omega_top-2)*n];
  // omega_fit = largest i <= omega_top with max_v omega_j(v) < 2^32 for 3 <= j <= i
  ged::DBuf omega_lv;
  int omega_top = 2, omega_fit = 2;
  // largest level of omega_lv shown free of 64-bit wrap-around everywhere
  // (each value exact), by max_v omega_i <= max_deg * max_v omega_{i-1}
  int omega_exact = 2;
  std::list<ged::DBuf> omega_old;  // replaced omega_lv buffers, freed with the graph
  // maxima known for levels 3 .. omax_top; omax_fit as omega_fit for them
  int omax_top = 2, omax_fit = 2;
  // deg(v) + omega_2(v) + omega_3(v) on the host (single-group level-3 push)
  std::vector<double> push_bound;
  // omega_2(v) on the host (push volumes decided before launch)
  std::vector<double> h_omega2;
  // omega_i(v) on the host for levels i >= 3 the graph holds (per-group
  // bounds of the stored levels of a single score)
  std::map<int, std::vector<double>> h_omega_lv;
  // omega_sum[i] = sum_v omega_i(v) for i = 1 .. (2 once omega2 is ready, then
  // omega_top once omega_lv holds levels 3..); exact for levels that fit 2^32
  std::vector<double> omega_sum;
  std::vector<uint32_t> stamp;  // host group-dedup stamps
  uint32_t stamp_gen = 0;
  ged::SplitWs split_ws;        // single-group scoring workspace
  ged::DBuf split_tmask;        // uint64 [n], zero between calls
  bool split_tmask_ready = false;
  ged::DBuf split_in;           // int64 offsets[2], int members[cap], int mcol[cap]
  ged::HBuf split_in_host;
  int split_cap = 0;
  // profiling
  ged::Profiler prof;
  ~ged_graph();
};

namespace ged {

// Partition for C columns (built on first use), at a row-split threshold of
// the LDS capacity / cut_div.
Partition &partition(ged_graph *g, int C, bool reverse = false, int cut_div = 1);
// The partition of a narrow_gather step with C columns (forward rows).
Partition &partition_narrow(ged_graph *g, int C, int cut_div = 1);
// The partition of a 16-bit (IN_CNT16) step with C >= 4 columns: blocks of
// kLdsDoubles / (C/4) arcs; source buckets only at C <= 8.
Partition &partition_quad(ged_graph *g, int C, int cut_div = 1);
// The forward C-column partition at cut_div 1 if it was built, else null
// (builds nothing).
const Partition *partition_if_built(ged_graph *g, int C);
// Precompute for (alpha, eps); throws HipError, returns status for arg errors.
int prepare(ged_graph *g, double alpha, double eps);
// W[ell] for arbitrary ell (extends the total-walk chain on demand).
double walk_total(ged_graph *g, int ell);
// Make the decayed total-walk levels t_0..t_L available (levels beyond ell*
// are computed on demand into prep.t_ext, which may move; t_levels does not).
void t_levels_to(ged_graph *g, int L);
// Pointer to level j (j <= ell* or an extended level).
const double *t_level(const ged_graph *g, int j);
// Tail bound B_ell(V) from W_ell = alpha^ell sum_x omega_ell(x): the
// combinatorial bound or the spectral one, as selected for the graph.
double comb_bound(ged_graph *g, double alpha, double W_ell);
// Upper estimate of sigma_max (ged_spectral.hip); computed once per graph.
double sigma_max(ged_graph *g);
int check_alpha_eps(ged_graph *g, double alpha, double eps);
// Device bytes of the handle's single-group score workspace.
size_t score_bytes_held(const ged_graph *g);
StepArgs base_args(ged_graph *g, bool reverse = false);
// Step launch, timed with HIP events around the main kernel when profiling is
// on for the graph (the only way library code launches walk-count steps).
void run_step(ged_graph *g, const Partition &p, const StepArgs &a, int in_mode, int out_mode,
              hipStream_t st, double extra_rows = 0);
// Algorithmic bytes of one step launch: row_ptr, col_idx (+ weights), the
// gathered input, the written output, the epilogue's mask reads and
// `extra_rows` further C-wide rows of 8-byte values per vertex that the
// epilogue streams.
double algo_bytes(const ged_graph *g, int C, int in_mode, int out_mode, double extra_rows = 0);
int score_group(ged_graph *g, const int32_t *S, int32_t s_len, double alpha, double eps,
                double *out, ged_score_info *info);
// Drop the batched-scoring workspace of a graph that is being destroyed.
void batch_forget(const ged_graph *g);
// Drop the greedy workspace of a graph that is being destroyed.
void greedy_forget(const ged_graph *g);
// Candidate batch width the greedy uses on g.
int greedy_width_for(const ged_graph *g);
// Upper bound of the device bytes a greedy run (walk length up to ell_max, k
// picks) can leave allocated on g, and the bytes its workspace holds now.
size_t greedy_footprint(ged_graph *g, int ell_max, int k);
size_t greedy_bytes_held(const ged_graph *g);

// Split scoring (ged_split.hip).
bool split_ok(const ged_graph *g);
SplitPlan split_plan(const ged_graph *g, int ell);
// Make sure per-graph split tables (omega2, tr, and the integer omega levels
// of the stored levels) exist for the prepared (alpha, eps), and set pl.lv32.
// The first call that needs new omega levels synchronizes the stream once to
// read their maxima.
void split_tables(ged_graph *g, SplitPlan &pl, hipStream_t st);
// Largest i <= L such that max_v omega_j(v) < 2^32 for 3 <= j <= i (L itself
// for L <= 2).  Computes the maxima by the integer chain the first time a
// level is asked for (synchronizes the stream once); stores no levels.
int omega_fit_level(ged_graph *g, int L, hipStream_t st);
// omega_2 as a host array (built on first use; synchronizes the stream then).
const std::vector<double> &omega2_host(ged_graph *g, hipStream_t st);
// Hub cut of the 16-bit level-2 layout for tiles of C columns under plan pl,
// or -1 when the layout does not apply (the plan's shape, C < 4, the graph's
// setting, or -- left to the library -- more than n/8 rows below the cut).
int split_c16_hub(ged_graph *g, const SplitPlan &pl, int C, hipStream_t st);
// 1 + the last vertex (internal order) with omega_2 > kC16Max: the least cut.
int least_c16_hub(ged_graph *g, hipStream_t st);
// Walk-count levels of the precomputation from the graph's exact integer
// counts omega_i (unweighted graphs): omega_prefix_levels gives how many
// levels those counts are held for (0 for weighted graphs);
// t_levels_from_omega writes t_1 .. t_L (level i at T + i*n) for L up to
// levels_cap, stopping at the first level whose tail bound is below eps,
// appends W_1 .. W_L to W and returns L.
constexpr int kTPrefixMax = 32;
int omega_prefix_levels(ged_graph *g);
int t_levels_from_omega(ged_graph *g, double alpha, double eps, int levels_cap, double *T,
                        std::vector<double> &W, hipStream_t st);
// Size a workspace for C columns and a worklist of wl_need entries; zero the
// count arrays if they are new or dirty.
void split_fit(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, size_t wl_need,
               hipStream_t st, bool counts_only = false);
// Worklist entries a group needs: min(n, sum of member degrees) + ceil(nnz/chunk).
size_t split_wl_need(const ged_graph *g, int64_t deg_sum);
// Grid of the worklist kernels for about `expected_entries` entries.
int split_wl_blocks(int64_t expected_entries);
// Dense levels s+1..a of a tile (the last one combining into the block
// partials of w.ws); the counts of levels <= s must be in place.
// counts (nullable) supplies the count levels when they live in another
// workspace than w's stored levels and partials.
void split_dense(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, const uint64_t *tmask,
                 hipStream_t st, bool profile = true, const SplitWs *counts = nullptr);
// Enqueue one tile of nc <= C groups (g0 .. g0+nc-1 of the device offsets /
// members / mcol arrays); scores go to out[0..nc).
// The phases of a tile, for callers that overlap them across tiles: member bits
// and integer levels (push), dense levels (split_dense), column sums of w's
// partials into out[0..C) (reduce), and clearing of what push wrote (clear).
// w's counts and tmask must not be shared with a tile in flight.
void split_tile_push(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, const int64_t *offs,
                     const int *mem, const int *mcol, int g0, int nc, int64_t tile_members,
                     uint64_t *tmask, hipStream_t st, bool set_tmask = true);
void split_tile_reduce(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, double *out,
                       hipStream_t st);
// fill: zero the count levels with a dense fill instead of replaying the
// pushes (split_clear_by_fill decides from the tile's estimated push volume).
void split_tile_clear(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C, const int64_t *offs,
                      const int *mem, const int *mcol, int g0, int nc, int64_t tile_members,
                      uint64_t *tmask, hipStream_t st, bool fill = false);
// Is a dense fill cheaper than replaying a tile's pushes?  push2_arcs: the
// sum of omega_2 over the tile's members, a bound on the arcs its level-2
// push wrote along.
bool split_clear_by_fill(const ged_graph *g, const SplitPlan &pl, int C, double push2_arcs);
// All four phases in order on one stream.  profile = false launches without
// profiling events (the server enqueues tiles from its own thread).
void enqueue_split_tile(ged_graph *g, SplitWs &w, const SplitPlan &pl, int C,
                        const int64_t *offs, const int *mem, const int *mcol, int g0, int nc,
                        int64_t tile_members, uint64_t *tmask, double *out, hipStream_t st,
                        bool profile = true, bool fill_clear = false);
// Map caller ids to internal ids, dropping duplicates inside the group;
// returns the sum of the members' degrees.
int64_t map_group(ged_graph *g, const int32_t *S, int64_t len, std::vector<int> &out);
int split_score(ged_graph *g, const int32_t *S, int32_t s_len, double *out);

// Run fn, translating HipError into a status code + message.
template <class F>
int guarded(F &&fn) {
  try {
    return fn();
  } catch (const HipError &e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc &) {
    return fail(GED_ERR_NOMEM, "host allocation failed");
  }
}

}  // namespace ged
