// Upper estimate of sigma_max for the spectral tail bound (Lemma
// "spectral-bound"; Section 2.1 defines sigma_max, the largest singular value
// of the adjacency matrix).
//
// sigma_max^2 is the Perron root of the nonnegative symmetric B = A^T A, and
// for every positive vector x the Collatz-Wielandt inequality gives
// rho(B) <= max_v (Bx)_v / x_v.  From x_0 = 1, for k = 1..kSigmaIters:
//     z = B x_{k-1},   c_k = max_v z_v / x_{k-1,v},
//     x_k = max((z + x_{k-1}) / max_v (z_v + x_{k-1,v}), 2^-990)
// (a power step on B + I, which also converges on bipartite graphs; the clamp
// keeps x positive), and sigma = sqrt(min_k c_k * (1 + 2^-40)), the factor
// covering the rounding of the sums.  Any value >= sigma_max keeps the bound
// valid.  The products run on the step kernels (C = 1, plain output); maxima
// are exact in any order, so the result does not depend on the reduction.
#include <math.h>

#include <algorithm>

#include "ged_internal.h"

namespace ged {

constexpr int kSigmaIters = 100;
constexpr int kMaxBlocks = 1024;

// Per block: max of z/x and of z + x over a grid-stride slice.
__global__ __launch_bounds__(kBlock) void k_cw_partial(const double *__restrict__ z,
                                                       const double *__restrict__ x, int64_t n,
                                                       double *__restrict__ part) {
  __shared__ double sr[kBlock], sm[kBlock];
  double r = 0.0, m = 0.0;
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock) {
    const double zv = z[v], xv = x[v];
    r = fmax(r, zv / xv);
    m = fmax(m, zv + xv);
  }
  sr[threadIdx.x] = r;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + s]);
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0];
    part[2 * blockIdx.x + 1] = sm[0];
  }
}

// One block: c_k -> cw[k], max(z + x) -> mz[0].
__global__ __launch_bounds__(kBlock) void k_cw_final(const double *__restrict__ part, int nb,
                                                     double *__restrict__ cw, int k,
                                                     double *__restrict__ mz) {
  __shared__ double sr[kBlock], sm[kBlock];
  double r = 0.0, m = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    r = fmax(r, part[2 * b]);
    m = fmax(m, part[2 * b + 1]);
  }
  sr[threadIdx.x] = r;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + s]);
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cw[k] = sr[0];
    mz[0] = sm[0];
  }
}

__global__ void k_cw_update(const double *__restrict__ z, double *__restrict__ x, int64_t n,
                            const double *__restrict__ mz) {
  const double m = mz[0];
  const double floor_v = 0x1p-990;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    x[v] = fmax((z[v] + x[v]) / m, floor_v);
}

double sigma_max(ged_graph *g) {
  if (g->sigma >= 0.0) return g->sigma;
  hipStream_t st = g->stream;
  const int64_t n = g->n;
  const bool directed = g->flags == GED_DIRECTED;
  Partition &pf = partition(g, 1);
  Partition &pr = partition(g, 1, directed);
  StepWs ws;
  ws.fit(pf);
  StepWs wsr;
  wsr.fit(pr);
  DBuf x, y, z, part, cw, mz;
  x.ensure(sizeof(double) * (size_t)n);
  y.ensure(sizeof(double) * (size_t)n);
  z.ensure(sizeof(double) * (size_t)n);
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks, (n + kBlock - 1) / kBlock));
  part.ensure(sizeof(double) * 2 * (size_t)nb);
  cw.ensure(sizeof(double) * kSigmaIters);
  mz.ensure(sizeof(double));
  launch_fill_f64(x.as<double>(), 1.0, (size_t)n, st);
  for (int k = 0; k < kSigmaIters; ++k) {
    StepArgs a = base_args(g);  // y = A x
    ws.into(a);
    a.C = 1;
    a.alpha = 1.0;
    a.X = x.as<const double>();
    a.Y = y.as<double>();
    launch_step(pf, a, IN_VEC, OUT_PLAIN, st);
    StepArgs b = base_args(g, directed);  // z = A^T y (the same rows when undirected)
    wsr.into(b);
    b.C = 1;
    b.alpha = 1.0;
    b.X = y.as<const double>();
    b.Y = z.as<double>();
    launch_step(pr, b, IN_VEC, OUT_PLAIN, st);
    hipLaunchKernelGGL(k_cw_partial, dim3(nb), dim3(kBlock), 0, st, z.as<const double>(),
                       x.as<const double>(), n, part.as<double>());
    hipLaunchKernelGGL(k_cw_final, dim3(1), dim3(kBlock), 0, st, part.as<const double>(), nb,
                       cw.as<double>(), k, mz.as<double>());
    hipLaunchKernelGGL(k_cw_update, dim3(nb), dim3(kBlock), 0, st, z.as<const double>(),
                       x.as<double>(), n, mz.as<const double>());
    GED_HIP(hipGetLastError());
  }
  double h[kSigmaIters];
  GED_HIP(hipMemcpyAsync(h, cw.p, sizeof(h), hipMemcpyDeviceToHost, st));
  GED_HIP(hipStreamSynchronize(st));
  double best = INFINITY;
  for (int k = 0; k < kSigmaIters; ++k) best = std::min(best, h[k]);
  g->sigma = sqrt(best * (1.0 + ldexp(1.0, -40)));
  return g->sigma;
}

}  // namespace ged
