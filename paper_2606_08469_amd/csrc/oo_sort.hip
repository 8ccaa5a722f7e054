// Spatial bucketing of the residual step's queries.
//
// The query kernel's cost is dominated by the texel gathers of the fine
// levels, whose tables (hundreds of MB) miss in the caches when queries come
// in sampling order. Grouping queries by a coarse octree cell before they
// are evaluated makes neighbouring query tiles read the same nodes' maps, so
// those lines are fetched once and then hit in L2. The grouping is a counting
// sort by the Morton code of the query's cell at octree level c = min(D, 4),
// with the secondary queries (q >= n_lhs) in a second key range, so the
// first n_lhs sorted positions are exactly the LHS queries the backward
// walks. The order inside a bucket is not fixed (LDS atomics hand out
// slots), which only changes the summation order of the gradients.
//
// Three passes over Q queries split into NB contiguous chunks:
//   1. per-chunk histograms in LDS          -> counts[NB][K]
//   2. per-bucket exclusive prefix over the chunks, bucket totals, and the
//      exclusive scan of the totals          -> counts (in place), start[K]
//   3. each chunk hands out slots from LDS cursors: order[pos] = q (the
//      query at sorted position pos) and rank[q] = pos.
// Only 4-byte indices move: the kernels that evaluate the sorted queries
// read positions and directions through order, and the residual assembly
// reads the sorted radiance through rank.
#include <hip/hip_runtime.h>

#include "oo_device.h"
#include "oo_internal.h"

namespace oo {

constexpr int kSortThreads = 1024;
constexpr int kSortMaxChunks = 256;

__device__ inline int sort_bucket(const float x[3], int D, int c, int64_t q, int64_t n_lhs) {
  const int sh = D - c;
  const int cx = quant_axis(x[0], D) >> sh, cy = quant_axis(x[1], D) >> sh, cz = quant_axis(x[2], D) >> sh;
  int code = 0;
  for (int b = 0; b < c; ++b)
    code |= (((cx >> b) & 1) | (((cy >> b) & 1) << 1) | (((cz >> b) & 1) << 2)) << (3 * b);
  return code + (q >= n_lhs ? (1 << (3 * c)) : 0);
}

__global__ __launch_bounds__(kSortThreads) void sort_hist_kernel(const QuerySrc src, int64_t Q, int64_t n_lhs, int D,
                                                                 int c, int K, int64_t chunk,
                                                                 int32_t* __restrict__ counts) {
  extern __shared__ int hist[];
  for (int b = threadIdx.x; b < K; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < Q ? lo + chunk : Q;
  for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) {
    float x[3];
    load_pos(src, q, x);
    atomicAdd(&hist[sort_bucket(x, D, c, q, n_lhs)], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < K; b += blockDim.x) counts[(int64_t)blockIdx.x * K + b] = hist[b];
}

// Thread b: exclusive prefix of bucket b's counts over the chunks (in place)
// and the bucket total.
__global__ __launch_bounds__(256) void sort_colscan_kernel(int32_t* __restrict__ counts, int NB, int K,
                                                           int32_t* __restrict__ total) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= K) return;
  constexpr int U = 16;
  int s = 0;
  for (int w0 = 0; w0 < NB; w0 += U) {
    int v[U];
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = w0 + j < NB ? counts[(int64_t)(w0 + j) * K + b] : 0;
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (w0 + j < NB) {
        counts[(int64_t)(w0 + j) * K + b] = s;
        s += v[j];
      }
  }
  total[b] = s;
}

// One workgroup: start[b] = sum of total[0 .. b-1].
__global__ __launch_bounds__(1024) void sort_start_kernel(const int32_t* __restrict__ total, int K,
                                                          int32_t* __restrict__ start) {
  __shared__ int part[1024];
  const int per = (K + 1023) / 1024, b0 = threadIdx.x * per;
  int s = 0;
  for (int j = 0; j < per; ++j)
    if (b0 + j < K) s += total[b0 + j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int j = 0; j < per; ++j)
    if (b0 + j < K) {
      start[b0 + j] = run;
      run += total[b0 + j];
    }
}

__global__ __launch_bounds__(kSortThreads) void sort_scatter_kernel(const QuerySrc src, int64_t Q, int64_t n_lhs,
                                                                    int D, int c, int K, int64_t chunk,
                                                                    const int32_t* __restrict__ prefix,
                                                                    const int32_t* __restrict__ start,
                                                                    int32_t* __restrict__ order,
                                                                    int32_t* __restrict__ rank) {
  extern __shared__ int cur[];
  for (int b = threadIdx.x; b < K; b += blockDim.x) cur[b] = start[b] + prefix[(int64_t)blockIdx.x * K + b];
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < Q ? lo + chunk : Q;
  for (int64_t q = lo + threadIdx.x; q < hi; q += blockDim.x) {
    float x[3];
    load_pos(src, q, x);
    const int pos = atomicAdd(&cur[sort_bucket(x, D, c, q, n_lhs)], 1);
    order[pos] = (int32_t)q;
    rank[q] = pos;
  }
}

SortShape sort_shape(int64_t Q, int D) {
  SortShape s;
  s.c = D < 4 ? D : 4;
  s.K = 2 << (3 * s.c);
  int64_t nb = (Q + kSortThreads - 1) / kSortThreads;
  s.NB = (int)(nb < 1 ? 1 : (nb > kSortMaxChunks ? kSortMaxChunks : nb));
  s.chunk = (Q + s.NB - 1) / s.NB;
  return s;
}

hipError_t launch_spatial_sort(const QuerySrc& src, int64_t Q, int64_t n_lhs, int D, int32_t* counts, int32_t* total,
                               int32_t* start, int32_t* order, int32_t* rank, hipStream_t st) {
  if (Q == 0) return hipSuccess;
  const SortShape s = sort_shape(Q, D);
  const size_t lds = (size_t)s.K * sizeof(int);
  hipLaunchKernelGGL(sort_hist_kernel, dim3(s.NB), dim3(kSortThreads), lds, st, src, Q, n_lhs, D, s.c, s.K, s.chunk,
                     counts);
  hipLaunchKernelGGL(sort_colscan_kernel, dim3((s.K + 255) / 256), dim3(256), 0, st, counts, s.NB, s.K, total);
  hipLaunchKernelGGL(sort_start_kernel, dim3(1), dim3(1024), 0, st, total, s.K, start);
  hipLaunchKernelGGL(sort_scatter_kernel, dim3(s.NB), dim3(kSortThreads), lds, st, src, Q, n_lhs, D, s.c, s.K, s.chunk,
                     counts, start, order, rank);
  return hipGetLastError();
}

}  // namespace oo
