// Optimiser step over the FP32 masters (Adam, lazy over feature-map blocks
// no query read, fused with the working-copy refresh and the gradient
// clear), and the marking of the nodes a residual batch read.
#include <hip/hip_runtime.h>

#include "oo_device.h"
#include "oo_internal.h"

namespace oo {

// Four elements per thread over the concatenated segments: segment s owns
// the thread indices [first[s], first[s + 1]). A thread reads the block
// flag of its first element; blocks are whole multiples of 4 elements
// (every table block is res^2 C or (res+1)^2 C with C in {4, 8}), so the
// four elements share it. The last thread of a segment may hold fewer than
// four elements.
template <class WT>
__global__ __launch_bounds__(256) void adam_kernel(const AdamArgs A) {
  const int64_t total = A.first[A.n_segs];
  for (int64_t tq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; tq < total;
       tq += (int64_t)gridDim.x * blockDim.x) {
    int s = 0;
    while (s + 1 < A.n_segs && tq >= A.first[s + 1]) ++s;
    const AdamSeg& S = A.seg[s];
    const int64_t i0 = (tq - A.first[s]) * 4;
    if (S.touched && !S.touched[i0 / S.block]) continue;
    const int cnt = S.n - i0 < 4 ? (int)(S.n - i0) : 4;
    for (int k = 0; k < cnt; ++k) {
      const int64_t i = i0 + k;
      const float g = S.grad[i];
      const float m = A.b1 * S.m[i] + (1.0f - A.b1) * g;
      const float v = A.b2 * S.v[i] + (1.0f - A.b2) * g * g;
      const float p = S.param[i] - A.lr * (m * A.inv_c1) / (sqrtf(v * A.inv_c2) + A.eps);
      S.m[i] = m;
      S.v[i] = v;
      S.param[i] = p;
      S.grad[i] = 0.0f;
      if (S.work) reinterpret_cast<WT*>(S.work)[i] = from_f32<WT>(p);
    }
  }
}

hipError_t launch_adam(const AdamArgs& A, oo_dtype wd, hipStream_t st) {
  const int64_t total = A.first[A.n_segs];
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  if (wd == OO_F16)
    hipLaunchKernelGGL(adam_kernel<f16>, dim3((unsigned)blocks), dim3(256), 0, st, A);
  else if (wd == OO_BF16)
    hipLaunchKernelGGL(adam_kernel<bf16>, dim3((unsigned)blocks), dim3(256), 0, st, A);
  else
    hipLaunchKernelGGL(adam_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, A);
  return hipGetLastError();
}

// touched[node] = 1 for every stored node index of the n backward queries
// ([rows][n], rows = levels x corners) that lies in [0, n_nodes).
__global__ __launch_bounds__(256) void touched_kernel(const int32_t* __restrict__ nidx, int64_t n, int64_t rows,
                                                      int64_t n_nodes, uint32_t* __restrict__ touched) {
  const int64_t total = n * rows, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int32_t v = nidx[e];
    if (v >= 0 && v < n_nodes) touched[v] = 1u;
  }
}

hipError_t launch_touched(const int32_t* nidx, int64_t n, int64_t rows, int64_t n_nodes, uint32_t* touched,
                          hipStream_t st) {
  const int64_t total = n * rows;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  hipLaunchKernelGGL(touched_kernel, dim3((unsigned)blocks), dim3(256), 0, st, nidx, n, rows, n_nodes, touched);
  return hipGetLastError();
}

}  // namespace oo
