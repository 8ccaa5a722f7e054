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
// four elements. Segments whose arrays are all 16-byte aligned (8-byte for
// a 16-bit working copy) move each array as one vector per thread.
__device__ inline float adam_update(const AdamArgs& A, float& p, float& m, float& v, float g) {
  m = A.b1 * m + (1.0f - A.b1) * g;
  v = A.b2 * v + (1.0f - A.b2) * g * g;
  p = p - A.lr * (m * A.inv_c1) / (sqrtf(v * A.inv_c2) + A.eps);
  return p;
}

template <class WT>
__global__ __launch_bounds__(256) void adam_kernel(const AdamArgs A) {
  const int64_t total = A.first[A.n_segs];
  typedef WT w4 __attribute__((ext_vector_type(4)));
  for (int64_t tq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; tq < total;
       tq += (int64_t)gridDim.x * blockDim.x) {
    int s = 0;
    while (s + 1 < A.n_segs && tq >= A.first[s + 1]) ++s;
    const AdamSeg& S = A.seg[s];
    const int64_t i0 = (tq - A.first[s]) * 4;
    if (S.touched && !S.touched[i0 / S.block]) continue;
    const int cnt = S.n - i0 < 4 ? (int)(S.n - i0) : 4;
    if (S.vec && cnt == 4) {
      float4 p = *reinterpret_cast<const float4*>(S.param + i0);
      float4 m = *reinterpret_cast<const float4*>(S.m + i0);
      float4 v = *reinterpret_cast<const float4*>(S.v + i0);
      const float4 g = *reinterpret_cast<const float4*>(S.grad + i0);
      adam_update(A, p.x, m.x, v.x, g.x);
      adam_update(A, p.y, m.y, v.y, g.y);
      adam_update(A, p.z, m.z, v.z, g.z);
      adam_update(A, p.w, m.w, v.w, g.w);
      *reinterpret_cast<float4*>(S.param + i0) = p;
      *reinterpret_cast<float4*>(S.m + i0) = m;
      *reinterpret_cast<float4*>(S.v + i0) = v;
      *reinterpret_cast<float4*>(S.grad + i0) = make_float4(0.f, 0.f, 0.f, 0.f);
      if (S.work) {
        w4 w;
        w[0] = from_f32<WT>(p.x);
        w[1] = from_f32<WT>(p.y);
        w[2] = from_f32<WT>(p.z);
        w[3] = from_f32<WT>(p.w);
        *reinterpret_cast<w4*>(reinterpret_cast<WT*>(S.work) + i0) = w;
      }
      continue;
    }
    for (int k = 0; k < cnt; ++k) {
      const int64_t i = i0 + k;
      float p = S.param[i], m = S.m[i], v = S.v[i];
      adam_update(A, p, m, v, S.grad[i]);
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
