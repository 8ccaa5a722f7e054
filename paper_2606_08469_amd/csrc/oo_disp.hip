// Backward of the disparity predictor (Sec. 3.3 disparity equation, Sec. 3.5
// hash-grid network): from each backward query's dLoss/d disparity to the
// predictor's MLP parameters and hash-table entries.
#include <hip/hip_runtime.h>

#include "oo_device.h"
#include "oo_internal.h"

namespace oo {

namespace {

// Per-lane rows in LDS, padded to odd strides so that a lane reading its own
// row and the wave reading one column both hit distinct banks.
constexpr int kTile = 64;
constexpr int kA0S = kDispK + 1;
constexpr int kHS = kDispH + 1;
// Parameters of the largest predictor (two hidden layers): W_0, b_0, W_1,
// b_1, W_out, b_out.
constexpr int kMaxP = kDispH * kDispK + kDispH + kDispH * kDispH + kDispH + kDispH + 1;
// rows, then the parameter sums
constexpr size_t kLds = sizeof(float) * (kTile * kA0S + 4 * kTile * kHS + kTile + kMaxP);

}  // namespace

// One wave per workgroup, persistent over 64-query tiles of the sorted
// backward queries. Per tile:
//  1. each lane recomputes its query's input and hidden activations, carries
//     its seed s = dLoss/d disparity back (delta of each hidden layer, with
//     ReLU'(0) = 0), adds the trilinear shares of the encoding's gradient to
//     the hash entries it read (FP32 atomics), and leaves activations and
//     deltas in LDS rows;
//  2. the wave adds the tile's dW = sum_q delta_{i+1} a_i^T and db = sum_q
//     delta_{i+1} to the workgroup's sums in LDS (lane j owns parameters j,
//     j + 64, ... of the flat layout W_0, b_0, (W_1, b_1,) W_out, b_out).
// Each workgroup writes its sums to partials[blockIdx][P] (reduced in
// workgroup order afterwards). Hidden units are handled kDispChunk at a
// time, as in the forward, to bound the registers a lane holds.
__global__ __launch_bounds__(64) void disparity_bwd_kernel(const DispArgs G, const QuerySrc src, int64_t Q,
                                                           const float* __restrict__ dd, float* __restrict__ dtables,
                                                           float* __restrict__ partials, int32_t P) {
  extern __shared__ float smem[];
  float* const a0s = smem;
  float* const h1s = a0s + kTile * kA0S;
  float* const h2s = h1s + kTile * kHS;
  float* const d1s = h2s + kTile * kHS;
  float* const d2s = d1s + kTile * kHS;
  float* const dos = d2s + kTile * kHS;
  float* const accs = dos + kTile;
  const int lane = threadIdx.x;
  const int K = kDispK, NL = G.n_layers;
  const bool two = NL == 3;
  // the weights: every lane reads the same address (scalar loads)
  const float* const w0s = G.W[0];
  const float* const w1s = G.W[1];
  const float* const Wout = two ? G.W[2] : G.W[1];
  for (int p = lane; p < P; p += kTile) accs[p] = 0.0f;
  __syncthreads();
  const int64_t n_tiles = (Q + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t q = tile * kTile + lane;
    const bool valid = q < Q;
    float x[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
    if (valid) load_query(src, q, x, d);
    const float s = valid ? dd[q] : 0.0f;
    float u[3];
    unit_dir3(d, u);
    float a[kDispK];
    disparity_input(G, x, u, a);
#pragma unroll
    for (int k = 0; k < kDispK; ++k) a0s[lane * kA0S + k] = a[k];
    dos[lane] = s;
    float* const h1r = h1s + lane * kHS;
    float* const d1r = d1s + lane * kHS;
    float* const d2r = d2s + lane * kHS;
    if (two) {
      {
        float z2[kDispH];
        disp_hidden2(G, w0s, w1s, a, z2, [&](int c, const float (&h1)[kDispChunk]) {
#pragma unroll
          for (int j = 0; j < kDispChunk; ++j) h1r[c + j] = h1[j];
        });
#pragma unroll
        for (int o = 0; o < kDispH; ++o) {
          const float h2 = fmaxf(z2[o], 0.0f);
          h2s[lane * kHS + o] = h2;
          d2r[o] = h2 > 0.0f ? Wout[o] * s : 0.0f;
        }
      }
      // delta_1 = ReLU'(z_1) (W_1^T delta_2), a chunk of units at a time
#pragma unroll 1
      for (int c = 0; c < kDispH; c += kDispChunk) {
        float t[kDispChunk];
#pragma unroll
        for (int j = 0; j < kDispChunk; ++j) t[j] = 0.0f;
#pragma unroll 4
        for (int o = 0; o < kDispH; ++o) {
          const float g2 = d2r[o];
#pragma unroll
          for (int j = 0; j < kDispChunk; ++j) t[j] += w1s[o * kDispH + c + j] * g2;
          __builtin_amdgcn_sched_barrier(0);  // bound the weights in flight
        }
#pragma unroll
        for (int j = 0; j < kDispChunk; ++j) d1r[c + j] = h1r[c + j] > 0.0f ? t[j] : 0.0f;
      }
    } else {
#pragma unroll 1
      for (int c = 0; c < kDispH; c += kDispChunk) {
        float h1[kDispChunk];
        disp_chunk0(G, w0s, c, a, h1);
#pragma unroll
        for (int j = 0; j < kDispChunk; ++j) {
          h1r[c + j] = h1[j];
          d1r[c + j] = h1[j] > 0.0f ? Wout[c + j] * s : 0.0f;
        }
      }
    }
    // the encoding's gradient (W_0^T delta_1, level by level) into the hash
    // entries of the query's eight vertices, with their trilinear weights
    if (s != 0.0f) {
#pragma unroll 1
      for (int i = 0; i < G.n_levels; ++i) {
        float g0 = 0.0f, g1 = 0.0f;
#pragma unroll 4
        for (int o = 0; o < kDispH; ++o) {
          const float d1 = d1r[o];
          g0 += w0s[o * kDispK + 2 * i] * d1;
          g1 += w0s[o * kDispK + 2 * i + 1] * d1;
          if ((o & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        const int N = G.res[i];
        int base[3];
        float f[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) hash_cell(x[ax], N, base[ax], f[ax]);
        float* tab = dtables + ((size_t)i << G.log2_T) * kDispF;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const float w = ((c & 1) ? f[0] : 1.0f - f[0]) * (((c >> 1) & 1) ? f[1] : 1.0f - f[1]) *
                          ((c >> 2) ? f[2] : 1.0f - f[2]);
          const uint32_t e = hash_entry(G, i, base[0] + (c & 1), base[1] + ((c >> 1) & 1), base[2] + (c >> 2));
          unsafeAtomicAdd(tab + (size_t)e * kDispF, w * g0);
          unsafeAtomicAdd(tab + (size_t)e * kDispF + 1, w * g1);
        }
      }
    }
    __syncthreads();
    // this tile's share of every parameter's gradient
    const int nW0 = kDispH * K;
#pragma unroll 1
    for (int p = lane; p < P; p += kTile) {
      float sum = 0.0f;
      if (p < nW0) {
        const int o = p / K, k = p % K;
        #pragma unroll 4
        for (int t = 0; t < kTile; ++t) sum += d1s[t * kHS + o] * a0s[t * kA0S + k];
      } else if (p < nW0 + kDispH) {
        const int o = p - nW0;
        #pragma unroll 4
        for (int t = 0; t < kTile; ++t) sum += d1s[t * kHS + o];
      } else {
        int r = p - nW0 - kDispH;
        const float* hl = h1s;
        bool done = false;
        if (two) {
          if (r < kDispH * kDispH) {
            const int o = r / kDispH, k = r % kDispH;
            #pragma unroll 4
            for (int t = 0; t < kTile; ++t) sum += d2s[t * kHS + o] * h1s[t * kHS + k];
            done = true;
          } else {
            r -= kDispH * kDispH;
            if (r < kDispH) {
              #pragma unroll 4
              for (int t = 0; t < kTile; ++t) sum += d2s[t * kHS + r];
              done = true;
            } else {
              r -= kDispH;
              hl = h2s;
            }
          }
        }
        if (!done) {
          if (r < kDispH) {  // output layer weights
            #pragma unroll 4
            for (int t = 0; t < kTile; ++t) sum += dos[t] * hl[t * kHS + r];
          } else {  // output bias
            #pragma unroll 4
            for (int t = 0; t < kTile; ++t) sum += dos[t];
          }
        }
      }
      accs[p] += sum;
    }
    __syncthreads();
  }
  float* part = partials + (int64_t)blockIdx.x * P;
  for (int p = lane; p < P; p += kTile) part[p] = accs[p];
}

int disparity_bwd_grid(int64_t Q) {
  const int64_t tiles = (Q + kTile - 1) / kTile;
  return (int)(tiles < 512 ? (tiles > 0 ? tiles : 1) : 512);
}

int32_t disparity_params(const DispArgs& G) {
  int32_t P = kDispH * G.K + kDispH;
  if (G.n_layers == 3) P += kDispH * kDispH + kDispH;
  return P + kDispH + 1;
}

hipError_t launch_disparity_bwd(const DispArgs& G, const QuerySrc& src, int64_t Q, const float* dd, float* dtables,
                                float* partials, int grid, hipStream_t st) {
  if (Q == 0) return hipSuccess;
  hipFuncSetAttribute((const void*)disparity_bwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds);
  hipLaunchKernelGGL(disparity_bwd_kernel, dim3(grid), dim3(kTile), kLds, st, G, src, Q, dd, dtables, partials,
                     disparity_params(G));
  return hipGetLastError();
}

}  // namespace oo
