// Backward of the disparity predictor (Sec. 3.3 disparity equation, Sec. 3.5
// hash-grid network): from each backward query's dLoss/d disparity to the
// predictor's MLP parameters and hash-table entries.
//
// Two passes over the sorted backward queries, a bounded number at a time:
//  1. one thread per query recomputes the predictor's input and hidden
//     activations, carries its seed s = dLoss/d disparity back through the
//     layers (ReLU'(0) = 0), adds the trilinear shares of the encoding's
//     gradient to the hash entries it read (FP32 atomics), and leaves its
//     activations and deltas as rows in memory;
//  2. the parameter gradients are matrix products over those rows,
//     dW | db of a layer = sum_q delta_q [a_q, 1]^T, on 16x16x4 FP32 MFMA
//     tiles with the queries along K; each workgroup leaves the sums over
//     its share of the queries in partials[blockIdx][P] (reduced in
//     workgroup order afterwards).
#include <hip/hip_runtime.h>

#include "oo_device.h"
#include "oo_internal.h"

namespace oo {

namespace {

// Rows of one pass: input (36 wide) and hidden rows are followed by a 1 (the
// bias column of the next product) and zeros up to a whole 16-column tile.
constexpr int kRowA = 48;
constexpr int kRowH = 80;
constexpr int kRowFloats = kRowA + kDispH + kRowH + kDispH + kRowH + 1;

struct DispRows {
  float* a0;  // [n][kRowA]  predictor input
  float* d1;  // [n][kDispH] delta of the first hidden layer
  float* h1;  // [n][kRowH]  first hidden layer (ReLU'd)
  float* d2;  // [n][kDispH] delta of the second hidden layer (two hidden layers)
  float* h2;  // [n][kRowH]  second hidden layer
  float* s;   // [n]         dLoss/d disparity
};

DispRows carve_rows(float* base, int64_t cap) {
  DispRows R;
  R.a0 = base;
  R.d1 = R.a0 + cap * kRowA;
  R.h1 = R.d1 + cap * kDispH;
  R.d2 = R.h1 + cap * kRowH;
  R.h2 = R.d2 + cap * kDispH;
  R.s = R.h2 + cap * kRowH;
  return R;
}

// Row tail: a 1 at column n, zeros up to `width` (n and width multiples of 4).
__device__ __forceinline__ void store_tail(float* row, int n, int width) {
  reinterpret_cast<float4*>(row + n)[0] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
  for (int k = n + 4; k < width; k += 4) reinterpret_cast<float4*>(row + k)[0] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__device__ __forceinline__ void store_chunk(float* row, const float (&v)[kDispChunk]) {
#pragma unroll
  for (int j = 0; j < kDispChunk; j += 4)
    reinterpret_cast<float4*>(row + j)[0] = make_float4(v[j], v[j + 1], v[j + 2], v[j + 3]);
}

// genc[k] += sum_j W_0[c + j][k] d1[j] for the encoding's columns k < 2 L_h.
__device__ __forceinline__ void add_enc_grad(const float* W0, int c, const float (&d1)[kDispChunk],
                                             float (&genc)[kDispF * kHashLevels]) {
  const cfloat_ptr Wc = uniform_ptr(W0 + c * kDispK);
#pragma unroll
  for (int j = 0; j < kDispChunk; ++j) {
#pragma unroll
    for (int k = 0; k < kDispF * kHashLevels; ++k) genc[k] += Wc[j * kDispK + k] * d1[j];
    if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the weights in flight
  }
}

}  // namespace

// The 16 values of one (query, level) (corner c, feature f at 2 c + f),
// summed over the lanes of `m` (a wave-uniform mask), transposed across the
// wave: afterwards lane l holds the sum of value 8 b0 + 4 b1 + 2 b2 + b3
// (b_k bit k of l). Four halving exchange steps and two plain ones: 17
// shuffles in place of 6 per value. Every lane of the wave takes part.
__device__ __forceinline__ float group_sum16(const float (&v)[16], uint64_t m, int lane) {
  const bool in = (m >> lane) & 1;
  float t[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) t[k] = in ? v[k] : 0.0f;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int half = 8 >> st;
    const bool upper = (lane >> st) & 1;
#pragma unroll
    for (int k = 0; k < half; ++k) {
      const float give = upper ? t[k] : t[k + half];
      const float keep = upper ? t[k + half] : t[k];
      t[k] = keep + __shfl_xor(give, 1 << st);
    }
  }
  t[0] += __shfl_xor(t[0], 16);
  t[0] += __shfl_xor(t[0], 32);
  return t[0];
}

// Pass 1: rows r < n of this pass are sorted positions q0 + r. Lanes past
// n stay (their seed is 0) so that every wave-wide exchange sees 64 lanes.
__global__ __launch_bounds__(256) void disparity_rows_kernel(const DispArgs G, const QuerySrc src, int64_t q0,
                                                             int64_t n, const float* __restrict__ dd,
                                                             float* __restrict__ dtables, const DispRows R) {
  const int64_t r0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = r0 < n;
  const int64_t r = valid ? r0 : 0;  // rows of lanes past n are not written
  const int lane = threadIdx.x & 63;
  const int64_t q = q0 + r;
  float x[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
  if (valid) load_query(src, q, x, d);
  const float s = valid ? dd[q] : 0.0f;
  float u[3];
  unit_dir3(d, u);
  float a[kDispK];
  disparity_input(G, x, u, a);
  float* const a0r = R.a0 + r * kRowA;
  if (valid) {
#pragma unroll
    for (int k = 0; k < kDispK; k += 4)
      reinterpret_cast<float4*>(a0r + k)[0] = make_float4(a[k], a[k + 1], a[k + 2], a[k + 3]);
    store_tail(a0r, kDispK, kRowA);
    R.s[r] = s;
  }
  // (selected, not indexed: a runtime index into the argument's arrays
  // would copy them to scratch memory)
  const bool two = G.n_layers == 3;
  const float* const W0 = G.W[0];
  const float* const W1 = G.W[1];
  const float* const Wout = two ? G.W[2] : G.W[1];
  float* const h1r = R.h1 + r * kRowH;
  float* const d1r = R.d1 + r * kDispH;
  float genc[kDispF * kHashLevels];
#pragma unroll
  for (int k = 0; k < kDispF * kHashLevels; ++k) genc[k] = 0.0f;
  if (two) {
    float d2[kDispH];
    {
      float z2[kDispH];
      disp_hidden2(G, W0, W1, a, z2, [&](int c, const float (&h1)[kDispChunk]) {
        if (valid) store_chunk(h1r + c, h1);
      });
      float* const h2r = R.h2 + r * kRowH;
      float* const d2r = R.d2 + r * kDispH;
#pragma unroll
      for (int o = 0; o < kDispH; o += 4) {
        float h2[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          h2[j] = fmaxf(z2[o + j], 0.0f);
          d2[o + j] = h2[j] > 0.0f ? Wout[o + j] * s : 0.0f;
        }
        if (valid) {
          reinterpret_cast<float4*>(h2r + o)[0] = make_float4(h2[0], h2[1], h2[2], h2[3]);
          reinterpret_cast<float4*>(d2r + o)[0] = make_float4(d2[o], d2[o + 1], d2[o + 2], d2[o + 3]);
        }
      }
      if (valid) store_tail(h2r, kDispH, kRowH);
    }
    // delta_1 = ReLU'(z_1) (W_1^T delta_2), a chunk of units at a time; the
    // chunk's activations come back from the row just written (a lane past n
    // reads row 0 and gets a zero delta: its delta_2 is zero)
#pragma unroll 1
    for (int c = 0; c < kDispH; c += kDispChunk) {
      float t[kDispChunk];
#pragma unroll
      for (int j = 0; j < kDispChunk; ++j) t[j] = 0.0f;
      const cfloat_ptr W1c = uniform_ptr(W1 + c);
#pragma unroll
      for (int o = 0; o < kDispH; ++o) {
#pragma unroll
        for (int j = 0; j < kDispChunk; ++j) t[j] += W1c[o * kDispH + j] * d2[o];
        if ((o & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
      float d1[kDispChunk];
#pragma unroll
      for (int j = 0; j < kDispChunk; j += 4) {
        const float4 h = reinterpret_cast<const float4*>(h1r + c + j)[0];
        d1[j] = h.x > 0.0f ? t[j] : 0.0f;
        d1[j + 1] = h.y > 0.0f ? t[j + 1] : 0.0f;
        d1[j + 2] = h.z > 0.0f ? t[j + 2] : 0.0f;
        d1[j + 3] = h.w > 0.0f ? t[j + 3] : 0.0f;
      }
      if (valid) store_chunk(d1r + c, d1);
      add_enc_grad(W0, c, d1, genc);
    }
  } else {
#pragma unroll 1
    for (int c = 0; c < kDispH; c += kDispChunk) {
      float h1[kDispChunk], d1[kDispChunk];
      disp_chunk0(G, W0, c, a, h1);
      const cfloat_ptr Woc = uniform_ptr(Wout + c);
#pragma unroll
      for (int j = 0; j < kDispChunk; ++j) d1[j] = h1[j] > 0.0f ? Woc[j] * s : 0.0f;
      if (valid) {
        store_chunk(h1r + c, h1);
        store_chunk(d1r + c, d1);
      }
      add_enc_grad(W0, c, d1, genc);
    }
  }
  if (valid) store_tail(h1r, kDispH, kRowH);
  // the encoding's gradient into the hash entries of the query's eight
  // vertices per level, with their trilinear weights. Lanes of the wave in
  // the same grid cell of a level read the same eight entries: while the
  // first pending lane's cell is shared by others, that group's sums go out
  // as one add per entry; the lanes left add their own shares.
  // (unrolled: genc is indexed by compile-time levels only)
  const uint64_t seeded = __ballot(s != 0.0f);
  if (seeded == 0) return;
#pragma unroll
  for (int i = 0; i < kHashLevels; ++i) {
    if (i >= G.n_levels) break;
    const float g0 = genc[2 * i], g1 = genc[2 * i + 1];
    const int N = G.res[i];
    int base[3];
    float f[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) hash_cell(x[ax], N, base[ax], f[ax]);
    float v[16];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float w = ((c & 1) ? f[0] : 1.0f - f[0]) * (((c >> 1) & 1) ? f[1] : 1.0f - f[1]) *
                      ((c >> 2) ? f[2] : 1.0f - f[2]);
      v[2 * c] = w * g0;
      v[2 * c + 1] = w * g1;
    }
    float* tab = dtables + ((size_t)i << G.log2_T) * kDispF;
    // cell key: base < N <= 2^11 per axis
    const uint32_t klo = (uint32_t)base[0] | ((uint32_t)base[1] << 16);
    const uint32_t khi = (uint32_t)base[2];
    uint64_t pend = seeded;
    while (pend) {
      const int ld = __builtin_ctzll(pend);
      const uint32_t llo = __builtin_amdgcn_readlane(klo, ld), lhi = __builtin_amdgcn_readlane(khi, ld);
      const uint64_t m = __ballot(klo == llo && khi == lhi) & pend;
      if (__builtin_popcountll(m) < 2) break;
      pend &= ~m;
      const float t = group_sum16(v, m, lane);
      if (lane < 16) {
        // lane l holds value 8 b0 + 4 b1 + 2 b2 + b3: corner and feature
        const int idx = ((lane & 1) << 3) | ((lane & 2) << 1) | ((lane & 4) >> 1) | ((lane & 8) >> 3);
        const int c = idx >> 1;
        const uint32_t e = hash_entry(G, i, (llo & 0xffffu) + (c & 1), (llo >> 16) + ((c >> 1) & 1), lhi + (c >> 2));
        if (t != 0.0f) unsafeAtomicAdd(tab + (size_t)e * kDispF + (idx & 1), t);
      }
    }
    if (pend) {
      // The lanes left add their own shares. An atomic instruction costs
      // one request per 64-byte chunk it touches, and a query's two
      // x-neighbouring vertices (both features) mostly sit in one chunk:
      // so four lanes take one (query, y, z) vertex pair, lane 4 j + 2 dx + f
      // adding feature f of vertex dx for the query of lane j + 16 h. Same
      // instruction count, a third of the requests.
      uint32_t ev[8];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        ev[c] = hash_entry(G, i, base[0] + (c & 1), base[1] + ((c >> 1) & 1), base[2] + (c >> 2));
      const int sub = lane & 3;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (((pend >> (16 * h)) & 0xffffu) == 0) continue;  // wave-uniform
        const int src = (lane >> 2) + 16 * h;
        const bool act = (pend >> src) & 1;
#pragma unroll
        for (int yz = 0; yz < 4; ++yz) {
          const int c0 = 2 * yz;  // vertex dx = 0 of this (y, z); dx = 1 is c0 + 1
          const float t0 = __shfl(v[2 * c0], src), t1 = __shfl(v[2 * c0 + 1], src);
          const float t2 = __shfl(v[2 * c0 + 2], src), t3 = __shfl(v[2 * c0 + 3], src);
          const uint32_t e0 = __shfl(ev[c0], src), e1 = __shfl(ev[c0 + 1], src);
          const float val = sub == 0 ? t0 : (sub == 1 ? t1 : (sub == 2 ? t2 : t3));
          const uint32_t e = sub < 2 ? e0 : e1;
          if (act) unsafeAtomicAdd(tab + (size_t)e * kDispF + (sub & 1), val);
        }
      }
    }
  }
}

namespace {

// One wave's product: NM x NN output tiles of sum_q A[q][16 (m0 + m) + i] *
// B[q][16 n + j] over rows [b, e), four queries per MFMA. With SEED the A
// operand is the seed column s[q] in row 0 (the output layer's delta).
template <int NM, int NN, bool SEED>
__device__ __forceinline__ void row_products(const float* __restrict__ A, int lda, int m0, const float* __restrict__ B,
                                             int ldb, int64_t b, int64_t e, int lane, f32x4 (&acc)[NM][NN]) {
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int nn = 0; nn < NN; ++nn) acc[m][nn] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int g = lane >> 4, i = lane & 15;
  constexpr int U = 4;  // MFMA steps per iteration (16 queries): loads of all four go out first
  for (int64_t q = b; q < e; q += 4 * U) {
    float av[U][NM], bv[U][NN];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = q + 4 * u + g;
      const bool ok = row < e;
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        if constexpr (SEED)
          av[u][m] = ok && i == 0 ? A[row] : 0.0f;
        else
          av[u][m] = ok ? A[row * lda + 16 * (m0 + m) + i] : 0.0f;
      }
#pragma unroll
      for (int nn = 0; nn < NN; ++nn) bv[u][nn] = ok ? B[row * ldb + 16 * nn + i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int nn = 0; nn < NN; ++nn)
          acc[m][nn] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u][m], bv[u][nn], acc[m][nn], 0, 0, 0);
  }
}

// Stores a wave's tiles into the flat parameter partials: element (o, k) of
// tile (m, n) is W[o][k] for k < n_in (rows o < n_out), b[o] for k = n_in.
template <int NM, int NN>
__device__ __forceinline__ void store_params(const f32x4 (&acc)[NM][NN], int m0, int n_in, int n_out, int w_off,
                                             int b_off, float* part, bool accumulate, int lane) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int nn = 0; nn < NN; ++nn)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int o = 16 * (m0 + m) + 4 * g + j, k = 16 * nn + i;
        if (o >= n_out || k > n_in) continue;
        float* p = part + (k < n_in ? w_off + o * n_in + k : b_off + o);
        *p = accumulate ? *p + acc[m][nn][j] : acc[m][nn][j];
      }
}

}  // namespace

// Pass 2: workgroup g takes rows [g per, (g + 1) per) of the pass. Its four
// waves split the products: with two hidden layers D1^T [A0 1] (4 x 3
// tiles), D2^T [H1 1] (two waves of 2 x 5) and s [H2 1] (1 x 5); with one,
// D1^T [A0 1] (two waves of 2 x 3) and s [H1 1].
__global__ __launch_bounds__(256) void disparity_params_kernel(const DispRows R, int64_t n, int two_hidden,
                                                               float* __restrict__ partials, int P, int accumulate) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + 3) / 4 * 4;
  const int64_t b = (int64_t)blockIdx.x * per, e = b + per < n ? b + per : n;
  float* const part = partials + (int64_t)blockIdx.x * P;
  const bool acc_in = accumulate != 0;
  // flat layout W_0, b_0, (W_1, b_1,) W_out, b_out
  const int w0 = 0, b0 = kDispH * kDispK;
  const int w1 = b0 + kDispH, b1 = w1 + kDispH * kDispH;
  const int wo = two_hidden ? b1 + kDispH : w1, bo = wo + kDispH;
  if (two_hidden) {
    if (wave == 0) {
      f32x4 acc[4][3];
      row_products<4, 3, false>(R.d1, kDispH, 0, R.a0, kRowA, b, e, lane, acc);
      store_params<4, 3>(acc, 0, kDispK, kDispH, w0, b0, part, acc_in, lane);
    } else if (wave <= 2) {
      const int m0 = 2 * (wave - 1);
      f32x4 acc[2][5];
      row_products<2, 5, false>(R.d2, kDispH, m0, R.h1, kRowH, b, e, lane, acc);
      store_params<2, 5>(acc, m0, kDispH, kDispH, w1, b1, part, acc_in, lane);
    } else {
      f32x4 acc[1][5];
      row_products<1, 5, true>(R.s, 0, 0, R.h2, kRowH, b, e, lane, acc);
      store_params<1, 5>(acc, 0, kDispH, 1, wo, bo, part, acc_in, lane);
    }
  } else {
    if (wave <= 1) {
      const int m0 = 2 * wave;
      f32x4 acc[2][3];
      row_products<2, 3, false>(R.d1, kDispH, m0, R.a0, kRowA, b, e, lane, acc);
      store_params<2, 3>(acc, m0, kDispK, kDispH, w0, b0, part, acc_in, lane);
    } else if (wave == 2) {
      f32x4 acc[1][5];
      row_products<1, 5, true>(R.s, 0, 0, R.h1, kRowH, b, e, lane, acc);
      store_params<1, 5>(acc, 0, kDispH, 1, wo, bo, part, acc_in, lane);
    }
  }
}

int disparity_bwd_grid(int64_t Q) {
  const int64_t chunks = (Q + 255) / 256;
  return (int)(chunks < 256 ? (chunks > 0 ? chunks : 1) : 256);
}

int64_t disparity_rows_cap(int64_t Q) {
  const int64_t cap = (Q + 63) / 64 * 64;
  return cap < kDispRowsMax ? cap : kDispRowsMax;
}

int64_t disparity_rows_floats(int64_t cap) { return cap * kRowFloats; }

int32_t disparity_params(const DispArgs& G) {
  int32_t P = kDispH * G.K + kDispH;
  if (G.n_layers == 3) P += kDispH * kDispH + kDispH;
  return P + kDispH + 1;
}

hipError_t launch_disparity_bwd(const DispArgs& G, const QuerySrc& src, int64_t Q, const float* dd, float* dtables,
                                float* rows, int64_t cap, float* partials, int grid, hipStream_t st) {
  if (Q == 0) return hipSuccess;
  const DispRows R = carve_rows(rows, cap);
  const int P = disparity_params(G);
  for (int64_t q0 = 0; q0 < Q; q0 += cap) {
    const int64_t n = Q - q0 < cap ? Q - q0 : cap;
    hipLaunchKernelGGL(disparity_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, G, src, q0, n, dd,
                       dtables, R);
    hipLaunchKernelGGL(disparity_params_kernel, dim3(grid), dim3(256), 0, st, R, n, G.n_layers == 3 ? 1 : 0, partials,
                       P, q0 > 0 ? 1 : 0);
  }
  return hipGetLastError();
}

}  // namespace oo
