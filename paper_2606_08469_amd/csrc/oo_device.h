// Device-side building blocks shared by the forward and backward kernels:
// octree descent, octahedral map, bilinear taps, texel gathers, and the
// matrix-core fragment conventions used by the decoder MLP.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "octaoctree.h"

namespace oo {

constexpr int kMaxLevels = OO_MAX_LEVELS;
constexpr int kMaxLayers = OO_MAX_LAYERS;
constexpr int kWave = 64;

// Kernel-argument copy of oo_tree (levels with no node point at level 0's
// table so that predicated dummy loads stay in bounds).
struct TreeArgs {
  int32_t L, C, D;
  int32_t interp;  // OO_INTERP_NODE_BILINEAR or OO_INTERP_PAPER
  int32_t res[kMaxLevels];
  int64_t off[kMaxLevels + 1];
  const uint32_t* nodes;
  const void* feat[kMaxLevels];
};

// Kernel-argument copy of oo_disparity (forward parameters). The GPU
// predictor has 16 hash levels of F = 2 features (its MLP input is 36
// wide, a compile-time shape, so the weight loads batch) and hidden layers
// of width 64; dense_mask bit i marks a level whose vertices are indexed
// densely (decided on the host in exact integer arithmetic).
constexpr int kHashLevels = OO_HASH_MAX_LEVELS;
constexpr int kDispF = 2;
constexpr int kDispH = 64;
constexpr int kDispK = kHashLevels * kDispF + 4;
struct DispArgs {
  int32_t n_levels, log2_T, n_layers, K;  // K = n_levels F + 4
  uint32_t dense_mask;
  int32_t res[kHashLevels];
  const float* tables;  // [n_levels][2^log2_T][F]
  const float* W[3];
  const float* b[3];
};

// Kernel-argument copy of oo_mlp.
struct MlpArgs {
  int32_t n_layers;  // Linear layers; n_layers - 1 hidden layers of width H
  int32_t K0;        // input width: levels * C features, then E surface attributes
  int32_t E;
  int32_t H;
  int32_t n_out;     // output width: 3 (RGB) for the decoder
  const void* W[kMaxLayers];  // [out][in] row-major, MT
  const float* b[kMaxLayers];
};

// Two query sources concatenated: q < nA reads (xA, dA)[q], else
// (xB, dB)[q - nA]. The residual step lists LHS points first, then the
// secondary hits.
struct QuerySrc {
  const float* xA;
  const float* dA;
  int64_t nA;
  const float* xB;
  const float* dB;
  // When set, query i is the source query idx[i] (a permutation into the
  // n queries above); an index outside [0, n) reads as x = 0, dir = +z.
  const int32_t* idx = nullptr;
  int64_t n = 0;
  // the decoder's E surface attributes per query, [nA][E] and [.][E]
  const float* gA = nullptr;
  const float* gB = nullptr;
  int32_t E = 0;
};

__device__ inline int64_t source_query(const QuerySrc& s, int64_t i) {
  if (!s.idx) return i;
  const int64_t q = s.idx[i];
  return q >= 0 && q < s.n ? q : -1;
}

__device__ inline void load_pos(const QuerySrc& s, int64_t i, float x[3]) {
  const int64_t q = source_query(s, i);
  if (q < 0) {
    x[0] = x[1] = x[2] = 0.0f;
    return;
  }
  const float* xp = q < s.nA ? s.xA + 3 * q : s.xB + 3 * (q - s.nA);
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = xp[a];
}

__device__ inline void load_query(const QuerySrc& s, int64_t i, float x[3], float d[3]) {
  const int64_t q = source_query(s, i);
  if (q < 0) {
    x[0] = x[1] = x[2] = 0.0f;
    d[0] = d[1] = 0.0f;
    d[2] = 1.0f;
    return;
  }
  const float* xp = q < s.nA ? s.xA + 3 * q : s.xB + 3 * (q - s.nA);
  const float* dp = q < s.nA ? s.dA + 3 * q : s.dB + 3 * (q - s.nA);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x[a] = xp[a];
    d[a] = dp[a];
  }
}

// Surface attributes k .. k + 3 of query i (zeros for an index outside the
// sources).
__device__ inline void load_attr4(const QuerySrc& s, int64_t i, int k, float v[4]) {
  const int64_t q = source_query(s, i);
  const float* gp = q < 0 ? nullptr : (q < s.nA ? s.gA + s.E * q : s.gB + s.E * (q - s.nA));
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = gp ? gp[k + c] : 0.0f;
}

// ---------------------------------------------------------------------------
// Disparity predictor: hash encoding of x and a small FP32 MLP per lane
// ---------------------------------------------------------------------------

// Level i of the hash encoding: the cell of x N_i (x clamped to the cube,
// the last cell closed) and the fraction in it. The product is formed in
// FP64, where it is exact, so the cell is the one the FP64 definition
// gives.
__device__ __forceinline__ void hash_cell(float xa, int N, int& base, float& f) {
  const double p = (double)fminf(fmaxf(xa, 0.0f), 1.0f) * (double)N;
  double fl = floor(p);
  if (fl > (double)(N - 1)) fl = (double)(N - 1);
  base = (int)fl;
  f = (float)(p - fl);
}

// Entry of grid vertex (a, b, c) of level i: dense, or the spatial hash
// (per-axis primes 1, 2654435761, 805459861, xor) modulo the table size.
__device__ __forceinline__ uint32_t hash_entry(const DispArgs& G, int i, uint32_t a, uint32_t b, uint32_t c) {
  if ((G.dense_mask >> i) & 1u) {
    const uint32_t N1 = (uint32_t)G.res[i] + 1u;
    return a + N1 * (b + N1 * c);
  }
  return (a ^ (b * 2654435761u) ^ (c * 805459861u)) & ((1u << G.log2_T) - 1u);
}

// The predictor's input [encoding, unit(w_r), 0] (zeros past it).
__device__ __forceinline__ void disparity_input(const DispArgs& G, const float x[3], const float u[3], float (&a)[kDispK]) {
#pragma unroll
  for (int k = 0; k < kDispK; ++k) a[k] = 0.0f;
#pragma unroll
  for (int i = 0; i < kHashLevels; ++i) {
    if (i < G.n_levels) {
      const int N = G.res[i];
      int base[3];
      float f[3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) hash_cell(x[ax], N, base[ax], f[ax]);
      const float2* tab = reinterpret_cast<const float2*>(G.tables) + ((size_t)i << G.log2_T);
      float2 r[8];
#pragma unroll
      for (int d = 0; d < 8; ++d)
        r[d] = tab[hash_entry(G, i, base[0] + (d & 1), base[1] + ((d >> 1) & 1), base[2] + (d >> 2))];
      float e0 = 0.0f, e1 = 0.0f;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const float w = ((d & 1) ? f[0] : 1.0f - f[0]) * (((d >> 1) & 1) ? f[1] : 1.0f - f[1]) *
                        ((d >> 2) ? f[2] : 1.0f - f[2]);
        e0 += w * r[d].x;
        e1 += w * r[d].y;
      }
      a[2 * i] = e0;
      a[2 * i + 1] = e1;
    }
  }
  const int nF = kDispF * G.n_levels;
#pragma unroll
  for (int k = 0; k < kDispK; ++k) {
    if (k == nF) a[k] = u[0];
    if (k == nF + 1) a[k] = u[1];
    if (k == nF + 2) a[k] = u[2];
  }
}

// The predictor's hidden units are formed kDispChunk at a time and streamed
// into the next layer, so that a lane holds its input, one chunk and the
// next layer's sums in registers. The weight addresses are uniform across
// the wave, so the weights come through the scalar cache.
constexpr int kDispChunk = 16;

// Weights read at wave-uniform addresses through the constant address
// space: the loads go through the scalar cache (scalar registers) even in
// kernels that store to global memory, where a plain pointer's loads could
// be clobbered and become vector loads. The weights are read-only while the
// predictor's kernels run.
typedef const __attribute__((address_space(4))) float* cfloat_ptr;
__device__ __forceinline__ cfloat_ptr uniform_ptr(const float* p) {
  asm volatile("" : "+s"(p));
  return (cfloat_ptr)p;
}

// Units c .. c + kDispChunk - 1 of the first hidden layer, ReLU'd:
// b_0[o] + sum_k W_0[o][k] a[k] (W: the first layer's weights, rows of
// kDispK).
__device__ __forceinline__ void disp_chunk0(const DispArgs& G, const float* W, int c, const float (&a)[kDispK],
                                            float (&h)[kDispChunk]) {
  const cfloat_ptr Wc = uniform_ptr(W + c * kDispK);
  const cfloat_ptr bc = uniform_ptr(G.b[0] + c);
#pragma unroll
  for (int j = 0; j < kDispChunk; ++j) {
    float z = bc[j];
#pragma unroll
    for (int k = 0; k < kDispK; ++k) z += Wc[j * kDispK + k] * a[k];
    h[j] = fmaxf(z, 0.0f);
    if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the weights in flight
  }
}

// Pre-activations of the second hidden layer (before its bias and ReLU)
// from the first layer's units, chunk by chunk; h1_out(c, h1) sees every
// chunk.
template <class Sink>
__device__ __forceinline__ void disp_hidden2(const DispArgs& G, const float* W0, const float* W1, const float (&a)[kDispK],
                                    float (&z2)[kDispH], Sink&& h1_out) {
#pragma unroll
  for (int o = 0; o < kDispH; ++o) z2[o] = G.b[1][o];
#pragma unroll 1
  for (int c = 0; c < kDispH; c += kDispChunk) {
    float h1[kDispChunk];
    disp_chunk0(G, W0, c, a, h1);
    h1_out(c, h1);
    const cfloat_ptr W1c = uniform_ptr(W1 + c);
#pragma unroll
    for (int o = 0; o < kDispH; ++o) {
#pragma unroll
      for (int j = 0; j < kDispChunk; ++j) z2[o] += W1c[o * kDispH + j] * h1[j];
      // a few units' weights in flight at a time: the scheduler would
      // otherwise hoist all of them into scalar registers and spill
      if ((o & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Predicted disparity d(x, w_r) of one lane's query (u = unit(w_r)).
__device__ __forceinline__ float predict_disparity(const DispArgs& G, const float x[3], const float u[3]) {
  float a[kDispK];
  disparity_input(G, x, u, a);
  // (selected, not indexed: a runtime index into the argument's arrays
  // would copy them to scratch memory)
  const bool two = G.n_layers == 3;
  const float* Wo = two ? G.W[2] : G.W[1];
  float d = (two ? G.b[2] : G.b[1])[0];
  if (two) {
    float z2[kDispH];
    disp_hidden2(G, G.W[0], G.W[1], a, z2, [](int, const float (&)[kDispChunk]) {});
#pragma unroll
    for (int o = 0; o < kDispH; ++o) d += Wo[o] * fmaxf(z2[o], 0.0f);
  } else {
#pragma unroll 1
    for (int c = 0; c < kDispH; c += kDispChunk) {
      float h1[kDispChunk];
      disp_chunk0(G, G.W[0], c, a, h1);
#pragma unroll
      for (int j = 0; j < kDispChunk; ++j) d += Wo[c + j] * h1[j];
    }
  }
  return d;
}

// Unit vector of a direction (zero stays zero).
__device__ __forceinline__ void unit_dir3(const float d[3], float u[3]) {
  const float n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const float inv = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = d[a] * inv;
}

// ---------------------------------------------------------------------------
// Spatial: quantisation and descent (containing node at every level)
// ---------------------------------------------------------------------------

// floor(x * 2^D) clamped to [0, 2^D - 1]; exact because the scale is a power
// of two. fmaxf maps NaN to 0.
__device__ inline int quant_axis(float xa, int D) {
  const float scale = (float)(1u << D);
  float v = floorf(xa * scale);
  v = fminf(fmaxf(v, 0.0f), scale - 1.0f);
  return (int)v;
}

// idx[l] = global index of the level-l node containing x, or -1. Level 0 is
// the root. The walk stops for the whole wave once no lane has a node left.
__device__ inline void descend(const TreeArgs& T, bool valid, const float x[3], int idx[kMaxLevels]) {
  const int D = T.D;
  const int qx = quant_axis(x[0], D), qy = quant_axis(x[1], D), qz = quant_axis(x[2], D);
  int cur = valid ? 0 : -1;
#pragma unroll
  for (int l = 0; l < kMaxLevels; ++l) idx[l] = -1;
  idx[0] = cur;
#pragma unroll
  for (int l = 1; l < kMaxLevels; ++l) {
    if (l > D || !__any(cur >= 0)) break;
    int nxt = -1;
    if (cur >= 0) {
      const uint32_t w = T.nodes[cur];
      const int sh = D - l;
      const int o = ((qx >> sh) & 1) | (((qy >> sh) & 1) << 1) | (((qz >> sh) & 1) << 2);
      const uint32_t m = w & 0xffu;
      nxt = ((m >> o) & 1u) ? (int)(w >> 8) + __popc(m & ((1u << o) - 1u)) : -1;
    }
    cur = nxt;
    idx[l] = cur;
  }
}

// ---------------------------------------------------------------------------
// Directional: octahedral map and bilinear taps
// ---------------------------------------------------------------------------

// u = (dx, dy) / (|dx| + |dy| + |dz|), lower hemisphere folded from the
// unfolded coordinates, (s, t) = (u + 1) / 2. sign(0) = +1.
// 1 / x for x > 0: the hardware reciprocal (about 1 ulp) refined by one
// Newton-Raphson step r' = r + r (1 - x r), a few instructions in place of
// the IEEE division sequence.
__device__ __forceinline__ float rcp_refined(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// 1 / sqrt(x) and sqrt(x) for normal x > 0: the hardware reciprocal square
// root refined by one Newton-Raphson step, y' = y + y (1 - x y^2) / 2, and
// sqrt(x) = x y' (a few ulp, in place of the correctly rounded sequences).
__device__ __forceinline__ float rsqrt_refined(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
}
__device__ __forceinline__ float sqrt_refined(float x) { return x > 0.0f ? x * rsqrt_refined(x) : 0.0f; }

__device__ inline void octa(const float d[3], float& s, float& t) {
  const float S = fabsf(d[0]) + fabsf(d[1]) + fabsf(d[2]);
  // one reciprocal for both coordinates (its rounding can put a coordinate
  // a unit past +-1; the clamp keeps the fold's 1 - |u| >= 0)
  const float iS = S > 0.0f ? rcp_refined(S) : 0.0f;
  float ux = fminf(fmaxf(d[0] * iS, -1.0f), 1.0f), uy = fminf(fmaxf(d[1] * iS, -1.0f), 1.0f);
  if (d[2] < 0.0f) {
    const float fx = (1.0f - fabsf(uy)) * (ux < 0.0f ? -1.0f : 1.0f);
    const float fy = (1.0f - fabsf(ux)) * (uy < 0.0f ? -1.0f : 1.0f);
    ux = fx;
    uy = fy;
  }
  s = 0.5f * (ux + 1.0f);
  t = 0.5f * (uy + 1.0f);
}

// Texel-centred bilinear tap k (k & 1: column +1, k >> 1: row +1) at
// resolution R. A tap beyond the map is moved across the octahedral seam:
// columns first (edges s = 0 and s = 1 meet themselves with t mirrored), then
// rows (edges t = 0 and t = 1 meet themselves with s mirrored).
// texel = j * R + i. For s, t in [0, 1] the unwrapped i and j lie in
// [-1, R], where a step past an edge lands on the edge texel itself: the wrap
// is a clamp plus a mirror of the other coordinate, written without branches.
// Out-of-range (s, t) still give in-range texels.
__device__ inline void tap(float s, float t, int R, int k, int& texel, float& w) {
  const float pu = s * (float)R - 0.5f, pv = t * (float)R - 0.5f;
  const float fi = floorf(pu), fj = floorf(pv);
  const float fu = pu - fi, fv = pv - fj;
  const int a = k & 1, b = k >> 1;
  int i = (int)fi + a, j = (int)fj + b;
  w = (a ? fu : 1.0f - fu) * (b ? fv : 1.0f - fv);
  const bool wrap_col = (unsigned)i >= (unsigned)R;
  j = wrap_col ? R - 1 - j : j;
  i = min(max(i, 0), R - 1);
  const bool wrap_row = (unsigned)j >= (unsigned)R;
  i = wrap_row ? R - 1 - i : i;
  j = min(max(j, 0), R - 1);
  texel = j * R + i;
}

// All four taps.
__device__ inline void taps(float s, float t, int R, int texel[4], float w[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) tap(s, t, R, k, texel[k], w[k]);
}

// ---------------------------------------------------------------------------
// Element types
// ---------------------------------------------------------------------------

typedef _Float16 f16;
typedef __bf16 bf16;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ inline float to_f32(float v) { return v; }
__device__ inline float to_f32(f16 v) { return (float)v; }
__device__ inline float to_f32(bf16 v) { return (float)v; }

template <class T>
__device__ inline T from_f32(float v);
template <>
__device__ inline float from_f32<float>(float v) { return v; }
template <>
__device__ inline f16 from_f32<f16>(float v) { return (f16)v; }
template <>
__device__ inline bf16 from_f32<bf16>(float v) { return (bf16)v; }

// Texel gather: acc[c] += w * table[texel][c] for C channels, read as one or
// two 16-byte (or one 8-byte) vector loads.
template <class TT, int C>
struct Texel;

template <int C>
struct Texel<float, C> {
  static_assert(C == 4 || C == 8, "C");
  struct raw {
    float4 v[C / 4];
  };
  __device__ static inline void load(const float* p, raw& r) {
#pragma unroll
    for (int v = 0; v < C / 4; ++v) r.v[v] = reinterpret_cast<const float4*>(p)[v];
  }
  __device__ static inline void acc(const raw& r, float w, float* a) {
#pragma unroll
    for (int v = 0; v < C / 4; ++v) {
      a[4 * v + 0] += w * r.v[v].x;
      a[4 * v + 1] += w * r.v[v].y;
      a[4 * v + 2] += w * r.v[v].z;
      a[4 * v + 3] += w * r.v[v].w;
    }
  }
};

template <class H16, int C>
struct Texel16 {
  static_assert(C == 4 || C == 8, "C");
  typedef H16 vec __attribute__((ext_vector_type(C)));
  typedef vec raw;
  __device__ static inline void load(const H16* p, raw& r) { r = *reinterpret_cast<const vec*>(p); }
  __device__ static inline void acc(const raw& r, float w, float* a) {
#pragma unroll
    for (int c = 0; c < C; ++c) a[c] += w * (float)r[c];
  }
};
template <int C>
struct Texel<f16, C> : Texel16<f16, C> {};
template <int C>
struct Texel<bf16, C> : Texel16<bf16, C> {};

// Per-level feature h_l of one query: the 4 taps of the level-l map of node
// idx (zeros when idx < 0). Loads are issued branch-free (a missing level
// reads texel 0 of the level table with weight 0).
template <class TT, int C>
__device__ inline void gather_level(const TreeArgs& T, int l, int idx, float s, float t, float* h) {
  const int R = T.res[l];
  int tx[4];
  float w[4];
  taps(s, t, R, tx, w);
  const bool ok = idx >= 0;
  const int64_t node = ok ? (int64_t)idx - T.off[l] : 0;
  const TT* base = reinterpret_cast<const TT*>(T.feat[l]);
  typename Texel<TT, C>::raw r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t e = ok ? ((node * R * R) + tx[k]) * C : 0;
    Texel<TT, C>::load(base + e, r[k]);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) h[c] = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) Texel<TT, C>::acc(r[k], ok ? w[k] : 0.0f, h);
}

// Levels l0, l0 + STRIDE, ... (G of them) of one query in one straight-line
// block: all 4G texel loads are issued before any is consumed, so a lane
// keeps 4G gathers in flight. Levels at or past T.L (and missing nodes) read
// texel 0 of a valid table with weight 0. idx[gi] is the node index of the
// gi-th of those levels.
template <class TT, int C, int G, int STRIDE = 1>
__device__ inline void gather_levels(const TreeArgs& T, int l0, const int* idx, float s, float t, float (*h)[C]) {
  typename Texel<TT, C>::raw r[G][4];
  float w[G][4];
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const int l = l0 + STRIDE * gi;
    const int R = T.res[l];
    int tx[4];
    taps(s, t, R, tx, w[gi]);
    const bool ok = l < T.L && idx[gi] >= 0;
    const int64_t node = ok ? (int64_t)idx[gi] - T.off[l] : 0;
    const TT* base = reinterpret_cast<const TT*>(T.feat[l]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t e = ok ? ((node * R * R) + tx[k]) * C : 0;
      Texel<TT, C>::load(base + e, r[gi][k]);
      if (!ok) w[gi][k] = 0.0f;
    }
  }
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
#pragma unroll
    for (int c = 0; c < C; ++c) h[gi][c] = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) Texel<TT, C>::acc(r[gi][k], w[gi][k], h[gi]);
  }
}

// Descent and gathers of one query, software-pipelined over the levels. At
// level l the lane first loads the node word that selects the level-(l+1)
// node, then issues the 4 texel loads of level l, and only then consumes the
// texels of level l-1; so while the dependent node-word chain advances, two
// levels of gathers are in flight behind it. put(l, h, node) receives each
// level's C features and node index (zeros and -1 where the tree has no
// node). The wave stops walking once none of its lanes has a node left.
template <class TT, int C, class Put>
__device__ inline void encode_pipelined(const TreeArgs& T, bool valid, const float x[3], float s, float t,
                                        Put&& put) {
  typedef typename Texel<TT, C>::raw Raw;
  const int D = T.D, L = T.L;
  const int qx = quant_axis(x[0], D), qy = quant_axis(x[1], D), qz = quant_axis(x[2], D);
  int cur = valid ? 0 : -1;
  Raw rp[4];
  float wp[4] = {0.f, 0.f, 0.f, 0.f};
  int np = -1;  // node of the level whose texels are in flight
  int l = 0;
  for (; l < L; ++l) {
    if (!__any(cur >= 0)) break;
    const bool has = cur >= 0;
    // 1. node word of the current node (selects the next level's node)
    uint32_t word = 0;
    if (l < D) word = T.nodes[has ? cur : 0];
    // 2. texels of level l
    Raw rn[4];
    float wn[4];
    {
      const int R = T.res[l];
      int tx[4];
      taps(s, t, R, tx, wn);
      const int64_t node = has ? (int64_t)cur - T.off[l] : 0;
      const TT* base = reinterpret_cast<const TT*>(T.feat[l]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Texel<TT, C>::load(base + (has ? (node * R * R + tx[k]) * C : 0), rn[k]);
        if (!has) wn[k] = 0.0f;
      }
    }
    // 3. features of level l - 1
    if (l > 0) {
      float h[C];
#pragma unroll
      for (int c = 0; c < C; ++c) h[c] = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) Texel<TT, C>::acc(rp[k], wp[k], h);
      put(l - 1, h, np);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      rp[k] = rn[k];
      wp[k] = wn[k];
    }
    np = cur;
    // 4. next level's node
    if (l < D) {
      const int sh = D - l - 1;
      const int o = ((qx >> sh) & 1) | (((qy >> sh) & 1) << 1) | (((qz >> sh) & 1) << 2);
      const uint32_t m = word & 0xffu;
      cur = (has && ((m >> o) & 1u)) ? (int)(word >> 8) + __popc(m & ((1u << o) - 1u)) : -1;
    }
  }
  // drain: the last level fetched, then zeros for levels never reached
  if (l > 0) {
    float h[C];
#pragma unroll
    for (int c = 0; c < C; ++c) h[c] = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) Texel<TT, C>::acc(rp[k], wp[k], h);
    put(l - 1, h, np);
  }
  float z[C];
#pragma unroll
  for (int c = 0; c < C; ++c) z[c] = 0.0f;
  for (; l < L; ++l) put(l, z, -1);
}

// ---------------------------------------------------------------------------
// The paper's scheme: the eight cells whose centres surround x, weighted
// trilinearly and renormalised over the cells that exist, each read by a
// barycentric lookup on a vertex map
// ---------------------------------------------------------------------------

// Along one axis at level l: the lower of the two cells around x (cell
// centres at (c + 1/2) 2^-l) and the trilinear fraction towards the upper
// one. x is clamped to the cube (fmaxf maps NaN to 0). x 2^l is exact, and
// so is the subtraction of 1/2 whenever x 2^l >= 1/2; below that the result
// lies in [-1/2, 0) and its floor is -1 however it rounds.
__device__ inline void cell_frac(float xa, int l, int& base, float& f) {
  const float xc = fminf(fmaxf(xa, 0.0f), 1.0f);
  const float p = xc * (float)(1u << l) - 0.5f;
  const float fl = floorf(p);
  base = (int)fl;
  f = p - fl;
}

// v[i] for a lane-varying i in [0, 8) without indexing a register array
// (which would spill it to scratch memory).
template <class V>
__device__ inline V pick8(const V v[8], int i) {
  const V a = (i & 1) ? v[1] : v[0], b = (i & 1) ? v[3] : v[2];
  const V c = (i & 1) ? v[5] : v[4], d = (i & 1) ? v[7] : v[6];
  const V ab = (i & 2) ? b : a, cd = (i & 2) ? d : c;
  return (i & 4) ? cd : ab;
}

// Nodes of the eight cells around x at level l >= 1 (corner d = dx | dy << 1
// | dz << 2 is cell base + (dx, dy, dz)), from the previous level's eight:
// a cell's parent is one of them, at corner ((cell >> 1) - pbase) per axis,
// which is 0 or 1. pnode/pword: the previous level's nodes (-1 if none) and
// their node words. Cells outside the cube, or whose parent has no such
// child, get -1.
__device__ inline void corners_next(int l, const int base[3], const int pbase[3], const int pnode[8],
                                    const uint32_t pword[8], int node[8]) {
  const unsigned n = 1u << l;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int cx = base[0] + (d & 1), cy = base[1] + ((d >> 1) & 1), cz = base[2] + (d >> 2);
    const bool in = (unsigned)cx < n && (unsigned)cy < n && (unsigned)cz < n;
    const int pd = (((cx >> 1) - pbase[0]) & 1) | ((((cy >> 1) - pbase[1]) & 1) << 1) | ((((cz >> 1) - pbase[2]) & 1) << 2);
    const int pn = pick8(pnode, pd);
    const uint32_t w = pick8(pword, pd);
    const int o = (cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2);
    const uint32_t m = w & 0xffu;
    node[d] = (in && pn >= 0 && ((m >> o) & 1u)) ? (int)(w >> 8) + __popc(m & ((1u << o) - 1u)) : -1;
  }
}

// Level-0 corners: only the root cell (0, 0, 0) exists.
__device__ inline void corners_root(bool valid, const int base[3], int node[8]) {
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const bool root = base[0] + (d & 1) == 0 && base[1] + ((d >> 1) & 1) == 0 && base[2] + (d >> 2) == 0;
    node[d] = valid && root ? 0 : -1;
  }
}

// Trilinear weights of the corners that have a node, divided by their sum
// (all zero when none has one).
__device__ inline void corner_weights(const float f[3], const int node[8], float w[8]) {
  float sum = 0.0f;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const float wx = (d & 1) ? f[0] : 1.0f - f[0];
    const float wy = ((d >> 1) & 1) ? f[1] : 1.0f - f[1];
    const float wz = (d >> 2) ? f[2] : 1.0f - f[2];
    w[d] = node[d] >= 0 ? wx * wy * wz : 0.0f;
    sum += w[d];
  }
  const float inv = sum > 0.0f ? rcp_refined(sum) : 0.0f;
#pragma unroll
  for (int d = 0; d < 8; ++d) w[d] *= inv;
}

// Storage slot of vertex (i, j) of an (R+1) x (R+1) map: a border vertex
// that is the same direction as another (edges s = 0 and s = 1 glued to
// themselves with t mirrored, t = 0 and t = 1 with s mirrored, corners the
// -z pole) uses the slot of the one with the lower index along the edge.
__device__ inline int vertex_slot(int i, int j, int R) {
  // i in [0, R]: i is 0 or R exactly when i - 1 wraps past R - 2 unsigned
  j = (unsigned)(i - 1) >= (unsigned)(R - 1) ? min(j, R - j) : j;
  i = (unsigned)(j - 1) >= (unsigned)(R - 1) ? min(i, R - i) : i;
  return (int)__umul24((unsigned)j, (unsigned)(R + 1)) + i;  // R < 2^23
}

// Barycentric lookup at (s, t) in [0, 1]^2 on a map of R x R grid cells:
// the cell is split along the diagonal parallel to its quadrant's equator
// segment (anti-diagonal where s - 1/2 and t - 1/2 have the same sign, main
// diagonal otherwise), so the triangle lies in one octahedron face.
// With GRAD, gu / gv receive the weights' derivatives with respect to
// pu = s R and pv = t R (constant inside the triangle).
template <bool GRAD>
__device__ __forceinline__ void bary_t(float s, float t, int R, int slot[3], float w[3], float gu[3], float gv[3]) {
  const float pu = s * (float)R, pv = t * (float)R;
  const int i = min(max((int)floorf(pu), 0), R - 1), j = min(max((int)floorf(pv), 0), R - 1);
  const float fu = pu - (float)i, fv = pv - (float)j;
  const bool same = (2 * i >= R) == (2 * j >= R);
  // up: the triangle of the cell's far half (above the anti-diagonal when
  // the cell is split along it, above the main diagonal otherwise). The four
  // cases, as selects (lanes of a wave take different ones):
  //   same, lower: (i, j) 1 - fu - fv, (i+1, j) fu,     (i, j+1) fv
  //   same, upper: (i+1, j+1) fu + fv - 1, (i, j+1) 1 - fu, (i+1, j) 1 - fv
  //   split, lower: (i, j) 1 - fu, (i+1, j) fu - fv, (i+1, j+1) fv
  //   split, upper: (i, j) 1 - fv, (i, j+1) fv - fu, (i+1, j+1) fu
  // every candidate first, so that the selects pick values (arms holding
  // arithmetic are turned into branches)
  const float sum = fu + fv, ou = 1.0f - fu, ov = 1.0f - fv;
  const float lo = ou - fv, hi = sum - 1.0f, duv = fu - fv, dvu = fv - fu;
  const bool up = (same && sum > 1.0f) || (!same && fu < fv);
  w[0] = same ? (up ? hi : lo) : (up ? ov : ou);
  w[1] = same ? (up ? ou : fu) : (up ? dvu : duv);
  w[2] = same ? (up ? ov : fv) : (up ? fu : fv);
  const int o0 = same && up ? 1 : 0;
  const int i0 = i + o0, j0 = j + o0;
  const int i1 = up ? i : i + 1, j1 = up ? j + 1 : j;
  const int i2 = same ? (up ? i + 1 : i) : i + 1, j2 = same ? (up ? j : j + 1) : j + 1;
  if constexpr (GRAD) {
    gu[0] = same ? (up ? 1.0f : -1.0f) : (up ? 0.0f : -1.0f);
    gv[0] = same ? (up ? 1.0f : -1.0f) : (up ? -1.0f : 0.0f);
    gu[1] = up ? -1.0f : 1.0f;
    gv[1] = same ? 0.0f : (up ? 1.0f : -1.0f);
    gu[2] = same ? 0.0f : (up ? 1.0f : 0.0f);
    gv[2] = same ? (up ? -1.0f : 1.0f) : (up ? 0.0f : 1.0f);
  }
  slot[0] = vertex_slot(i0, j0, R);
  slot[1] = vertex_slot(i1, j1, R);
  slot[2] = vertex_slot(i2, j2, R);
}

__device__ __forceinline__ void bary(float s, float t, int R, int slot[3], float w[3]) {
  bary_t<false>(s, t, R, slot, w, nullptr, nullptr);
}

// d(s, t) / d v of octa(v), on the piece octa() evaluates (sign(0) = +1).
__device__ __forceinline__ void octa_jacobian(const float v[3], float J[2][3]) {
  const float S = fabsf(v[0]) + fabsf(v[1]) + fabsf(v[2]);
  float du[2][3];
  const float iS = S > 0.0f ? rcp_refined(S) : 0.0f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) du[a][b] = (a == b ? iS : 0.0f) - v[a] * (v[b] < 0.0f ? -iS : iS) * iS;
  if (v[2] < 0.0f) {
    const float sxy = (v[0] < 0.0f) == (v[1] < 0.0f) ? -1.0f : 1.0f;  // -sign(u_x) sign(u_y)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float fx = sxy * du[1][b], fy = sxy * du[0][b];
      du[0][b] = fx;
      du[1][b] = fy;
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = 0.5f * du[a][b];
}

// Shifted lookup of the level-l cell base + corner d: v = (x - centre) disp
// + u with centre (cell + 1/2) / 2^l; dv = x - centre (= d v / d disp).
// x is clamped to the cube as for the cells.
__device__ __forceinline__ void shifted_dir(const float x[3], int l, const int base[3], int d, float disp, const float u[3],
                                   float v[3], float dv[3]) {
  const float inv = ldexpf(1.0f, -l);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int bit = (d >> a) & 1;
    const float xc = fminf(fmaxf(x[a], 0.0f), 1.0f);
    dv[a] = xc - ((float)(base[a] + bit) + 0.5f) * inv;
    v[a] = dv[a] * disp + u[a];
  }
}

// The eight corners' shifted directions share their per-axis terms: axis a
// of corner d is v[(d >> a) & 1][a] (the same arithmetic as shifted_dir).
struct ShiftAxes {
  float v[2][3];
};
__device__ __forceinline__ void shift_axes(const float x[3], int l, const int base[3], float disp, const float u[3],
                                           ShiftAxes& A) {
  const float inv = ldexpf(1.0f, -l);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float xc = fminf(fmaxf(x[a], 0.0f), 1.0f);
#pragma unroll
    for (int bit = 0; bit < 2; ++bit) A.v[bit][a] = (xc - ((float)(base[a] + bit) + 0.5f) * inv) * disp + u[a];
  }
}

// Level feature of the paper's scheme: sum over the corners and the three
// vertices of w_corner * w_vertex * T[node][slot]. Loads go out a batch of
// corners at a time (12 entries of 16 bytes, or 6 of 32 bytes); corners
// without a node read entry 0 of the level with weight 0.
template <class TT, int C>
__device__ inline void gather_paper_level(const TreeArgs& T, int l, const int node[8], const float wc[8],
                                          const int slot[3], const float wv[3], float* h) {
  typedef typename Texel<TT, C>::raw Raw;
  constexpr int CB = sizeof(TT) * C > 16 ? 2 : 4;  // corners per batch
  const int R = T.res[l];
  const int64_t E = (int64_t)(R + 1) * (R + 1);
  const TT* base = reinterpret_cast<const TT*>(T.feat[l]);
#pragma unroll
  for (int c = 0; c < C; ++c) h[c] = 0.0f;
#pragma unroll
  for (int b0 = 0; b0 < 8; b0 += CB) {
    Raw r[CB][3];
#pragma unroll
    for (int dd = 0; dd < CB; ++dd) {
      const int d = b0 + dd;
      const bool ok = node[d] >= 0;
      const int64_t nb = ok ? ((int64_t)node[d] - T.off[l]) * E : 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) Texel<TT, C>::load(base + (ok ? (nb + slot[k]) * C : 0), r[dd][k]);
    }
#pragma unroll
    for (int dd = 0; dd < CB; ++dd)
#pragma unroll
      for (int k = 0; k < 3; ++k) Texel<TT, C>::acc(r[dd][k], wc[b0 + dd] * wv[k], h);
  }
}

// The same level feature with the disparity shift: corner d's cell is read
// at its own direction (x - centre) disp + u (one barycentric lookup per
// corner).
template <class TT, int C>
__device__ __forceinline__ void gather_paper_level_shift(const TreeArgs& T, int l, const int node[8], const float wc[8],
                                                const float x[3], const int base[3], float disp, const float u[3],
                                                float* h) {
  typedef typename Texel<TT, C>::raw Raw;
  constexpr int CB = sizeof(TT) * C > 16 ? 2 : 4;  // corners per batch
  const int R = T.res[l];
  const int64_t E = (int64_t)(R + 1) * (R + 1);
  const int64_t off = T.off[l];
  const TT* tab = reinterpret_cast<const TT*>(T.feat[l]);
  ShiftAxes A;
  shift_axes(x, l, base, disp, u, A);
#pragma unroll
  for (int c = 0; c < C; ++c) h[c] = 0.0f;
#pragma unroll
  for (int b0 = 0; b0 < 8; b0 += CB) {
    Raw r[CB][3];
    float wv[CB][3];
#pragma unroll
    for (int dd = 0; dd < CB; ++dd) {
      const int d = b0 + dd;
      const float v[3] = {A.v[d & 1][0], A.v[(d >> 1) & 1][1], A.v[d >> 2][2]};
      float s, t;
      octa(v, s, t);
      int slot[3];
      bary(s, t, R, slot, wv[dd]);
      const bool ok = node[d] >= 0;
      const int64_t nb = ok ? ((int64_t)node[d] - off) * E : 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) Texel<TT, C>::load(tab + (ok ? (nb + slot[k]) * C : 0), r[dd][k]);
    }
#pragma unroll
    for (int dd = 0; dd < CB; ++dd)
#pragma unroll
      for (int k = 0; k < 3; ++k) Texel<TT, C>::acc(r[dd][k], wc[b0 + dd] * wv[dd][k], h);
  }
}

// Encoding of one query in the paper's scheme, level by level: the eight
// corners' nodes follow from the previous level's (their node words are
// loaded while this level's entries are gathered). put(l, h, node) receives
// each level's C features and the eight corner nodes. Once no lane of the
// wave has a corner left, deeper levels are empty too (their cells' parents
// are among this level's corners) and get zeros.
// With SHIFT every corner's cell is read along its shifted direction
// (disparity disp, unit lookup direction u).
template <class TT, int C, bool SHIFT = false, class Put>
__device__ __forceinline__ void encode_paper(const TreeArgs& T, bool valid, const float x[3], float s, float t, Put&& put,
                                    float disp = 0.0f, const float* u = nullptr) {
  const int L = T.L, D = T.D;
  int base[3], pbase[3], node[8], pnode[8];
  uint32_t pword[8];
  float f[3];
  int l = 0;
  for (; l < L; ++l) {
#pragma unroll
    for (int a = 0; a < 3; ++a) cell_frac(x[a], l, base[a], f[a]);
    if (l == 0)
      corners_root(valid, base, node);
    else
      corners_next(l, base, pbase, pnode, pword, node);
    bool any = false;
#pragma unroll
    for (int d = 0; d < 8; ++d) any |= node[d] >= 0;
    if (!__any(any)) break;
    // node words for the next level, then this level's entries
#pragma unroll
    for (int d = 0; d < 8; ++d) pword[d] = (l < D && node[d] >= 0) ? T.nodes[node[d]] : 0u;
    float wc[8];
    corner_weights(f, node, wc);
    float h[C];
    if constexpr (SHIFT) {
      gather_paper_level_shift<TT, C>(T, l, node, wc, x, base, disp, u, h);
    } else {
      float wv[3];
      int slot[3];
      bary(s, t, T.res[l], slot, wv);
      gather_paper_level<TT, C>(T, l, node, wc, slot, wv, h);
    }
    put(l, h, node);
#pragma unroll
    for (int a = 0; a < 3; ++a) pbase[a] = base[a];
#pragma unroll
    for (int d = 0; d < 8; ++d) pnode[d] = node[d];
  }
  float z[C];
#pragma unroll
  for (int c = 0; c < C; ++c) z[c] = 0.0f;
  int none[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) none[d] = -1;
  for (; l < L; ++l) put(l, z, none);
}

// ---------------------------------------------------------------------------
// Matrix-core fragments for the decoder
// ---------------------------------------------------------------------------
//
// Queries run along the N dimension of every 16x16 output tile, neurons along
// M. An output tile gives lane l the rows 16m + 4g + j (j = 0..3) of column
// q = l % 16, with g = l / 16. A K-chunk of 32 inputs is held as 8 slots per
// lane; slot i of lane l (group g) carries input neuron
//     nu(kb, g, i) = 32 kb + 16 (i >> 2) + 4 g + (i & 3),
// so that output tiles 2kb and 2kb+1 of one layer are, unchanged, the
// K-chunk kb of the next layer. Operands A (weights) and B (activations) use
// the same nu, so every product pairs matching neurons. FP16/BF16 issue one
// 16x16x32 MFMA per chunk; FP32 issues eight 16x16x4 MFMAs, one per slot.

__host__ __device__ inline int nu(int kb, int g, int i) { return 32 * kb + 16 * (i >> 2) + 4 * g + (i & 3); }

template <class MT>
struct FragT;
template <>
struct FragT<f16> {
  typedef f16x8 type;
};
template <>
struct FragT<bf16> {
  typedef bf16x8 type;
};
template <>
struct FragT<float> {
  typedef f32x8 type;
};

__device__ inline f32x4 mma(const f16x8& a, const f16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mma(const bf16x8& a, const bf16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mma(const f32x8& a, const f32x8& b, f32x4 c) {
#pragma unroll
  for (int i = 0; i < 8; ++i) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[i], c, 0, 0, 0);
  return c;
}

// Position of input neuron k inside a fragment: chunk kb, lane group g, slot i.
__device__ inline void nu_inv(int k, int& kb, int& g, int& i) {
  kb = k >> 5;
  const int r = k & 31;
  g = (r & 15) >> 2;
  i = ((r >> 4) << 2) | (r & 3);
}

// Activation tile in LDS for one 16-query N-tile set, fragment-major:
// element (q, k) of a tile with KB chunks lives at
//   ((q / 16) * KB + kb) * 64 * 8 + (16 g + q % 16) * 8 + i.
// Reading chunk kb of N-tile t is then one contiguous 8-element read per lane.
template <class MT>
__device__ inline int htile_index(int q, int k, int KB) {
  int kb, g, i;
  nu_inv(k, kb, g, i);
  return (((q >> 4) * KB + kb) * kWave + (g << 4) + (q & 15)) * 8 + i;
}

// Four consecutive inputs k0..k0+3 (k0 % 4 == 0) of query q: they share
// (kb, g) and occupy slots 4h..4h+3, so one vector store writes them.
template <class MT>
__device__ inline void htile_put4(MT* tile, int KB, int q, int k0, const float v[4]) {
  const int idx = htile_index<MT>(q, k0, KB);
  typedef MT v4 __attribute__((ext_vector_type(4)));
  v4 x;
  x[0] = from_f32<MT>(v[0]);
  x[1] = from_f32<MT>(v[1]);
  x[2] = from_f32<MT>(v[2]);
  x[3] = from_f32<MT>(v[3]);
  *reinterpret_cast<v4*>(tile + idx) = x;
}

template <class MT>
__device__ inline typename FragT<MT>::type htile_get(const MT* tile, int KB, int t, int kb, int lane) {
  return *reinterpret_cast<const typename FragT<MT>::type*>(tile + ((t * KB + kb) * kWave + lane) * 8);
}

// Weight fragment (A operand) of a row-major [n_out][n_in] matrix with
// leading dimension ld (a multiple of 4, zero padded beyond n_in), for output
// tile m and chunk kb. Slots 0..3 and 4..7 are 4 consecutive columns each,
// so the fragment is two vector loads; columns past the row read as zero.
template <class MT>
__device__ inline typename FragT<MT>::type wfrag_global(const MT* W, int n_out, int n_in, int ld, int m, int kb,
                                                        int lane) {
  typedef MT v4 __attribute__((ext_vector_type(4)));
  typename FragT<MT>::type a;
  const int row = 16 * m + (lane & 15), g = lane >> 4;
  const bool rok = row < n_out;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int col = 32 * kb + 16 * h + 4 * g;
    v4 v;
    if (rok && col < n_in) {
      v = *reinterpret_cast<const v4*>(W + (int64_t)row * ld + col);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = from_f32<MT>(0.0f);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) a[4 * h + j] = v[j];
  }
  return a;
}

// B-operand chunk kb built from two output tiles (2kb, 2kb+1) of the
// previous layer: bias already added; ReLU applied when relu is set.
template <class MT>
__device__ inline typename FragT<MT>::type chain_frag(const f32x4& lo, const f32x4& hi, bool relu) {
  typename FragT<MT>::type b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float a0 = relu ? fmaxf(lo[j], 0.0f) : lo[j];
    const float a1 = relu ? fmaxf(hi[j], 0.0f) : hi[j];
    b[j] = from_f32<MT>(a0);
    b[4 + j] = from_f32<MT>(a1);
  }
  return b;
}

// FP16: round first, then the ReLU on packed halves (rounding keeps the
// sign, so the result is the same and the max runs on pairs).
template <>
__device__ inline FragT<f16>::type chain_frag<f16>(const f32x4& lo, const f32x4& hi, bool relu) {
  FragT<f16>::type b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    b[j] = from_f32<f16>(lo[j]);
    b[4 + j] = from_f32<f16>(hi[j]);
  }
  if (relu) {
    typedef f16 h2 __attribute__((ext_vector_type(2)));
    const h2 z = {(f16)0.0f, (f16)0.0f};
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
      h2 v = {b[j], b[j + 1]};
      v = __builtin_elementwise_max(v, z);
      b[j] = v[0];
      b[j + 1] = v[1];
    }
  }
  return b;
}

// Returns p unchanged but opaque to the optimiser. Weight fragments are
// loop-invariant in the persistent tile loops; laundering their base pointer
// per iteration keeps the compiler from hoisting every fragment load out of
// the loop and pinning hundreds of registers. The loads then hit L2.
template <class P>
__device__ inline P* launder_ptr(P* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Same for a lane-varying integer: values derived from it are recomputed
// where they are used instead of being hoisted and held in registers.
__device__ inline int launder_lane(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Orders this wave's LDS writes before its following LDS reads.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// XCD-aware work split: workgroups are dispatched round-robin over the 8
// XCDs, so workgroup b runs on XCD b % 8. Each XCD takes one contiguous range
// of tiles (neighbouring queries share nodes and texels, and each XCD has
// its own L2); inside it the workers stride through the range.
struct TileRange {
  int64_t first, end, stride;
};
__device__ inline TileRange xcd_tiles(int64_t n_tiles, int workers_per_wg, int worker) {
  const int G = gridDim.x;
  TileRange r;
  if (G % 8 != 0 || G < 8) {
    r.first = (int64_t)blockIdx.x * workers_per_wg + worker;
    r.end = n_tiles;
    r.stride = (int64_t)G * workers_per_wg;
    return r;
  }
  const int xcd = blockIdx.x & 7, per = G >> 3;
  const int64_t lo = n_tiles * xcd / 8, hi = n_tiles * (xcd + 1) / 8;
  r.first = lo + (int64_t)(blockIdx.x >> 3) * workers_per_wg + worker;
  r.end = hi;
  r.stride = (int64_t)per * workers_per_wg;
  return r;
}

// ---------------------------------------------------------------------------
// BSDF sample weight of the residual's Monte-Carlo target (forward and the
// backward's full-mode seeds use the same one)
// ---------------------------------------------------------------------------
// GGX + Lambert sample weight f |n.wi| / pdf for unit n, wo, wi. The GGX
// denominator (n.h)^2 (a^2 - 1) + 1 is evaluated as a^2 (n.h)^2 + |n x h|^2,
// which avoids the cancellation near the specular peak. Smith's separable
// G_1(c) = 2c / (c + sqrt(a^2 + (1 - a^2) c^2)) cancels against the
// 4 cos_i cos_o of the microfacet term, leaving D F / ((ci + si)(co + so)).
__device__ __forceinline__ void bsdf_weight(const float n[3], const float wo[3], const float wi[3], const float alb[3],
                                   float alpha, float F0, float pdf, float w[3]) {
  const float ci = n[0] * wi[0] + n[1] * wi[1] + n[2] * wi[2];
  const float co = n[0] * wo[0] + n[1] * wo[1] + n[2] * wo[2];
  if (!(ci > 0.0f) || !(co > 0.0f)) {
    w[0] = w[1] = w[2] = 0.0f;
    return;
  }
  float h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
  const float ihl = rsqrt_refined(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) h[a] *= ihl;
  const float nh = n[0] * h[0] + n[1] * h[1] + n[2] * h[2];
  const float cx = n[1] * h[2] - n[2] * h[1], cy = n[2] * h[0] - n[0] * h[2], cz = n[0] * h[1] - n[1] * h[0];
  const float a2 = alpha * alpha;
  const float den = a2 * nh * nh + (cx * cx + cy * cy + cz * cz);
  const float vh = 1.0f - (wi[0] * h[0] + wi[1] * h[1] + wi[2] * h[2]);
  const float vh2 = vh * vh;
  const float F = F0 + (1.0f - F0) * (vh2 * vh2 * vh);
  const float gi = ci + sqrt_refined(a2 + (1.0f - a2) * ci * ci), go = co + sqrt_refined(a2 + (1.0f - a2) * co * co);
  const float spec = a2 * F * rcp_refined(3.14159265358979f * den * den * gi * go);
  const float sc = ci * rcp_refined(pdf);
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = (alb[c] * (1.0f / 3.14159265358979f) + spec) * sc;
}
__device__ __forceinline__ void load_unit(const float* p, float v[3]) {
  v[0] = p[0];
  v[1] = p[1];
  v[2] = p[2];
  const float l2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const float il = l2 > 0.0f ? rsqrt_refined(l2) : 1.0f;
  v[0] *= il;
  v[1] *= il;
  v[2] *= il;
}

}  // namespace oo
