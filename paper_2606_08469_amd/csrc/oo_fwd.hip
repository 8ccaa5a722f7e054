// Forward kernels: standalone encoding, standalone decoder, the fused
// encode + decode query, the residual assembly with its FP64 loss
// reduction, and the FP32 -> FP16/BF16 parameter cast.
#include <hip/hip_runtime.h>

#include "oo_device.h"
#include "oo_internal.h"

namespace oo {

// ---------------------------------------------------------------------------
// Standalone encoding: one thread per query, h written row-major to memory.
// ---------------------------------------------------------------------------
// MODE: 0 node + bilinear, 1 the paper's scheme, 2 the paper's scheme with
// the disparity shift (predicted per query from G).
template <class TT, class HT, int C, int MODE>
__global__ __launch_bounds__(256) void encode_kernel(const TreeArgs T, const float* __restrict__ x,
                                                     const float* __restrict__ dir, int64_t B,
                                                     HT* __restrict__ h_out, int32_t* __restrict__ idx_out,
                                                     const DispArgs G) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < B;
  float xq[3] = {0.f, 0.f, 0.f}, dq[3] = {0.f, 0.f, 1.f};
  if (valid) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xq[a] = x[3 * q + a];
      dq[a] = dir[3 * q + a];
    }
  }
  typedef HT vC __attribute__((ext_vector_type(C)));
  if constexpr (MODE > 0) {
    // the eight cells around x per level, barycentric vertex maps
    float s, t;
    octa(dq, s, t);
    float u[3] = {0.f, 0.f, 0.f}, disp = 0.0f;
    if constexpr (MODE == 2) {
      unit_dir3(dq, u);
      disp = predict_disparity(G, xq, u);
    }
    const int L = T.L;
    HT* hrow = h_out + (valid ? q : 0) * (int64_t)(L * C);
    encode_paper<TT, C, MODE == 2>(T, valid, xq, s, t, [&](int l, const float (&h)[C], const int (&node)[8]) {
      if (!valid) return;
      vC v;
#pragma unroll
      for (int c = 0; c < C; ++c) v[c] = from_f32<HT>(h[c]);
      *reinterpret_cast<vC*>(hrow + l * C) = v;
      if (idx_out) {
        int4* o = reinterpret_cast<int4*>(idx_out + (q * L + l) * 8);
        o[0] = make_int4(node[0], node[1], node[2], node[3]);
        o[1] = make_int4(node[4], node[5], node[6], node[7]);
      }
    }, disp, u);
    return;
  }
  int idx[kMaxLevels];
  descend(T, valid, xq, idx);
  if (!valid) return;
  float s, t;
  octa(dq, s, t);
  const int L = T.L;
  HT* hrow = h_out + q * (int64_t)(L * C);
#pragma unroll
  for (int l0 = 0; l0 < kMaxLevels; l0 += 4) {
    if (l0 >= L) break;
    float h[4][C];
    gather_levels<TT, C, 4>(T, l0, &idx[l0], s, t, h);
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
      const int l = l0 + gi;
      if (l < L) {
        vC v;
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = from_f32<HT>(h[gi][c]);
        *reinterpret_cast<vC*>(hrow + l * C) = v;
        if (idx_out) idx_out[q * L + l] = idx[l];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Decoder forward on one wave's 64-query activation tile.
// ---------------------------------------------------------------------------

// Weight fragments: packed in LDS in fragment order (zero padded), or read
// straight from the row-major matrices. Packed layout: layer 0 first
// ((H/16) x KB0 fragments), then each hidden layer ((H/16) x (H/32)), then
// the output layer (H/32); one fragment is 64 lanes x 8 elements.
template <class MT, bool WLDS>
struct WFrag {
  const MT* lds;
  int KB0;
  __device__ inline typename FragT<MT>::type get(const MlpArgs& M, int layer, int m, int kb, int lane) const {
    if constexpr (WLDS) {
      const int MH = M.H / 16, KH = M.H / 32;
      int base, KB;
      if (layer == 0) {
        base = 0;
        KB = KB0;
      } else {
        base = MH * KB0 + (layer - 1) * MH * KH;
        KB = KH;
      }
      return *reinterpret_cast<const typename FragT<MT>::type*>(lds + ((base + m * KB + kb) * kWave + lane) * 8);
    } else {
      const int n_in = layer == 0 ? M.K0 : M.H;
      const int n_out = layer == M.n_layers - 1 ? M.n_out : M.H;
      return wfrag_global<MT>(launder_ptr(reinterpret_cast<const MT*>(M.W[layer])), n_out, n_in, n_in, m, kb, lane);
    }
  }
};

__device__ inline f32x4 bias_tile(const float* b, int n_out, int m, int lane) {
  f32x4 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = 16 * m + 4 * (lane >> 4) + j;
    v[j] = row < n_out ? b[row] : 0.0f;
  }
  return v;
}

// Runs the MLP on N-tiles t0 .. t0+NT-1 of the activation tile and returns
// the output tile per N-tile (rows 0..2 = RGB in lanes 0..15).
template <class MT, int H, int NT, class WSrc>
__device__ inline void mlp_forward_tiles(const MlpArgs& M, const WSrc& W, const MT* htile, int KB0, int t0,
                                         int lane, f32x4 out[NT]) {
  // M is a kernel argument: indexing its arrays reads the argument segment.
  typedef typename FragT<MT>::type frag;
  constexpr int MH = H / 16, KH = H / 32;
  f32x4 acc[MH][NT];
  // layer 0: K0 -> H
#pragma unroll
  for (int m = 0; m < MH; ++m) {
    const f32x4 bt = bias_tile(M.b[0], H, m, lane);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = bt;
  }
  // Each K-chunk's weight fragments are all read before its MFMAs, so their
  // LDS latency overlaps instead of stalling every pair of MFMAs.
  for (int kb = 0; kb < KB0; ++kb) {
    frag bf[NT], a[MH];
#pragma unroll
    for (int t = 0; t < NT; ++t) bf[t] = htile_get<MT>(htile, KB0, t0 + t, kb, lane);
#pragma unroll
    for (int m = 0; m < MH; ++m) a[m] = W.get(M, 0, m, kb, lane);
    __builtin_amdgcn_sched_barrier(0);  // (the scheduler would sink each read to its MFMAs)
#pragma unroll
    for (int m = 0; m < MH; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = mma(a[m], bf[t], acc[m][t]);
  }
  // hidden layers H -> H
  for (int layer = 1; layer < M.n_layers - 1; ++layer) {
    frag bf[KH][NT];
#pragma unroll
    for (int kb = 0; kb < KH; ++kb)
#pragma unroll
      for (int t = 0; t < NT; ++t) bf[kb][t] = chain_frag<MT>(acc[2 * kb][t], acc[2 * kb + 1][t], true);
#pragma unroll
    for (int m = 0; m < MH; ++m) {
      const f32x4 bt = bias_tile(M.b[layer], H, m, lane);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = bt;
    }
#pragma unroll
    for (int kb = 0; kb < KH; ++kb) {
      frag a[MH];
#pragma unroll
      for (int m = 0; m < MH; ++m) a[m] = W.get(M, layer, m, kb, lane);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < MH; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = mma(a[m], bf[kb][t], acc[m][t]);
    }
  }
  // output layer H -> 3
  const int lo = M.n_layers - 1;
  const f32x4 bt = bias_tile(M.b[lo], M.n_out, 0, lane);
#pragma unroll
  for (int t = 0; t < NT; ++t) out[t] = bt;
#pragma unroll
  for (int kb = 0; kb < KH; ++kb) {
    const frag a = W.get(M, lo, 0, kb, lane);
#pragma unroll
    for (int t = 0; t < NT; ++t) out[t] = mma(a, chain_frag<MT>(acc[2 * kb][t], acc[2 * kb + 1][t], true), out[t]);
  }
}

// Packs every layer's weights into LDS in fragment order (zero padded).
template <class MT>
__device__ inline void pack_weights_lds(const MlpArgs& M, MT* lds) {
  int offset = 0;
  for (int layer = 0; layer < M.n_layers; ++layer) {
    const int n_in = layer == 0 ? M.K0 : M.H;
    const int n_out = layer == M.n_layers - 1 ? 3 : M.H;
    const int KB = (n_in + 31) / 32;
    const int total = ((n_out + 15) / 16) * KB * kWave * 8;
    const MT* src = reinterpret_cast<const MT*>(M.W[layer]);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int i = e & 7, lane = (e >> 3) & 63, frag = e >> 9;
      const int kb = frag % KB, m = frag / KB;
      const int row = 16 * m + (lane & 15), col = nu(kb, lane >> 4, i);
      lds[offset + e] = (row < n_out && col < n_in) ? src[(int64_t)row * n_in + col] : from_f32<MT>(0.0f);
    }
    offset += total;
  }
}

template <class MT>
__host__ __device__ inline int packed_weight_elems(int n_layers, int K0, int H) {
  int total = 0;
  for (int layer = 0; layer < n_layers; ++layer) {
    const int n_in = layer == 0 ? K0 : H;
    const int n_out = layer == n_layers - 1 ? 3 : H;
    total += ((n_out + 15) / 16) * ((n_in + 31) / 32) * kWave * 8;
  }
  return total;
}

template <class MT, int NT>
__device__ inline void store_rgb(const f32x4 out[NT], int t0, int64_t q_base, int64_t Q, int lane, float* rgb) {
  if (lane < 16) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t q = q_base + 16 * (t0 + t) + lane;
      if (q < Q) {
        rgb[3 * q + 0] = out[t][0];
        rgb[3 * q + 1] = out[t][1];
        rgb[3 * q + 2] = out[t][2];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fused query: encode 64 queries per wave into LDS, decode them there.
// ---------------------------------------------------------------------------
// Queries q < n_idx also store their node index per level in idx_out
// (level-major [L][n_idx]) and their octahedral coordinates in uv_out, which
// the residual backward reads instead of descending and mapping again.
// In the paper's scheme the stored indices are the eight corner cells'
// nodes per level ([L][8][n_idx]) and the query's position is kept too
// (pos_out, [n_idx]); the backward recomputes the trilinear weights from it.
// MODE as for encode_kernel; with the shift the query's disparity goes to
// pos_out's w and its unit lookup direction to wdir_out.
template <class TT, class MT, int C, int H, bool WLDS, int MODE>
__global__ __launch_bounds__(512) void query_kernel(const TreeArgs T, const MlpArgs M, const QuerySrc src,
                                                    int64_t Q, float* __restrict__ rgb, const QueryOut O,
                                                    const DispArgs G) {
  int32_t* __restrict__ idx_out = O.idx;
  float2* __restrict__ uv_out = O.uv;
  float4* __restrict__ pos_out = O.pos;
  const int64_t n_idx = O.n_idx;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  // N-tiles per decoder pass: all four with 16-bit operands, LDS weights
  // and 64-wide layers (each weight fragment read then serves four MFMAs;
  // at width 128 the accumulators would spill)
  constexpr int NT = sizeof(MT) == 2 && WLDS && H == 64 ? 4 : 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, waves = blockDim.x >> 6;
  const int KB0 = (M.K0 + 31) / 32;
  const int wl_elems = WLDS ? packed_weight_elems<MT>(M.n_layers, M.K0, M.H) : 0;
  MT* wl = reinterpret_cast<MT*>(smem);
  MT* htile = wl + wl_elems + wave * (4 * KB0 * kWave * 8);
  if (WLDS) pack_weights_lds<MT>(M, wl);
  {  // zero the K padding of this lane's row once
    const float z[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = M.K0; k < 32 * KB0; k += 4) htile_put4<MT>(htile, KB0, lane, k, z);
  }
  __syncthreads();
  const WFrag<MT, WLDS> W{wl, KB0};
  const int64_t n_tiles = (Q + 63) / 64;
  const TileRange tr = xcd_tiles(n_tiles, waves, wave);
  for (int64_t tile = tr.first; tile < tr.end; tile += tr.stride) {
    const int64_t q = tile * 64 + lane;
    const bool valid = q < Q;
    float x[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
    if (valid) load_query(src, q, x, d);
    float s, t;
    octa(d, s, t);
    const bool keep = q < n_idx;
    if (keep) uv_out[q] = make_float2(s, t);
    if constexpr (MODE > 0) {
      float u[3] = {0.f, 0.f, 0.f}, disp = 0.0f;
      if constexpr (MODE >= 2) {
        unit_dir3(d, u);
        disp = predict_disparity(G, x, u);
        if (keep) O.wdir[q] = make_float4(u[0], u[1], u[2], 0.0f);
      }
      if (keep) pos_out[q] = make_float4(x[0], x[1], x[2], disp);
      encode_paper<TT, C, MODE >= 2>(T, valid, x, s, t, [&](int l, const float (&h)[C], const int (&node)[8]) {
#pragma unroll
        for (int c = 0; c < C; c += 4) htile_put4<MT>(htile, KB0, lane, l * C + c, &h[c]);
        if (keep)
#pragma unroll
          for (int d = 0; d < 8; ++d) idx_out[(l * 8 + d) * n_idx + q] = node[d];  // coalesced across lanes
      }, disp, u);
    } else {
      encode_pipelined<TT, C>(T, valid, x, s, t, [&](int l, const float* h, int node) {
#pragma unroll
        for (int c = 0; c < C; c += 4) htile_put4<MT>(htile, KB0, lane, l * C + c, &h[c]);
        if (keep) idx_out[l * n_idx + q] = node;  // level-major: coalesced across lanes
      });
    }
    // the decoder's surface attributes follow the level features
    for (int k = 0; k < M.E; k += 4) {
      float g4[4] = {0.f, 0.f, 0.f, 0.f};
      if (valid) load_attr4(src, q, k, g4);
      htile_put4<MT>(htile, KB0, lane, M.K0 - M.E + k, g4);
    }
    wave_lds_sync();
#pragma unroll
    for (int t0 = 0; t0 < 4; t0 += NT) {
      f32x4 out[NT];
      mlp_forward_tiles<MT, H, NT>(M, W, htile, KB0, t0, lane, out);
      store_rgb<MT, NT>(out, t0, tile * 64, Q, lane, rgb);
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Standalone decoder: h rows from memory into the LDS tile, then decode.
// ---------------------------------------------------------------------------
template <class MT, int H, bool WLDS>
__global__ __launch_bounds__(512) void mlp_kernel(const MlpArgs M, const MT* __restrict__ h, int64_t Q,
                                                  float* __restrict__ rgb) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  // N-tiles per pass: with 16-bit operands and the weights in LDS all
  // four, so that each weight fragment read serves four MFMAs (the other
  // variants would spill)
  constexpr int NT = sizeof(MT) == 2 && WLDS ? 4 : 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, waves = blockDim.x >> 6;
  const int KB0 = (M.K0 + 31) / 32;
  const int wl_elems = WLDS ? packed_weight_elems<MT>(M.n_layers, M.K0, M.H) : 0;
  MT* wl = reinterpret_cast<MT*>(smem);
  MT* htile = wl + wl_elems + wave * (4 * KB0 * kWave * 8);
  if (WLDS) pack_weights_lds<MT>(M, wl);
  {
    const float z[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = M.K0; k < 32 * KB0; k += 4) htile_put4<MT>(htile, KB0, lane, k, z);
  }
  __syncthreads();
  const WFrag<MT, WLDS> W{wl, KB0};
  const int64_t n_tiles = (Q + 63) / 64;
  const TileRange tr = xcd_tiles(n_tiles, waves, wave);
  // 16-bit rows: a tile's rows are P pieces of 16 bytes each; this lane
  // reads pieces lane + 64 i, i = 0 .. P-1, walked by row and position
  // without a division per piece
  constexpr int EP = 16 / sizeof(MT);
  const int P = M.K0 / EP > 0 ? M.K0 / EP : 1;
  const int step_r = 64 / P, step_m = 64 % P;
  const int lane_r = lane / P, lane_m = lane % P;
  for (int64_t tile = tr.first; tile < tr.end; tile += tr.stride) {
    // With 16-bit rows the wave reads the tile's 64 contiguous rows as
    // 16-byte pieces in order (coalesced; EP entries each, K0 a multiple of
    // EP), eight of a lane's pieces (at most 16, K0 <= 128) loaded before
    // any of them is stored, so their latencies overlap; the pieces go to
    // their fragment slots unconverted. Otherwise each lane reads its own
    // row four entries at a time (FP32 measured faster that way).
    const int64_t q0 = tile * 64;
    const int nrow = Q - q0 < 64 ? (int)(Q - q0) : 64;
    if (sizeof(MT) == 2 && M.K0 % EP == 0) {
      typedef MT vP __attribute__((ext_vector_type(EP)));
      typedef MT v4 __attribute__((ext_vector_type(4)));
      constexpr int kMaxPieces = 128 / EP, kBatch = 8;
      const vP* src = reinterpret_cast<const vP*>(h + q0 * (int64_t)M.K0);
      int r = lane_r, m = lane_m;  // row and position of piece lane + 64 i
#pragma unroll 1
      for (int i0 = 0; i0 < kMaxPieces; i0 += kBatch) {
        vP xs[kBatch];
        int rs[kBatch], ms[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          const int i = i0 + j;
          rs[j] = r;
          ms[j] = m;
          xs[j] = vP{};
          if (i < P && r < nrow) xs[j] = src[lane + 64 * i];
          m += step_m;
          r += step_r;
          if (m >= P) {
            m -= P;
            ++r;
          }
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          if (i0 + j < P) {
#pragma unroll
            for (int c = 0; c < EP; c += 4) {
              const v4 x4 = {xs[j][c], xs[j][c + 1], xs[j][c + 2], xs[j][c + 3]};
              *reinterpret_cast<v4*>(htile + htile_index<MT>(rs[j], ms[j] * EP + c, KB0)) = x4;
            }
          }
        }
      }
    } else {
      typedef MT v4 __attribute__((ext_vector_type(4)));
      const int64_t q = q0 + lane;
      const v4* row = reinterpret_cast<const v4*>(h + (q < Q ? q : 0) * (int64_t)M.K0);
      for (int k = 0; k < M.K0; k += 4) {
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (q < Q) {
          const v4 r = row[k >> 2];
#pragma unroll
          for (int c = 0; c < 4; ++c) v[c] = to_f32(r[c]);
        }
        htile_put4<MT>(htile, KB0, lane, k, v);
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int t0 = 0; t0 < 4; t0 += NT) {
      f32x4 out[NT];
      mlp_forward_tiles<MT, H, NT>(M, W, htile, KB0, t0, lane, out);
      store_rgb<MT, NT>(out, t0, tile * 64, Q, lane, rgb);
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Shifted encode of the residual's sorted queries into decoder input rows:
// one thread per query (the paper's scheme with the disparity shift, each
// query's disparity read from O.disp). Row q of h_rows (K0 = L C + E
// entries of MT) holds the level features, then the surface attributes;
// queries q < n_idx also leave what the backward reads (corner nodes,
// octahedral coordinates, position and disparity, lookup direction), as
// the fused query does. Without the decoder's registers the encode runs at
// several more waves per SIMD, which its dependent gathers need; the
// standalone decoder then reads the rows.
// ---------------------------------------------------------------------------
template <class TT, class MT, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(C == 4 ? 4 : 3))) void encode_rows_kernel(const TreeArgs T, const QuerySrc src, int64_t Q, int K0,
                                                          int E, MT* __restrict__ h_rows, const QueryOut O) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < Q;
  float x[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
  if (valid) load_query(src, q, x, d);
  float s, t;
  octa(d, s, t);
  float u[3];
  unit_dir3(d, u);
  const float disp = valid ? O.disp[q] : 0.0f;
  const bool keep = q < O.n_idx;
  if (keep) {
    O.uv[q] = make_float2(s, t);
    O.wdir[q] = make_float4(u[0], u[1], u[2], 0.0f);
    O.pos[q] = make_float4(x[0], x[1], x[2], disp);
  }
  typedef MT vC __attribute__((ext_vector_type(C)));
  MT* const row = h_rows + (valid ? q : 0) * (int64_t)K0;
  encode_paper<TT, C, true>(T, valid, x, s, t, [&](int l, const float (&h)[C], const int (&node)[8]) {
    if (valid) {
      vC v;
#pragma unroll
      for (int c = 0; c < C; ++c) v[c] = from_f32<MT>(h[c]);
      *reinterpret_cast<vC*>(row + l * C) = v;
    }
    if (keep)
#pragma unroll
      for (int dd = 0; dd < 8; ++dd) O.idx[(l * 8 + dd) * O.n_idx + q] = node[dd];  // coalesced across lanes
  }, disp, u);
  if (!valid) return;
  typedef MT v4 __attribute__((ext_vector_type(4)));
  for (int k = 0; k < E; k += 4) {
    float g4[4];
    load_attr4(src, q, k, g4);
    v4 v;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = from_f32<MT>(g4[c]);
    *reinterpret_cast<v4*>(row + K0 - E + k) = v;
  }
}

// ---------------------------------------------------------------------------
// Disparity predictor on the matrix cores: each wave encodes 64 queries'
// positions (hash grid) and lookup directions into its FP32 activation tile
// and runs the predictor's MLP on it like the decoder's, writing d per
// query. FP32 path: 16x16x4 FP32 MFMA, weights from L2. 16-bit path
// (SPLIT): every operand is split into two BF16 parts, x = hi + lo with
// hi = bf16(x) and lo = bf16(x - hi) (about 16 significant bits, FP32's
// exponent range), and each product is hi hi + hi lo + lo hi on 16x16x32
// BF16 MFMA with FP32 accumulation: three MFMAs of 16 cycles for each
// eight FP32 ones of 32. The weights are split once per workgroup into LDS.
// hi + lo holds x to 2^-16 relative (each part rounds to 8 significant
// bits) and the dropped lo lo term is below 2^-16 of the product, so each
// product carries at most about 3 * 2^-16 relative error. (A plain 16-bit
// predictor moves shifted lookups across triangle edges often enough to
// break its gradients' agreement.)
// ---------------------------------------------------------------------------

// Packs the predictor's FP32 weights into LDS in fragment order, split into
// BF16 hi (at hi) and lo (at hi + the packed size) parts.
__device__ inline void pack_weights_split(const MlpArgs& M, bf16* hi, int total_elems) {
  int offset = 0;
  for (int layer = 0; layer < M.n_layers; ++layer) {
    const int n_in = layer == 0 ? M.K0 : M.H;
    const int n_out = layer == M.n_layers - 1 ? M.n_out : M.H;
    const int KB = (n_in + 31) / 32;
    const int total = ((n_out + 15) / 16) * KB * kWave * 8;
    const float* src = static_cast<const float*>(M.W[layer]);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int i = e & 7, lane = (e >> 3) & 63, frag = e >> 9;
      const int kb = frag % KB, m = frag / KB;
      const int row = 16 * m + (lane & 15), col = nu(kb, lane >> 4, i);
      const float w = (row < n_out && col < n_in) ? src[(int64_t)row * n_in + col] : 0.0f;
      const bf16 h = from_f32<bf16>(w);
      hi[offset + e] = h;
      hi[total_elems + offset + e] = from_f32<bf16>(w - to_f32(h));
    }
    offset += total;
  }
}

__device__ __forceinline__ void split8(const float (&v)[8], bf16x8& h, bf16x8& l) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bf16 a = from_f32<bf16>(v[i]);
    h[i] = a;
    l[i] = from_f32<bf16>(v[i] - to_f32(a));
  }
}

// acc += A B with A, B split: hi hi + hi lo + lo hi.
__device__ __forceinline__ f32x4 mma_split(const bf16x8& ah, const bf16x8& al, const bf16x8& bh, const bf16x8& bl,
                                           f32x4 c) {
  c = mma(ah, bh, c);
  c = mma(ah, bl, c);
  return mma(al, bh, c);
}

// The predictor's MLP (width 64) on N-tiles t0 .. t0+NT-1 with split
// operands; out[t] rows 0.. = d in lanes 0..15. The input's first K-chunk
// (the 32 hash features) comes from the wave's one-chunk FP32 tile; the
// second holds only the unit direction (inputs 32..34, input 35 zero),
// which the lanes of group 0 take from the lane that owns the query, so the
// tile needs half the LDS.
static_assert(kDispK == 36, "the predictor's input is 32 hash features, the unit direction and a zero");
template <int NT>
__device__ inline void disp_mlp_split(const MlpArgs& M, const WFrag<bf16, true>& Wh, const WFrag<bf16, true>& Wl,
                                      const float* htile, const float u[3], int t0, int lane, f32x4 out[NT]) {
  constexpr int MH = kDispH / 16, KH = kDispH / 32;
  f32x4 acc[MH][NT];
#pragma unroll
  for (int m = 0; m < MH; ++m) {
    const f32x4 bt = bias_tile(M.b[0], kDispH, m, lane);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = bt;
  }
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    bf16x8 bh[NT], bl[NT], ah[MH], al[MH];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float v[8];
      if (kb == 0) {
        const f32x8 x = htile_get<float>(htile, 1, t0 + t, 0, lane);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = x[i];
      } else {
        // slot i < 4 of group g holds input 32 + 4g + i; the rest are >= 48
        const int src = 16 * (t0 + t) + (lane & 15);
        const float s0 = __shfl(u[0], src), s1 = __shfl(u[1], src), s2 = __shfl(u[2], src);
        const bool g0 = (lane >> 4) == 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.0f;
        v[0] = g0 ? s0 : 0.0f;
        v[1] = g0 ? s1 : 0.0f;
        v[2] = g0 ? s2 : 0.0f;
      }
      split8(v, bh[t], bl[t]);
    }
#pragma unroll
    for (int m = 0; m < MH; ++m) {
      ah[m] = Wh.get(M, 0, m, kb, lane);
      al[m] = Wl.get(M, 0, m, kb, lane);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int m = 0; m < MH; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = mma_split(ah[m], al[m], bh[t], bl[t], acc[m][t]);
  }
  // ReLU'd outputs of tiles (2kb, 2kb+1) are the next layer's chunk kb
  auto chain = [&](int kb, int t, bf16x8& h, bf16x8& l) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = fmaxf(acc[2 * kb][t][j], 0.0f);
      v[4 + j] = fmaxf(acc[2 * kb + 1][t][j], 0.0f);
    }
    split8(v, h, l);
  };
  for (int layer = 1; layer < M.n_layers - 1; ++layer) {
    bf16x8 bh[KH][NT], bl[KH][NT];
#pragma unroll
    for (int kb = 0; kb < KH; ++kb)
#pragma unroll
      for (int t = 0; t < NT; ++t) chain(kb, t, bh[kb][t], bl[kb][t]);
#pragma unroll
    for (int m = 0; m < MH; ++m) {
      const f32x4 bt = bias_tile(M.b[layer], kDispH, m, lane);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = bt;
    }
#pragma unroll
    for (int kb = 0; kb < KH; ++kb) {
      bf16x8 ah[MH], al[MH];
#pragma unroll
      for (int m = 0; m < MH; ++m) {
        ah[m] = Wh.get(M, layer, m, kb, lane);
        al[m] = Wl.get(M, layer, m, kb, lane);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int m = 0; m < MH; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = mma_split(ah[m], al[m], bh[kb][t], bl[kb][t], acc[m][t]);
    }
  }
  const int lo = M.n_layers - 1;
  const f32x4 bo = bias_tile(M.b[lo], M.n_out, 0, lane);
#pragma unroll
  for (int t = 0; t < NT; ++t) out[t] = bo;
#pragma unroll
  for (int kb = 0; kb < KH; ++kb) {
    const bf16x8 ah = Wh.get(M, lo, 0, kb, lane), al = Wl.get(M, lo, 0, kb, lane);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x8 bh, bl;
      chain(kb, t, bh, bl);
      out[t] = mma_split(ah, al, bh, bl, out[t]);
    }
  }
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void disparity_fwd_kernel(const DispArgs G, const MlpArgs P, const QuerySrc src,
                                                            int64_t Q, float* __restrict__ d_out) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  constexpr int NT = 2;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, waves = blockDim.x >> 6;
  const int KB0 = (P.K0 + 31) / 32;
  const int KBT = SPLIT ? 1 : KB0;  // K-chunks the FP32 tile holds
  const int wl_elems = SPLIT ? packed_weight_elems<bf16>(P.n_layers, P.K0, P.H) : 0;
  bf16* const wl = reinterpret_cast<bf16*>(smem);
  float* const htile = reinterpret_cast<float*>(wl + 2 * wl_elems) + wave * (4 * KBT * kWave * 8);
  if (SPLIT) pack_weights_split(P, wl, wl_elems);
  {  // zero the K padding of this lane's row once
    const float z[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = P.K0; k < 32 * KBT; k += 4) htile_put4<float>(htile, KBT, lane, k, z);
  }
  if (SPLIT) __syncthreads();
  const WFrag<float, false> W{nullptr, KB0};
  const WFrag<bf16, true> Wh{wl, KB0}, Wlo{wl + wl_elems, KB0};
  const int64_t n_tiles = (Q + 63) / 64;
  const TileRange tr = xcd_tiles(n_tiles, waves, wave);
  for (int64_t tile = tr.first; tile < tr.end; tile += tr.stride) {
    const int64_t q = tile * 64 + lane;
    float x[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f}, u[3];
    if (q < Q) load_query(src, q, x, d);
    unit_dir3(d, u);
    float a[kDispK];
    disparity_input(G, x, u, a);
#pragma unroll
    for (int k = 0; k < (SPLIT ? 32 : kDispK); k += 4) htile_put4<float>(htile, KBT, lane, k, &a[k]);
    wave_lds_sync();
#pragma unroll
    for (int t0 = 0; t0 < 4; t0 += NT) {
      f32x4 out[NT];
      if constexpr (SPLIT)
        disp_mlp_split<NT>(P, Wh, Wlo, htile, u, t0, lane, out);
      else
        mlp_forward_tiles<float, kDispH, NT>(P, W, htile, KB0, t0, lane, out);
      if (lane < 16) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int64_t qq = tile * 64 + 16 * (t0 + t) + lane;
          if (qq < Q) d_out[qq] = out[t][0];
        }
      }
    }
    wave_lds_sync();
  }
}

// ---------------------------------------------------------------------------
// Residual assembly (rendering-equation RHS) and loss partials.
// ---------------------------------------------------------------------------

// One group of G lanes per LHS point (G = N rounded up to a power of two,
// at most 64): lane k of the group weighs secondary sample k (and k + G, ...)
// so the per-sample inputs are read coalesced; the group sums its products
// with lane shuffles in a fixed order. The group leader forms
// T = Le + (1/N) sum_k w_k * L(x2_k) and r = L - T and writes the outputs;
// each block leaves one FP64 partial of sum r^2 (or (r / rho)^2).
__global__ __launch_bounds__(256) void combine_kernel(const ResidualArgs A, int G, const float* __restrict__ Lq,
                                                      const int32_t* __restrict__ rank, float* __restrict__ lhs_out, float* __restrict__ rhs_out,
                                                      float* __restrict__ resid_out, double* __restrict__ partials) {
  __shared__ double red[4];
  const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  const int64_t b = gid / G;
  const int k0 = (int)(gid % G);
  const bool valid = b < A.B;
  float s[3] = {0.f, 0.f, 0.f};
  if (valid && !A.target_override && A.N > 0) {
    float n[3], wo[3], alb[3] = {A.albedo[3 * b], A.albedo[3 * b + 1], A.albedo[3 * b + 2]};
    load_unit(A.n + 3 * b, n);
    load_unit(A.wo + 3 * b, wo);
    const float alpha = A.rough[b];
    for (int k = k0; k < A.N; k += G) {
      const int64_t bk = b * A.N + k;
      float wi[3], w[3];
      load_unit(A.wi + 3 * bk, wi);
      bsdf_weight(n, wo, wi, alb, alpha, A.F0, A.pdf ? A.pdf[bk] : 1.0f, w);
      const int64_t qk = A.B + bk;
      const float* Lk = Lq + 3 * (rank ? (int64_t)rank[qk] : qk);
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c] += w[c] * Lk[c];
    }
  }
  for (int off = G >> 1; off > 0; off >>= 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += __shfl_xor(s[c], off, G);
  double acc = 0.0;
  if (valid && k0 == 0) {
    const float* Lb = Lq + 3 * (rank ? (int64_t)rank[b] : b);
    float L[3] = {Lb[0], Lb[1], Lb[2]};
    float T[3];
    if (A.target_override) {
#pragma unroll
      for (int c = 0; c < 3; ++c) T[c] = A.target_override[3 * b + c];
    } else {
      const float invN = A.N > 0 ? 1.0f / (float)A.N : 0.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) T[c] = A.Le[3 * b + c] + s[c] * invN;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float r = L[c] - T[c];
      lhs_out[3 * b + c] = L[c];
      rhs_out[3 * b + c] = T[c];
      resid_out[3 * b + c] = r;
      double rr = (double)r;
      if (A.loss_kind == 1) {
        const double rho = fmax((double)L[c] + (double)T[c], 0.0) + (double)A.eps;
        rr /= rho;
      }
      acc += rr * rr;
    }
  }
  // fixed order: within each wave by shuffles, then the four waves in turn
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Fixed-order sum of the block partials: loss = sum / (3B).
__global__ __launch_bounds__(256) void loss_reduce_kernel(const double* __restrict__ partials, int n, int64_t B,
                                                          double* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = B > 0 ? red[0] / (3.0 * (double)B) : 0.0;
}

// Eight elements per thread and iteration (two 16-byte loads, one store of
// 8 x sizeof(DT) bytes) when both pointers allow it, both loads issued before
// either is converted; the tail and unaligned arrays go element by element.
template <class DT>
__global__ __launch_bounds__(256) void cast_kernel(const float* __restrict__ src, DT* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nv = 0;
  if ((reinterpret_cast<uintptr_t>(src) % 16) == 0 && (reinterpret_cast<uintptr_t>(dst) % (8 * sizeof(DT))) == 0) {
    nv = n / 8;
    typedef DT v8 __attribute__((ext_vector_type(8)));
    for (int64_t i = i0; i < nv; i += stride) {
      // streamed once: non-temporal loads and stores keep the masters and
      // the working copy from displacing cached data
      typedef float f4 __attribute__((ext_vector_type(4)));
      const f4 a = __builtin_nontemporal_load(reinterpret_cast<const f4*>(src) + 2 * i);
      const f4 b = __builtin_nontemporal_load(reinterpret_cast<const f4*>(src) + 2 * i + 1);
      v8 o;
      o[0] = from_f32<DT>(a.x);
      o[1] = from_f32<DT>(a.y);
      o[2] = from_f32<DT>(a.z);
      o[3] = from_f32<DT>(a.w);
      o[4] = from_f32<DT>(b.x);
      o[5] = from_f32<DT>(b.y);
      o[6] = from_f32<DT>(b.z);
      o[7] = from_f32<DT>(b.w);
      __builtin_nontemporal_store(o, reinterpret_cast<v8*>(dst) + i);
    }
  }
  for (int64_t i = 8 * nv + i0; i < n; i += stride) dst[i] = from_f32<DT>(src[i]);
}

// Node indices the residual forward stored for its backward queries
// ([L][Qb], sorted positions), returned per source query ([Qb][L]). Sorted
// position p holds source query order[p]; a value outside [0, Qb) is skipped.
// With K = 8 (the paper's scheme) each level holds the eight corners:
// [L][8][Qb] in, [Qb][L][8] out.
__global__ __launch_bounds__(256) void saved_nodes_kernel(const int32_t* __restrict__ nidx,
                                                          const int32_t* __restrict__ order, int64_t Qb, int L, int K,
                                                          int32_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Qb) return;
  const int64_t q = order[p];
  if (q < 0 || q >= Qb) return;
  for (int l = 0; l < L; ++l)
    for (int k = 0; k < K; ++k) out[(q * L + l) * K + k] = nidx[((int64_t)l * K + k) * Qb + p];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

static int max_lds() {
  static int lds = 0;
  if (!lds) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (lds <= 0) lds = 65536;
  }
  return lds;
}

template <class TT, class HT, int C>
static hipError_t launch_encode_t(const TreeArgs& T, const float* x, const float* d, int64_t B, void* h,
                                  int32_t* idx, const DispArgs& G, hipStream_t st) {
  const int64_t blocks = (B + 255) / 256;
  HT* hp = reinterpret_cast<HT*>(h);
  if (T.interp != OO_INTERP_PAPER)
    hipLaunchKernelGGL((encode_kernel<TT, HT, C, 0>), dim3((unsigned)blocks), dim3(256), 0, st, T, x, d, B, hp, idx, G);
  else if (G.n_levels == 0)
    hipLaunchKernelGGL((encode_kernel<TT, HT, C, 1>), dim3((unsigned)blocks), dim3(256), 0, st, T, x, d, B, hp, idx, G);
  else if constexpr (sizeof(HT) == 4)  // the shifted encoding writes FP32 features only
    hipLaunchKernelGGL((encode_kernel<TT, HT, C, 2>), dim3((unsigned)blocks), dim3(256), 0, st, T, x, d, B, hp, idx, G);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class TT, int C>
static hipError_t launch_encode_h(const TreeArgs& T, const float* x, const float* d, int64_t B, void* h,
                                  oo_dtype hd, int32_t* idx, const DispArgs& G, hipStream_t st) {
  switch (hd) {
    case OO_F32: return launch_encode_t<TT, float, C>(T, x, d, B, h, idx, G, st);
    case OO_F16: return launch_encode_t<TT, f16, C>(T, x, d, B, h, idx, G, st);
    default: return launch_encode_t<TT, bf16, C>(T, x, d, B, h, idx, G, st);
  }
}

hipError_t launch_encode(const TreeArgs& T, oo_dtype td, const float* x, const float* d, int64_t B, void* h,
                         oo_dtype hd, int32_t* idx, const DispArgs& G, hipStream_t st) {
  if (B == 0) return hipSuccess;
  if (td == OO_F32)
    return T.C == 4 ? launch_encode_h<float, 4>(T, x, d, B, h, hd, idx, G, st)
                    : launch_encode_h<float, 8>(T, x, d, B, h, hd, idx, G, st);
  if (td == OO_F16)
    return T.C == 4 ? launch_encode_h<f16, 4>(T, x, d, B, h, hd, idx, G, st)
                    : launch_encode_h<f16, 8>(T, x, d, B, h, hd, idx, G, st);
  return T.C == 4 ? launch_encode_h<bf16, 4>(T, x, d, B, h, hd, idx, G, st)
                  : launch_encode_h<bf16, 8>(T, x, d, B, h, hd, idx, G, st);
}

// Grid of the tile kernels for a workgroup of `waves` waves using lds bytes.
static int tile_grid(int64_t Q, int waves, size_t lds) {
  const int64_t n_tiles = (Q + 63) / 64;
  // LDS per CU on gfx950 is 160 KiB: one or two workgroups fit per CU.
  const int per_cu = lds * 2 <= (size_t)160 * 1024 ? 2 : 1;
  int64_t g = (int64_t)device_cus() * per_cu;
  const int64_t need = (n_tiles + waves - 1) / waves;
  if (g > need) g = need;
  if (g >= 8) g -= g % 8;
  return (int)(g > 0 ? g : 1);
}

// The shape without weights in LDS: as many 64-query tiles as fit, up to 8.
template <class MT>
static void tile_launch_shape_plain(const MlpArgs& M, int64_t Q, int& waves, size_t& lds, int& grid) {
  const int KB0 = (M.K0 + 31) / 32;
  const size_t tile_bytes = (size_t)4 * KB0 * kWave * 8 * sizeof(MT);
  waves = 8;
  while (waves > 1 && waves * tile_bytes > (size_t)max_lds()) --waves;
  lds = waves * tile_bytes;
  grid = tile_grid(Q, waves, lds);
}

// Workgroup shape for the tile kernels: up to 8 waves, each with a 64-query
// activation tile, plus the packed weights when they fit next to them.
template <class MT>
static void tile_launch_shape(const MlpArgs& M, int64_t Q, bool& wlds, int& waves, size_t& lds, int& grid) {
  const int KB0 = (M.K0 + 31) / 32;
  const size_t tile_bytes = (size_t)4 * KB0 * kWave * 8 * sizeof(MT);
  const size_t wbytes = (size_t)packed_weight_elems<MT>(M.n_layers, M.K0, M.H) * sizeof(MT);
  const size_t cap = (size_t)max_lds();
  waves = 8;
  wlds = true;
  while (waves > 4 && wbytes + waves * tile_bytes > cap) --waves;
  if (wlds && wbytes + waves * tile_bytes > cap) wlds = false;
  if (!wlds) {
    waves = 8;
    while (waves > 1 && waves * tile_bytes > cap) --waves;
  }
  lds = (wlds ? wbytes : 0) + waves * tile_bytes;
  grid = tile_grid(Q, waves, lds);
}


template <class TT, class MT, int C, int H, int MODE>
static hipError_t launch_query_p(const TreeArgs& T, const MlpArgs& M, const QuerySrc& src, int64_t Q, float* rgb,
                                 const QueryOut& O, const DispArgs& G, hipStream_t st) {
  bool wlds;
  int waves, grid;
  size_t lds;
  tile_launch_shape<MT>(M, Q, wlds, waves, lds, grid);
  if (wlds && MODE >= 2) {  // the shifted variants: keep one of each
    wlds = false;
    tile_launch_shape_plain<MT>(M, Q, waves, lds, grid);
  }
  if (wlds) {
    auto k = query_kernel<TT, MT, C, H, true, MODE >= 2 ? 1 : MODE>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, st, T, M, src, Q, rgb, O, G);
  } else {
    auto k = query_kernel<TT, MT, C, H, false, MODE>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, st, T, M, src, Q, rgb, O, G);
  }
  return hipGetLastError();
}

template <class TT, class MT, int C, int H>
static hipError_t launch_query_t(const TreeArgs& T, const MlpArgs& M, const QuerySrc& src, int64_t Q, float* rgb,
                                 const QueryOut& O, const DispArgs& G, hipStream_t st) {
  if (T.interp != OO_INTERP_PAPER) return launch_query_p<TT, MT, C, H, 0>(T, M, src, Q, rgb, O, G, st);
  if (G.n_levels == 0) return launch_query_p<TT, MT, C, H, 1>(T, M, src, Q, rgb, O, G, st);
  return launch_query_p<TT, MT, C, H, 2>(T, M, src, Q, rgb, O, G, st);
}

template <class TT, class MT, int C>
static hipError_t launch_query_c(const TreeArgs& T, const MlpArgs& M, const QuerySrc& src, int64_t Q, float* rgb,
                                 const QueryOut& O, const DispArgs& G, hipStream_t st) {
  return M.H == 64 ? launch_query_t<TT, MT, C, 64>(T, M, src, Q, rgb, O, G, st)
                   : launch_query_t<TT, MT, C, 128>(T, M, src, Q, rgb, O, G, st);
}

hipError_t launch_query(const TreeArgs& T, oo_dtype td, const MlpArgs& M, oo_dtype md, const QuerySrc& src,
                        int64_t Q, float* rgb, const QueryOut& O, const DispArgs& G, hipStream_t st) {
  if (Q == 0) return hipSuccess;
  if (td == OO_F32)
    return T.C == 4 ? launch_query_c<float, float, 4>(T, M, src, Q, rgb, O, G, st)
                    : launch_query_c<float, float, 8>(T, M, src, Q, rgb, O, G, st);
  if (td == OO_F16)
    return T.C == 4 ? launch_query_c<f16, f16, 4>(T, M, src, Q, rgb, O, G, st)
                    : launch_query_c<f16, f16, 8>(T, M, src, Q, rgb, O, G, st);
  return T.C == 4 ? launch_query_c<bf16, bf16, 4>(T, M, src, Q, rgb, O, G, st)
                  : launch_query_c<bf16, bf16, 8>(T, M, src, Q, rgb, O, G, st);
  (void)md;
}

template <class MT, int H>
static hipError_t launch_mlp_t(const MlpArgs& M, const void* h, int64_t Q, float* rgb, hipStream_t st) {
  bool wlds;
  int waves, grid;
  size_t lds;
  tile_launch_shape<MT>(M, Q, wlds, waves, lds, grid);
  if (wlds) {
    auto k = mlp_kernel<MT, H, true>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, st, M, reinterpret_cast<const MT*>(h), Q, rgb);
  } else {
    auto k = mlp_kernel<MT, H, false>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, st, M, reinterpret_cast<const MT*>(h), Q, rgb);
  }
  return hipGetLastError();
}

hipError_t launch_mlp(const MlpArgs& M, oo_dtype md, const void* h, int64_t Q, float* rgb, hipStream_t st) {
  if (Q == 0) return hipSuccess;
  if (md == OO_F32) return M.H == 64 ? launch_mlp_t<float, 64>(M, h, Q, rgb, st) : launch_mlp_t<float, 128>(M, h, Q, rgb, st);
  if (md == OO_F16) return M.H == 64 ? launch_mlp_t<f16, 64>(M, h, Q, rgb, st) : launch_mlp_t<f16, 128>(M, h, Q, rgb, st);
  return M.H == 64 ? launch_mlp_t<bf16, 64>(M, h, Q, rgb, st) : launch_mlp_t<bf16, 128>(M, h, Q, rgb, st);
}

static int combine_group(int N) {
  int G = 1;
  while (G < N && G < 64) G <<= 1;
  return G;
}

int combine_blocks(int64_t B, int N) { return (int)((B * combine_group(N) + 255) / 256); }

hipError_t launch_combine(const ResidualArgs& A, const float* Lq, const int32_t* rank, float* lhs, float* rhs,
                          float* resid, double* partials, double* loss, hipStream_t st) {
  const int G = combine_group(A.target_override ? 0 : A.N);
  const int nb = combine_blocks(A.B, A.target_override ? 0 : A.N);
  if (nb > 0)
    hipLaunchKernelGGL(combine_kernel, dim3(nb), dim3(256), 0, st, A, G, Lq, rank, lhs, rhs, resid, partials);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, st, partials, nb, A.B, loss);
  return hipGetLastError();
}

hipError_t launch_saved_nodes(const int32_t* nidx, const int32_t* order, int64_t Qb, int L, int K, int32_t* out,
                              hipStream_t st) {
  if (Qb == 0) return hipSuccess;
  hipLaunchKernelGGL(saved_nodes_kernel, dim3((unsigned)((Qb + 255) / 256)), dim3(256), 0, st, nidx, order, Qb, L,
                     K, out);
  return hipGetLastError();
}

hipError_t launch_cast(const float* src, void* dst, oo_dtype dt, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // one 8-element vector per thread (measured faster than a smaller grid
  // striding over the array); arrays beyond 2^33 elements stride
  int64_t blocks = (n / 8 + 255) / 256;
  if (blocks > (1 << 22)) blocks = 1 << 22;
  if (blocks < 1) blocks = 1;
  if (dt == OO_F32)
    hipLaunchKernelGGL(cast_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, src, (float*)dst, n);
  else if (dt == OO_F16)
    hipLaunchKernelGGL(cast_kernel<f16>, dim3((unsigned)blocks), dim3(256), 0, st, src, (f16*)dst, n);
  else
    hipLaunchKernelGGL(cast_kernel<bf16>, dim3((unsigned)blocks), dim3(256), 0, st, src, (bf16*)dst, n);
  return hipGetLastError();
}

template <class TT, class MT, int C>
static void launch_encode_rows_t(const TreeArgs& T, const QuerySrc& src, int64_t Q, int K0, int E, void* h_rows,
                                 const QueryOut& O, hipStream_t st) {
  hipLaunchKernelGGL((encode_rows_kernel<TT, MT, C>), dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, st, T, src, Q,
                     K0, E, reinterpret_cast<MT*>(h_rows), O);
}

hipError_t launch_encode_rows(const TreeArgs& T, oo_dtype td, const MlpArgs& M, const QuerySrc& src, int64_t Q,
                              void* h_rows, const QueryOut& O, hipStream_t st) {
  if (Q == 0) return hipSuccess;
  // the tables and the decoder share one dtype in the product paths
  if (td == OO_F32)
    T.C == 4 ? launch_encode_rows_t<float, float, 4>(T, src, Q, M.K0, M.E, h_rows, O, st)
             : launch_encode_rows_t<float, float, 8>(T, src, Q, M.K0, M.E, h_rows, O, st);
  else if (td == OO_F16)
    T.C == 4 ? launch_encode_rows_t<f16, f16, 4>(T, src, Q, M.K0, M.E, h_rows, O, st)
             : launch_encode_rows_t<f16, f16, 8>(T, src, Q, M.K0, M.E, h_rows, O, st);
  else
    T.C == 4 ? launch_encode_rows_t<bf16, bf16, 4>(T, src, Q, M.K0, M.E, h_rows, O, st)
             : launch_encode_rows_t<bf16, bf16, 8>(T, src, Q, M.K0, M.E, h_rows, O, st);
  return hipGetLastError();
}

hipError_t launch_disparity_fwd(const DispArgs& G, oo_dtype md, const QuerySrc& src, int64_t Q, float* d_out,
                                hipStream_t st) {
  if (Q == 0) return hipSuccess;
  MlpArgs P{};
  P.n_layers = G.n_layers;
  P.K0 = kDispK;
  P.E = 0;
  P.H = kDispH;
  P.n_out = 1;
  for (int i = 0; i < kMaxLayers; ++i) {
    P.W[i] = i < G.n_layers ? G.W[i] : nullptr;
    P.b[i] = i < G.n_layers ? G.b[i] : nullptr;
  }
  // four-wave workgroups, two per CU: four 16 KiB FP32 tiles, or for the
  // split variant the hi and lo weight copies (2 x 18 KiB) and four 8 KiB
  // one-chunk tiles
  const bool split = md != OO_F32;
  constexpr int waves = 4;
  const size_t wbytes = split ? (size_t)2 * packed_weight_elems<bf16>(P.n_layers, P.K0, P.H) * sizeof(bf16) : 0;
  const int kbt = split ? 1 : (P.K0 + 31) / 32;
  const size_t lds = wbytes + (size_t)waves * 4 * kbt * kWave * 8 * sizeof(float);
  const int grid = tile_grid(Q, waves, lds);
  if (split) {
    hipFuncSetAttribute((const void*)disparity_fwd_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(disparity_fwd_kernel<true>, dim3(grid), dim3(64 * waves), lds, st, G, P, src, Q, d_out);
  } else {
    hipFuncSetAttribute((const void*)disparity_fwd_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(disparity_fwd_kernel<false>, dim3(grid), dim3(64 * waves), lds, st, G, P, src, Q, d_out);
  }
  return hipGetLastError();
}

}  // namespace oo
