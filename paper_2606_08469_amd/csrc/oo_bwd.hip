// Backward of the residual step: seeds, the fused recompute + decoder
// backward kernel, the feature-gradient scatter, and the fixed-order dW/db
// reduction.
//
// One workgroup (8 waves with 16-bit operands, 16 with FP32) handles 64
// queries at a time:
//  1. encode: node indices and octahedral coordinates come from the forward;
//     one lane per wave for each query (8 or 16), each gathering whole texels
//     of its levels; h written to the layer-0 activation buffer as
//     [feature][query];
//  2. forward recompute of the hidden layers on matrix cores, activations
//     kept in LDS as [neuron][query];
//  3. backward: delta chained through W^T on matrix cores; dW of every layer
//     contracted over the workgroup's 64 queries, each wave owning a share of
//     the dW tiles in registers for the whole kernel; dh of every query
//     written to memory.
// dW/db leave as one partial per workgroup (accumulated over the launches
// of one backward), reduced in a fixed order later. A separate,
// high-occupancy kernel scatters w_tap * dh into the FP32 feature gradient
// tables with hardware float atomics; the caller runs it on a second stream
// so that it overlaps the next launch of the fused kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "oo_device.h"
#include "oo_internal.h"

namespace oo {

constexpr int kQW = 64;  // queries per workgroup tile

struct BwdLayout {
  int KB0, R0;
  size_t act0, act1, seed, total;
};

__host__ __device__ inline BwdLayout bwd_layout(int K0, int H, int n_layers, int L, int msz) {
  BwdLayout b;
  b.KB0 = (K0 + 31) / 32;
  b.R0 = (K0 + 15) / 16 * 16;
  size_t o = 0;
  b.act0 = o;
  o += (size_t)b.R0 * kQW * msz;
  b.act1 = o;  // hidden-layer activations a_1 .. a_{n_layers-1}, H rows each;
  o += (size_t)(n_layers - 1) * H * kQW * msz;  // the backward overwrites a_i with delta_i
  b.seed = o;  // output-layer seeds, 16 rows (3 used)
  o += (size_t)16 * kQW * msz;
  b.total = o;
  return b;
  (void)L;
}

// [row][query] buffer of 64 queries, 16-byte chunks XOR-swizzled by row so
// that 16 lanes reading 16 rows at one query offset hit distinct banks.
__device__ inline int tq_index(int row, int q) { return row * kQW + ((((q >> 3) ^ (row & 7))) << 3) + (q & 7); }

template <class MT>
__device__ inline typename FragT<MT>::type tq_frag(const MT* buf, int row, int chunk) {
  return *reinterpret_cast<const typename FragT<MT>::type*>(buf + row * kQW + ((chunk ^ (row & 7)) << 3));
}

// Packs an n_rows x n_cols row-major matrix (leading dimension ld) into
// matrix-core A-fragment order: fragment (m, kb) holds, for lane l and slot
// i, A[16 m + l % 16][nu(kb, l / 16, i)], zero outside the matrix. One
// 16-byte LDS read then gives a lane its fragment.
template <class MT>
__device__ inline void pack_frags_lds(const MT* src, int n_rows, int n_cols, int ld, MT* dst) {
  const int KB = (n_cols + 31) / 32, total = ((n_rows + 15) / 16) * KB * kWave * 8;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = e & 7, lane = (e >> 3) & 63, frag = e >> 9;
    const int kb = frag % KB, m = frag / KB;
    const int row = 16 * m + (lane & 15), col = nu(kb, lane >> 4, i);
    dst[e] = (row < n_rows && col < n_cols) ? src[(int64_t)row * ld + col] : from_f32<MT>(0.0f);
  }
}

template <class MT>
__device__ inline typename FragT<MT>::type lds_frag(const MT* packed, int KB, int m, int kb, int lane) {
  return *reinterpret_cast<const typename FragT<MT>::type*>(packed + ((m * KB + kb) * kWave + lane) * 8);
}

// Weights kept packed in LDS next to the activation buffers: W_i and W_i^T
// of every hidden-to-hidden layer 0 < i < n_layers - 1 (H x H each), then
// W_0^T (K0 x H), which forms dh, then W_0 (H x K0) for the recompute.
__host__ __device__ inline size_t hidden_weight_elems(int H, int n_layers) {
  return (size_t)(n_layers > 2 ? n_layers - 2 : 0) * 2 * H * H;
}
__host__ __device__ inline size_t lds_weight_bytes(int K0, int H, int n_layers, int msz) {
  const size_t wt0 = (size_t)((K0 + 15) / 16) * (H / 32) * kWave * 8;  // W_0^T: K0 rows, H inputs
  const size_t w0 = (size_t)(H / 16) * ((K0 + 31) / 32) * kWave * 8;   // W_0: H rows, K0 inputs
  return (hidden_weight_elems(H, n_layers) + wt0 + w0) * msz;
}


// Waves per workgroup. The LDS holds one workgroup per CU, and the feature
// scatter, which runs beside this kernel on a second stream, gets the wave
// slots the workgroup leaves free. With 16-bit operands 8 waves (two per SIMD,
// up to 256 registers each, an eighth of the dW tiles per wave) measured
// faster for the pair than 16 waves of 128 registers. FP32 reads its weights
// from L2 (they do not fit in LDS) and needs the latency hiding of 16 waves.
template <class MT>
__host__ __device__ constexpr int bwd_waves() {
  return sizeof(MT) == 4 ? 16 : 8;
}

// With 16-bit operands a K-chunk's operand reads all go out before its
// MFMAs (a scheduling barrier keeps them there; otherwise each read is
// waited on next to its MFMA). FP32 fragments take 8 registers each and its
// 16-wave workgroups hide the latency; there the batching measured slower,
// so FP32 keeps the compiler's interleaved schedule.
template <class MT>
__host__ __device__ constexpr bool batch_reads() {
  return sizeof(MT) == 2;
}

// dW tiles of one layer owned by this wave: tile tau = wave + NW u.
template <class MT, int NW, int U>
__device__ inline void dw_layer(f32x4 (&acc)[U], const MT* dT, const MT* act, int n_out, int n_in, int wave, int lane) {
  const int MM = (n_out + 15) / 16, NK = (n_in + 15) / 16;
  const int r16 = lane & 15, g = lane >> 4;
  if constexpr (!batch_reads<MT>()) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int tau = wave + NW * u;
      if (tau < MM * NK) {
        const int mm = tau / NK, nk = tau % NK;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          const auto a = tq_frag<MT>(dT, 16 * mm + r16, 4 * kk + g);
          const auto b = tq_frag<MT>(act, 16 * nk + r16, 4 * kk + g);
          acc[u] = mma(a, b, acc[u]);
        }
      }
      // keep the scheduler from hoisting every tile's LDS reads at once
      __builtin_amdgcn_sched_barrier(0);
    }
    return;
  }
  // two tiles at a time: their eight operand reads go out before the four
  // MFMAs (all tiles' reads at once would hold too many registers)
#pragma unroll
  for (int u0 = 0; u0 < U; u0 += 2) {
    typename FragT<MT>::type a[2][2], b[2][2];
#pragma unroll
    for (int du = 0; du < 2; ++du) {
      const int tau = wave + NW * (u0 + du);
      if (u0 + du < U && tau < MM * NK) {
        const int mm = tau / NK, nk = tau % NK;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          a[du][kk] = tq_frag<MT>(dT, 16 * mm + r16, 4 * kk + g);
          b[du][kk] = tq_frag<MT>(act, 16 * nk + r16, 4 * kk + g);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int du = 0; du < 2; ++du) {
      const int tau = wave + NW * (u0 + du);
      if (u0 + du < U && tau < MM * NK)
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) acc[u0 + du] = mma(a[du][kk], b[du][kk], acc[u0 + du]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int NW, int U>
__device__ inline void dw_store(const f32x4 (&acc)[U], float* part, int64_t off, int n_out, int n_in, int wave,
                                int lane, bool add) {
  const int MM = (n_out + 15) / 16, NK = (n_in + 15) / 16;
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int tau = wave + NW * u;
    if (tau < MM * NK) {
      const int mm = tau / NK, nk = tau % NK;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = 16 * mm + 4 * g + j, k = 16 * nk + r16;
        if (n < n_out && k < n_in) {
          float& dst = part[off + (int64_t)n * n_in + k];
          dst = add ? dst + acc[u][j] : acc[u][j];
        }
      }
    }
  }
}

// B-operand chunk kb for query column col, read from a [row][query] buffer:
// slot i holds row nu(kb, g, i); rows >= n_rows read as zero.
template <class MT>
__device__ inline typename FragT<MT>::type tq_bfrag(const MT* buf, int kb, int g, int col, int n_rows) {
  typename FragT<MT>::type b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int row = nu(kb, g, i);
    b[i] = row < n_rows ? buf[tq_index(row, col)] : from_f32<MT>(0.0f);
  }
  return b;
}

// Writes this wave's output tiles (M-tiles m0 .. m0+MT2-1 of query columns
// 16 nt .. 16 nt + 15) into a [row][query] buffer, rows >= n_rows as zeros.
template <class MT, int MT2>
__device__ inline void store_tq(MT* buf, const f32x4 (&acc)[MT2], int m0, int n_tiles, int n_rows, int nt, int lane,
                                bool relu) {
  const int col = 16 * nt + (lane & 15), g = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < MT2; ++mi) {
    const int m = m0 + mi;
    if (m < n_tiles) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * m + 4 * g + j;
        float v = row < n_rows ? acc[mi][j] : 0.0f;
        if (relu) v = fmaxf(v, 0.0f);
        buf[tq_index(row, col)] = from_f32<MT>(v);
      }
    }
  }
}

// Workgroup of bwd_waves<MT>() waves on 64 queries. In the layer chains wave w
// works on query columns 16 (w % 4) .. +15 and on the share w / 4 of the
// output rows; the layers exchange activations and deltas through the
// [row][query] buffers. With WL the hidden-to-hidden weights W_i and W_i^T,
// W_0^T and W_0 are packed into LDS once per workgroup (their per-tile
// fragment loads from L2 dominated the layer chains); the output layer's
// weights are read from L2.
// NHH: hidden-to-hidden layers whose dW the kernel accumulates in registers
// (up to 3 at width 64; at width 128 one, or three for a four-hidden-layer
// decoder).
template <class TT, class MT, int C, int H, bool WL, bool PAPER, int NHH>
__global__ __launch_bounds__(64 * bwd_waves<MT>()) void bwd_kernel(const TreeArgs T, const MlpArgs M, const MlpArgs Mt,
                                                             const BwdArgs A, const ParamLayout PL) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  typedef typename FragT<MT>::type frag;
  const int64_t Q = A.Q, ldn = A.ldn, n_seed = A.n_seed;
  const int32_t* __restrict__ nidx = A.nidx;
  const float2* __restrict__ uv = A.uv;
  const float* __restrict__ seeds = A.seeds;
  const int32_t* __restrict__ order = A.order;
  float* __restrict__ partials = A.partials;
  float* __restrict__ dh_out = A.dh;
  constexpr int NW = bwd_waves<MT>();
  constexpr int kMSplit = NW / 4;                  // waves sharing one query column block
  constexpr int kLanesPerQuery = 64 * NW / kQW;
  constexpr int MH = H / 16, MH2 = MH / kMSplit;
  constexpr int U0 = (MH * 8 + NW - 1) / NW, UH = (MH * MH + NW - 1) / NW;
  constexpr int UO = (MH + NW - 1) / NW;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar branches
  const int nt = wave & 3, mh = wave >> 2, col = 16 * nt + r16;  // mh = 0 with 4 waves
  const int K0 = M.K0, NL = M.n_layers, L = T.L, LC = L * C;
  const BwdLayout lay = bwd_layout(K0, H, NL, L, (int)sizeof(MT));
  const int KB0 = lay.KB0, R0 = lay.R0;
  MT* const act0 = reinterpret_cast<MT*>(smem + lay.act0);
  MT* const act1 = reinterpret_cast<MT*>(smem + lay.act1);
  // input activation buffer of layer i: a_0 = h, a_i = ReLU(z_{i-1})
  auto act = [&](int i) { return i == 0 ? act0 : act1 + (size_t)(i - 1) * H * kQW; };
  MT* const seedb = reinterpret_cast<MT*>(smem + lay.seed);
  // Buffer of the gradient flowing into layer i's output: the seeds for the
  // output layer, else the buffer of a_{i+1}, which step i + 1 overwrote with
  // delta_{i+1} once a_{i+1} was no longer needed.
  auto din = [&](int i) { return i == NL - 1 ? seedb : act(i + 1); };
  // packed weights: layer i at hw + 2 (i - 1) H^2 (W_i), + H^2 (W_i^T);
  // then W_0^T, then W_0
  MT* const hw = reinterpret_cast<MT*>(smem + lay.total);
  MT* const wt0 = hw + hidden_weight_elems(H, NL);
  MT* const w0p = wt0 + (size_t)((K0 + 15) / 16) * (H / 32) * kWave * 8;
  if (WL) {
    for (int i = 1; i < NL - 1; ++i) {
      pack_frags_lds<MT>(reinterpret_cast<const MT*>(M.W[i]), H, H, H, hw + (size_t)2 * (i - 1) * H * H);
      pack_frags_lds<MT>(reinterpret_cast<const MT*>(Mt.W[i]), H, H, H, hw + (size_t)(2 * (i - 1) + 1) * H * H);
    }
    pack_frags_lds<MT>(reinterpret_cast<const MT*>(Mt.W[0]), K0, H, H, wt0);  // W_0^T is [K0][H]
    pack_frags_lds<MT>(reinterpret_cast<const MT*>(M.W[0]), H, K0, K0, w0p);  // W_0 is [H][K0]
  }

  f32x4 acc0[U0], accH[NHH][UH], accO[UO];
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < U0; ++u) acc0[u] = z4;
#pragma unroll
  for (int h = 0; h < NHH; ++h)
#pragma unroll
    for (int u = 0; u < UH; ++u) accH[h][u] = z4;
#pragma unroll
  for (int u = 0; u < UO; ++u) accO[u] = z4;
  float dbO = 0.0f, db0 = 0.0f, dbH[NHH];
#pragma unroll
  for (int h = 0; h < NHH; ++h) dbH[h] = 0.0f;

  // Zero the layer-0 padding rows [K0, R0) once.
  for (int e = tid; e < (R0 - K0) * kQW; e += blockDim.x) act0[tq_index(K0 + e / kQW, e % kQW)] = from_f32<MT>(0.0f);
  __syncthreads();

  const int64_t n_tiles = (Q + kQW - 1) / kQW;
  const TileRange tr = xcd_tiles(n_tiles, 1, 0);  // neighbouring tiles share an XCD's L2
  for (int64_t tile = tr.first; tile < tr.end; tile += tr.stride) {
    const int64_t qbase = tile * kQW;
    // Lane-derived LDS addresses are loop-invariant; recompute them per tile
    // rather than holding a hundred of them in registers across the loop.
    const int tid = launder_lane(threadIdx.x), lane = tid & 63, g = lane >> 4, r16 = lane & 15;
    const int col = 16 * nt + r16;
    // ---- 1. encode: node indices come from the forward (no second walk of
    //      the tree); kLanesPerQuery lanes per query gather its levels -----
    {
      const int ql = tid / kLanesPerQuery, part = tid % kLanesPerQuery;
      const int64_t q = qbase + ql;
      // octahedral coordinates stored by the forward; clamped so the taps
      // stay inside the map even for a workspace the forward did not fill
      const float2 p = q < Q ? uv[q] : make_float2(0.5f, 0.5f);
      const float s = fminf(fmaxf(p.x, 0.0f), 1.0f), t = fminf(fmaxf(p.y, 0.0f), 1.0f);
      // this lane's levels part, part + kLanesPerQuery, ...: all their
      // gathers in flight
      constexpr int G = kMaxLevels / kLanesPerQuery;
      if constexpr (PAPER) {
        // the eight corner nodes per level come from the forward ([L][8][Q]),
        // the trilinear weights from the stored position
        const float4 xp = q < Q ? A.pos[q] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float xq[3] = {xp.x, xp.y, xp.z};
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
          const int l = part + kLanesPerQuery * gi;
          if (l < L) {
            int node[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) {
              int v = q < Q ? nidx[((int64_t)l * 8 + d) * ldn + q] : -1;
              node[d] = (v < T.off[l] || v >= T.off[l + 1]) ? -1 : v;  // never index outside level l
            }
            int base[3], slot[3];
            float f[3], wc[8], wv[3], h[C];
#pragma unroll
            for (int a = 0; a < 3; ++a) cell_frac(xq[a], l, base[a], f[a]);
            corner_weights(f, node, wc);
            if (A.shift) {  // each corner's cell along its shifted direction
              const float4 w4 = q < Q ? A.wdir[q] : make_float4(0.f, 0.f, 0.f, 0.f);
              const float u[3] = {w4.x, w4.y, w4.z};
              gather_paper_level_shift<TT, C>(T, l, node, wc, xq, base, xp.w, u, h);
            } else {
              bary(s, t, T.res[l], slot, wv);
              gather_paper_level<TT, C>(T, l, node, wc, slot, wv, h);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) act0[tq_index(l * C + c, ql)] = from_f32<MT>(h[c]);
          }
        }
      } else {
        int lidx[G];
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
          const int l = part + kLanesPerQuery * gi;
          int v = (l < L && q < Q) ? nidx[(int64_t)l * ldn + q] : -1;  // nidx is level-major [L][Q]
          if (l < L && (v < T.off[l] || v >= T.off[l + 1])) v = -1;  // never index outside level l
          lidx[gi] = v;
        }
        float h[G][C];
        gather_levels<TT, C, G, kLanesPerQuery>(T, part, lidx, s, t, h);
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
          const int l = part + kLanesPerQuery * gi;
          if (l < L) {
#pragma unroll
            for (int c = 0; c < C; ++c) act0[tq_index(l * C + c, ql)] = from_f32<MT>(h[gi][c]);
          }
        }
      }
      // the decoder's surface attributes, rows L C .. K0 - 1, read in the
      // caller's query order
      if (M.E > 0) {
        int64_t qs = q < Q ? (order ? (int64_t)order[q] : q) : -1;
        const float* gp = (qs < 0 || qs >= A.n_src) ? nullptr : (qs < A.nA ? A.gA + M.E * qs : A.gB + M.E * (qs - A.nA));
        for (int k = 4 * part; k < M.E; k += 4 * kLanesPerQuery)
#pragma unroll
          for (int c = 0; c < 4; ++c) act0[tq_index(LC + k + c, ql)] = from_f32<MT>(gp ? gp[k + c] : 0.0f);
      }
    }
    __syncthreads();

    // ---- 2. forward recompute of the hidden layers ------------------------
    {
      f32x4 acc[MH2];
      const MT* W0 = launder_ptr(reinterpret_cast<const MT*>(M.W[0]));
      const float* b0 = launder_ptr(M.b[0]);
#pragma unroll
      for (int mi = 0; mi < MH2; ++mi)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[mi][j] = b0[16 * (mh * MH2 + mi) + 4 * g + j];
      // per K-chunk, every operand read goes out before the chunk's MFMAs
      // (the scheduler would otherwise wait on each read next to its MFMA)
      for (int kb = 0; kb < KB0; ++kb) {
        const frag b = tq_bfrag<MT>(act0, kb, g, col, K0);
        if constexpr (batch_reads<MT>()) {
          frag a[MH2];
#pragma unroll
          for (int mi = 0; mi < MH2; ++mi) {
            const int m = mh * MH2 + mi;
            a[mi] = WL ? lds_frag<MT>(w0p, KB0, m, kb, lane) : wfrag_global<MT>(W0, H, K0, K0, m, kb, lane);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int mi = 0; mi < MH2; ++mi) acc[mi] = mma(a[mi], b, acc[mi]);
        } else {
#pragma unroll
          for (int mi = 0; mi < MH2; ++mi) {
            const int m = mh * MH2 + mi;
            acc[mi] = mma(WL ? lds_frag<MT>(w0p, KB0, m, kb, lane) : wfrag_global<MT>(W0, H, K0, K0, m, kb, lane), b,
                          acc[mi]);
          }
        }
      }
      store_tq<MT, MH2>(act(1), acc, mh * MH2, MH, H, nt, lane, true);
      for (int layer = 1; layer < NL - 1; ++layer) {
        __syncthreads();  // a_layer complete
        const MT* Wl = launder_ptr(reinterpret_cast<const MT*>(M.W[layer]));
        const float* bl = launder_ptr(M.b[layer]);
        const MT* a = act(layer);
#pragma unroll
        for (int mi = 0; mi < MH2; ++mi)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[mi][j] = bl[16 * (mh * MH2 + mi) + 4 * g + j];
        const MT* Wp = hw + (size_t)2 * (layer - 1) * H * H;
#pragma unroll
        for (int kb = 0; kb < H / 32; ++kb) {
          const frag b = tq_bfrag<MT>(a, kb, g, col, H);
          if constexpr (batch_reads<MT>()) {
            frag wa[MH2];
#pragma unroll
            for (int mi = 0; mi < MH2; ++mi) {
              const int m = mh * MH2 + mi;
              wa[mi] = WL ? lds_frag<MT>(Wp, H / 32, m, kb, lane) : wfrag_global<MT>(Wl, H, H, H, m, kb, lane);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mi = 0; mi < MH2; ++mi) acc[mi] = mma(wa[mi], b, acc[mi]);
          } else {
#pragma unroll
            for (int mi = 0; mi < MH2; ++mi) {
              const int m = mh * MH2 + mi;
              acc[mi] = mma(WL ? lds_frag<MT>(Wp, H / 32, m, kb, lane) : wfrag_global<MT>(Wl, H, H, H, m, kb, lane), b,
                            acc[mi]);
            }
          }
        }
        store_tq<MT, MH2>(act(layer + 1), acc, mh * MH2, MH, H, nt, lane, true);
      }
    }

    // ---- 3. backward ------------------------------------------------------
    if (mh == 0) {  // seeds of the output layer into the seed buffer, rows 0..15
      const int64_t q = qbase + col;
      // seeds are stored in the caller's query order
      int64_t qs = q < Q ? q : -1;
      if (order && qs >= 0) {
        qs = order[q];
        if (qs >= n_seed) qs = -1;
      }
      f32x4 so[1];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 4 * g + j;
        so[0][j] = (row < 3 && qs >= 0) ? seeds[3 * qs + row] : 0.0f;
      }
      store_tq<MT, 1>(seedb, so, 0, 1, 3, nt, lane, false);
    }
    // One layer of the backward: with delta_{i+1} (the gradient at layer i's
    // output) in din(i), dW_i over the workgroup's 64 queries into this
    // wave's accumulators accs, db_i, then delta_i into a_i's buffer (or dh
    // for i = 0).
    // Each call site gets its own accumulator array, and the lane index is
    // re-laundered so addresses are not kept live from one layer to the next.
    auto step = [&](auto& accs, float& dbr, int i) {
      const int ln = launder_lane(lane), gs = ln >> 4, cs = 16 * nt + (ln & 15);
      const int n_out = i == NL - 1 ? 3 : H, n_in = i == 0 ? K0 : H;
      __syncthreads();  // din(i) and the activations are complete
      const MT* dT = din(i);
      dw_layer<MT, NW>(accs, dT, act(i), n_out, n_in, wave, ln);
      if (tid < n_out) {
        float sum = 0.0f;
#pragma unroll
        for (int c = 0; c < kQW / 8; ++c) {
          const auto v = tq_frag<MT>(dT, tid, c);
#pragma unroll
          for (int e = 0; e < 8; ++e) sum += to_f32(v[e]);
        }
        dbr += sum;
      }
      const MT* Wt = launder_ptr(reinterpret_cast<const MT*>(Mt.W[i]));  // [n_in][ldt], ldt = n_out rounded up to 4
      const int ldt = (n_out + 3) & ~3;
      const int KBo = (n_out + 31) / 32;
      if (i > 0) {
        f32x4 dacc[MH2];
#pragma unroll
        for (int mi = 0; mi < MH2; ++mi) dacc[mi] = z4;
        const bool hid = WL && i < NL - 1;  // W_i^T packed in LDS
        const MT* Wp = hw + (size_t)(2 * (i - 1) + 1) * H * H;
        for (int kb = 0; kb < KBo; ++kb) {
          const frag b = tq_bfrag<MT>(dT, kb, gs, cs, n_out);
          if constexpr (batch_reads<MT>()) {
            frag wa[MH2];
#pragma unroll
            for (int mi = 0; mi < MH2; ++mi) {
              const int m = mh * MH2 + mi;
              wa[mi] = hid ? lds_frag<MT>(Wp, H / 32, m, kb, ln) : wfrag_global<MT>(Wt, H, n_out, ldt, m, kb, ln);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mi = 0; mi < MH2; ++mi) dacc[mi] = mma(wa[mi], b, dacc[mi]);
          } else {
#pragma unroll
            for (int mi = 0; mi < MH2; ++mi) {
              const int m = mh * MH2 + mi;
              dacc[mi] = mma(hid ? lds_frag<MT>(Wp, H / 32, m, kb, ln) : wfrag_global<MT>(Wt, H, n_out, ldt, m, kb, ln),
                             b, dacc[mi]);
            }
          }
        }
        // ReLU'(z) = 1 where the layer-i input activation is positive
        const MT* a = act(i);
#pragma unroll
        for (int mi = 0; mi < MH2; ++mi)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int n = 16 * (mh * MH2 + mi) + 4 * gs + j;
            if (!(to_f32(a[tq_index(n, cs)]) > 0.0f)) dacc[mi][j] = 0.0f;
          }
        __syncthreads();  // every wave has read din(i) and a_i
        store_tq<MT, MH2>(act(i), dacc, mh * MH2, MH, H, nt, ln, false);
      } else {
        // dh = W_0^T delta_1 over the level-feature rows only: the surface
        // attributes are inputs, not parameters
        constexpr int MK2 = 8 / kMSplit;  // up to 8 row tiles of dh (L C <= 128)
        const int MK = (LC + 15) / 16;
        f32x4 dacc[MK2];
#pragma unroll
        for (int mi = 0; mi < MK2; ++mi) dacc[mi] = z4;
        for (int kb = 0; kb < KBo; ++kb) {
          const frag b = tq_bfrag<MT>(dT, kb, gs, cs, n_out);
          if constexpr (batch_reads<MT>()) {
            frag wa[MK2];
#pragma unroll
            for (int mi = 0; mi < MK2; ++mi) {
              const int m = mh * MK2 + mi;
              if (m < MK)
                wa[mi] = WL ? lds_frag<MT>(wt0, H / 32, m, kb, ln) : wfrag_global<MT>(Wt, K0, n_out, ldt, m, kb, ln);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mi = 0; mi < MK2; ++mi)
              if (mh * MK2 + mi < MK) dacc[mi] = mma(wa[mi], b, dacc[mi]);
          } else {
#pragma unroll
            for (int mi = 0; mi < MK2; ++mi)
              if (mh * MK2 + mi < MK) {
                const int m = mh * MK2 + mi;
                dacc[mi] = mma(WL ? lds_frag<MT>(wt0, H / 32, m, kb, ln) : wfrag_global<MT>(Wt, K0, n_out, ldt, m, kb, ln),
                               b, dacc[mi]);
              }
          }
        }
        // dh of query column cs, rows 16m + 4g .. +3: one 16-byte store each
        const int64_t q = qbase + cs;
        if (q < Q) {
#pragma unroll
          for (int mi = 0; mi < MK2; ++mi) {
            const int k = 16 * (mh * MK2 + mi) + 4 * gs;
            if (mh * MK2 + mi < MK && k < LC)
              *reinterpret_cast<float4*>(dh_out + q * LC + k) = make_float4(dacc[mi][0], dacc[mi][1], dacc[mi][2], dacc[mi][3]);
          }
        }
      }
    };
    step(accO, dbO, NL - 1);
#pragma unroll
    for (int hh = NHH - 1; hh >= 0; --hh)
      if (hh + 1 < NL - 1) step(accH[hh], dbH[hh], hh + 1);
    step(acc0, db0, 0);
    __syncthreads();  // LDS buffers are reused by the next tile
  }

  // ---- partials ------------------------------------------------------------
  float* part = partials + (int64_t)blockIdx.x * PL.P;
  for (int i = 0; i < NL; ++i) {
    const int n_out = PL.n_out[i], n_in = PL.n_in[i];
    if (i == NL - 1)
      dw_store<NW, UO>(accO, part, PL.w_off[i], n_out, n_in, wave, lane, A.accumulate);
    else if (i == 0)
      dw_store<NW, U0>(acc0, part, PL.w_off[i], n_out, n_in, wave, lane, A.accumulate);
    else {
#pragma unroll
      for (int hh = 0; hh < NHH; ++hh)
        if (hh == i - 1) dw_store<NW, UH>(accH[hh], part, PL.w_off[i], n_out, n_in, wave, lane, A.accumulate);
    }
    float dbv = i == NL - 1 ? dbO : db0;
#pragma unroll
    for (int hh = 0; hh < NHH; ++hh)
      if (i > 0 && i < NL - 1 && hh == i - 1) dbv = dbH[hh];
    if (tid < n_out) {
      float& dst = part[PL.b_off[i] + tid];
      dst = A.accumulate ? dst + dbv : dbv;
    }
  }
}

// Seeds of the backward: LHS point b gets 2 r_b grad_loss (divided by the
// squared detached normaliser for the relative loss); with the gradient
// through the target, secondary query (b, k) gets -seed_b * w_bk / N. The
// 1 / (3B) mean factor is applied later in FP32, so that 16-bit matrix-core
// operands stay far from underflow.
__device__ inline void bsdf_weight_b(const ResidualArgs& A, int64_t b, int k, float w[3]);

__global__ __launch_bounds__(256) void seed_kernel(const ResidualArgs A, const float* __restrict__ resid,
                                                   const float* __restrict__ rhs, const double* __restrict__ grad_loss,
                                                   int full, float* __restrict__ seeds) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.B) return;
  const float gam = (float)(*grad_loss);
  float sd[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float r = resid[3 * b + c];
    float v = 2.0f * r * gam;
    if (A.loss_kind == 1) {
      const float T = rhs[3 * b + c], Lh = r + T;
      const float rho = fmaxf(Lh + T, 0.0f) + A.eps;
      v /= rho * rho;
    }
    sd[c] = v;
    seeds[3 * b + c] = v;
  }
  if (full && A.N > 0) {
    const float invN = 1.0f / (float)A.N;
    for (int k = 0; k < A.N; ++k) {
      float w[3];
      bsdf_weight_b(A, b, k, w);
      const int64_t q = A.B + b * A.N + k;
#pragma unroll
      for (int c = 0; c < 3; ++c) seeds[3 * q + c] = -sd[c] * w[c] * invN;
    }
  }
}

// Wt[i][o] = W[o][i], rows of Wt padded with zeros to ld = n_out rounded up
// to a multiple of 4.
__global__ __launch_bounds__(256) void transpose_kernel(const void* __restrict__ W, void* __restrict__ Wt, int n_out,
                                                        int n_in, int esz) {
  const int ld = (n_out + 3) & ~3;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ld * n_in) return;
  const int i = e / ld, o = e % ld;
  if (esz == 4)
    reinterpret_cast<float*>(Wt)[e] = o < n_out ? reinterpret_cast<const float*>(W)[o * n_in + i] : 0.0f;
  else
    reinterpret_cast<uint16_t*>(Wt)[e] = o < n_out ? reinterpret_cast<const uint16_t*>(W)[o * n_in + i] : (uint16_t)0;
}

// dst[p] += scale * sum over workgroups of partial[g][p], summed in FP64 in
// workgroup order.
__global__ __launch_bounds__(256) void dw_reduce_kernel(const float* __restrict__ partials, int grid, int64_t P,
                                                        const ReduceDst D, float scale) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
#pragma unroll 8
  for (int g = 0; g < grid; ++g) s += (double)partials[(int64_t)g * P + p];
  int seg = 0;
  while (seg + 1 < D.n_seg && p >= D.start[seg + 1]) ++seg;
  D.dst[seg][p - D.start[seg]] += (float)(s * (double)scale);
}

// ---------------------------------------------------------------------------
// BSDF weight of sample (b, k), as the forward residual assembly forms it.
// ---------------------------------------------------------------------------
__device__ inline void bsdf_weight_b(const ResidualArgs& A, int64_t b, int k, float w[3]) {
  const int64_t bk = b * A.N + k;
  float n[3], wo[3], wi[3];
  load_unit(A.n + 3 * b, n);
  load_unit(A.wo + 3 * b, wo);
  load_unit(A.wi + 3 * bk, wi);
  const float alb[3] = {A.albedo[3 * b], A.albedo[3 * b + 1], A.albedo[3 * b + 2]};
  bsdf_weight(n, wo, wi, alb, A.rough[b], A.F0, A.pdf ? A.pdf[bk] : 1.0f, w);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int cu_count() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
  }
  return cus;
}

constexpr size_t kLdsBytes = 160 * 1024;

// LDS of the backward workgroup: the buffers, plus the packed hidden weights
// when both fit.
static size_t bwd_lds_total(int K0, int H, int n_layers, int L, int msz, bool& wl) {
  const size_t base = bwd_layout(K0, H, n_layers, L, msz).total;
  const size_t hwb = lds_weight_bytes(K0, H, n_layers, msz);
  wl = base + hwb <= kLdsBytes;
  return wl ? base + hwb : base;
}

size_t bwd_lds_bytes(const MlpArgs& M, oo_dtype md, int L) {
  bool wl;
  return bwd_lds_total(M.K0, M.H, M.n_layers, L, md == OO_F32 ? 4 : 2, wl);
}

// Persistent grid: as many workgroups as fit on the chip at once (LDS
// bound, 160 KiB per CU on gfx950), so that there is one dW partial per
// resident workgroup.
int bwd_grid(const MlpArgs& M, oo_dtype md, int L, int64_t Q) {
  const int64_t n_tiles = (Q + kQW - 1) / kQW;
  const size_t lds = bwd_lds_bytes(M, md, L);
  int per_cu = (int)(kLdsBytes / (lds ? lds : 1));
  const int by_waves = 16 / (md == OO_F32 ? bwd_waves<float>() : bwd_waves<f16>());  // at most 16 waves per CU
  if (per_cu > by_waves) per_cu = by_waves;
  per_cu = per_cu < 1 ? 1 : per_cu;
  int64_t g = (int64_t)cu_count() * per_cu;
  if (g > n_tiles) g = n_tiles;
  return (int)(g > 0 ? g : 1);
}

hipError_t launch_seeds(const ResidualArgs& A, const float* resid, const float* rhs, const double* grad_loss,
                        int full, float* seeds, hipStream_t st) {
  if (A.B == 0) return hipSuccess;
  hipLaunchKernelGGL(seed_kernel, dim3((unsigned)((A.B + 255) / 256)), dim3(256), 0, st, A, resid, rhs, grad_loss,
                     full, seeds);
  return hipGetLastError();
}

hipError_t launch_transpose_weights(const MlpArgs& M, oo_dtype md, void* const* Wt, hipStream_t st) {
  const int esz = md == OO_F32 ? 4 : 2;
  for (int i = 0; i < M.n_layers; ++i) {
    const int n_in = i == 0 ? M.K0 : M.H, n_out = i == M.n_layers - 1 ? 3 : M.H;
    const int n = n_in * ((n_out + 3) & ~3);
    hipLaunchKernelGGL(transpose_kernel, dim3((n + 255) / 256), dim3(256), 0, st, M.W[i], Wt[i], n_out, n_in, esz);
  }
  return hipGetLastError();
}

template <class TT, class MT, int C, int H>
static hipError_t launch_bwd_t(const TreeArgs& T, const MlpArgs& M, const MlpArgs& Mt, const BwdArgs& A,
                               const ParamLayout& PL, int grid, hipStream_t st) {
  bool wl;
  const size_t lds = bwd_lds_total(M.K0, H, M.n_layers, T.L, (int)sizeof(MT), wl);
  const bool paper = T.interp == OO_INTERP_PAPER;
  constexpr int NH = H == 128 ? 1 : 3;
  auto k = wl ? (paper ? bwd_kernel<TT, MT, C, H, true, true, NH> : bwd_kernel<TT, MT, C, H, true, false, NH>)
              : (paper ? bwd_kernel<TT, MT, C, H, false, true, NH> : bwd_kernel<TT, MT, C, H, false, false, NH>);
  if (H == 128 && M.n_layers > 3)  // four hidden layers: their weights do not fit in LDS
    k = paper ? bwd_kernel<TT, MT, C, H, false, true, 3> : bwd_kernel<TT, MT, C, H, false, false, 3>;
  hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * bwd_waves<MT>()), lds, st, T, M, Mt, A, PL);
  return hipGetLastError();
}

template <class TT, class MT, int C>
static hipError_t launch_bwd_c(const TreeArgs& T, const MlpArgs& M, const MlpArgs& Mt, const BwdArgs& A,
                               const ParamLayout& PL, int grid, hipStream_t st) {
  return M.H == 64 ? launch_bwd_t<TT, MT, C, 64>(T, M, Mt, A, PL, grid, st)
                   : launch_bwd_t<TT, MT, C, 128>(T, M, Mt, A, PL, grid, st);
}

hipError_t launch_bwd(const TreeArgs& T, oo_dtype td, const MlpArgs& M, oo_dtype md, void* const* Wt,
                      const BwdArgs& A, const ParamLayout& PL, int grid, hipStream_t st) {
  if (A.Q == 0) return hipSuccess;
  MlpArgs Mt = M;
  for (int i = 0; i < M.n_layers; ++i) Mt.W[i] = Wt[i];
  if (td == OO_F32)
    return T.C == 4 ? launch_bwd_c<float, float, 4>(T, M, Mt, A, PL, grid, st)
                    : launch_bwd_c<float, float, 8>(T, M, Mt, A, PL, grid, st);
  if (td == OO_F16)
    return T.C == 4 ? launch_bwd_c<f16, f16, 4>(T, M, Mt, A, PL, grid, st) : launch_bwd_c<f16, f16, 8>(T, M, Mt, A, PL, grid, st);
  return T.C == 4 ? launch_bwd_c<bf16, bf16, 4>(T, M, Mt, A, PL, grid, st)
                  : launch_bwd_c<bf16, bf16, 8>(T, M, Mt, A, PL, grid, st);
  (void)md;
}

// Feature-gradient scatter: one lane per (query, tap, channel), level by
// level, queries along the grid, so one atomic instruction of a wave covers
// whole bilinear footprints (4C consecutive lanes per query). The memory-side
// atomic units work on 64-byte chunks, one chunk per instruction and chunk
// touched, so the two taps of a footprint row (2C contiguous floats) mostly
// share one chunk and a 2x2 map (the finest levels) takes two chunks per
// query. This request rate, not bandwidth, bounds the step; privatising
// coarse-level maps in LDS does not pay here, because LDS float atomics
// retire about one lane per clock per CU. Each lane adds
// w_tap * dh[q][l C + c] * post_scale with a hardware FP32 atomic. Node
// indices and octahedral coordinates come from the forward ([L][Q] and [Q]);
// indices are range-checked and coordinates clamped, and the taps are
// recomputed from the coordinates.
template <int C>
__global__ __launch_bounds__(256) void scatter_kernel(const TreeArgs T, int64_t Q, const int32_t* __restrict__ nidx,
                                                      int64_t ldn,
                                                      const float2* __restrict__ uv, const float* __restrict__ dh,
                                                      float post_scale, const GradArgs G) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, n = Q * 4 * C;
  for (int l = 0; l < T.L; ++l) {
    const int R = T.res[l];
    float* const pad = G.pad[l];
    for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < n; gid += stride) {
      const int64_t q = gid / (4 * C);
      const int k = (int)(gid / C) & 3;
      const int c = (int)(gid % C);
      const int id = nidx[(int64_t)l * ldn + q];
      if (id < T.off[l] || id >= T.off[l + 1]) continue;
      const float2 p = uv[q];
      const float s = fminf(fmaxf(p.x, 0.0f), 1.0f), t = fminf(fmaxf(p.y, 0.0f), 1.0f);
      const float gv = dh[q * (int64_t)(T.L * C) + l * C + c] * post_scale;
      const int64_t node = id - T.off[l];
      if (pad) {
        // pair buffer: the tap at unwrapped (i0 + a, j0 + b) goes to slot a
        // of the pair starting at column i0 in unwrapped row j0 + b, so both
        // taps of a footprint row share one 64-byte chunk; i0, j0 in
        // [-1, R - 1] for s, t in [0, 1] (the same arithmetic as tap())
        const float pu = s * (float)R - 0.5f, pv = t * (float)R - 0.5f;
        const float fi = floorf(pu), fj = floorf(pv);
        const float fu = pu - fi, fv = pv - fj;
        const int a = k & 1, b = k >> 1;
        const int i0 = (int)fi, jr = (int)fj + b;
        const float wk = (a ? fu : 1.0f - fu) * (b ? fv : 1.0f - fv);
        const int64_t slot = ((node * (R + 2) + (jr + 1)) * (R + 1) + (i0 + 1)) * 2 + a;
        unsafeAtomicAdd(pad + slot * C + c, wk * gv);
      } else {
        int txk;
        float wk;
        tap(s, t, R, k, txk, wk);
        unsafeAtomicAdd(G.dfeat[l] + (node * R * R + txk) * C + c, wk * gv);
      }
    }
  }
}

// Feature-gradient scatter of the paper's scheme: 8 C lanes per (query,
// level), one per (corner, channel), corner-major. A lane adds
// w_corner * w_vertex * dh[q][l C + c] * post_scale to the three vertices
// its corner's cell reads. The renormalisation needs to know which of the
// query's eight corners exist: one ballot over the wave, read at this
// lane's group of 8 C lanes (all lanes of a group share the query, so they
// run the loop the same number of times). Corner nodes come from the
// forward ([L][8][Q], range-checked), positions and octahedral coordinates
// too; weights are recomputed.
// With the disparity shift (S.wdir set) corner d's vertices and weights
// follow its own direction v = (x - centre) disp + u, and the lane adds its
// share of dLoss/d disparity,
//   w_corner * dh[q][l C + c] * post_scale * sum_k (d w_k / d disp) T[k][c],
// with d w_k / d disp = R (dw_k/dpu ds + dw_k/dpv dt), (ds, dt) = J_octa(v)
// (x - centre); the 8 C lanes of a (query, level) are summed over the wave
// before one atomic add into dd[q].
template <class TT, int C>
__global__ __launch_bounds__(256) void scatter_paper_kernel(const TreeArgs T, int64_t Q,
                                                            const int32_t* __restrict__ nidx, int64_t ldn,
                                                            const float2* __restrict__ uv,
                                                            const float4* __restrict__ pos,
                                                            const float* __restrict__ dh, float post_scale,
                                                            const GradArgs G, const ShiftArgs S) {
  constexpr int U = 8 * C;
  static_assert(64 % U == 0, "a lane group must not straddle waves");
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, n = Q * U;
  const int gbase = (int)(threadIdx.x & 63) / U * U;
  for (int l = 0; l < T.L; ++l) {
    const int R = T.res[l];
    const int64_t E = (int64_t)(R + 1) * (R + 1);
    float* const dst = G.dfeat[l];
    for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < n; gid += stride) {
      const int64_t q = gid / U;
      const int d = (int)(gid / C) & 7;
      const int c = (int)(gid % C);
      const int id = nidx[((int64_t)l * 8 + d) * ldn + q];
      const bool ok = id >= T.off[l] && id < T.off[l + 1];
      const uint64_t gb = __ballot(ok) >> gbase;
      int node[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) node[e] = ((gb >> (e * C)) & 1u) ? 0 : -1;
      const float4 xp = pos[q];
      const float xq[3] = {xp.x, xp.y, xp.z};
      int base[3], slot[3];
      float f[3], wc[8], wv[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) cell_frac(xq[a], l, base[a], f[a]);
      corner_weights(f, node, wc);
      const float gv = dh[q * (int64_t)(T.L * C) + l * C + c] * post_scale * pick8(wc, d);
      const int64_t nb = ok ? ((int64_t)id - T.off[l]) * E : 0;
      if (S.wdir) {
        const float4 w4 = S.wdir[q];
        const float u[3] = {w4.x, w4.y, w4.z};
        float v[3], dv[3], s, t, J[2][3], gu[3], gvv[3];
        shifted_dir(xq, l, base, d, xp.w, u, v, dv);
        octa(v, s, t);
        octa_jacobian(v, J);
        bary_t<true>(s, t, R, slot, wv, gu, gvv);
        const float ds = J[0][0] * dv[0] + J[0][1] * dv[1] + J[0][2] * dv[2];
        const float dt = J[1][0] * dv[0] + J[1][1] * dv[1] + J[1][2] * dv[2];
        float contrib = 0.0f;
        if (ok) {
          const TT* tab = reinterpret_cast<const TT*>(T.feat[l]);
#pragma unroll
          for (int k = 0; k < 3; ++k)
            contrib += (float)R * (gu[k] * ds + gvv[k] * dt) * to_f32(tab[(nb + slot[k]) * C + c]);
          contrib *= gv;
        }
        // the group's 8 C lanes share (q, l): sum them, one add per group
#pragma unroll
        for (int off = U / 2; off >= 1; off >>= 1) contrib += __shfl_xor(contrib, off);
        if ((gid % U) == 0 && contrib != 0.0f) unsafeAtomicAdd(S.dd + q, contrib);
      } else {
        const float2 p = uv[q];
        bary(fminf(fmaxf(p.x, 0.0f), 1.0f), fminf(fmaxf(p.y, 0.0f), 1.0f), R, slot, wv);
      }
      if (!ok) continue;
#pragma unroll
      for (int k = 0; k < 3; ++k) unsafeAtomicAdd(dst + (nb + slot[k]) * C + c, wv[k] * gv);
    }
  }
}

template <class TT>
static void launch_scatter_paper(const TreeArgs& T, int64_t Q, const int32_t* nidx, int64_t ldn, const float2* uv,
                                 const float4* pos, const float* dh, float post_scale, const GradArgs& G,
                                 const ShiftArgs& S, hipStream_t st) {
  int64_t blocks = (Q * 8 * T.C + 255) / 256;
  if (blocks > 256 * 16) blocks = 256 * 16;
  if (T.C == 4)
    hipLaunchKernelGGL((scatter_paper_kernel<TT, 4>), dim3((unsigned)blocks), dim3(256), 0, st, T, Q, nidx, ldn, uv,
                       pos, dh, post_scale, G, S);
  else
    hipLaunchKernelGGL((scatter_paper_kernel<TT, 8>), dim3((unsigned)blocks), dim3(256), 0, st, T, Q, nidx, ldn, uv,
                       pos, dh, post_scale, G, S);
}

hipError_t launch_scatter(const TreeArgs& T, oo_dtype td, int64_t Q, const int32_t* nidx, int64_t ldn,
                          const float2* uv, const float4* pos, const float* dh, float post_scale, const GradArgs& G,
                          const ShiftArgs& S, hipStream_t st) {
  if (Q == 0) return hipSuccess;
  if (T.interp == OO_INTERP_PAPER) {
    if (td == OO_F32)
      launch_scatter_paper<float>(T, Q, nidx, ldn, uv, pos, dh, post_scale, G, S, st);
    else if (td == OO_F16)
      launch_scatter_paper<f16>(T, Q, nidx, ldn, uv, pos, dh, post_scale, G, S, st);
    else
      launch_scatter_paper<bf16>(T, Q, nidx, ldn, uv, pos, dh, post_scale, G, S, st);
    return hipGetLastError();
  }
  // a persistent grid walks every level: block scheduling stays out of the
  // way of the atomic stream
  int64_t blocks = (Q * 4 * T.C + 255) / 256;
  if (blocks > 256 * 16) blocks = 256 * 16;
  if (T.C == 4)
    hipLaunchKernelGGL(scatter_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, T, Q, nidx, ldn, uv, dh, post_scale,
                       G);
  else
    hipLaunchKernelGGL(scatter_kernel<8>, dim3((unsigned)blocks), dim3(256), 0, st, T, Q, nidx, ldn, uv, dh, post_scale,
                       G);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * i + 3 < n)
    reinterpret_cast<float4*>(p)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  else
    for (int64_t e = 4 * i; e < n; ++e) p[e] = 0.0f;
}

// Moves level l's pair-buffer sums into its feature gradient: the unwrapped
// texel (ii, jj), ii and jj in [-1, R], collects slot 0 of the pair starting
// at ii and slot 1 of the pair starting at ii - 1, and lands on the texel
// the seam wrap of tap() maps it to (several unwrapped texels of the border
// land on one texel, hence the atomic add).
template <int C>
__global__ __launch_bounds__(256) void pad_fold_kernel(const TreeArgs T, const GradArgs G, int l, int64_t nodes) {
  const int R = T.res[l];
  const int64_t n = nodes * (R + 2) * (R + 2) * C;
  const float* __restrict__ pad = G.pad[l];
  float* __restrict__ dst = G.dfeat[l];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < n; gid += stride) {
    const int c = (int)(gid % C);
    int64_t r = gid / C;
    const int ii = (int)(r % (R + 2)) - 1;
    r /= R + 2;
    const int jj = (int)(r % (R + 2)) - 1;
    const int64_t node = r / (R + 2);
    const int64_t row = (node * (R + 2) + (jj + 1)) * (R + 1);
    float v = 0.0f;
    if (ii <= R - 1) v += pad[((row + (ii + 1)) * 2 + 0) * C + c];
    if (ii >= 0) v += pad[((row + ii) * 2 + 1) * C + c];
    if (v == 0.0f) continue;
    int i = ii, j = jj;
    if ((unsigned)i >= (unsigned)R) j = R - 1 - j;
    i = min(max(i, 0), R - 1);
    if ((unsigned)j >= (unsigned)R) i = R - 1 - i;
    j = min(max(j, 0), R - 1);
    unsafeAtomicAdd(dst + ((node * R + j) * R + i) * C + c, v);
  }
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = ((n + 3) / 4 + 255) / 256;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_pad_fold(const TreeArgs& T, const GradArgs& G, hipStream_t st) {
  for (int l = 0; l < T.L; ++l) {
    if (!G.pad[l]) continue;
    const int R = T.res[l];
    const int64_t nodes = (int64_t)T.off[l + 1] - T.off[l];
    const int64_t n = nodes * (R + 2) * (R + 2) * T.C;
    if (n == 0) continue;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 16) blocks = 256 * 16;
    if (T.C == 4)
      hipLaunchKernelGGL(pad_fold_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, T, G, l, nodes);
    else
      hipLaunchKernelGGL(pad_fold_kernel<8>, dim3((unsigned)blocks), dim3(256), 0, st, T, G, l, nodes);
  }
  return hipGetLastError();
}

// FP64 inner products of FP32 arrays in a fixed order: block k of group g
// sums elements k * 256 + t + (256 * kDotBlocks) j (thread t, j = 0, 1, ...)
// into per-thread FP64 accumulators, reduces them in a fixed tree and writes
// partial [g][k]; dot_final sums the kDotBlocks partials of a group in a
// fixed tree. b[g] == NULL squares a[g].
__global__ __launch_bounds__(256) void dot_partial_kernel(const DotArgs D, double* __restrict__ partials) {
  __shared__ double red[256];
  const int g = blockIdx.y;
  const float* __restrict__ a = D.a[g];
  const float* __restrict__ b = D.b[g] ? D.b[g] : D.a[g];
  const int64_t n = D.n[g], stride = (int64_t)256 * kDotBlocks;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) acc += (double)a[i] * (double)b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[(int64_t)g * kDotBlocks + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void dot_final_kernel(const double* __restrict__ partials, double* __restrict__ out) {
  __shared__ double red[256];
  const int g = blockIdx.x;
  double acc = 0.0;
  for (int k = threadIdx.x; k < kDotBlocks; k += 256) acc += partials[(int64_t)g * kDotBlocks + k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[g] = red[0];
}

// Partial sums of the allocation-free inner-product entry point: one
// kDotGroups x kDotBlocks array of doubles (128 KiB) per device, held until
// the process ends. Host code never passes `scratch` itself to a kernel: its
// name on the host is a stand-in, not a device address. dot_scratch looks up
// the current device's copy once (hipGetSymbolAddress, with that device
// current) and hands out that address.
static __device__ __align__(256) double scratch[kDotGroups * kDotBlocks];

hipError_t dot_scratch(double** partials) {
  static std::mutex m;
  static double* ptr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(m);
  if (!ptr[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    ptr[dev] = static_cast<double*>(p);
  }
  *partials = ptr[dev];
  return hipSuccess;
}

hipError_t launch_dot(const DotArgs& D, int n_groups, double* partials, double* out, hipStream_t st) {
  if (n_groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks, n_groups), dim3(256), 0, st, D, partials);
  hipLaunchKernelGGL(dot_final_kernel, dim3(n_groups), dim3(256), 0, st, partials, out);
  return hipGetLastError();
}

hipError_t launch_dw_reduce(const float* partials, int grid, const ParamLayout& PL, const ReduceDst& D, float scale,
                            hipStream_t st) {
  const int64_t blocks = (PL.P + 255) / 256;
  hipLaunchKernelGGL(dw_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, partials, grid, PL.P, D, scale);
  return hipGetLastError();
}

}  // namespace oo
