// Launchers shared between the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "octaoctree.h"
#include "oo_device.h"

namespace oo {

// Residual inputs as the kernels read them.
struct ResidualArgs {
  int64_t B;
  int32_t N;
  const float *n, *wo, *albedo, *Le, *rough, *wi, *pdf, *target_override;
  float F0;
  int32_t loss_kind;
  float eps;
};

// Feature-gradient targets. pad[l], when set, is the level's pair buffer:
// the scatter adds level l's taps there at their unwrapped positions and
// pad_fold moves the sums into dfeat[l] (see scatter_kernel).
struct GradArgs {
  float* dfeat[kMaxLevels];
  float* pad[kMaxLevels];
};

// Floats of a level's pair buffer: per node, R + 2 rows (unwrapped rows -1
// .. R) of R + 1 pairs (pairs starting at columns -1 .. R - 1) of two texels
// of C channels.
inline int64_t pad_floats(int R, int64_t nodes, int C) { return nodes * (R + 2) * (R + 1) * 2 * C; }

// Flat parameter layout of the dW/db partials: layer i's W block at
// w_off[i] (n_out x n_in), its b block at b_off[i].
struct ParamLayout {
  int32_t n_layers;
  int32_t n_in[kMaxLayers], n_out[kMaxLayers];
  int64_t w_off[kMaxLayers], b_off[kMaxLayers];
  int64_t P;
};

struct ReduceDst {
  int32_t n_seg;
  int64_t start[2 * kMaxLayers + 1];
  float* dst[2 * kMaxLayers];
};

hipError_t launch_encode(const TreeArgs& T, oo_dtype td, const float* x, const float* d, int64_t B, void* h,
                         oo_dtype hd, int32_t* idx, const DispArgs& G, hipStream_t st);
hipError_t launch_mlp(const MlpArgs& M, oo_dtype md, const void* h, int64_t Q, float* rgb, hipStream_t st);
// Queries q < n_idx also store their node index per level (idx_out,
// [L][n_idx]; the paper's scheme: the eight corner nodes, [L][8][n_idx], and
// the position, pos_out [n_idx]) and octahedral coordinates (uv_out,
// [n_idx]).
// With the disparity predictor (G.n_levels > 0; the paper's scheme only)
// the fused kernel predicts each query's disparity, stores it in pos_out's
// w and the unit lookup direction in wdir_out ([n_idx]).
struct QueryOut {
  int32_t* idx;
  float2* uv;
  float4* pos;
  float4* wdir;
  int64_t n_idx;
  const float* disp = nullptr;  // per-query disparity, read by the shifted encode into rows
};
// The predictor's d for Q queries (matrix cores), into d_out [Q]: FP32 for
// an FP32 model, split BF16 operands (hi + lo) for a 16-bit one.
hipError_t launch_disparity_fwd(const DispArgs& G, oo_dtype md, const QuerySrc& src, int64_t Q, float* d_out,
                                hipStream_t st);
// The shifted encode of the Q sorted queries (disparity from O.disp) into
// decoder input rows h_rows [Q][M.K0] of the tables' dtype (level features,
// then the M.E surface attributes), with the backward's outputs in O.
hipError_t launch_encode_rows(const TreeArgs& T, oo_dtype td, const MlpArgs& M, const QuerySrc& src, int64_t Q,
                              void* h_rows, const QueryOut& O, hipStream_t st);
hipError_t launch_query(const TreeArgs& T, oo_dtype td, const MlpArgs& M, oo_dtype md, const QuerySrc& src,
                        int64_t Q, float* rgb, const QueryOut& O, const DispArgs& G, hipStream_t st);

// Spatial bucketing of the residual queries: NB chunks, K buckets (octree
// cell level c). Workspace: counts [NB][K], total [K], start [K] int32;
// outputs order [Q] (source query of each sorted position) and rank [Q]
// (sorted position of each source query).
struct SortShape {
  int c, K, NB;
  int64_t chunk;
};
SortShape sort_shape(int64_t Q, int D);
hipError_t launch_spatial_sort(const QuerySrc& src, int64_t Q, int64_t n_lhs, int D, int32_t* counts, int32_t* total,
                               int32_t* start, int32_t* order, int32_t* rank, hipStream_t st);
int combine_blocks(int64_t B, int N);
// Lq row of query q is rank[q] when rank is set, else q.
hipError_t launch_combine(const ResidualArgs& A, const float* Lq, const int32_t* rank, float* lhs, float* rhs,
                          float* resid, double* partials, double* loss, hipStream_t st);
hipError_t launch_cast(const float* src, void* dst, oo_dtype dt, int64_t n, hipStream_t st);
hipError_t launch_saved_nodes(const int32_t* nidx, const int32_t* order, int64_t Qb, int L, int K, int32_t* out,
                              hipStream_t st);

// Backward.
int bwd_grid(const MlpArgs& M, oo_dtype md, int L, int64_t Q);
size_t bwd_lds_bytes(const MlpArgs& M, oo_dtype md, int L);
hipError_t launch_seeds(const ResidualArgs& A, const float* resid, const float* rhs, const double* grad_loss,
                        int full, float* seeds, hipStream_t st);
hipError_t launch_transpose_weights(const MlpArgs& M, oo_dtype md, void* const* Wt, hipStream_t st);
// One backward launch over Q consecutive sorted positions: node indices
// nidx[l * ldn + q], coordinates uv[q], order[q] (source query, whose seed
// row is read if it is below n_seed), dh[q][K0] out, one dW/db partial per
// workgroup into partials [grid][P] (added to what is there when
// accumulate is set).
struct BwdArgs {
  int64_t Q;
  const int32_t* nidx;  // [L][ldn], or [L][8][ldn] in the paper's scheme
  int64_t ldn;
  const float2* uv;
  const float4* pos;    // the paper's scheme: query positions, [Q]
  const float* seeds;
  const int32_t* order;
  int64_t n_seed;
  float* partials;
  float* dh;            // [Q][L C]: dLoss/dh of the level features
  int accumulate;
  // the decoder's surface attributes in the caller's query order: [nA][E]
  // for the first nA queries, [n_src - nA][E] for the rest
  const float* gA = nullptr;
  const float* gB = nullptr;
  int64_t nA = 0, n_src = 0;
  // the disparity shift: unit lookup directions [Q] (the disparity is in
  // pos[q].w)
  const float4* wdir = nullptr;
  int shift = 0;
};
hipError_t launch_bwd(const TreeArgs& T, oo_dtype td, const MlpArgs& M, oo_dtype md, void* const* Wt,
                      const BwdArgs& A, const ParamLayout& PL, int grid, hipStream_t st);
// Feature-gradient scatter. With the disparity shift (wdir set; the
// paper's scheme) it also adds each query's dLoss/d disparity into dd[q]
// (dd cleared by the caller), reading the tables (feat, type td) it
// differentiates through.
struct ShiftArgs {
  const float4* wdir = nullptr;
  float* dd = nullptr;
};
hipError_t launch_scatter(const TreeArgs& T, oo_dtype td, int64_t Q, const int32_t* nidx, int64_t ldn,
                          const float2* uv, const float4* pos, const float* dh, float post_scale, const GradArgs& G,
                          const ShiftArgs& S, hipStream_t st);
// Disparity predictor backward over the Q sorted backward queries (x, dir
// from src; dd[q] = dLoss/d disparity), at most `cap` queries per pass
// through the row buffer `rows` (disparity_rows_floats(cap) floats):
// hash-table gradients added into dtables, MLP parameter sums per
// workgroup into partials [grid][P] with P = disparity_params(G) (flat W_0,
// b_0, (W_1, b_1,) W_out, b_out).
constexpr int64_t kDispRowsMax = 262144;
int disparity_bwd_grid(int64_t Q);
int64_t disparity_rows_cap(int64_t Q);
int64_t disparity_rows_floats(int64_t cap);
int32_t disparity_params(const DispArgs& G);
hipError_t launch_disparity_bwd(const DispArgs& G, const QuerySrc& src, int64_t Q, const float* dd, float* dtables,
                                float* rows, int64_t cap, float* partials, int grid, hipStream_t st);
hipError_t launch_dw_reduce(const float* partials, int grid, const ParamLayout& PL, const ReduceDst& D, float scale,
                            hipStream_t st);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t st);

// FP64 inner products of up to kDotGroups pairs of FP32 arrays (b == NULL:
// a . a). partials: [n_groups][kDotBlocks] doubles.
constexpr int kDotGroups = OO_DOT_MAX_GROUPS;
constexpr int kDotBlocks = OO_DOT_BLOCKS;
struct DotArgs {
  const float* a[kDotGroups];
  const float* b[kDotGroups];
  int64_t n[kDotGroups];
};
hipError_t launch_dot(const DotArgs& D, int n_groups, double* partials, double* out, hipStream_t st);
// Device address of the current device's library-owned partials array
// ([kDotGroups][kDotBlocks] doubles), looked up on first use per device.
constexpr int kMaxDevices = 64;
hipError_t dot_scratch(double** partials);
hipError_t launch_pad_fold(const TreeArgs& T, const GradArgs& G, hipStream_t st);

// Optimiser step: segments and the thread range each owns (4 elements per
// thread), hyper-parameters with the bias corrections folded in.
struct AdamSeg {
  float *param, *grad, *m, *v;
  void* work;
  int64_t n;
  const uint32_t* touched;
  int64_t block;
  int vec;  // every array aligned for one vector of 4 elements per thread
};
struct AdamArgs {
  int32_t n_segs;
  AdamSeg seg[OO_ADAM_MAX_SEGMENTS];
  int64_t first[OO_ADAM_MAX_SEGMENTS + 1];
  float lr, b1, b2, eps, inv_c1, inv_c2;
};
hipError_t launch_adam(const AdamArgs& A, oo_dtype work_dtype, hipStream_t st);
hipError_t launch_touched(const int32_t* nidx, int64_t n, int64_t rows, int64_t n_nodes, uint32_t* touched,
                          hipStream_t st);

}  // namespace oo
