/*
 * FP64 CPU oracle for the OctaOctree query and the neural-radiosity residual
 * step (OctaOctree Neural Radiosity, Sec. 3.2-3.6).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the HIP library
 * against a plain, slow, obviously correct implementation. Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no source, header, table or helper with the HIP library.
 *
 * Conventions
 *  - Every FP32 input is widened exactly to double; all arithmetic is FP64.
 *  - Feature tables are the FP32 master copies, laid out per level as
 *    [n_l][R_l][R_l][C] texels (row = t direction, column = s direction),
 *    or with ORA_INTERP_PAPER as [n_l][R_l + 1][R_l + 1][C] map vertices.
 *  - Node words: (first_child << 8) | child_mask, first_child a global node
 *    index, child octant o = bx | by << 1 | bz << 2. Leaves hold 0.
 *  - Levels 0..D; level 0 is the root.
 *  - Functions that can fail return 0 on success, a negative code otherwise.
 *
 * Parity status per function is listed in the comment above each one.
 */
#ifndef OCTAOCTREE_ORACLE_H
#define OCTAOCTREE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAX_LEVELS 16
#define ORA_MAX_LAYERS 7

/* Interpolation schemes of a level feature. */
#define ORA_INTERP_NODE_BILINEAR 0  /* containing node, bilinear on R x R texels */
#define ORA_INTERP_PAPER 1          /* 8 neighbouring cells (trilinear,
                                       renormalised over non-empty cells),
                                       barycentric on (R+1)^2 vertices */

/* The decoder reads [h, g]: the L*C level features, then E = dims[0] - L*C
 * per-query surface attributes g (Sec. 3.5: position, mirror direction,
 * normal, albedo, roughness; E = 0 reads h only). */
typedef struct {
  int32_t n_layers;                          /* number of Linear layers */
  int32_t dims[ORA_MAX_LAYERS + 1];          /* dims[0] = L*C + E, dims[n_layers] = 3 */
  const float* W[ORA_MAX_LAYERS];            /* [dims[i+1]][dims[i]] row-major */
  const float* b[ORA_MAX_LAYERS];            /* [dims[i+1]] */
} ora_mlp;

/* The disparity predictor g_psi (Sec. 3.3 disparity equation, Sec. 3.5): a
 * multi-resolution hash encoding of x (Instant-NGP style) followed by a
 * small MLP on [encoding, unit w_r, 0] with one linear output, d.
 *  - Level i has N_i cells per side (Instant-NGP's geometric series
 *    floor(N_0 b^i), evaluated by the caller). Its eight grid vertices
 *    around x N_i (x clamped to the cube; the last cell is closed) are read
 *    with the trilinear weights of x N_i's fraction in the cell.
 *  - Level i's table has 2^log2_T entries of F features. Vertex (a, b, c)
 *    is entry a + (N_i + 1) (b + (N_i + 1) c) when (N_i + 1)^3 <= 2^log2_T,
 *    else the spatial hash (a * 1) xor (b * 2654435761) xor (c * 805459861)
 *    in 32-bit arithmetic, modulo 2^log2_T.
 *  - mlp.dims[0] = n_levels F + 4, mlp.dims[mlp.n_layers] = 1. */
#define ORA_HASH_MAX_LEVELS 16
#define ORA_HASH_MAX_F 8
typedef struct {
  int32_t n_levels;                          /* hash-grid levels, <= ORA_HASH_MAX_LEVELS */
  int32_t F;                                 /* features per entry */
  int32_t log2_T;                            /* entries per level = 2^log2_T */
  int32_t res[ORA_HASH_MAX_LEVELS];          /* N_i cells per side */
  const float* tables;                       /* [n_levels][2^log2_T][F] */
  ora_mlp mlp;
} ora_disparity;

typedef struct {
  int32_t n_levels;                          /* L = D + 1 */
  int32_t C;                                 /* features per texel */
  int32_t res[ORA_MAX_LEVELS];               /* R_l texels (cells) per side */
  int64_t level_offset[ORA_MAX_LEVELS + 1];  /* level l = [off_l, off_{l+1}) */
  const uint32_t* nodes;
  const float* feat[ORA_MAX_LEVELS];         /* FP32 masters */
  int32_t interp;                            /* ORA_INTERP_* */
  /* ORA_INTERP_PAPER only: the disparity predictor, or NULL for none (the
   * "no direction offset" lookup along w_r). With it, neighbouring cell j
   * of a level (centre c_j) is read along v_j = (x - c_j) d + w_r / |w_r|
   * (Sec. 3.3, shifted-direction equation, second form), where d is the
   * query's predicted disparity and w_r its lookup direction. */
  const ora_disparity* disp;
} ora_tree;

typedef struct {
  int64_t B;
  int32_t N;
  const float *x, *dir, *n, *wo, *albedo, *Le; /* [B][3] */
  const float* rough;                          /* [B] GGX alpha */
  const float *x2, *dir2, *wi;                 /* [B][N][3] */
  const float* pdf;                            /* [B][N] or NULL (== 1) */
  const float* target_override;                /* [B][3] or NULL */
  double F0;
  int32_t loss_kind;                           /* 0 mean L2, 1 relative L2 */
  double eps;
  int32_t grad_through_rhs;                    /* 0 detached target, 1 full */
  const float* attr;                           /* [B][E] decoder attributes of the LHS queries */
  const float* attr2;                          /* [B][N][E] those of the secondary queries */
} ora_batch;

/* Octree construction from surface samples (refinement rule: a node at level
 * l < D holding more than tau samples gets its non-empty children). */
int ora_build_octree(const float* samples, int64_t n, int32_t D, int32_t tau,
                     uint32_t* nodes_out, int64_t capacity,
                     int64_t* level_offset_out, int64_t* n_nodes_out);

/* Integer cell coordinates of x at the finest level D, clamped. [B][3]. */
void ora_quantize(const float* x, int64_t B, int32_t D, int64_t* q_out);

/* Node containing x at every level, -1 where the tree has no node. [B][L]. */
void ora_descend(const ora_tree* t, const float* x, int64_t B, int32_t* idx_out);

/* Octahedral projection and fold (Sec. 3.3), remapped to [0,1]^2. [B][2]. */
void ora_octa(const float* dir, int64_t B, double* st_out);

/* Inverse of ora_octa: unit direction for a map coordinate. [B][3]. */
void ora_octa_decode(const double* st, int64_t B, double* dir_out);

/* Four bilinear taps at resolution R: texel (i, j) pairs [B][4][2] and
 * weights [B][4]. */
void ora_taps(const double* st, int64_t B, int32_t R, int32_t* ij_out, double* w_out);

/* Entries of one node's map: R^2 texels, or (R + 1)^2 vertices with
 * ORA_INTERP_PAPER. */
int64_t ora_map_entries(int32_t R, int32_t interp);

/* Barycentric vertex lookup (Sec. 3.3) at map resolution R (cells per side):
 * the three vertices (i, j) of the triangle holding (s, t), as found on the
 * unfolded grid [B][3][2], their weights [B][3], and each vertex's
 * canonical storage index j * (R + 1) + i after the seam identification
 * [B][3]. */
void ora_bary(const double* st, int64_t B, int32_t R, int32_t* ij_out, double* w_out, int32_t* vidx_out);

/* The eight octree cells around x at level l (Sec. 3.4): global node index
 * of each (-1 where the cell is empty or outside the cube) [B][8], integer
 * cell coordinates [B][8][3], and trilinear weights renormalised over the
 * non-empty cells [B][8] (all zero when every cell is empty). Corner
 * d = dx | dy << 1 | dz << 2. */
void ora_neighbours(const ora_tree* t, const float* x, int64_t B, int32_t l, int32_t* idx_out,
                    int64_t* cell_out, double* w_out);

/* Concatenated per-level features h [B][L*C] and node indices [B][L]
 * (idx_out may be NULL; the containing node per level in both schemes). */
void ora_encode(const ora_tree* t, const float* x, const float* dir, int64_t B,
                double* h_out, int32_t* idx_out);

/* Hash encoding of x [B][n_levels F], with each level's eight vertex
 * entries [B][n_levels][8] and trilinear weights [B][n_levels][8] (either
 * output may be NULL). Vertex d = dx | dy << 1 | dz << 2. */
void ora_hash_encode(const ora_disparity* g, const float* x, int64_t B, double* enc_out, int64_t* idx_out,
                     double* w_out);

/* Predicted disparity d(x, w_r) of each query [B]. */
void ora_disparity_fwd(const ora_disparity* g, const float* x, const float* dir, int64_t B, double* d_out);

/* Decoder MLP on FP64 inputs h [B][dims[0]] -> out [B][dims[n_layers]]. */
void ora_mlp_fwd(const ora_mlp* m, const double* h, int64_t B, double* out);

/* Encode + MLP, queries processed in parallel over nthreads (<= 0: all).
 * attr: [B][E] decoder attributes appended after h (NULL when E = 0). */
void ora_query_fwd(const ora_tree* t, const ora_mlp* m, const float* x, const float* dir, const float* attr,
                   int64_t B, double* rgb_out, int32_t nthreads);

/* BSDF sample weight f_r * |n . wi| / pdf for every (b, k): [B][N][3]. */
void ora_bsdf_weight(const ora_batch* bt, double* w_out);

/* Residual forward: LHS radiance, RHS target, residual [B][3] and loss. */
int ora_residual_fwd(const ora_tree* t, const ora_mlp* m, const ora_batch* bt,
                     double* lhs_out, double* rhs_out, double* resid_out, double* loss_out,
                     int32_t nthreads);

/* Residual backward for upstream gradient grad_loss. Gradients accumulate
 * (+=) into dfeat[l] ([n_l][R_l][R_l][C]), dW[i], db[i], all FP64. With a
 * disparity predictor (t->disp) its gradients accumulate into dtables
 * ([n_levels][2^log2_T][F]), gdW[i] and gdb[i]; these may be NULL
 * otherwise. dd_out (may be NULL): dL/d disparity of each backward query
 * (the LHS queries, then with grad_through_rhs the secondary ones). */
int ora_residual_bwd(const ora_tree* t, const ora_mlp* m, const ora_batch* bt, double grad_loss,
                     double* const* dfeat, double* const* dW, double* const* db,
                     double* dtables, double* const* gdW, double* const* gdb, double* dd_out,
                     int32_t nthreads);

/* One Adam step (Kingma and Ba, Algorithm 1) over n FP32 parameters with
 * FP32 moments, all updated in place after widening to FP64:
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * With `touched` set, the array is split into blocks of `block` entries and
 * only blocks whose flag is non-zero are updated (a node's map that no query
 * of the batch read keeps its parameters and moments); touched == NULL
 * updates every entry. Results are rounded back to FP32 (p, m, v). */
void ora_adam(float* p, const float* g, float* m, float* v, int64_t n, const uint32_t* touched, int64_t block,
              int32_t t, double lr, double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
