/*
 * liboctaoctree: the OctaOctree query and neural-radiosity residual step on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: OctaOctree Neural Radiosity for Real-time Glossy Material Rendering.
 *  - Sec. 3.3: a direction is projected onto the octahedron, its lower
 *    hemisphere folded, and the result remapped to [0,1]^2.
 *  - Sec. 3.4: an adaptive octree over the scene; every non-empty cell at
 *    every level holds a C-channel octahedral feature map; the per-level
 *    features are concatenated into h (dimension levels * C).
 *  - Sec. 3.5: a small MLP decodes h into RGB radiance.
 *  - Sec. 3.2: the residual step compares the prediction at (x, w_o) with a
 *    Monte-Carlo estimate of the rendering equation's right-hand side built
 *    from predictions at secondary hits.
 *  - Sec. 3.6: the target is detached from the gradient.
 *
 * Two interpolation schemes per level (oo_tree.interp):
 *  - OO_INTERP_NODE_BILINEAR: each level reads the node that contains x
 *    (the paper's "no octree interpolation" variant, Sec. 4.4). Each map
 *    has R x R texels, read by a bilinear fetch at texel centres. The
 *    octahedral seams are glued: the edges s = 0 and s = 1 each meet
 *    themselves with t mirrored, and the edges t = 0 and t = 1 with s
 *    mirrored.
 *  - OO_INTERP_PAPER: the paper's own scheme. The eight octree cells whose
 *    centres surround x are weighted trilinearly, renormalised over the
 *    cells that exist (Sec. 3.4, level-feature equation). Each is read by
 *    the barycentric lookup of Sec. 3.3 on a map of (R+1) x (R+1)
 *    vertices. Every grid cell of the map is split along the diagonal
 *    parallel to its quadrant's equator segment, so triangles follow the
 *    octahedron's faces. Border vertices that are one direction share one
 *    slot (the lower index along the edge; the four corners use slot 0).
 *    Without a disparity predictor (oo_tree.disparity = NULL) all eight
 *    cells use the lookup direction; with one, each cell is read along
 *    its own disparity-shifted direction (oo_disparity below).
 *  - The decoder reads h, followed by the query's surface attributes when
 *    its input is wider than h (oo_mlp, oo_residual_batch).
 *  - The BSDF is Lambert plus GGX.
 *
 * Conventions for every entry point:
 *  - Return value: OO_OK (0) or a negative status. oo_last_error() holds a
 *    message for the calling thread.
 *  - Array pointers are DEVICE pointers owned by the caller unless marked
 *    "host". The library allocates no device memory. Scratch memory comes
 *    from a caller-provided workspace, except for oo_dot_f64_noalloc, whose
 *    partial sums sit in a fixed 128 KiB device array of the library's code
 *    object.
 *  - Device work is enqueued asynchronously on the given hipStream_t (NULL
 *    is the default stream). Device faults surface at the caller's next
 *    synchronisation. oo_build_octree runs on the host and is synchronous.
 *  - B = 0 (no queries) is a valid no-op.
 *  - Gradient outputs accumulate (+=). The caller zeroes them.
 *  - Inputs are FP32 unless a dtype field says otherwise. FP32 arrays need
 *    4-byte alignment. Feature tables need 16-byte alignment.
 *  - Points are expected in the unit cube. Coordinates outside it are
 *    clamped to the boundary cells. NaN inputs give unspecified results.
 */
#ifndef OCTAOCTREE_H
#define OCTAOCTREE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OO_MAX_LEVELS 16
#define OO_MAX_LAYERS 7

/* Status codes. */
#define OO_OK 0
#define OO_EINVAL (-1)        /* invalid argument (shape, pointer, alignment) */
#define OO_ECAPACITY (-2)     /* output capacity too small; needed size written */
#define OO_EHIP (-3)          /* a HIP runtime call failed */
#define OO_EUNSUPPORTED (-4)  /* valid but not implemented (e.g. a layer width) */

typedef enum { OO_F32 = 0, OO_F16 = 1, OO_BF16 = 2 } oo_dtype;

/*
 * The octree and its feature maps (Sec. 3.4). All pointers are device
 * pointers.
 *  - n_levels: L = D + 1 levels, 0 (root) ..= D, with 1 <= L <= 16.
 *  - C: channels per texel, 4 or 8.
 *  - res[l]: the level-l map is res[l] x res[l] texels (cells). A power of
 *    two in [2, 64], or in [2, 512] with OO_INTERP_PAPER (the paper's
 *    coarsest vertex maps have 2^8 + 1 vertices per side).
 *  - level_offset: the nodes of level l have global indices
 *    [level_offset[l], level_offset[l+1]).
 *  - nodes: one 32-bit word per node, breadth first; within a level, nodes
 *    are ordered by parent, then octant.
 *    word = (first_child << 8) | child_mask. Bit o of the mask is set when
 *    the child in octant o = bx | by << 1 | bz << 2 exists. first_child is
 *    the global index of the lowest existing child. A leaf's word is 0.
 *  - feat[l]: level-l table of feat_dtype, channels contiguous, 16-byte
 *    aligned. Row index is t (v), column index is s (u).
 *    OO_INTERP_NODE_BILINEAR: [n_l][res][res][C] texels.
 *    OO_INTERP_PAPER: [n_l][res + 1][res + 1][C] vertices. Vertex (i, j)
 *    sits at (s, t) = (i / res, j / res). A border vertex that repeats
 *    another's direction is never read.
 *  - interp: OO_INTERP_NODE_BILINEAR (0) or OO_INTERP_PAPER (1).
 *  - disparity: see oo_disparity below; NULL unless interp = 1.
 */
#define OO_INTERP_NODE_BILINEAR 0
#define OO_INTERP_PAPER 1

/*
 * The disparity predictor g_psi (Sec. 3.3, disparity equation; Sec. 3.5:
 * a multi-resolution hash encoding followed by a small MLP). All FP32
 * device pointers.
 *  - Hash encoding of x (Instant-NGP style): level i has res[i] = N_i
 *    cells per side (1 <= N_i <= 2^20). x, clamped to the cube, scaled by
 *    N_i lies in cell floor(x N_i) (the last cell closed at x = 1); its
 *    eight vertices are read with the trilinear weights of the fraction.
 *    Vertex (a, b, c) is entry a + (N_i + 1) (b + (N_i + 1) c) when
 *    (N_i + 1)^3 <= 2^log2_T, else ((a * 1) xor (b * 2654435761) xor
 *    (c * 805459861)) mod 2^log2_T in 32-bit arithmetic.
 *  - tables: [n_levels][2^log2_T][F] with n_levels = 16 and F = 2
 *    (Instant-NGP's shape), 1 <= log2_T <= 24, 8-byte aligned.
 *  - The MLP reads [encoding (n_levels F), unit(w_r) (3), 0]: n_layers = 2
 *    or 3 Linear layers (one or two hidden layers of width 64; the paper's
 *    has two), W[i] row-major [dims[i+1]][dims[i]] FP32, b[i] [dims[i+1]];
 *    dims[0] = 36, dims[n_layers] = 1 (the disparity d, linear output).
 *    ReLU between. Other shapes are refused with OO_EUNSUPPORTED.
 *  - Arithmetic: FP32, except that the residual forward of a 16-bit decoder
 *    (oo_mlp dtype FP16/BF16) runs the MLP on split BF16 operands (each
 *    FP32 value as hi + lo, three BF16 products per FP32 one, FP32
 *    accumulation; about 16 significant bits).
 *  - dtables, dW, db: gradient accumulators (same shapes) that the residual
 *    backward adds the predictor's gradients into (+=); NULL for calls
 *    that do not differentiate.
 * With a predictor, cell j of a level (centre c_j = (cell + 1/2) / 2^l) is
 * read along v_j = (x - c_j) d + w_r / |w_r| (Sec. 3.3, shifted-direction
 * equation, second form; x clamped to the cube as for the cells); the
 * octahedral map needs no normalisation of v_j.
 */
#define OO_HASH_MAX_LEVELS 16
typedef struct {
  int32_t n_levels;
  int32_t F;
  int32_t log2_T;
  int32_t res[OO_HASH_MAX_LEVELS];
  const float* tables;
  int32_t n_layers;
  int32_t dims[5];
  const float* W[4];
  const float* b[4];
  float* dtables;
  float* dW[4];
  float* db[4];
} oo_disparity;

typedef struct {
  int32_t n_levels;
  int32_t C;
  int32_t res[OO_MAX_LEVELS];
  int64_t level_offset[OO_MAX_LEVELS + 1];
  const uint32_t* nodes;
  oo_dtype feat_dtype;
  const void* feat[OO_MAX_LEVELS];
  int32_t interp;
  /* OO_INTERP_PAPER only: the disparity predictor shifting each cell's
   * lookup direction, or NULL for the lookup along w_r (Sec. 4.4's ablation
   * without a direction offset). */
  const oo_disparity* disparity;
} oo_tree;

/*
 * The decoder MLP (Sec. 3.5). Hidden layers use ReLU; the output layer is
 * linear.
 *  - n_layers: number of Linear layers, 2..5 (the paper's decoder has four
 *    hidden layers of width 128: n_layers = 5).
 *  - dims[0] = n_levels * C + E, a multiple of 4, at most 128. The decoder
 *    reads [h, g]: the n_levels * C level features, then E >= 0 surface
 *    attributes per query (Sec. 3.5: position, mirror direction, normal,
 *    albedo, roughness: 13 values; the caller pads g with zero columns to
 *    make dims[0] a multiple of 4, which leaves the function unchanged and
 *    gives the padding weights zero gradient). E = 0 decodes h alone.
 *    dims[n_layers] = 3. Every hidden width is the same: 64 or 128.
 *  - W[i]: [dims[i+1]][dims[i]] row-major in `dtype`. Also the operand type
 *    of the matrix cores. Accumulation is always FP32.
 *  - b[i]: [dims[i+1]] FP32.
 */
typedef struct {
  int32_t n_layers;
  int32_t dims[OO_MAX_LAYERS + 1];
  oo_dtype dtype;
  const void* W[OO_MAX_LAYERS];
  const float* b[OO_MAX_LAYERS];
} oo_mlp;

/*
 * Octree construction on the host (Sec. 3.4 sparse octree of non-empty cells;
 * Sec. 4.1 o-cnn-style structure).
 *  - Refinement rule: the root always exists. A node at level l < max_depth
 *    holding MORE than split_threshold samples gets every child octant that
 *    holds at least one sample.
 *  - samples_xyz_host: host [n][3] FP32 points in the unit cube.
 *  - Size query: call with nodes_out_host == NULL. Then only
 *    *n_nodes_out_host and level_offset_out_host are written.
 *  - capacity: size of nodes_out_host in words. If it is too small the call
 *    returns OO_ECAPACITY and still writes the needed count.
 *  - level_offset_out_host: host [max_depth + 2].
 *  - Returns OO_EUNSUPPORTED if the tree needs more than 2^24 nodes.
 */
int oo_build_octree(const float* samples_xyz_host, int64_t n, int32_t max_depth,
                    int32_t split_threshold, uint32_t* nodes_out_host, int64_t capacity,
                    int64_t* level_offset_out_host, int64_t* n_nodes_out_host);

/*
 * Encoding query (Sec. 3.3-3.4): the octahedral coordinate of dir and, per
 * level, the interpolated feature of the tree's scheme.
 *  - x, dir: [B][3] FP32.
 *  - h_out: [B][n_levels * C] in h_dtype. Level-major, channels contiguous.
 *    A level with no node to read contributes zeros.
 *  - node_idx_out: may be NULL. OO_INTERP_NODE_BILINEAR: [B][n_levels], the
 *    global node index per level, -1 where the tree has no node.
 *    OO_INTERP_PAPER: [B][n_levels][8], the nodes of the eight cells around
 *    x, -1 for an empty cell or one outside the cube. Corner d = dx | dy << 1
 *    | dz << 2; its cell is floor(x 2^l - 1/2) + (dx, dy, dz).
 */
int oo_encode_query(const oo_tree* tree, const float* x, const float* dir, int64_t B, void* h_out,
                    oo_dtype h_dtype, int32_t* node_idx_out, hipStream_t stream);

/*
 * Decoder forward on materialised features (Sec. 3.5).
 *  - h: [B][dims[0]] in h_dtype. h_dtype must equal mlp->dtype.
 *  - rgb_out: [B][3] FP32.
 */
int oo_mlp_fwd(const oo_mlp* mlp, const void* h, oo_dtype h_dtype, int64_t B, float* rgb_out,
               hipStream_t stream);

/*
 * Fused query forward: encode + decode in one kernel. h stays on chip
 * (Sec. 3.6, rendering: one query and one decoder evaluation per visible
 * point).
 *  - x, dir: [B][3] FP32. rgb_out: [B][3] FP32.
 *  - attr: [B][E] FP32, the decoder's surface attributes g (E = dims[0] -
 *    n_levels * C); NULL when E = 0, required otherwise.
 *  - Supported type pairs (tree->feat_dtype, mlp->dtype): (F32, F32),
 *    (F16, F16), (BF16, BF16).
 */
int oo_query_fwd(const oo_tree* tree, const oo_mlp* mlp, const float* x, const float* dir, const float* attr,
                 int64_t B, float* rgb_out, hipStream_t stream);

/*
 * One batch of the neural-radiosity residual (Sec. 3.2 Monte-Carlo RHS;
 * Sec. 3.6 loss). All pointers are device pointers.
 *  - B: number of LHS points. N: secondary samples per point, N >= 0.
 *  - Per point, [B][3] FP32: x, dir (lookup direction of the LHS query),
 *    n (normal), wo (outgoing direction), albedo, Le (emission).
 *  - rough: [B] FP32, the GGX alpha.
 *  - Per sample, [B][N][3] FP32: x2 (secondary hit), dir2 (lookup
 *    direction at the hit), wi (sampled incident direction).
 *  - pdf: [B][N] FP32, or NULL for 1.
 *  - attr: [B][E] FP32, the decoder's surface attributes g of the LHS
 *    queries; attr2: [B][N][E] those of the secondary hits (E = dims[0] -
 *    n_levels * C). Both NULL when E = 0; attr2 is not read with
 *    target_override.
 *  - target_override: [B][3] FP32. When set, it replaces the RHS estimate
 *    and no RHS query is made. Finite-difference checks use this to freeze
 *    the target.
 *  - F0: Schlick reflectance at normal incidence.
 *  - loss_kind: 0 = mean L2 over the 3B entries. 1 = relative L2 with the
 *    detached normaliser max(LHS + T, 0) + eps (Sec. 3.6).
 *  - grad_through_rhs: 0 = target detached (the paper's choice). 1 = the
 *    gradient also flows into the RHS queries.
 *  - BSDF: f = albedo/pi + D G F / (4 cos_i cos_o) with GGX D, Smith's
 *    separable G, Schlick's F. Sample weight: f |n . wi| / pdf. n, wo and wi
 *    are normalised first. A direction below either horizon weighs 0.
 */
typedef struct {
  int64_t B;
  int32_t N;
  const float *x, *dir, *n, *wo, *albedo, *Le;
  const float* rough;
  const float *x2, *dir2, *wi;
  const float* pdf;
  const float* target_override;
  float F0;
  int32_t loss_kind;
  float eps;
  int32_t grad_through_rhs;
  const float *attr, *attr2;
} oo_residual_batch;

/* Workspace size in bytes that the residual forward and backward need for
 * this problem (it depends on the batch and on the MLP's dtype). The same
 * workspace serves both calls; both take its size and return OO_EINVAL,
 * before launching anything, when it is smaller than this. */
int oo_residual_workspace_bytes(const oo_tree* tree, const oo_mlp* mlp,
                                const oo_residual_batch* batch, size_t* bytes);

/*
 * Residual forward.
 *  - The B (1 + N) queries are first bucketed by the octree cell that holds
 *    them (a counting sort on the Morton code of a coarse cell, LHS queries
 *    first) and evaluated in that order, so neighbouring query tiles read
 *    the same nodes' maps; outputs are in the caller's order. Requires
 *    B (1 + N) < 2^31 (else OO_EUNSUPPORTED).
 *  - Outputs, each [B][3] FP32: lhs_out = L(x, dir);
 *    rhs_out = T = Le + (1/N) sum_k w_k * L(x2_k, dir2_k), or the override;
 *    resid_out = lhs - T.
 *  - loss_out: device FP64 scalar, sum over entries of r^2 / (3B). The
 *    relative loss divides each r by its normaliser first.
 *  - The loss reduction runs in FP64 in a fixed order, so repeated calls
 *    give identical bits.
 */
int oo_radiosity_residual_fwd(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch,
                              float* lhs_out, float* rhs_out, float* resid_out, double* loss_out,
                              void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * Residual backward. The texel gathers and the decoder forward are
 * recomputed, not stored; the node index per level comes from the forward.
 *  - workspace: the one the forward of this batch used, unchanged since.
 *    The forward leaves there the bucketed query order and, for every query
 *    the backward processes, its node indices and octahedral coordinates.
 *    Indices found outside their level or outside the batch, and
 *    coordinates outside [0, 1] (a workspace the forward did not fill), are
 *    treated as missing nodes, as no seed, and clamped; nothing outside the
 *    tables or the batch is dereferenced.
 *  - resid, rhs: the forward's outputs for the same batch and parameters.
 *  - grad_loss: device FP64 scalar, dLoss_total/dloss.
 *  - dfeat[l]: FP32 [n_l][res][res][C]. Receives += the feature gradient by
 *    atomic scatter; the summation order is not fixed.
 *  - dW[i], db[i]: FP32, shaped like the layer. Receive += the reduced
 *    gradient. The reduction over workgroups runs in a fixed order, but
 *    which queries share a workgroup follows the bucketed order, which is
 *    not fixed inside a bucket: results agree to rounding, not bitwise,
 *    from call to call.
 *  - Gradients are for the tables and weights the forward read. In
 *    mixed-precision runs those are the FP16/BF16 working copies, and the
 *    gradient is applied to the FP32 masters.
 *  - Streams: with at least 65,536 backward queries the work runs in up to
 *    four chunks, and the feature scatter of each chunk runs on a second
 *    stream that the library creates once per device (default priority),
 *    ordered by events: it starts after that chunk's decoder backward on
 *    `stream`, and `stream` waits for the last scatter before the dW/db
 *    reduction. To the caller the call behaves as work enqueued on `stream`.
 */
int oo_radiosity_residual_bwd(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch,
                              const float* resid, const float* rhs, const double* grad_loss,
                              float* const* dfeat, float* const* dW, float* const* db, void* workspace,
                              size_t workspace_bytes, hipStream_t stream);

/*
 * Node index per level that the residual forward found for each query the
 * backward processes (Sec. 3.4: the node containing the point at every
 * level), read back from the workspace in the caller's query order.
 *  - tree, mlp, batch: as passed to the forward; workspace: the one it
 *    filled, unchanged since (its size is checked as in the forward).
 *  - node_idx_out: [Qb][n_levels] int32, -1 where the tree has no node
 *    (OO_INTERP_PAPER: [Qb][n_levels][8], the eight neighbouring cells'
 *    nodes as in oo_encode_query).
 *    Qb = B (the LHS queries) with the target detached, B (1 + N) with
 *    grad_through_rhs (LHS queries first, then query (b, k) at B + b N + k).
 *  - The indices are those the fused query kernel computed during the
 *    forward and that the backward reads; nothing is recomputed.
 */
int oo_residual_node_indices(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch,
                             const void* workspace, size_t workspace_bytes, int32_t* node_idx_out,
                             hipStream_t stream);

/*
 * FP64 inner products of FP32 arrays, for the gradient norms and
 * directional derivatives that finite-difference checks of the residual
 * adjoint (Sec. 3.6) compare against.
 *  - a[g], b[g]: device FP32 arrays of n[g] elements, g < n_groups <=
 *    OO_DOT_MAX_GROUPS. b == NULL, or b[g] == NULL, takes b[g] = a[g]
 *    (squared norm). a, b and n are host arrays of pointers / sizes.
 *  - out: device FP64 [n_groups], out[g] = sum_i a[g][i] * b[g][i].
 *  - partials: device FP64 scratch of n_groups * OO_DOT_BLOCKS elements,
 *    owned by the caller.
 *  - Each product is formed and summed in FP64, in an order that depends
 *    only on n[g]: repeated calls give identical bits.
 */
#define OO_DOT_MAX_GROUPS 64
#define OO_DOT_BLOCKS 256
int oo_dot_f64(const float* const* a, const float* const* b, const int64_t* n, int32_t n_groups, double* out,
               double* partials, hipStream_t stream);

/*
 * oo_dot_f64 for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same inner products, with the partial sums kept in an array the library
 * owns instead of a caller workspace.
 *  - a, b, n, n_groups, out: as in oo_dot_f64. The result bits are those of
 *    oo_dot_f64 on the same input (same kernels, same summation order).
 *  - The array holds OO_DOT_MAX_GROUPS x OO_DOT_BLOCKS doubles (128 KiB) per
 *    device, set up on the first call on that device and kept until the
 *    process ends. n_groups > OO_DOT_MAX_GROUPS is refused with OO_EINVAL;
 *    group lengths are not limited.
 *  - The call allocates nothing on the device or through any library.
 *  - Every call on one device shares that device's array: calls that overlap
 *    on one device (different streams or host threads without ordering)
 *    race and give wrong sums. Calls ordered on one stream are safe; each
 *    call overwrites every partial it reads, so nothing needs clearing.
 */
int oo_dot_f64_noalloc(const float* const* a, const float* const* b, const int64_t* n, int32_t n_groups,
                       double* out, hipStream_t stream);

/*
 * Optimiser step over the FP32 masters. The paper trains its tables and
 * networks jointly by gradient descent on the residual loss (Sec. 3.6, 4.1)
 * but does not name the optimiser; this is Adam (Kingma and Ba,
 * Algorithm 1), fused with the refresh of the 16-bit working copy and the
 * clearing of the gradient, and lazy over feature-map blocks that no query
 * of the batch read.
 *  - segments: host array of n_segs <= OO_ADAM_MAX_SEGMENTS descriptors, each
 *    a contiguous parameter array (a level's table, a layer's W or b):
 *    param, grad, m, v are device FP32 arrays of n elements; work is the
 *    working copy (n elements of cfg->work_dtype) or NULL; touched is NULL
 *    (update every element) or a device array of per-block flags with
 *    `block` elements per flag (a node's map: res^2 C, or (res+1)^2 C in the
 *    paper's scheme), of which only blocks with a non-zero flag are touched.
 *  - For every updated element, in FP32:
 *      m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *      param -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 *    then work = RNE(param) and grad = 0. Elements of untouched blocks are
 *    not read or written.
 *  - cfg->step is t >= 1. param, grad, m, v and work must not overlap.
 */
#define OO_ADAM_MAX_SEGMENTS 32
typedef struct {
  float lr, beta1, beta2, eps;
  int32_t step;
  oo_dtype work_dtype;
} oo_adam_config;
typedef struct {
  float* param;
  float* grad;
  float* m;
  float* v;
  void* work;
  int64_t n;
  const uint32_t* touched;
  int64_t block;
} oo_adam_segment;
int oo_adam_step(const oo_adam_config* cfg, const oo_adam_segment* segments, int32_t n_segs, hipStream_t stream);

/*
 * Marks the nodes the residual forward's backward queries read: for each
 * stored node index (the node per level, or the eight corner cells' nodes in
 * the paper's scheme), touched[node] = 1. touched: device [n_nodes] uint32,
 * global node indices; the caller clears it first. tree, mlp, batch,
 * workspace: as passed to the forward, unchanged since. The flags of a
 * level, offset by its first node, are the `touched` blocks of that level's
 * table in oo_adam_step.
 */
int oo_touched_nodes(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch, const void* workspace,
                     size_t workspace_bytes, uint32_t* touched, hipStream_t stream);

/* FP32 -> FP16/BF16 (round to nearest even) or FP32 copy, n elements. Used
 * to refresh working copies from FP32 masters. */
int oo_cast_params(const float* src_fp32, void* dst, oo_dtype dst_dtype, int64_t n, hipStream_t stream);

/*
 * Opt-in launch timing (a measurement aid, not part of the method). Between
 * oo_profile_begin and oo_profile_end every entry point records a pair of
 * HIP events on its stream around each group of kernels it launches, for up
 * to `capacity` groups (later groups are not timed). oo_profile_end waits
 * for the recorded events, writes per kind the summed milliseconds
 * (total_ms) and the number of timed groups (launches), each an array of
 * OO_PROF_KINDS entries or NULL, and releases the events. Kinds: sort =
 * query bucketing (4 kernels), query = fused encode + decode, combine =
 * residual assembly + loss reduction (2 kernels), backward = recompute +
 * decoder backward, scatter = feature-gradient atomics, seeds = backward
 * seeds + clear of the coarse levels' gradient pair buffers, dw_reduce =
 * fold of those buffers into the feature gradients + dW/db reduction; the
 * others are one kernel each. Timing a call adds two event records per group; the events
 * are host-side objects, no device memory is allocated.
 */
#define OO_PROF_KINDS 11
enum {
  OO_PROF_SORT = 0,
  OO_PROF_QUERY = 1,
  OO_PROF_COMBINE = 2,
  OO_PROF_SEEDS = 3,
  OO_PROF_TRANSPOSE = 4,
  OO_PROF_BACKWARD = 5,
  OO_PROF_SCATTER = 6,
  OO_PROF_DW_REDUCE = 7,
  OO_PROF_CAST = 8,
  OO_PROF_ENCODE = 9,
  OO_PROF_MLP = 10
};
int oo_profile_begin(int32_t capacity);
int oo_profile_end(double* total_ms, int64_t* launches);
/* Name of a kind ("" when out of range). */
const char* oo_profile_kind_name(int32_t kind);

/* Message for the last failed call on this thread ("" if none). */
const char* oo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* OCTAOCTREE_H */
