/*
 * FP64 CPU oracle for the OctaOctree query and the neural-radiosity residual
 * step. TEST INFRASTRUCTURE ONLY: see octaoctree_oracle.h.
 *
 * Each function follows the paper's steps in order, one query at a time, in
 * double precision, with no blocking or fusion. Where the paper is silent the
 * readings are stated at the function (they are the same readings the GPU
 * library is held to):
 *  - two interpolation schemes (ora_tree.interp):
 *    ORA_INTERP_NODE_BILINEAR reads the containing node at every level (the
 *    paper's "no octree interpolation" variant, Sec. 4.4) with a
 *    texel-centred bilinear fetch on an R x R map and the octahedral seam
 *    identification; ORA_INTERP_PAPER is the paper's own: the 8 neighbouring
 *    cells blended trilinearly and renormalised over the non-empty ones
 *    (Sec. 3.4, level-feature equation), each read by the barycentric
 *    lookup on an (R+1) x (R+1) vertex map (Sec. 3.3);
 *  - the decoder reads the concatenated levels h only (no G-buffer inputs);
 *  - the BSDF is Lambert + GGX (Smith separable, Schlick Fresnel).
 *
 * Parity pins (tests/test_oracle_*.py): brute-force containment for the
 * descent, closed-form octahedral vectors and the decode round trip, bilinear
 * weight / reproduction / seam-continuity properties, dense-layer products,
 * BSDF special cases, the constant-radiance residual closed form, and FP64
 * central finite differences for the adjoint.
 */
#include "octaoctree_oracle.h"

#define ORA_MAX_WIDTH 256  /* widest layer of either MLP */

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Spatial: quantisation and octree (Sec. 3.4 sparse octree; Sec. 4.1)       */
/* ------------------------------------------------------------------------ */

/* Cell coordinate along one axis at depth D: floor(x * 2^D) clamped to the
 * cube. Cells are half-open, so x == 1 lands in the last cell. The scaling by
 * a power of two is exact in floating point. */
static int64_t quant_axis(float xa, int32_t D) {
  double v = floor((double)xa * ldexp(1.0, D));
  int64_t maxq = ((int64_t)1 << D) - 1;
  if (!(v >= 0.0)) return 0; /* negative, or NaN (unspecified, clamped) */
  if (v > (double)maxq) return maxq;
  return (int64_t)v;
}

void ora_quantize(const float* x, int64_t B, int32_t D, int64_t* q_out) {
  for (int64_t b = 0; b < B; ++b)
    for (int a = 0; a < 3; ++a) q_out[3 * b + a] = quant_axis(x[3 * b + a], D);
}

/* Octant of the child at level l + 1 that contains cell q (finest-level
 * coordinates): bit a of the octant is bit (D - l - 1) of q_a. */
static int child_octant(const int64_t q[3], int32_t shift) {
  int bx = (int)((q[0] >> shift) & 1);
  int by = (int)((q[1] >> shift) & 1);
  int bz = (int)((q[2] >> shift) & 1);
  return bx | (by << 1) | (bz << 2);
}

typedef struct {
  int64_t* start;
  int64_t* count;
  uint32_t* mask;
  int64_t* first_child;
  int64_t n, cap;
} node_list;

static int node_push(node_list* L, int64_t start, int64_t count) {
  if (L->n == L->cap) {
    int64_t nc = L->cap ? 2 * L->cap : 1024;
    int64_t* s = (int64_t*)realloc(L->start, nc * sizeof(int64_t));
    if (!s) return -1;
    L->start = s;
    int64_t* c = (int64_t*)realloc(L->count, nc * sizeof(int64_t));
    if (!c) return -1;
    L->count = c;
    uint32_t* m = (uint32_t*)realloc(L->mask, nc * sizeof(uint32_t));
    if (!m) return -1;
    L->mask = m;
    int64_t* f = (int64_t*)realloc(L->first_child, nc * sizeof(int64_t));
    if (!f) return -1;
    L->first_child = f;
    L->cap = nc;
  }
  L->start[L->n] = start;
  L->count[L->n] = count;
  L->mask[L->n] = 0;
  L->first_child[L->n] = 0;
  L->n++;
  return 0;
}

/* Builds the tree top-down. The root always exists. Every node at level
 * l < D holding more than tau samples is refined, and only its non-empty
 * children are created ("every non-empty cell stores a map", Sec. 3.4).
 * Nodes are numbered breadth first; within a level by parent, then octant.
 * Each node owns a contiguous run of a sample permutation, which a stable
 * counting split by octant divides among its children. */
int ora_build_octree(const float* samples, int64_t n, int32_t D, int32_t tau,
                     uint32_t* nodes_out, int64_t capacity,
                     int64_t* level_offset_out, int64_t* n_nodes_out) {
  if (n < 0 || D < 0 || D > ORA_MAX_LEVELS - 1 || tau < 0) return -1;
  if ((n > 0 && !samples) || !level_offset_out || !n_nodes_out) return -1;

  int64_t* q = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(int64_t));
  int64_t* perm = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t* tmp = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  node_list L;
  memset(&L, 0, sizeof(L));
  int rc = 0;
  if (!q || !perm || !tmp) { rc = -5; goto done; }
  ora_quantize(samples, n, D, q);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;

  int64_t level_offset[ORA_MAX_LEVELS + 2];
  level_offset[0] = 0;
  if (node_push(&L, 0, n)) { rc = -5; goto done; }
  level_offset[1] = 1;

  for (int32_t l = 0; l < D; ++l) {
    int32_t shift = D - l - 1;
    for (int64_t v = level_offset[l]; v < level_offset[l + 1]; ++v) {
      int64_t s0 = L.start[v], cnt = L.count[v];
      if (cnt <= tau) continue; /* leaf */
      int64_t bucket[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int64_t s = s0; s < s0 + cnt; ++s) bucket[child_octant(&q[3 * perm[s]], shift)]++;
      int64_t pos[8];
      pos[0] = s0;
      for (int o = 1; o < 8; ++o) pos[o] = pos[o - 1] + bucket[o - 1];
      for (int64_t s = s0; s < s0 + cnt; ++s) {
        int o = child_octant(&q[3 * perm[s]], shift);
        tmp[pos[o]++] = perm[s];
      }
      memcpy(&perm[s0], &tmp[s0], (size_t)cnt * sizeof(int64_t));
      int64_t first = L.n, run = s0;
      uint32_t mask = 0;
      for (int o = 0; o < 8; ++o) {
        if (bucket[o] > 0) {
          if (node_push(&L, run, bucket[o])) { rc = -5; goto done; }
          mask |= 1u << o;
        }
        run += bucket[o];
      }
      L.mask[v] = mask;
      L.first_child[v] = first;
    }
    level_offset[l + 2] = L.n;
  }

  for (int32_t l = 0; l <= D + 1; ++l) level_offset_out[l] = level_offset[l];
  *n_nodes_out = L.n;
  if (L.n > ((int64_t)1 << 24)) { rc = -4; goto done; } /* first_child needs 24 bits */
  if (!nodes_out) goto done;
  if (capacity < L.n) { rc = -2; goto done; }
  for (int64_t v = 0; v < L.n; ++v)
    nodes_out[v] = L.mask[v] ? (((uint32_t)L.first_child[v] << 8) | L.mask[v]) : 0u;

done:
  free(q);
  free(perm);
  free(tmp);
  free(L.start);
  free(L.count);
  free(L.mask);
  free(L.first_child);
  return rc;
}

static int popcount8(uint32_t m) {
  int c = 0;
  for (int i = 0; i < 8; ++i) c += (int)((m >> i) & 1u);
  return c;
}

/* Containing node at every level: start at the root; at level l the child
 * octant of the query's cell selects a child of the level-(l-1) node, whose
 * index is first_child plus the number of existing children with a smaller
 * octant. A missing child ends the descent (index -1 below). */
static void descend_one(const ora_tree* t, const float* x3, int32_t* idx) {
  int32_t D = t->n_levels - 1;
  int64_t q[3];
  for (int a = 0; a < 3; ++a) q[a] = quant_axis(x3[a], D);
  int64_t cur = 0;
  idx[0] = 0;
  for (int32_t l = 1; l <= D; ++l) {
    if (cur >= 0) {
      uint32_t word = t->nodes[cur];
      uint32_t mask = word & 0xffu;
      int64_t first = (int64_t)(word >> 8);
      int o = child_octant(q, D - l);
      if ((mask >> o) & 1u)
        cur = first + popcount8(mask & ((1u << o) - 1u));
      else
        cur = -1;
    }
    idx[l] = (int32_t)cur;
  }
}

void ora_descend(const ora_tree* t, const float* x, int64_t B, int32_t* idx_out) {
  for (int64_t b = 0; b < B; ++b) descend_one(t, &x[3 * b], &idx_out[(int64_t)t->n_levels * b]);
}

/* ------------------------------------------------------------------------ */
/* Directional: octahedral map (Sec. 3.3) and bilinear taps                  */
/* ------------------------------------------------------------------------ */

static double sign_pos(double v) { return v < 0.0 ? -1.0 : 1.0; } /* sign(0) = +1 */

/* u = (wx, wy) / (|wx| + |wy| + |wz|); for wz < 0 the lower hemisphere is
 * folded with both new coordinates computed from the unfolded u; then
 * (s, t) = (u + 1) / 2. The zero vector maps to the map centre. */
static void octa_vec(const double* d, double* st) {
  double dx = d[0], dy = d[1], dz = d[2];
  double S = fabs(dx) + fabs(dy) + fabs(dz);
  double ux = 0.0, uy = 0.0;
  if (S > 0.0) {
    ux = dx / S;
    uy = dy / S;
  }
  if (dz < 0.0) {
    double fx = (1.0 - fabs(uy)) * sign_pos(ux);
    double fy = (1.0 - fabs(ux)) * sign_pos(uy);
    ux = fx;
    uy = fy;
  }
  st[0] = 0.5 * (ux + 1.0);
  st[1] = 0.5 * (uy + 1.0);
}

static void octa_one(const float* d, double* st) {
  double v[3] = {d[0], d[1], d[2]};
  octa_vec(v, st);
}

/* Derivative of (s, t) = octa(v) with respect to v, J[2][3], differentiated
 * piece by piece on the piece octa(v) evaluates (|a|' = sign(a) with
 * sign(0) = +1, as in the map). Upper hemisphere:
 * d u_a / d v_b = [a == b] / S - v_a sign(v_b) / S^2 with S = |v|_1. The
 * lower fold (1 - |u_y|) sign(u_x), (1 - |u_x|) sign(u_y) swaps and
 * negates: d f_x = -sign(u_x) sign(u_y) d u_y, d f_y = -sign(u_x) sign(u_y)
 * d u_x. Then (s, t) = (u + 1) / 2. */
static void octa_jacobian(const double* v, double J[2][3]) {
  double S = fabs(v[0]) + fabs(v[1]) + fabs(v[2]);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
  if (!(S > 0.0)) return;
  double du[2][3];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) du[a][b] = (a == b ? 1.0 / S : 0.0) - v[a] * sign_pos(v[b]) / (S * S);
  if (v[2] < 0.0) {
    double sx = sign_pos(v[0] / S), sy = sign_pos(v[1] / S);
    for (int b = 0; b < 3; ++b) {
      double fx = -sx * sy * du[1][b], fy = -sx * sy * du[0][b];
      du[0][b] = fx;
      du[1][b] = fy;
    }
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) J[a][b] = 0.5 * du[a][b];
}

void ora_octa(const float* dir, int64_t B, double* st_out) {
  for (int64_t b = 0; b < B; ++b) octa_one(&dir[3 * b], &st_out[2 * b]);
}

/* Inverse map: a point of the unfolded square inside the diamond
 * |u| + |v| <= 1 is on the upper hemisphere with z = 1 - |u| - |v|; a point
 * outside it is unfolded first. */
void ora_octa_decode(const double* st, int64_t B, double* dir_out) {
  for (int64_t b = 0; b < B; ++b) {
    double u = 2.0 * st[2 * b] - 1.0, v = 2.0 * st[2 * b + 1] - 1.0;
    double z = 1.0 - fabs(u) - fabs(v);
    if (z < 0.0) {
      double nu = (1.0 - fabs(v)) * sign_pos(u);
      double nv = (1.0 - fabs(u)) * sign_pos(v);
      u = nu;
      v = nv;
    }
    double len = sqrt(u * u + v * v + z * z);
    dir_out[3 * b] = u / len;
    dir_out[3 * b + 1] = v / len;
    dir_out[3 * b + 2] = z / len;
  }
}

/* Texel (i, j) has its centre at ((i + 0.5) / R, (j + 0.5) / R). The four
 * texels around (s, t) get the usual bilinear weights. A tap outside the map
 * is moved to the texel it touches across the octahedral seam: the edges
 * s = 0 and s = 1 are each glued to themselves with t mirrored, and the edges
 * t = 0 and t = 1 with s mirrored. Column wrap is applied first, then row
 * wrap, so a corner tap lands on the diagonally opposite map corner. */
static void taps_one(double s, double t, int32_t R, int32_t ij[8], double w[4]) {
  double pu = s * R - 0.5, pv = t * R - 0.5;
  double fi = floor(pu), fj = floor(pv);
  double fu = pu - fi, fv = pv - fj;
  int32_t i0 = (int32_t)fi, j0 = (int32_t)fj;
  for (int k = 0; k < 4; ++k) {
    int a = k & 1, bb = k >> 1;
    int32_t i = i0 + a, j = j0 + bb;
    w[k] = (a ? fu : 1.0 - fu) * (bb ? fv : 1.0 - fv);
    if (i < 0) {
      i = -1 - i;
      j = R - 1 - j;
    } else if (i >= R) {
      i = 2 * R - 1 - i;
      j = R - 1 - j;
    }
    if (j < 0) {
      i = R - 1 - i;
      j = -1 - j;
    } else if (j >= R) {
      i = R - 1 - i;
      j = 2 * R - 1 - j;
    }
    ij[2 * k] = i;
    ij[2 * k + 1] = j;
  }
}

void ora_taps(const double* st, int64_t B, int32_t R, int32_t* ij_out, double* w_out) {
  for (int64_t b = 0; b < B; ++b) taps_one(st[2 * b], st[2 * b + 1], R, &ij_out[8 * b], &w_out[4 * b]);
}

/* ------------------------------------------------------------------------ */
/* Encoding: per-level features, concatenated level by level (Sec. 3.4)      */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* The paper's interpolation: barycentric vertex maps (Sec. 3.3) and the     */
/* 8-cell trilinear blend renormalised over non-empty cells (Sec. 3.4)      */
/* ------------------------------------------------------------------------ */

int64_t ora_map_entries(int32_t R, int32_t interp) {
  return interp == ORA_INTERP_PAPER ? (int64_t)(R + 1) * (R + 1) : (int64_t)R * R;
}

/* Vertex (i, j) of the unfolded grid sits at (i / R, j / R). Points of the
 * map border that are one direction share one storage slot: the edges
 * s = 0 and s = 1 are each glued to themselves with t mirrored, the edges
 * t = 0 and t = 1 with s mirrored, and the four corners are the -z pole. */
static int32_t vertex_slot(int32_t i, int32_t j, int32_t R) {
  if (i == 0 || i == R) j = j < R - j ? j : R - j;
  if (j == 0 || j == R) i = i < R - i ? i : R - i;
  return j * (R + 1) + i;
}

/* Each octahedron face, unfolded, is a right isosceles triangle whose
 * hypotenuse lies on one of the lines |2s - 1| + |2t - 1| = 1 (the equator)
 * and whose legs lie on the map's border or on its centre lines. Subdividing
 * every face uniformly gives grid cells split along the diagonal parallel
 * to their quadrant's equator segment: the anti-diagonal in the quadrants
 * where s - 1/2 and t - 1/2 have the same sign, the main diagonal in the
 * other two. The query's cell and half give the triangle; its weights are
 * the barycentric coordinates of (s R, t R). */
static void bary_one(double s, double t, int32_t R, int32_t ij[6], double w[3]) {
  double pu = s * R, pv = t * R;
  int32_t i = (int32_t)floor(pu), j = (int32_t)floor(pv);
  if (i > R - 1) i = R - 1;
  if (j > R - 1) j = R - 1;
  if (i < 0) i = 0;
  if (j < 0) j = 0;
  double fu = pu - i, fv = pv - j;
  int same_side = (2 * i >= R) == (2 * j >= R);
  int32_t v[3][2];
  if (same_side) {
    if (fu + fv <= 1.0) {
      v[0][0] = i;     v[0][1] = j;     w[0] = 1.0 - fu - fv;
      v[1][0] = i + 1; v[1][1] = j;     w[1] = fu;
      v[2][0] = i;     v[2][1] = j + 1; w[2] = fv;
    } else {
      v[0][0] = i + 1; v[0][1] = j + 1; w[0] = fu + fv - 1.0;
      v[1][0] = i;     v[1][1] = j + 1; w[1] = 1.0 - fu;
      v[2][0] = i + 1; v[2][1] = j;     w[2] = 1.0 - fv;
    }
  } else {
    if (fu >= fv) {
      v[0][0] = i;     v[0][1] = j;     w[0] = 1.0 - fu;
      v[1][0] = i + 1; v[1][1] = j;     w[1] = fu - fv;
      v[2][0] = i + 1; v[2][1] = j + 1; w[2] = fv;
    } else {
      v[0][0] = i;     v[0][1] = j;     w[0] = 1.0 - fv;
      v[1][0] = i;     v[1][1] = j + 1; w[1] = fv - fu;
      v[2][0] = i + 1; v[2][1] = j + 1; w[2] = fu;
    }
  }
  for (int k = 0; k < 3; ++k) {
    ij[2 * k] = v[k][0];
    ij[2 * k + 1] = v[k][1];
  }
}

void ora_bary(const double* st, int64_t B, int32_t R, int32_t* ij_out, double* w_out, int32_t* vidx_out) {
  for (int64_t b = 0; b < B; ++b) {
    int32_t ij[6];
    bary_one(st[2 * b], st[2 * b + 1], R, ij, &w_out[3 * b]);
    for (int k = 0; k < 3; ++k) {
      ij_out[6 * b + 2 * k] = ij[2 * k];
      ij_out[6 * b + 2 * k + 1] = ij[2 * k + 1];
      vidx_out[3 * b + k] = vertex_slot(ij[2 * k], ij[2 * k + 1], R);
    }
  }
}

static double det3(const double a[3][3]) {
  return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
         a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}

/* Derivatives of the barycentric weights with respect to (pu, pv) = (s R,
 * t R) inside the triangle with grid vertices ij: the weights solve
 * sum_k w_k (i_k, j_k, 1) = (pu, pv, 1), so each derivative is that system
 * solved for a unit right-hand side (Cramer's rule). */
static void bary_grad(const int32_t ij[6], double dw_du[3], double dw_dv[3]) {
  double M[3][3];
  for (int k = 0; k < 3; ++k) {
    M[0][k] = ij[2 * k];
    M[1][k] = ij[2 * k + 1];
    M[2][k] = 1.0;
  }
  double det = det3(M);
  for (int r = 0; r < 2; ++r) {
    double* out = r == 0 ? dw_du : dw_dv;
    for (int k = 0; k < 3; ++k) {
      double A[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = b == k ? (a == r ? 1.0 : 0.0) : M[a][b];
      out[k] = det3(A) / det;
    }
  }
}

/* Node of the level-l cell with integer coordinates c, found by walking
 * down from the root along the cell's octants; -1 if the cell is outside
 * the cube or has no node. */
static int64_t cell_node(const ora_tree* t, int32_t l, const int64_t c[3]) {
  int64_t n = (int64_t)1 << l;
  for (int a = 0; a < 3; ++a)
    if (c[a] < 0 || c[a] >= n) return -1;
  int64_t cur = 0;
  for (int32_t k = 1; k <= l; ++k) {
    uint32_t word = t->nodes[cur];
    uint32_t mask = word & 0xffu;
    int o = child_octant(c, l - k);
    if (!((mask >> o) & 1u)) return -1;
    cur = (int64_t)(word >> 8) + popcount8(mask & ((1u << o) - 1u));
  }
  return cur;
}

/* Cell centres at level l sit at (c + 1/2) / 2^l. The eight cells whose
 * centres surround x (clamped to the cube) get the standard trilinear
 * weights; cells outside the cube or without a node are dropped and the
 * remaining weights rescaled to sum to 1 (all zero if none remains). */
static void neighbours_one(const ora_tree* t, const float* x3, int32_t l, int32_t idx[8], int64_t cells[24],
                           double w[8]) {
  int64_t base[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    double xa = (double)x3[a];
    if (!(xa >= 0.0)) xa = 0.0;
    if (xa > 1.0) xa = 1.0;
    double p = xa * ldexp(1.0, l) - 0.5;
    double fl = floor(p);
    base[a] = (int64_t)fl;
    f[a] = p - fl;
  }
  double sum = 0.0;
  for (int d = 0; d < 8; ++d) {
    int64_t c[3];
    double wd = 1.0;
    for (int a = 0; a < 3; ++a) {
      int bit = (d >> a) & 1;
      c[a] = base[a] + bit;
      wd *= bit ? f[a] : 1.0 - f[a];
      cells[3 * d + a] = c[a];
    }
    idx[d] = (int32_t)cell_node(t, l, c);
    w[d] = idx[d] >= 0 ? wd : 0.0;
    sum += w[d];
  }
  for (int d = 0; d < 8; ++d) w[d] = sum > 0.0 ? w[d] / sum : 0.0;
}

void ora_neighbours(const ora_tree* t, const float* x, int64_t B, int32_t l, int32_t* idx_out,
                    int64_t* cell_out, double* w_out) {
  for (int64_t b = 0; b < B; ++b) neighbours_one(t, &x[3 * b], l, &idx_out[8 * b], &cell_out[24 * b], &w_out[8 * b]);
}

/* ------------------------------------------------------------------------ */
/* Encoding: per-level features, concatenated level by level (Sec. 3.4)      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t idx[ORA_MAX_LEVELS];       /* containing node per level */
  int32_t ij[ORA_MAX_LEVELS][8];     /* bilinear taps (texel i, j) */
  double w[ORA_MAX_LEVELS][4];
  int32_t nb[ORA_MAX_LEVELS][8];     /* paper: the 8 neighbouring cells' nodes */
  double nbw[ORA_MAX_LEVELS][8];     /* their renormalised trilinear weights */
  int32_t vert[ORA_MAX_LEVELS][8][3]; /* paper: storage slots of each cell's 3 vertices */
  double vw[ORA_MAX_LEVELS][8][3];    /* their barycentric weights */
  double dvw[ORA_MAX_LEVELS][8][3];   /* their derivatives with respect to the disparity */
  /* with a disparity predictor: the query's disparity, its hash-grid
   * vertices and weights, and (backward) the gradient at the encoding */
  double disp;
  double dd;                          /* backward: dL/d disparity */
  int64_t hidx[ORA_HASH_MAX_LEVELS][8];
  double hw[ORA_HASH_MAX_LEVELS][8];
  double denc[ORA_HASH_MAX_LEVELS * ORA_HASH_MAX_F];
} query_taps;

static double disparity_one(const ora_disparity* g, const float* x3, const float* d3, int64_t hidx[][8],
                            double hw[][8], double act[][ORA_MAX_WIDTH], double pre[][ORA_MAX_WIDTH]);
static void unit_dir(const float* d3, double u[3]);

/* Everything a query reads, per level. Paper scheme with a disparity
 * predictor: cell j (integer coordinates c, centre (c + 1/2) / 2^l) is read
 * along v_j = (x - centre) d + unit(w_r), with x clamped to the cube as for
 * the cells; d (v_j) / d d = x - centre, carried through the octahedral
 * map and the triangle's barycentric weights to dvw. */
static void query_locate(const ora_tree* t, const float* x3, const float* d3, query_taps* qt) {
  double st[2];
  descend_one(t, x3, qt->idx);
  octa_one(d3, st);
  int shift = t->interp == ORA_INTERP_PAPER && t->disp != NULL;
  double xc[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0};
  qt->disp = 0.0;
  if (shift) {
    double act[ORA_MAX_LAYERS + 1][ORA_MAX_WIDTH], pre[ORA_MAX_LAYERS][ORA_MAX_WIDTH];
    qt->disp = disparity_one(t->disp, x3, d3, qt->hidx, qt->hw, act, pre);
    unit_dir(d3, u);
    for (int a = 0; a < 3; ++a) {
      double xa = (double)x3[a];
      if (!(xa >= 0.0)) xa = 0.0;
      if (xa > 1.0) xa = 1.0;
      xc[a] = xa;
    }
  }
  for (int32_t l = 0; l < t->n_levels; ++l) {
    int32_t R = t->res[l];
    if (t->interp == ORA_INTERP_PAPER) {
      int64_t cells[24];
      neighbours_one(t, x3, l, qt->nb[l], cells, qt->nbw[l]);
      for (int d = 0; d < 8; ++d) {
        double sd[2] = {st[0], st[1]}, dv[3] = {0.0, 0.0, 0.0}, J[2][3];
        if (shift) {
          double v[3];
          for (int a = 0; a < 3; ++a) {
            dv[a] = xc[a] - ((double)cells[3 * d + a] + 0.5) / ldexp(1.0, l);
            v[a] = dv[a] * qt->disp + u[a];
          }
          octa_vec(v, sd);
          octa_jacobian(v, J);
        }
        int32_t ij[6];
        bary_one(sd[0], sd[1], R, ij, qt->vw[l][d]);
        for (int k = 0; k < 3; ++k) qt->vert[l][d][k] = vertex_slot(ij[2 * k], ij[2 * k + 1], R);
        double gu[3] = {0.0, 0.0, 0.0}, gv[3] = {0.0, 0.0, 0.0}, ds = 0.0, dt = 0.0;
        if (shift) {
          bary_grad(ij, gu, gv);
          for (int a = 0; a < 3; ++a) {
            ds += J[0][a] * dv[a];
            dt += J[1][a] * dv[a];
          }
        }
        for (int k = 0; k < 3; ++k) qt->dvw[l][d][k] = R * (gu[k] * ds + gv[k] * dt);
      }
    } else {
      taps_one(st[0], st[1], R, qt->ij[l], qt->w[l]);
    }
  }
}

/* Offset of map entry `slot` of node idx at level l. */
static int64_t entry_base(const ora_tree* t, int32_t l, int32_t idx, int64_t slot) {
  int64_t local = (int64_t)idx - t->level_offset[l];
  return (local * ora_map_entries(t->res[l], t->interp) + slot) * t->C;
}

/* Offset of texel (i, j) of node idx at level l in that level's table. */
static int64_t texel_base(const ora_tree* t, int32_t l, int32_t idx, int32_t i, int32_t j) {
  int64_t R = t->res[l];
  int64_t local = (int64_t)idx - t->level_offset[l];
  return ((local * R + j) * R + i) * t->C;
}

/* Bilinear scheme: h_l = sum over taps of w * T_l[node][j][i][:]; a level
 * without a node contributes zeros. Paper scheme: h_l = sum over the 8
 * neighbouring cells of their renormalised trilinear weight times the
 * barycentric blend of that cell's three vertices; empty cells contribute
 * nothing. */
static void encode_from_taps(const ora_tree* t, const query_taps* qt, double* h) {
  int32_t C = t->C;
  for (int32_t l = 0; l < t->n_levels; ++l) {
    for (int32_t c = 0; c < C; ++c) h[l * C + c] = 0.0;
    if (t->interp == ORA_INTERP_PAPER) {
      for (int d = 0; d < 8; ++d) {
        if (qt->nb[l][d] < 0) continue;
        for (int k = 0; k < 3; ++k) {
          int64_t base = entry_base(t, l, qt->nb[l][d], qt->vert[l][d][k]);
          double wk = qt->nbw[l][d] * qt->vw[l][d][k];
          for (int32_t c = 0; c < C; ++c) h[l * C + c] += wk * (double)t->feat[l][base + c];
        }
      }
      continue;
    }
    if (qt->idx[l] < 0) continue;
    for (int k = 0; k < 4; ++k) {
      int64_t base = texel_base(t, l, qt->idx[l], qt->ij[l][2 * k], qt->ij[l][2 * k + 1]);
      for (int32_t c = 0; c < C; ++c) h[l * C + c] += qt->w[l][k] * (double)t->feat[l][base + c];
    }
  }
}

void ora_encode(const ora_tree* t, const float* x, const float* dir, int64_t B, double* h_out,
                int32_t* idx_out) {
  int64_t HC = (int64_t)t->n_levels * t->C;
  for (int64_t b = 0; b < B; ++b) {
    query_taps qt;
    query_locate(t, &x[3 * b], &dir[3 * b], &qt);
    encode_from_taps(t, &qt, &h_out[HC * b]);
    if (idx_out)
      for (int32_t l = 0; l < t->n_levels; ++l) idx_out[(int64_t)t->n_levels * b + l] = qt.idx[l];
  }
}

/* ------------------------------------------------------------------------ */
/* Decoder MLP (Sec. 3.5): ReLU hidden layers, linear output                 */
/* ------------------------------------------------------------------------ */


/* Forward pass of one row. act[i] receives the input of layer i (act[0] = h)
 * and pre[i] the pre-activation of layer i. */
static void mlp_row(const ora_mlp* m, const double* h, double act[][ORA_MAX_WIDTH],
                    double pre[][ORA_MAX_WIDTH], double* out) {
  for (int32_t k = 0; k < m->dims[0]; ++k) act[0][k] = h[k];
  for (int32_t i = 0; i < m->n_layers; ++i) {
    int32_t fin = m->dims[i], fout = m->dims[i + 1];
    for (int32_t o = 0; o < fout; ++o) {
      double z = (double)m->b[i][o];
      for (int32_t k = 0; k < fin; ++k) z += (double)m->W[i][(int64_t)o * fin + k] * act[i][k];
      pre[i][o] = z;
      if (i + 1 < m->n_layers)
        act[i + 1][o] = z > 0.0 ? z : 0.0;
      else
        out[o] = z;
    }
  }
}

void ora_mlp_fwd(const ora_mlp* m, const double* h, int64_t B, double* out) {
  static __thread double act[ORA_MAX_LAYERS + 1][ORA_MAX_WIDTH];
  static __thread double pre[ORA_MAX_LAYERS][ORA_MAX_WIDTH];
  int32_t din = m->dims[0], dout = m->dims[m->n_layers];
  for (int64_t b = 0; b < B; ++b) mlp_row(m, &h[din * b], act, pre, &out[dout * b]);
}

/* Reverse pass through the dense layers for the output gradient in delta:
 * dW/db accumulate delta_{i+1} a_i^T and delta_{i+1}, the gradient moves
 * through W_i^T and the ReLU mask (ReLU'(0) = 0); delta ends as the gradient
 * at the input. */
static void mlp_backprop(const ora_mlp* m, double act[][ORA_MAX_WIDTH], double pre[][ORA_MAX_WIDTH],
                         double* delta, double* const* dW, double* const* db) {
  double prev[ORA_MAX_WIDTH];
  for (int32_t i = m->n_layers - 1; i >= 0; --i) {
    int32_t fin = m->dims[i], fout = m->dims[i + 1];
    for (int32_t o = 0; o < fout; ++o) {
      db[i][o] += delta[o];
      for (int32_t k = 0; k < fin; ++k) dW[i][(int64_t)o * fin + k] += delta[o] * act[i][k];
    }
    for (int32_t k = 0; k < fin; ++k) {
      double s = 0.0;
      for (int32_t o = 0; o < fout; ++o) s += (double)m->W[i][(int64_t)o * fin + k] * delta[o];
      if (i > 0 && !(pre[i - 1][k] > 0.0)) s = 0.0;
      prev[k] = s;
    }
    for (int32_t k = 0; k < fin; ++k) delta[k] = prev[k];
  }
}

/* ------------------------------------------------------------------------ */
/* Disparity predictor: hash encoding + small MLP (Sec. 3.3, Sec. 3.5)       */
/* ------------------------------------------------------------------------ */

/* Entry of grid vertex c of hash level i: dense when the level's
 * (N + 1)^3 vertices fit in the table, else the spatial hash of Instant-NGP
 * (per-axis primes 1, 2654435761, 805459861, xor, 32-bit wrap-around),
 * modulo the table size. */
static int64_t hash_slot(const ora_disparity* g, int32_t i, const int64_t c[3]) {
  int64_t N1 = (int64_t)g->res[i] + 1;
  int64_t T = (int64_t)1 << g->log2_T;
  if (N1 * N1 * N1 <= T) return c[0] + N1 * (c[1] + N1 * c[2]);
  uint32_t h = ((uint32_t)c[0] * 1u) ^ ((uint32_t)c[1] * 2654435761u) ^ ((uint32_t)c[2] * 805459861u);
  return (int64_t)(h & (uint32_t)(T - 1));
}

/* Level i: x (clamped to the cube) scaled by N_i lies in cell
 * floor(x N_i) (the last cell closed at x = 1); its eight vertices get the
 * trilinear weights of the fraction. enc[i F + f] = sum_d w_d T_i[slot_d][f]. */
static void hash_encode_one(const ora_disparity* g, const float* x3, double* enc, int64_t idx[][8],
                            double w[][8]) {
  int64_t T = (int64_t)1 << g->log2_T;
  for (int32_t i = 0; i < g->n_levels; ++i) {
    int64_t N = g->res[i], base[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
      double xa = (double)x3[a];
      if (!(xa >= 0.0)) xa = 0.0;
      if (xa > 1.0) xa = 1.0;
      double p = xa * (double)N;
      double fl = floor(p);
      if (fl > (double)(N - 1)) fl = (double)(N - 1);
      base[a] = (int64_t)fl;
      f[a] = p - fl;
    }
    for (int32_t e = 0; e < g->F; ++e) enc[i * g->F + e] = 0.0;
    for (int d = 0; d < 8; ++d) {
      int64_t c[3];
      double wd = 1.0;
      for (int a = 0; a < 3; ++a) {
        int bit = (d >> a) & 1;
        c[a] = base[a] + bit;
        wd *= bit ? f[a] : 1.0 - f[a];
      }
      int64_t slot = hash_slot(g, i, c);
      idx[i][d] = slot;
      w[i][d] = wd;
      const float* row = g->tables + ((int64_t)i * T + slot) * g->F;
      for (int32_t e = 0; e < g->F; ++e) enc[i * g->F + e] += wd * (double)row[e];
    }
  }
}

void ora_hash_encode(const ora_disparity* g, const float* x, int64_t B, double* enc_out, int64_t* idx_out,
                     double* w_out) {
  int64_t E = (int64_t)g->n_levels * g->F;
  for (int64_t b = 0; b < B; ++b) {
    double enc[ORA_HASH_MAX_LEVELS * ORA_HASH_MAX_F];
    int64_t idx[ORA_HASH_MAX_LEVELS][8];
    double w[ORA_HASH_MAX_LEVELS][8];
    hash_encode_one(g, &x[3 * b], enc, idx, w);
    for (int64_t e = 0; e < E; ++e)
      if (enc_out) enc_out[E * b + e] = enc[e];
    for (int32_t i = 0; i < g->n_levels; ++i)
      for (int d = 0; d < 8; ++d) {
        if (idx_out) idx_out[(b * g->n_levels + i) * 8 + d] = idx[i][d];
        if (w_out) w_out[(b * g->n_levels + i) * 8 + d] = w[i][d];
      }
  }
}

/* Unit vector of a direction (the zero vector stays zero). */
static void unit_dir(const float* d3, double u[3]) {
  double n = sqrt((double)d3[0] * d3[0] + (double)d3[1] * d3[1] + (double)d3[2] * d3[2]);
  for (int a = 0; a < 3; ++a) u[a] = n > 0.0 ? (double)d3[a] / n : 0.0;
}

/* d = MLP([hash encoding of x, unit(w_r), 0]); act / pre are the MLP's
 * activations for the backward. */
static double disparity_one(const ora_disparity* g, const float* x3, const float* d3, int64_t hidx[][8],
                            double hw[][8], double act[][ORA_MAX_WIDTH], double pre[][ORA_MAX_WIDTH]) {
  double in[ORA_MAX_WIDTH], out[ORA_MAX_WIDTH], u[3];
  int32_t E = g->n_levels * g->F;
  hash_encode_one(g, x3, in, hidx, hw);
  unit_dir(d3, u);
  in[E] = u[0];
  in[E + 1] = u[1];
  in[E + 2] = u[2];
  in[E + 3] = 0.0;
  mlp_row(&g->mlp, in, act, pre, out);
  return out[0];
}

void ora_disparity_fwd(const ora_disparity* g, const float* x, const float* dir, int64_t B, double* d_out) {
  for (int64_t b = 0; b < B; ++b) {
    int64_t hidx[ORA_HASH_MAX_LEVELS][8];
    double hw[ORA_HASH_MAX_LEVELS][8];
    double act[ORA_MAX_LAYERS + 1][ORA_MAX_WIDTH], pre[ORA_MAX_LAYERS][ORA_MAX_WIDTH];
    d_out[b] = disparity_one(g, &x[3 * b], &dir[3 * b], hidx, hw, act, pre);
  }
}

/* Number of decoder attributes after the level features. */
static int32_t attr_dims(const ora_tree* t, const ora_mlp* m) { return m->dims[0] - t->n_levels * t->C; }

/* Decoder input of one query: the level features, then its attributes. */
static void decoder_input(const ora_tree* t, const ora_mlp* m, const query_taps* qt, const float* e, double* h) {
  encode_from_taps(t, qt, h);
  int32_t LC = t->n_levels * t->C, E = attr_dims(t, m);
  for (int32_t k = 0; k < E; ++k) h[LC + k] = (double)e[k];
}

void ora_query_fwd(const ora_tree* t, const ora_mlp* m, const float* x, const float* dir, const float* attr,
                   int64_t B, double* rgb_out, int32_t nthreads) {
  int32_t dout = m->dims[m->n_layers];
  int32_t E = attr_dims(t, m);
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
  for (int64_t b = 0; b < B; ++b) {
    double h[ORA_MAX_WIDTH];
    double act[ORA_MAX_LAYERS + 1][ORA_MAX_WIDTH];
    double pre[ORA_MAX_LAYERS][ORA_MAX_WIDTH];
    query_taps qt;
    query_locate(t, &x[3 * b], &dir[3 * b], &qt);
    decoder_input(t, m, &qt, E > 0 ? &attr[E * b] : NULL, h);
    mlp_row(m, h, act, pre, &rgb_out[dout * b]);
  }
  (void)nthreads;
}

/* ------------------------------------------------------------------------ */
/* BSDF weight (rendering equation, Sec. 3.2)                                */
/* ------------------------------------------------------------------------ */

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* f_r = albedo / pi + D G F / (4 cos_i cos_o) with the GGX distribution
 * D = a^2 / (pi ((n.h)^2 (a^2 - 1) + 1)^2), the separable Smith term
 * G1(c) = 2c / (c + sqrt(a^2 + (1 - a^2) c^2)), Schlick's Fresnel
 * F = F0 + (1 - F0)(1 - wi.h)^5, and a = roughness. The sample weight is
 * f_r |n . wi| / pdf; directions below either horizon weigh zero. */
static void normalize3(double* v) {
  double l = sqrt(dot3(v, v));
  if (l > 0.0)
    for (int a = 0; a < 3; ++a) v[a] /= l;
}

static void bsdf_one(const float* n3, const float* wo3, const float* wi3, const float* alb3,
                     double alpha, double F0, double pdf, double w[3]) {
  double n[3], wo[3], wi[3];
  for (int a = 0; a < 3; ++a) {
    n[a] = n3[a];
    wo[a] = wo3[a];
    wi[a] = wi3[a];
  }
  /* directions are unit vectors: FP32 inputs are normalised first */
  normalize3(n);
  normalize3(wo);
  normalize3(wi);
  double ci = dot3(n, wi), co = dot3(n, wo);
  if (ci <= 0.0 || co <= 0.0) {
    w[0] = w[1] = w[2] = 0.0;
    return;
  }
  double hv[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
  double hl = sqrt(dot3(hv, hv));
  for (int a = 0; a < 3; ++a) hv[a] /= hl;
  double nh = dot3(n, hv);
  double a2 = alpha * alpha;
  double den = nh * nh * (a2 - 1.0) + 1.0;
  double Dm = a2 / (PI * den * den);
  double g1i = 2.0 * ci / (ci + sqrt(a2 + (1.0 - a2) * ci * ci));
  double g1o = 2.0 * co / (co + sqrt(a2 + (1.0 - a2) * co * co));
  double F = F0 + (1.0 - F0) * pow(1.0 - dot3(wi, hv), 5.0);
  double spec = Dm * g1i * g1o * F / (4.0 * ci * co);
  for (int c = 0; c < 3; ++c) w[c] = ((double)alb3[c] / PI + spec) * fabs(ci) / pdf;
}

void ora_bsdf_weight(const ora_batch* bt, double* w_out) {
  for (int64_t b = 0; b < bt->B; ++b)
    for (int32_t k = 0; k < bt->N; ++k) {
      int64_t bk = b * bt->N + k;
      double p = bt->pdf ? (double)bt->pdf[bk] : 1.0;
      bsdf_one(&bt->n[3 * b], &bt->wo[3 * b], &bt->wi[3 * bk], &bt->albedo[3 * b],
               (double)bt->rough[b], bt->F0, p, &w_out[3 * bk]);
    }
}

/* ------------------------------------------------------------------------ */
/* Residual step (Sec. 3.2 Monte-Carlo target, Sec. 3.6 loss)                */
/* ------------------------------------------------------------------------ */

/* LHS radiance at (x, d), RHS target T = L_e + (1/N) sum_k w_k * L(x'_k, d'_k)
 * (or the override), and the residual r = LHS - T. */
static int residual_parts(const ora_tree* t, const ora_mlp* m, const ora_batch* bt, double* lhs,
                          double* T, double* r, int32_t nthreads) {
  int64_t B = bt->B;
  int32_t N = bt->N;
  ora_query_fwd(t, m, bt->x, bt->dir, bt->attr, B, lhs, nthreads);
  if (bt->target_override) {
    for (int64_t i = 0; i < 3 * B; ++i) T[i] = (double)bt->target_override[i];
  } else {
    for (int64_t i = 0; i < 3 * B; ++i) T[i] = (double)bt->Le[i];
    if (N > 0) {
      double* rhsq = (double*)malloc((size_t)(B * N * 3) * sizeof(double));
      double* w = (double*)malloc((size_t)(B * N * 3) * sizeof(double));
      if (!rhsq || !w) {
        free(rhsq);
        free(w);
        return -5;
      }
      ora_query_fwd(t, m, bt->x2, bt->dir2, bt->attr2, B * N, rhsq, nthreads);
      ora_bsdf_weight(bt, w);
      for (int64_t b = 0; b < B; ++b)
        for (int c = 0; c < 3; ++c) {
          double acc = 0.0;
          for (int32_t k = 0; k < N; ++k) acc += w[3 * (b * N + k) + c] * rhsq[3 * (b * N + k) + c];
          T[3 * b + c] += acc / (double)N;
        }
      free(rhsq);
      free(w);
    }
  }
  for (int64_t i = 0; i < 3 * B; ++i) r[i] = lhs[i] - T[i];
  return 0;
}

/* Normaliser of the relative loss, treated as a constant: the sum of
 * prediction and target, clamped at zero, plus eps. */
static double rel_norm(double lhs, double T, double eps) {
  double s = lhs + T;
  return (s > 0.0 ? s : 0.0) + eps;
}

static int check_inputs(const ora_tree* t, const ora_mlp* m, const ora_batch* bt) {
  if (!t || !m || !bt || bt->B < 0 || bt->N < 0) return -1;
  if (t->n_levels < 1 || t->n_levels > ORA_MAX_LEVELS) return -1;
  if (m->n_layers < 1 || m->n_layers > ORA_MAX_LAYERS) return -1;
  if (attr_dims(t, m) < 0 || m->dims[m->n_layers] != 3) return -1;
  if (attr_dims(t, m) > 0 && bt->B > 0 && (!bt->attr || (bt->N > 0 && !bt->target_override && !bt->attr2)))
    return -1;
  for (int32_t i = 0; i <= m->n_layers; ++i)
    if (m->dims[i] < 1 || m->dims[i] > ORA_MAX_WIDTH) return -1;
  if (m->dims[0] > ORA_MAX_WIDTH) return -1;
  const ora_disparity* g = t->disp;
  if (g && t->interp == ORA_INTERP_PAPER) {
    if (g->n_levels < 1 || g->n_levels > ORA_HASH_MAX_LEVELS || g->F < 1 || g->F > ORA_HASH_MAX_F) return -1;
    if (g->log2_T < 1 || g->log2_T > 30 || !g->tables) return -1;
    for (int32_t i = 0; i < g->n_levels; ++i)
      if (g->res[i] < 1 || g->res[i] > (1 << 20)) return -1;
    const ora_mlp* gm = &g->mlp;
    if (gm->n_layers < 1 || gm->n_layers > ORA_MAX_LAYERS) return -1;
    if (gm->dims[0] != g->n_levels * g->F + 4 || gm->dims[gm->n_layers] != 1) return -1;
    for (int32_t i = 0; i <= gm->n_layers; ++i)
      if (gm->dims[i] < 1 || gm->dims[i] > ORA_MAX_WIDTH) return -1;
  }
  return 0;
}

int ora_residual_fwd(const ora_tree* t, const ora_mlp* m, const ora_batch* bt, double* lhs_out,
                     double* rhs_out, double* resid_out, double* loss_out, int32_t nthreads) {
  int rc = check_inputs(t, m, bt);
  if (rc) return rc;
  int64_t B = bt->B;
  rc = residual_parts(t, m, bt, lhs_out, rhs_out, resid_out, nthreads);
  if (rc) return rc;
  double acc = 0.0;
  for (int64_t i = 0; i < 3 * B; ++i) {
    double r = resid_out[i];
    if (bt->loss_kind == 1) r /= rel_norm(lhs_out[i], rhs_out[i], bt->eps);
    acc += r * r;
  }
  *loss_out = B > 0 ? acc / (3.0 * (double)B) : 0.0;
  return 0;
}

/* Reverse pass of one query for the radiance seed g: the dense-layer
 * gradients (ReLU'(0) = 0) added to dW/db, then dh = W_1^T delta_1 written
 * to dh_out, and the query's node indices, taps and weights to qt, from which
 * scatter_query later adds each tap's share of dh to the texel it read. */
static void backprop_query(const ora_tree* t, const ora_mlp* m, const float* x3, const float* d3, const float* e,
                           const double g[3], double* const* dW, double* const* db, double* const* gdW,
                           double* const* gdb, query_taps* qt, double* dh_out) {
  double h[ORA_MAX_WIDTH];
  double act[ORA_MAX_LAYERS + 1][ORA_MAX_WIDTH];
  double pre[ORA_MAX_LAYERS][ORA_MAX_WIDTH];
  double out[ORA_MAX_WIDTH];
  double delta[ORA_MAX_WIDTH];
  query_locate(t, x3, d3, qt);
  decoder_input(t, m, qt, e, h);
  mlp_row(m, h, act, pre, out);

  int32_t nl = m->n_layers;
  for (int32_t o = 0; o < m->dims[nl]; ++o) delta[o] = g[o];
  mlp_backprop(m, act, pre, delta, dW, db);
  /* delta now holds dL/dh. */
  for (int32_t k = 0; k < m->dims[0]; ++k) dh_out[k] = delta[k];
  if (!(t->interp == ORA_INTERP_PAPER && t->disp)) return;
  /* dL/dd = sum over levels, cells and vertices of
   * w_cell * (d w_vertex / d d) * <T[cell][vertex], dL/dh_l>, then through
   * the predictor's MLP to its weights and its input; the encoding part of
   * the input gradient is kept for the hash-table scatter. */
  const ora_disparity* gp = t->disp;
  int32_t C = t->C;
  double dd = 0.0;
  for (int32_t l = 0; l < t->n_levels; ++l)
    for (int d = 0; d < 8; ++d) {
      if (qt->nb[l][d] < 0) continue;
      for (int k = 0; k < 3; ++k) {
        int64_t base = entry_base(t, l, qt->nb[l][d], qt->vert[l][d][k]);
        double s = 0.0;
        for (int32_t c = 0; c < C; ++c) s += (double)t->feat[l][base + c] * dh_out[l * C + c];
        dd += qt->nbw[l][d] * qt->dvw[l][d][k] * s;
      }
    }
  qt->dd = dd;
  double gact[ORA_MAX_LAYERS + 1][ORA_MAX_WIDTH], gpre[ORA_MAX_LAYERS][ORA_MAX_WIDTH];
  disparity_one(gp, x3, d3, qt->hidx, qt->hw, gact, gpre);
  double gdelta[ORA_MAX_WIDTH];
  gdelta[0] = dd;
  mlp_backprop(&gp->mlp, gact, gpre, gdelta, gdW, gdb);
  for (int32_t k = 0; k < gp->n_levels * gp->F; ++k) qt->denc[k] = gdelta[k];
}

/* Adjoint of the level features: each tap's share w_tap * dh_l is added to
 * the texel the tap read, at the node that holds the query at that level
 * (paper scheme: each of the 24 cell-vertex reads gets its weight times
 * dh_l). */
static void scatter_query(const ora_tree* t, const query_taps* qt, const double* dh, double* const* dfeat,
                          double* dtables) {
  int32_t C = t->C;
  if (t->interp == ORA_INTERP_PAPER && t->disp) {
    /* hash-table entries: each vertex's trilinear share of dL/d enc */
    const ora_disparity* g = t->disp;
    int64_t T = (int64_t)1 << g->log2_T;
    for (int32_t i = 0; i < g->n_levels; ++i)
      for (int d = 0; d < 8; ++d)
        for (int32_t e = 0; e < g->F; ++e)
          dtables[((int64_t)i * T + qt->hidx[i][d]) * g->F + e] += qt->hw[i][d] * qt->denc[i * g->F + e];
  }
  for (int32_t l = 0; l < t->n_levels; ++l) {
    if (t->interp == ORA_INTERP_PAPER) {
      for (int d = 0; d < 8; ++d) {
        if (qt->nb[l][d] < 0) continue;
        for (int k = 0; k < 3; ++k) {
          int64_t base = entry_base(t, l, qt->nb[l][d], qt->vert[l][d][k]);
          double wk = qt->nbw[l][d] * qt->vw[l][d][k];
          for (int32_t c = 0; c < C; ++c) dfeat[l][base + c] += wk * dh[l * C + c];
        }
      }
      continue;
    }
    if (qt->idx[l] < 0) continue;
    for (int k = 0; k < 4; ++k) {
      int64_t base = texel_base(t, l, qt->idx[l], qt->ij[l][2 * k], qt->ij[l][2 * k + 1]);
      for (int32_t c = 0; c < C; ++c) dfeat[l][base + c] += qt->w[l][k] * dh[l * C + c];
    }
  }
}

/* Seed of backward query q (q < B: the LHS query of point q; otherwise the
 * RHS query (b, k) of point b = (q - B) / N, only with the gradient through
 * the target). */
static void query_seed(const ora_batch* bt, int32_t E, const double* lhs, const double* T, const double* r,
                       const double* w, double grad_loss, int64_t q, double g[3], const float** x3,
                       const float** d3, const float** e) {
  int64_t B = bt->B;
  int64_t b = q < B ? q : (q - B) / bt->N;
  for (int c = 0; c < 3; ++c) {
    double gc = 2.0 * r[3 * b + c] * grad_loss / (3.0 * (double)B);
    if (bt->loss_kind == 1) {
      double rho = rel_norm(lhs[3 * b + c], T[3 * b + c], bt->eps);
      gc /= rho * rho;
    }
    g[c] = gc;
  }
  if (q < B) {
    *x3 = &bt->x[3 * q];
    *d3 = &bt->dir[3 * q];
    *e = E > 0 ? &bt->attr[E * q] : NULL;
    return;
  }
  int64_t bk = q - B;
  for (int c = 0; c < 3; ++c) g[c] = -g[c] * w[3 * bk + c] / (double)bt->N;
  *x3 = &bt->x2[3 * bk];
  *d3 = &bt->dir2[3 * bk];
  *e = E > 0 ? &bt->attr2[E * bk] : NULL;
}

/* Gradient of the loss scaled by grad_loss. With the target detached (the
 * paper's choice) only the LHS query receives the seed
 * 2 r grad_loss / (3B) (divided by the squared normaliser for the relative
 * loss). With grad_through_rhs each RHS query (b, k) also receives
 * -seed_b * w_bk / N.
 * Queries are processed in blocks: the per-query reverse passes of a block
 * run in parallel (each thread adds into its own dW/db), then the block's
 * feature-gradient shares are added in query order on one thread, and at the
 * end the threads' dW/db are summed in thread order. */
#define ORA_BWD_BLOCK 16384
int ora_residual_bwd(const ora_tree* t, const ora_mlp* m, const ora_batch* bt, double grad_loss,
                     double* const* dfeat, double* const* dW, double* const* db,
                     double* dtables, double* const* gdW, double* const* gdb, double* dd_out,
                     int32_t nthreads) {
  int rc = check_inputs(t, m, bt);
  if (rc) return rc;
  int64_t B = bt->B;
  int32_t N = bt->N;
  if (B == 0) return 0;
  int nt = 1;
#ifdef _OPENMP
  nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  (void)nthreads;
  const ora_mlp* gm = (t->interp == ORA_INTERP_PAPER && t->disp) ? &t->disp->mlp : NULL;
  if (gm && (!dtables || !gdW || !gdb)) return -1;
  int64_t P = 0, PG = 0;
  for (int32_t i = 0; i < m->n_layers; ++i) P += (int64_t)m->dims[i + 1] * (m->dims[i] + 1);
  if (gm)
    for (int32_t i = 0; i < gm->n_layers; ++i) PG += (int64_t)gm->dims[i + 1] * (gm->dims[i] + 1);
  P += PG;
  int32_t K0 = m->dims[0];
  double* lhs = (double*)malloc((size_t)(3 * B) * sizeof(double));
  double* T = (double*)malloc((size_t)(3 * B) * sizeof(double));
  double* r = (double*)malloc((size_t)(3 * B) * sizeof(double));
  double* w = NULL;
  double* priv = (double*)calloc((size_t)nt * (size_t)P, sizeof(double));
  query_taps* qts = (query_taps*)malloc((size_t)ORA_BWD_BLOCK * sizeof(query_taps));
  double* dhs = (double*)malloc((size_t)ORA_BWD_BLOCK * (size_t)K0 * sizeof(double));
  if (!lhs || !T || !r || !priv || !qts || !dhs) { rc = -5; goto done; }
  rc = residual_parts(t, m, bt, lhs, T, r, nthreads);
  if (rc) goto done;
  int full = bt->grad_through_rhs && !bt->target_override && N > 0;
  if (full) {
    w = (double*)malloc((size_t)(3 * B * N) * sizeof(double));
    if (!w) { rc = -5; goto done; }
    ora_bsdf_weight(bt, w);
  }
  int64_t Qb = full ? B * (1 + N) : B;
  for (int64_t q0 = 0; q0 < Qb; q0 += ORA_BWD_BLOCK) {
    int64_t nq = Qb - q0 < ORA_BWD_BLOCK ? Qb - q0 : ORA_BWD_BLOCK;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      double* mine = priv + (int64_t)tid * P;
      double* pdW[ORA_MAX_LAYERS];
      double* pdb[ORA_MAX_LAYERS];
      double* pgW[ORA_MAX_LAYERS];
      double* pgb[ORA_MAX_LAYERS];
      int64_t o = 0;
      for (int32_t i = 0; i < m->n_layers; ++i) {
        pdW[i] = mine + o;
        o += (int64_t)m->dims[i + 1] * m->dims[i];
        pdb[i] = mine + o;
        o += m->dims[i + 1];
      }
      for (int32_t i = 0; gm && i < gm->n_layers; ++i) {
        pgW[i] = mine + o;
        o += (int64_t)gm->dims[i + 1] * gm->dims[i];
        pgb[i] = mine + o;
        o += gm->dims[i + 1];
      }
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
      for (int64_t j = 0; j < nq; ++j) {
        double g[3];
        const float *x3, *d3, *e;
        query_seed(bt, attr_dims(t, m), lhs, T, r, w, grad_loss, q0 + j, g, &x3, &d3, &e);
        backprop_query(t, m, x3, d3, e, g, pdW, pdb, pgW, pgb, &qts[j], &dhs[j * K0]);
      }
    }
    for (int64_t j = 0; j < nq; ++j) scatter_query(t, &qts[j], &dhs[j * K0], dfeat, dtables);
    if (gm && dd_out)
      for (int64_t j = 0; j < nq; ++j) dd_out[q0 + j] = qts[j].dd;
  }
  for (int th = 0; th < nt; ++th) {
    const double* mine = priv + (int64_t)th * P;
    int64_t o = 0;
    for (int32_t i = 0; i < m->n_layers; ++i) {
      int64_t nw = (int64_t)m->dims[i + 1] * m->dims[i];
      for (int64_t e = 0; e < nw; ++e) dW[i][e] += mine[o + e];
      o += nw;
      for (int32_t e = 0; e < m->dims[i + 1]; ++e) db[i][e] += mine[o + e];
      o += m->dims[i + 1];
    }
    for (int32_t i = 0; gm && i < gm->n_layers; ++i) {
      int64_t nw = (int64_t)gm->dims[i + 1] * gm->dims[i];
      for (int64_t e = 0; e < nw; ++e) gdW[i][e] += mine[o + e];
      o += nw;
      for (int32_t e = 0; e < gm->dims[i + 1]; ++e) gdb[i][e] += mine[o + e];
      o += gm->dims[i + 1];
    }
  }
done:
  free(lhs);
  free(T);
  free(r);
  free(w);
  free(priv);
  free(qts);
  free(dhs);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Optimiser step over the FP32 masters                                      */
/* ------------------------------------------------------------------------ */

/* Adam as stated by Kingma and Ba (Algorithm 1), with the bias corrections
 * written out; blocks of a feature table whose node no query read are left
 * alone (their gradient is zero, and their moments are not decayed). */
void ora_adam(float* p, const float* g, float* m, float* v, int64_t n, const uint32_t* touched, int64_t block,
              int32_t t, double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    if (touched && !touched[i / block]) continue;
    double gi = (double)g[i];
    double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
    double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
    double step = lr * (mi / c1) / (sqrt(vi / c2) + eps);
    m[i] = (float)mi;
    v[i] = (float)vi;
    p[i] = (float)((double)p[i] - step);
  }
}
