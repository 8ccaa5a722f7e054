// C-ABI of liboctaoctree: argument validation, host octree construction,
// workspace layout and kernel dispatch. Declarations and their contracts are
// in include/octaoctree.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "octaoctree.h"
#include "oo_internal.h"

using namespace oo;

namespace {

thread_local char g_err[512] = "";

// The backward runs in up to kMaxChunks chunks of at least kChunkQueries
// sorted positions; the feature scatter of chunk c runs on a second stream
// while the backward kernel works on chunk c + 1 (the scatter is bound by
// the memory-side atomic units, the backward by latency, so they overlap).
constexpr int kMaxChunks = 4;
constexpr int64_t kChunkQueries = 32768;

int bwd_chunks(int64_t Qb) {
  int64_t n = Qb / kChunkQueries;
  return (int)(n < 1 ? 1 : (n > kMaxChunks ? kMaxChunks : n));
}


int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return OO_OK;
  return fail(OO_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// --- opt-in launch timing ----------------------------------------------------
// While enabled, every kernel launch group records a pair of events on the
// caller's stream around itself; oo_profile_end sums their elapsed times per
// kind.
const char* const kProfNames[OO_PROF_KINDS] = {"bucket_sort", "query",    "combine",   "seeds",
                                               "transpose",   "backward", "scatter",   "dw_reduce",
                                               "cast",        "encode",   "mlp_decode"};

struct Profiler {
  std::mutex m;
  bool on = false;
  std::vector<hipEvent_t> ev;  // 2 per slot
  std::vector<int> kind;
  int used = 0;
};
Profiler g_prof;

struct ProfScope {
  int slot = -1;
  hipStream_t st;
  ProfScope(int kind, hipStream_t s) : st(s) {
    std::lock_guard<std::mutex> lk(g_prof.m);
    if (!g_prof.on || g_prof.used >= (int)g_prof.kind.size()) return;
    slot = g_prof.used++;
    g_prof.kind[slot] = kind;
    (void)hipEventRecord(g_prof.ev[2 * slot], st);
  }
  ~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], st);
  }
};

// Second stream per device for the overlapped feature scatter, with the
// events that order it against the caller's stream. Created on first use at
// the default priority; the enqueue sequence that uses it is serialised.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ev[kMaxChunks + 1] = {};
};
std::mutex g_side_m;
SideStream g_side[64];

hipError_t side_stream(SideStream*& out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  SideStream& S = g_side[dev];
  if (!S.s) {
    if ((e = hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking)) != hipSuccess) return e;
    for (auto& ev : S.ev)
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  }
  out = &S;
  return hipSuccess;
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

int check_tree(const oo_tree* t, TreeArgs& A) {
  if (!t) return fail(OO_EINVAL, "tree is NULL");
  if (t->n_levels < 1 || t->n_levels > OO_MAX_LEVELS)
    return fail(OO_EINVAL, "n_levels must be in [1, %d], got %d", OO_MAX_LEVELS, t->n_levels);
  if (t->C != 4 && t->C != 8) return fail(OO_EINVAL, "C must be 4 or 8, got %d", t->C);
  if (t->feat_dtype != OO_F32 && t->feat_dtype != OO_F16 && t->feat_dtype != OO_BF16)
    return fail(OO_EINVAL, "unknown feat_dtype %d", (int)t->feat_dtype);
  if (!t->nodes) return fail(OO_EINVAL, "nodes is NULL");
  if (t->interp != OO_INTERP_NODE_BILINEAR && t->interp != OO_INTERP_PAPER)
    return fail(OO_EINVAL, "interp must be OO_INTERP_NODE_BILINEAR or OO_INTERP_PAPER, got %d", t->interp);
  if (t->level_offset[0] != 0 || t->level_offset[1] != 1)
    return fail(OO_EINVAL, "level_offset must start 0, 1 (one root node)");
  A.L = t->n_levels;
  A.C = t->C;
  A.D = t->n_levels - 1;
  A.interp = t->interp;
  A.nodes = t->nodes;
  for (int l = 0; l < OO_MAX_LEVELS; ++l) {
    A.res[l] = 2;
    A.feat[l] = nullptr;
  }
  for (int l = 0; l <= OO_MAX_LEVELS; ++l) A.off[l] = l <= t->n_levels ? t->level_offset[l] : t->level_offset[t->n_levels];
  // vertex maps reach 2^8 + 1 vertices per side in the paper's configuration
  const int rmax = t->interp == OO_INTERP_PAPER ? 512 : 64;
  for (int l = 0; l < t->n_levels; ++l) {
    if (!pow2_in(t->res[l], 2, rmax))
      return fail(OO_EINVAL, "res[%d] = %d is not a power of two in [2, %d]", l, t->res[l], rmax);
    if (t->level_offset[l + 1] < t->level_offset[l]) return fail(OO_EINVAL, "level_offset must be non-decreasing");
    A.res[l] = t->res[l];
    const bool has_nodes = t->level_offset[l + 1] > t->level_offset[l];
    if (has_nodes) {
      if (!t->feat[l]) return fail(OO_EINVAL, "feat[%d] is NULL", l);
      if (reinterpret_cast<uintptr_t>(t->feat[l]) % 16) return fail(OO_EINVAL, "feat[%d] is not 16-byte aligned", l);
      A.feat[l] = t->feat[l];
    }
  }
  if (t->level_offset[t->n_levels] > (int64_t(1) << 24))
    return fail(OO_EUNSUPPORTED, "more than 2^24 nodes");
  // Levels without nodes, and the unused slots past n_levels, are never read
  // with a non-zero weight; point them at level 0 so that the kernels'
  // predicated loads (texel 0) stay in bounds.
  for (int l = 0; l < OO_MAX_LEVELS; ++l)
    if (!A.feat[l]) A.feat[l] = A.feat[0];
  return OO_OK;
}

// LC: the level features' width n_levels * C; the rest of dims[0] are the
// decoder's surface attributes.
int check_mlp(const oo_mlp* m, int LC, MlpArgs& A) {
  if (!m) return fail(OO_EINVAL, "mlp is NULL");
  if (m->n_layers < 2 || m->n_layers > 5) return fail(OO_EUNSUPPORTED, "n_layers must be in [2, 5], got %d", m->n_layers);
  if (m->dtype != OO_F32 && m->dtype != OO_F16 && m->dtype != OO_BF16)
    return fail(OO_EINVAL, "unknown mlp dtype %d", (int)m->dtype);
  const int K0 = m->dims[0];
  if (K0 < LC) return fail(OO_EINVAL, "dims[0] = %d is smaller than n_levels * C = %d", K0, LC);
  if (K0 > 128) return fail(OO_EUNSUPPORTED, "input width %d > 128", K0);
  if (K0 % 4) return fail(OO_EUNSUPPORTED, "input width %d must be a multiple of 4 (pad the attributes)", K0);
  if (m->dims[m->n_layers] != 3) return fail(OO_EINVAL, "last dim must be 3, got %d", m->dims[m->n_layers]);
  const int H = m->dims[1];
  for (int i = 1; i < m->n_layers; ++i)
    if (m->dims[i] != H) return fail(OO_EUNSUPPORTED, "hidden widths must all be equal");
  if (H != 64 && H != 128) return fail(OO_EUNSUPPORTED, "hidden width must be 64 or 128, got %d", H);
  for (int i = 0; i < m->n_layers; ++i)
    if (!m->W[i] || !m->b[i]) return fail(OO_EINVAL, "W[%d] or b[%d] is NULL", i, i);
  A.n_layers = m->n_layers;
  A.K0 = K0;
  A.E = K0 - LC;
  A.H = H;
  A.n_out = 3;
  for (int i = 0; i < OO_MAX_LAYERS; ++i) {
    A.W[i] = i < m->n_layers ? m->W[i] : nullptr;
    A.b[i] = i < m->n_layers ? m->b[i] : nullptr;
  }
  return OO_OK;
}

// The disparity predictor of the paper's scheme (G.n_levels = 0 without
// one). grads: the call differentiates, so the gradient accumulators are
// required too.
int check_disparity(const oo_tree* t, DispArgs& G, bool grads) {
  G = DispArgs{};
  const oo_disparity* p = t->disparity;
  if (!p) return OO_OK;
  if (t->interp != OO_INTERP_PAPER) return fail(OO_EINVAL, "a disparity predictor needs interp = OO_INTERP_PAPER");
  if (p->n_levels != kHashLevels)
    return fail(OO_EUNSUPPORTED, "disparity n_levels must be %d, got %d", kHashLevels, p->n_levels);
  if (p->F != kDispF) return fail(OO_EUNSUPPORTED, "disparity F must be %d, got %d", kDispF, p->F);
  if (p->log2_T < 1 || p->log2_T > 24) return fail(OO_EINVAL, "disparity log2_T must be in [1, 24], got %d", p->log2_T);
  if (!p->tables || reinterpret_cast<uintptr_t>(p->tables) % 8)
    return fail(OO_EINVAL, "disparity tables must be non-NULL and 8-byte aligned");
  if (p->n_layers != 2 && p->n_layers != 3)
    return fail(OO_EUNSUPPORTED, "disparity n_layers must be 2 or 3, got %d", p->n_layers);
  const int K = p->n_levels * p->F + 4;
  if (p->dims[0] != K) return fail(OO_EINVAL, "disparity dims[0] = %d must be n_levels F + 4 = %d", p->dims[0], K);
  for (int i = 1; i < p->n_layers; ++i)
    if (p->dims[i] != kDispH) return fail(OO_EUNSUPPORTED, "disparity hidden widths must be %d", kDispH);
  if (p->dims[p->n_layers] != 1) return fail(OO_EINVAL, "disparity output width must be 1");
  G.n_levels = p->n_levels;
  G.log2_T = p->log2_T;
  G.n_layers = p->n_layers;
  G.K = K;
  G.tables = p->tables;
  G.dense_mask = 0;
  for (int i = 0; i < p->n_levels; ++i) {
    if (p->res[i] < 1 || p->res[i] > (1 << 20))
      return fail(OO_EINVAL, "disparity res[%d] = %d must be in [1, 2^20]", i, p->res[i]);
    G.res[i] = p->res[i];
    const uint64_t n1 = (uint64_t)p->res[i] + 1;
    if (n1 * n1 * n1 <= (uint64_t(1) << p->log2_T)) G.dense_mask |= 1u << i;
  }
  for (int i = 0; i < p->n_layers; ++i) {
    if (!p->W[i] || !p->b[i]) return fail(OO_EINVAL, "disparity W[%d] or b[%d] is NULL", i, i);
    G.W[i] = p->W[i];
    G.b[i] = p->b[i];
    if (grads && (!p->dW[i] || !p->db[i])) return fail(OO_EINVAL, "disparity dW[%d] or db[%d] is NULL", i, i);
  }
  if (grads && !p->dtables) return fail(OO_EINVAL, "disparity dtables is NULL");
  return OO_OK;
}

int check_pair(const oo_tree* t, const oo_mlp* m) {
  if (t->feat_dtype != m->dtype)
    return fail(OO_EUNSUPPORTED, "feature dtype %d and MLP dtype %d must match", (int)t->feat_dtype, (int)m->dtype);
  return OO_OK;
}

int check_batch(const oo_residual_batch* b, ResidualArgs& A) {
  if (!b) return fail(OO_EINVAL, "batch is NULL");
  if (b->B < 0 || b->N < 0) return fail(OO_EINVAL, "B and N must be >= 0");
  if (b->loss_kind != 0 && b->loss_kind != 1) return fail(OO_EINVAL, "loss_kind must be 0 or 1");
  if (b->B > 0) {
    if (!b->x || !b->dir) return fail(OO_EINVAL, "x and dir are required");
    if (!b->target_override) {
      if (!b->Le) return fail(OO_EINVAL, "Le is required without target_override");
      if (b->N > 0 && (!b->n || !b->wo || !b->albedo || !b->rough || !b->x2 || !b->dir2 || !b->wi))
        return fail(OO_EINVAL, "n, wo, albedo, rough, x2, dir2 and wi are required when N > 0");
    }
  }
  A.B = b->B;
  A.N = b->target_override ? 0 : b->N;
  A.n = b->n;
  A.wo = b->wo;
  A.albedo = b->albedo;
  A.Le = b->Le;
  A.rough = b->rough;
  A.wi = b->wi;
  A.pdf = b->pdf;
  A.target_override = b->target_override;
  A.F0 = b->F0;
  A.loss_kind = b->loss_kind;
  A.eps = b->eps;
  return OO_OK;
}

// The surface attributes that the decoder reads: of the LHS queries, and of
// the secondary hits when the RHS is estimated.
int check_attrs(const oo_residual_batch* b, const ResidualArgs& A, const MlpArgs& M) {
  if (M.E == 0 || A.B == 0) return OO_OK;
  if (!b->attr) return fail(OO_EINVAL, "attr is required: the decoder reads %d surface attributes", M.E);
  if (A.N > 0 && !b->attr2) return fail(OO_EINVAL, "attr2 is required when N > 0 without target_override");
  return OO_OK;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Workspace {
  size_t Lq, lossp, seeds, nidx, uv, pos, dh, wt[OO_MAX_LAYERS], dwp, order, rank, scount, stotal, sstart, gpad, total;
  size_t wdir, dd, gdwp, dsp, drows, hrows;  // the disparity predictor's: lookup directions, dLoss/d
                                             // disparity, parameter partials, disparity of every query,
                                             // backward rows, decoder input rows
  int ggrid;
  int64_t dcap;  // queries per pass of the predictor's backward
  int K;  // node indices stored per level and backward query: 1, or 8 corners in the paper's scheme
  int64_t pad_off[OO_MAX_LEVELS];  // float offset of each level's pair buffer in gpad, or -1
  int64_t pad_total;               // floats in gpad
  int64_t Qb;
  int grid;
  ParamLayout PL;
};

void param_layout(const MlpArgs& M, ParamLayout& PL) {
  PL.n_layers = M.n_layers;
  int64_t off = 0;
  for (int i = 0; i < M.n_layers; ++i) {
    PL.n_in[i] = i == 0 ? M.K0 : M.H;
    PL.n_out[i] = i == M.n_layers - 1 ? 3 : M.H;
    PL.w_off[i] = off;
    off += (int64_t)PL.n_in[i] * PL.n_out[i];
    PL.b_off[i] = off;
    off += PL.n_out[i];
  }
  PL.P = off;
}

// Levels whose feature gradients go through pair buffers: the leading
// levels with maps of at least 8x8 texels whose buffers fit in 64 MiB
// together. There a footprint row always costs one 64-byte atomic request
// instead of 1.5 on average; their tables are small and nearly every query
// touches them, so the clear and the fold cost little.
constexpr size_t kPadBudget = size_t(64) << 20;

Workspace workspace_layout(const MlpArgs& M, oo_dtype md, const oo_residual_batch* b, const oo_tree* tree) {
  Workspace w;
  const int L = tree->n_levels;
  const int64_t B = b->B;
  const int N = b->target_override ? 0 : b->N;
  const int64_t Qf = B * (1 + N);
  const bool full = b->grad_through_rhs && !b->target_override && N > 0;
  const int64_t Qb = full ? Qf : B;
  param_layout(M, w.PL);
  w.grid = bwd_grid(M, md, L, Qb);
  size_t o = 0;
  w.Lq = o;
  o = align256(o + (size_t)Qf * 3 * sizeof(float));
  w.lossp = o;
  o = align256(o + (size_t)(combine_blocks(B, N) + 1) * sizeof(double));
  w.seeds = o;
  o = align256(o + (size_t)Qb * 3 * sizeof(float));
  w.Qb = Qb;
  const bool paper = tree->interp == OO_INTERP_PAPER;
  w.K = paper ? 8 : 1;
  // node index per level of every backward query, written by the forward,
  // [L][Qb] (paper's scheme: the eight corner cells' nodes, [L][8][Qb])
  w.nidx = o;
  o = align256(o + (size_t)Qb * L * w.K * sizeof(int32_t));
  w.uv = o;  // octahedral coordinates of every backward query, written by the forward, [Qb]
  o = align256(o + (size_t)Qb * sizeof(float2));
  w.pos = o;  // paper's scheme: position of every backward query, [Qb]
  o = align256(o + (paper ? (size_t)Qb * sizeof(float4) : 0));
  w.dh = o;  // dLoss/dh of every backward query, [Qb][L C] FP32
  o = align256(o + (size_t)Qb * L * tree->C * sizeof(float));
  // with the disparity predictor: unit lookup direction [Qb] float4 and
  // dLoss/d disparity [Qb] of every backward query, and the predictor's
  // parameter partials [ggrid][P]
  const bool shift = paper && tree->disparity;
  w.ggrid = shift ? disparity_bwd_grid(Qb) : 0;
  w.wdir = o;
  o = align256(o + (shift ? (size_t)Qb * sizeof(float4) : 0));
  w.dd = o;
  o = align256(o + (shift ? (size_t)Qb * sizeof(float) : 0));
  w.dsp = o;  // [Qf], sorted order
  o = align256(o + (shift ? (size_t)Qf * sizeof(float) : 0));
  w.hrows = o;  // decoder input rows of the shifted encode, [Qf][K0] in the MLP's dtype
  o = align256(o + (shift ? (size_t)Qf * M.K0 * (md == OO_F32 ? 4 : 2) : 0));
  w.gdwp = o;
  if (shift) {
    const oo_disparity* p = tree->disparity;
    size_t P = (size_t)p->dims[1] * p->dims[0] + p->dims[1] + (size_t)p->dims[p->n_layers] * p->dims[p->n_layers - 1] +
               p->dims[p->n_layers];
    if (p->n_layers == 3) P += (size_t)p->dims[2] * p->dims[1] + p->dims[2];
    o = align256(o + (size_t)w.ggrid * P * sizeof(float));
  }
  w.dcap = shift ? disparity_rows_cap(Qb) : 0;
  w.drows = o;
  o = align256(o + (size_t)disparity_rows_floats(w.dcap) * sizeof(float));
  const size_t esz = md == OO_F32 ? 4 : 2;
  for (int i = 0; i < M.n_layers; ++i) {
    w.wt[i] = o;
    o = align256(o + (size_t)w.PL.n_in[i] * ((w.PL.n_out[i] + 3) & ~3) * esz);
  }
  w.dwp = o;  // dW/db partials, [grid][P], accumulated over the backward's chunks
  o = align256(o + (size_t)w.grid * w.PL.P * sizeof(float));
  // spatially bucketed queries, written by the forward and read by both passes
  const SortShape ss = sort_shape(Qf, L - 1);
  w.order = o;
  o = align256(o + (size_t)Qf * sizeof(int32_t));
  w.rank = o;
  o = align256(o + (size_t)Qf * sizeof(int32_t));
  w.scount = o;
  o = align256(o + (size_t)ss.NB * ss.K * sizeof(int32_t));
  w.stotal = o;
  o = align256(o + (size_t)ss.K * sizeof(int32_t));
  w.sstart = o;
  o = align256(o + (size_t)ss.K * sizeof(int32_t));
  // coarse-level pair buffers of the feature-gradient scatter
  w.gpad = o;
  w.pad_total = 0;
  bool open = tree->C == 8 && !paper;  // the paper's scheme scatters to vertices directly
  for (int l = 0; l < OO_MAX_LEVELS; ++l) {
    w.pad_off[l] = -1;
    if (l >= L || !open) continue;
    const int R = tree->res[l];
    const int64_t nodes = tree->level_offset[l + 1] - tree->level_offset[l];
    const int64_t f = pad_floats(R, nodes, tree->C);
    if (R < 8 || (size_t)(w.pad_total + f) * sizeof(float) > kPadBudget) {
      open = false;
      continue;
    }
    w.pad_off[l] = w.pad_total;
    w.pad_total += f;
  }
  o = align256(o + (size_t)w.pad_total * sizeof(float));
  w.total = o;
  return w;
}

// --- host octree construction ---------------------------------------------
// Morton codes of the samples' finest cells, sorted once: every node is then
// a contiguous run of the sorted codes sharing a prefix, and its children are
// the sub-runs split by the next octant digit, already in octant order.

inline int64_t quant_host(float v, int D) {
  const float scale = (float)(1u << D);
  float f = std::floor(v * scale);
  if (!(f >= 0.0f)) f = 0.0f;
  if (f > scale - 1.0f) f = scale - 1.0f;
  return (int64_t)f;
}

inline uint64_t morton3(uint64_t x, uint64_t y, uint64_t z, int D) {
  uint64_t code = 0;
  for (int bit = 0; bit < D; ++bit) {
    code |= ((x >> bit) & 1ull) << (3 * bit);
    code |= ((y >> bit) & 1ull) << (3 * bit + 1);
    code |= ((z >> bit) & 1ull) << (3 * bit + 2);
  }
  return code;
}

}  // namespace

extern "C" {

const char* oo_last_error(void) { return g_err; }

int oo_profile_begin(int32_t capacity) {
  g_err[0] = 0;
  if (capacity < 1 || capacity > (1 << 20)) return fail(OO_EINVAL, "capacity must be in [1, 2^20]");
  std::lock_guard<std::mutex> lk(g_prof.m);
  if (g_prof.on) return fail(OO_EINVAL, "profiling already enabled");
  g_prof.ev.assign(2 * (size_t)capacity, nullptr);
  for (auto& e : g_prof.ev) {
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      for (auto& x : g_prof.ev)
        if (x) (void)hipEventDestroy(x);
      g_prof.ev.clear();
      return hip_status(r, "hipEventCreate");
    }
  }
  g_prof.kind.assign(capacity, -1);
  g_prof.used = 0;
  g_prof.on = true;
  return OO_OK;
}

int oo_profile_end(double* total_ms, int64_t* launches) {
  g_err[0] = 0;
  std::lock_guard<std::mutex> lk(g_prof.m);
  if (!g_prof.on) return fail(OO_EINVAL, "profiling is not enabled");
  int rc = OO_OK;
  for (int k = 0; k < OO_PROF_KINDS; ++k) {
    if (total_ms) total_ms[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  for (int i = 0; i < g_prof.used && rc == OO_OK; ++i) {
    hipError_t r = hipEventSynchronize(g_prof.ev[2 * i + 1]);
    float ms = 0.0f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]);
    if (r != hipSuccess) {
      rc = hip_status(r, "profile event");
      break;
    }
    if (total_ms) total_ms[g_prof.kind[i]] += ms;
    if (launches) launches[g_prof.kind[i]] += 1;
  }
  for (auto& e : g_prof.ev) (void)hipEventDestroy(e);
  g_prof.ev.clear();
  g_prof.kind.clear();
  g_prof.used = 0;
  g_prof.on = false;
  return rc;
}

const char* oo_profile_kind_name(int32_t kind) { return kind >= 0 && kind < OO_PROF_KINDS ? kProfNames[kind] : ""; }

int oo_build_octree(const float* samples, int64_t n, int32_t max_depth, int32_t split_threshold, uint32_t* nodes_out,
                    int64_t capacity, int64_t* level_offset_out, int64_t* n_nodes_out) {
  g_err[0] = 0;
  if (n < 0) return fail(OO_EINVAL, "n must be >= 0");
  if (max_depth < 0 || max_depth > OO_MAX_LEVELS - 1) return fail(OO_EINVAL, "max_depth must be in [0, %d]", OO_MAX_LEVELS - 1);
  if (split_threshold < 0) return fail(OO_EINVAL, "split_threshold must be >= 0");
  if ((n > 0 && !samples) || !level_offset_out || !n_nodes_out) return fail(OO_EINVAL, "NULL argument");
  const int D = max_depth;
  std::vector<uint64_t> code((size_t)n);
  for (int64_t i = 0; i < n; ++i)
    code[i] = morton3(quant_host(samples[3 * i], D), quant_host(samples[3 * i + 1], D),
                      quant_host(samples[3 * i + 2], D), D);
  std::sort(code.begin(), code.end());

  struct Node {
    int64_t lo, hi;
    uint32_t word;
  };
  std::vector<Node> nodes;
  nodes.push_back({0, n, 0u});
  std::vector<int64_t> lo(D + 2, 0);
  lo[0] = 0;
  lo[1] = 1;
  for (int l = 0; l < D; ++l) {
    const int shift = 3 * (D - l - 1);
    for (int64_t v = lo[l]; v < lo[l + 1]; ++v) {
      const int64_t a = nodes[v].lo, b = nodes[v].hi;
      if (b - a <= split_threshold) continue;
      const int64_t first = (int64_t)nodes.size();
      uint32_t mask = 0;
      int64_t s = a;
      while (s < b) {
        const unsigned o = (unsigned)((code[s] >> shift) & 7ull);
        const uint64_t key = code[s] >> shift;
        int64_t e = s;
        while (e < b && (code[e] >> shift) == key) ++e;
        mask |= 1u << o;
        nodes.push_back({s, e, 0u});
        s = e;
      }
      nodes[v].word = ((uint32_t)first << 8) | mask;
    }
    lo[l + 2] = (int64_t)nodes.size();
  }
  const int64_t total = (int64_t)nodes.size();
  for (int l = 0; l <= D + 1; ++l) level_offset_out[l] = lo[l];
  *n_nodes_out = total;
  if (total > (int64_t(1) << 24)) return fail(OO_EUNSUPPORTED, "tree needs %lld nodes (> 2^24)", (long long)total);
  if (!nodes_out) return OO_OK;
  if (capacity < total) return fail(OO_ECAPACITY, "capacity %lld < %lld nodes", (long long)capacity, (long long)total);
  for (int64_t v = 0; v < total; ++v) nodes_out[v] = nodes[v].word;
  return OO_OK;
}

int oo_encode_query(const oo_tree* tree, const float* x, const float* dir, int64_t B, void* h_out, oo_dtype h_dtype,
                    int32_t* node_idx_out, hipStream_t stream) {
  g_err[0] = 0;
  TreeArgs T;
  int rc = check_tree(tree, T);
  if (rc) return rc;
  if (B < 0) return fail(OO_EINVAL, "B must be >= 0");
  if (h_dtype != OO_F32 && h_dtype != OO_F16 && h_dtype != OO_BF16) return fail(OO_EINVAL, "unknown h_dtype");
  DispArgs G;
  if ((rc = check_disparity(tree, G, false))) return rc;
  if (G.n_levels > 0 && h_dtype != OO_F32)
    return fail(OO_EUNSUPPORTED, "the shifted encoding writes FP32 features only");
  if (B == 0) return OO_OK;
  if (!x || !dir || !h_out) return fail(OO_EINVAL, "x, dir and h_out are required");
  ProfScope ps(OO_PROF_ENCODE, stream);
  return hip_status(launch_encode(T, tree->feat_dtype, x, dir, B, h_out, h_dtype, node_idx_out, G, stream),
                    "encode_query launch");
}

int oo_mlp_fwd(const oo_mlp* mlp, const void* h, oo_dtype h_dtype, int64_t B, float* rgb_out, hipStream_t stream) {
  g_err[0] = 0;
  if (!mlp) return fail(OO_EINVAL, "mlp is NULL");
  MlpArgs M;
  int rc = check_mlp(mlp, mlp->dims[0], M);
  if (rc) return rc;
  if (h_dtype != mlp->dtype) return fail(OO_EINVAL, "h_dtype must equal mlp->dtype");
  if (B < 0) return fail(OO_EINVAL, "B must be >= 0");
  if (B == 0) return OO_OK;
  if (!h || !rgb_out) return fail(OO_EINVAL, "h and rgb_out are required");
  ProfScope ps(OO_PROF_MLP, stream);
  return hip_status(launch_mlp(M, mlp->dtype, h, B, rgb_out, stream), "mlp_fwd launch");
}

int oo_query_fwd(const oo_tree* tree, const oo_mlp* mlp, const float* x, const float* dir, const float* attr, int64_t B,
                 float* rgb_out, hipStream_t stream) {
  g_err[0] = 0;
  TreeArgs T;
  MlpArgs M;
  int rc = check_tree(tree, T);
  if (rc) return rc;
  if ((rc = check_mlp(mlp, tree->n_levels * tree->C, M))) return rc;
  if ((rc = check_pair(tree, mlp))) return rc;
  DispArgs G;
  if ((rc = check_disparity(tree, G, false))) return rc;
  if (B < 0) return fail(OO_EINVAL, "B must be >= 0");
  if (B == 0) return OO_OK;
  if (!x || !dir || !rgb_out) return fail(OO_EINVAL, "x, dir and rgb_out are required");
  if (M.E > 0 && !attr) return fail(OO_EINVAL, "attr is required: the decoder reads %d surface attributes", M.E);
  QuerySrc src{x, dir, B, x, dir};
  src.gA = src.gB = attr;
  src.E = M.E;
  ProfScope ps(OO_PROF_QUERY, stream);
  const QueryOut O{nullptr, nullptr, nullptr, nullptr, 0};
  return hip_status(launch_query(T, tree->feat_dtype, M, mlp->dtype, src, B, rgb_out, O, G, stream),
                    "query_fwd launch");
}

int oo_residual_workspace_bytes(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch, size_t* bytes) {
  g_err[0] = 0;
  TreeArgs T;
  MlpArgs M;
  ResidualArgs A;
  int rc = check_tree(tree, T);
  if (rc) return rc;
  if ((rc = check_mlp(mlp, tree->n_levels * tree->C, M))) return rc;
  if ((rc = check_pair(tree, mlp))) return rc;
  if ((rc = check_batch(batch, A))) return rc;
  DispArgs G;
  if ((rc = check_disparity(tree, G, false))) return rc;
  if (!bytes) return fail(OO_EINVAL, "bytes is NULL");
  *bytes = workspace_layout(M, mlp->dtype, batch, tree).total;
  return OO_OK;
}

int oo_radiosity_residual_fwd(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch, float* lhs_out,
                              float* rhs_out, float* resid_out, double* loss_out, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
  g_err[0] = 0;
  TreeArgs T;
  MlpArgs M;
  ResidualArgs A;
  int rc = check_tree(tree, T);
  if (rc) return rc;
  if ((rc = check_mlp(mlp, tree->n_levels * tree->C, M))) return rc;
  if ((rc = check_pair(tree, mlp))) return rc;
  if ((rc = check_batch(batch, A))) return rc;
  if ((rc = check_attrs(batch, A, M))) return rc;
  DispArgs G;
  if ((rc = check_disparity(tree, G, false))) return rc;
  if (!loss_out || !workspace) return fail(OO_EINVAL, "loss_out and workspace are required");
  if (A.B > 0 && (!lhs_out || !rhs_out || !resid_out)) return fail(OO_EINVAL, "lhs_out, rhs_out, resid_out are required");
  const Workspace w = workspace_layout(M, mlp->dtype, batch, tree);
  if (workspace_bytes < w.total)
    return fail(OO_EINVAL, "workspace of %zu bytes is smaller than the %zu this problem needs", workspace_bytes,
                w.total);
  char* ws = static_cast<char*>(workspace);
  float* Lq = reinterpret_cast<float*>(ws + w.Lq);
  double* lossp = reinterpret_cast<double*>(ws + w.lossp);
  int32_t* nidx = reinterpret_cast<int32_t*>(ws + w.nidx);
  const int64_t Q = A.B * (1 + A.N);
  if (Q > INT32_MAX) return fail(OO_EUNSUPPORTED, "B (1 + N) = %lld exceeds 2^31 - 1 queries", (long long)Q);
  QuerySrc src{batch->x, batch->dir, A.B, A.N > 0 ? batch->x2 : batch->x, A.N > 0 ? batch->dir2 : batch->dir};
  src.gA = batch->attr;
  src.gB = A.N > 0 ? batch->attr2 : batch->attr;
  src.E = M.E;
  // bucket the queries by octree cell (LHS first) and evaluate them in that
  // order: Lq and the stored node indices are in sorted order
  int32_t* order = reinterpret_cast<int32_t*>(ws + w.order);
  int32_t* rank = reinterpret_cast<int32_t*>(ws + w.rank);
  hipError_t e;
  {
    ProfScope ps(OO_PROF_SORT, stream);
    e = launch_spatial_sort(src, Q, A.B, tree->n_levels - 1, reinterpret_cast<int32_t*>(ws + w.scount),
                            reinterpret_cast<int32_t*>(ws + w.stotal), reinterpret_cast<int32_t*>(ws + w.sstart),
                            order, rank, stream);
  }
  if (e != hipSuccess) return hip_status(e, "query bucketing launch");
  QuerySrc sorted = src;
  sorted.idx = order;
  sorted.n = Q;
  {
    ProfScope ps(OO_PROF_QUERY, stream);
    QueryOut O{nidx, reinterpret_cast<float2*>(ws + w.uv), reinterpret_cast<float4*>(ws + w.pos),
               G.n_levels ? reinterpret_cast<float4*>(ws + w.wdir) : nullptr, w.Qb};
    if (G.n_levels) {
      // every query's disparity on the matrix cores, the shifted encode into
      // decoder input rows, then the decoder over the rows
      float* dsp = reinterpret_cast<float*>(ws + w.dsp);
      e = launch_disparity_fwd(G, mlp->dtype, sorted, Q, dsp, stream);
      if (e != hipSuccess) return hip_status(e, "disparity launch");
      O.disp = dsp;
      void* hrows = ws + w.hrows;
      e = launch_encode_rows(T, tree->feat_dtype, M, sorted, Q, hrows, O, stream);
      if (e != hipSuccess) return hip_status(e, "shifted encode launch");
      e = launch_mlp(M, mlp->dtype, hrows, Q, Lq, stream);
    } else {
      e = launch_query(T, tree->feat_dtype, M, mlp->dtype, sorted, Q, Lq, O, G, stream);
    }
  }
  if (e != hipSuccess) return hip_status(e, "residual query launch");
  ProfScope ps(OO_PROF_COMBINE, stream);
  return hip_status(launch_combine(A, Lq, rank, lhs_out, rhs_out, resid_out, lossp, loss_out, stream), "combine launch");
}

int oo_radiosity_residual_bwd(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch,
                              const float* resid, const float* rhs, const double* grad_loss, float* const* dfeat,
                              float* const* dW, float* const* db, void* workspace, size_t workspace_bytes,
                              hipStream_t stream) {
  g_err[0] = 0;
  TreeArgs T;
  MlpArgs M;
  ResidualArgs A;
  int rc = check_tree(tree, T);
  if (rc) return rc;
  if ((rc = check_mlp(mlp, tree->n_levels * tree->C, M))) return rc;
  if ((rc = check_pair(tree, mlp))) return rc;
  if ((rc = check_batch(batch, A))) return rc;
  if ((rc = check_attrs(batch, A, M))) return rc;
  DispArgs G;
  if ((rc = check_disparity(tree, G, true))) return rc;
  if (!grad_loss || !dfeat || !dW || !db || !workspace) return fail(OO_EINVAL, "NULL argument");
  if (A.B == 0) return OO_OK;
  if (!resid || !rhs) return fail(OO_EINVAL, "resid and rhs are required");
  GradArgs GA;
  for (int l = 0; l < OO_MAX_LEVELS; ++l) GA.dfeat[l] = GA.pad[l] = nullptr;
  for (int l = 0; l < tree->n_levels; ++l) {
    const bool has_nodes = tree->level_offset[l + 1] > tree->level_offset[l];
    if (has_nodes && !dfeat[l]) return fail(OO_EINVAL, "dfeat[%d] is NULL", l);
    GA.dfeat[l] = dfeat[l];
  }
  for (int i = 0; i < mlp->n_layers; ++i)
    if (!dW[i] || !db[i]) return fail(OO_EINVAL, "dW[%d] or db[%d] is NULL", i, i);
  const Workspace w = workspace_layout(M, mlp->dtype, batch, tree);
  if (workspace_bytes < w.total)
    return fail(OO_EINVAL, "workspace of %zu bytes is smaller than the %zu this problem needs", workspace_bytes,
                w.total);
  char* ws = static_cast<char*>(workspace);
  float* const gpad = reinterpret_cast<float*>(ws + w.gpad);
  for (int l = 0; l < tree->n_levels; ++l)
    if (w.pad_off[l] >= 0 && GA.dfeat[l]) GA.pad[l] = gpad + w.pad_off[l];
  float* seeds = reinterpret_cast<float*>(ws + w.seeds);
  const int32_t* nidx = reinterpret_cast<const int32_t*>(ws + w.nidx);
  float* partials = reinterpret_cast<float*>(ws + w.dwp);
  void* Wt[OO_MAX_LAYERS];
  for (int i = 0; i < mlp->n_layers; ++i) Wt[i] = ws + w.wt[i];
  const bool full = batch->grad_through_rhs && !batch->target_override && batch->N > 0;
  const int64_t Qb = full ? A.B * (1 + A.N) : A.B;
  const float post_scale = (float)(1.0 / (3.0 * (double)A.B));
  hipError_t e;
  {
    ProfScope ps(OO_PROF_SEEDS, stream);
    e = launch_seeds(A, resid, rhs, grad_loss, full ? 1 : 0, seeds, stream);
    if (e == hipSuccess) e = launch_fill_zero(gpad, w.pad_total, stream);
    if (e == hipSuccess && G.n_levels) e = launch_fill_zero(reinterpret_cast<float*>(ws + w.dd), Qb, stream);
  }
  if (e != hipSuccess) return hip_status(e, "seed launch");
  {
    ProfScope ps(OO_PROF_TRANSPOSE, stream);
    e = launch_transpose_weights(M, mlp->dtype, Wt, stream);
  }
  if (e != hipSuccess) return hip_status(e, "transpose launch");
  // the forward's bucketed order: its first Qb sorted positions are the
  // backward's queries (all LHS queries come first); node indices and
  // octahedral coordinates were stored at those positions
  const int32_t* order = reinterpret_cast<const int32_t*>(ws + w.order);
  const float2* uv = reinterpret_cast<const float2*>(ws + w.uv);
  const float4* pos = reinterpret_cast<const float4*>(ws + w.pos);
  float* dh = reinterpret_cast<float*>(ws + w.dh);
  const int nc = bwd_chunks(Qb);
  const int64_t chunk = ((Qb + nc - 1) / nc + 63) / 64 * 64;  // whole 64-query tiles
  {
    std::lock_guard<std::mutex> lk(g_side_m);
    SideStream* side = nullptr;
    if (nc > 1 && (e = side_stream(side)) != hipSuccess) return hip_status(e, "side stream");
    for (int c = 0; c < nc; ++c) {
      const int64_t q0 = c * chunk, qn = std::min(Qb - q0, chunk);
      if (qn <= 0) break;
      const int64_t LC = (int64_t)tree->n_levels * tree->C;
      BwdArgs B{qn, nidx + q0, Qb, uv + q0, pos + q0, seeds, order + q0, Qb, partials, dh + q0 * LC, c > 0};
      B.gA = batch->attr;
      B.gB = A.N > 0 ? batch->attr2 : batch->attr;
      B.nA = A.B;
      B.n_src = A.B * (1 + A.N);
      ShiftArgs SA;
      if (G.n_levels) {
        B.wdir = reinterpret_cast<const float4*>(ws + w.wdir) + q0;
        B.shift = 1;
        SA.wdir = B.wdir;
        SA.dd = reinterpret_cast<float*>(ws + w.dd) + q0;
      }
      {
        ProfScope ps(OO_PROF_BACKWARD, stream);
        e = launch_bwd(T, tree->feat_dtype, M, mlp->dtype, Wt, B, w.PL, w.grid, stream);
      }
      if (e != hipSuccess) return hip_status(e, "backward launch");
      hipStream_t ss = stream;
      if (side) {  // the scatter of this chunk waits for its dh only
        if ((e = hipEventRecord(side->ev[c], stream)) != hipSuccess) return hip_status(e, "event record");
        if ((e = hipStreamWaitEvent(side->s, side->ev[c], 0)) != hipSuccess) return hip_status(e, "stream wait");
        ss = side->s;
      }
      {
        ProfScope ps(OO_PROF_SCATTER, ss);
        e = launch_scatter(T, tree->feat_dtype, qn, nidx + q0, Qb, uv + q0, pos + q0, dh + q0 * LC, post_scale, GA, SA,
                           ss);
      }
      if (e != hipSuccess) return hip_status(e, "scatter launch");
    }
    if (side) {  // the caller's stream continues after the last scatter
      if ((e = hipEventRecord(side->ev[kMaxChunks], side->s)) != hipSuccess) return hip_status(e, "event record");
      if ((e = hipStreamWaitEvent(stream, side->ev[kMaxChunks], 0)) != hipSuccess) return hip_status(e, "stream wait");
    }
  }
  ReduceDst D;
  D.n_seg = 2 * mlp->n_layers;
  for (int i = 0; i < mlp->n_layers; ++i) {
    D.start[2 * i] = w.PL.w_off[i];
    D.dst[2 * i] = dW[i];
    D.start[2 * i + 1] = w.PL.b_off[i];
    D.dst[2 * i + 1] = db[i];
  }
  D.start[D.n_seg] = w.PL.P;
  ProfScope ps(OO_PROF_DW_REDUCE, stream);
  if ((e = launch_pad_fold(T, GA, stream)) != hipSuccess) return hip_status(e, "gradient fold launch");
  if ((e = launch_dw_reduce(partials, w.grid, w.PL, D, post_scale, stream)) != hipSuccess)
    return hip_status(e, "dW reduce launch");
  if (!G.n_levels) return OO_OK;
  // the disparity predictor: from each backward query's dLoss/d disparity
  // (summed by the scatter) to its MLP and hash tables
  const oo_disparity* gp = tree->disparity;
  QuerySrc src{batch->x, batch->dir, A.B, A.N > 0 ? batch->x2 : batch->x, A.N > 0 ? batch->dir2 : batch->dir};
  src.idx = order;
  src.n = A.B * (1 + A.N);
  float* gpart = reinterpret_cast<float*>(ws + w.gdwp);
  if ((e = launch_disparity_bwd(G, src, Qb, reinterpret_cast<const float*>(ws + w.dd), gp->dtables,
                                reinterpret_cast<float*>(ws + w.drows), w.dcap, gpart, w.ggrid, stream)) != hipSuccess)
    return hip_status(e, "disparity backward launch");
  ParamLayout GL;
  ReduceDst GD;
  GL.n_layers = gp->n_layers;
  GD.n_seg = 2 * gp->n_layers;
  int64_t off = 0;
  for (int i = 0; i < gp->n_layers; ++i) {
    GL.n_in[i] = gp->dims[i];
    GL.n_out[i] = gp->dims[i + 1];
    GL.w_off[i] = off;
    GD.start[2 * i] = off;
    GD.dst[2 * i] = gp->dW[i];
    off += (int64_t)gp->dims[i] * gp->dims[i + 1];
    GL.b_off[i] = off;
    GD.start[2 * i + 1] = off;
    GD.dst[2 * i + 1] = gp->db[i];
    off += gp->dims[i + 1];
  }
  GL.P = off;
  GD.start[GD.n_seg] = off;
  return hip_status(launch_dw_reduce(gpart, w.ggrid, GL, GD, 1.0f, stream), "disparity reduce launch");
}

int oo_residual_node_indices(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch,
                             const void* workspace, size_t workspace_bytes, int32_t* node_idx_out,
                             hipStream_t stream) {
  g_err[0] = 0;
  TreeArgs T;
  MlpArgs M;
  ResidualArgs A;
  int rc = check_tree(tree, T);
  if (rc) return rc;
  if ((rc = check_mlp(mlp, tree->n_levels * tree->C, M))) return rc;
  if ((rc = check_pair(tree, mlp))) return rc;
  if ((rc = check_batch(batch, A))) return rc;
  DispArgs G;
  if ((rc = check_disparity(tree, G, false))) return rc;
  if (!workspace) return fail(OO_EINVAL, "workspace is required");
  const Workspace w = workspace_layout(M, mlp->dtype, batch, tree);
  if (workspace_bytes < w.total)
    return fail(OO_EINVAL, "workspace of %zu bytes is smaller than the %zu this problem needs", workspace_bytes,
                w.total);
  if (w.Qb == 0) return OO_OK;
  if (!node_idx_out) return fail(OO_EINVAL, "node_idx_out is required");
  const char* ws = static_cast<const char*>(workspace);
  return hip_status(launch_saved_nodes(reinterpret_cast<const int32_t*>(ws + w.nidx),
                                       reinterpret_cast<const int32_t*>(ws + w.order), w.Qb, tree->n_levels, w.K,
                                       node_idx_out, stream),
                    "node index readback launch");
}

}  // extern "C"

namespace {

int dot_args(const float* const* a, const float* const* b, const int64_t* n, int32_t n_groups, double* out,
             DotArgs& D) {
  if (n_groups < 0 || n_groups > OO_DOT_MAX_GROUPS)
    return fail(OO_EINVAL, "n_groups must be in [0, %d], got %d", OO_DOT_MAX_GROUPS, n_groups);
  if (n_groups == 0) return OO_OK;
  if (!a || !n || !out) return fail(OO_EINVAL, "a, n and out are required");
  for (int g = 0; g < OO_DOT_MAX_GROUPS; ++g) {
    D.a[g] = D.b[g] = nullptr;
    D.n[g] = 0;
  }
  for (int g = 0; g < n_groups; ++g) {
    if (n[g] < 0) return fail(OO_EINVAL, "n[%d] must be >= 0", g);
    if (n[g] > 0 && !a[g]) return fail(OO_EINVAL, "a[%d] is NULL", g);
    D.a[g] = a[g];
    D.b[g] = b ? b[g] : nullptr;
    D.n[g] = n[g];
  }
  return OO_OK;
}

}  // namespace

extern "C" {

int oo_dot_f64(const float* const* a, const float* const* b, const int64_t* n, int32_t n_groups, double* out,
               double* partials, hipStream_t stream) {
  g_err[0] = 0;
  DotArgs D;
  int rc = dot_args(a, b, n, n_groups, out, D);
  if (rc || n_groups == 0) return rc;
  if (!partials) return fail(OO_EINVAL, "partials is required");
  return hip_status(launch_dot(D, n_groups, partials, out, stream), "dot launch");
}

int oo_dot_f64_noalloc(const float* const* a, const float* const* b, const int64_t* n, int32_t n_groups,
                       double* out, hipStream_t stream) {
  g_err[0] = 0;
  if (n_groups > OO_DOT_MAX_GROUPS)
    return fail(OO_EINVAL, "n_groups = %d exceeds the %d groups the library's static partials array holds", n_groups,
                OO_DOT_MAX_GROUPS);
  DotArgs D;
  int rc = dot_args(a, b, n, n_groups, out, D);
  if (rc || n_groups == 0) return rc;
  double* partials = nullptr;
  hipError_t e = dot_scratch(&partials);
  if (e != hipSuccess) return hip_status(e, "static partials lookup");
  // every partial is overwritten by the launch: nothing to clear
  return hip_status(launch_dot(D, n_groups, partials, out, stream), "dot launch");
}

int oo_adam_step(const oo_adam_config* cfg, const oo_adam_segment* segs, int32_t n_segs, hipStream_t stream) {
  g_err[0] = 0;
  if (!cfg) return fail(OO_EINVAL, "cfg is NULL");
  if (n_segs < 0 || n_segs > OO_ADAM_MAX_SEGMENTS)
    return fail(OO_EINVAL, "n_segs must be in [0, %d], got %d", OO_ADAM_MAX_SEGMENTS, n_segs);
  if (cfg->step < 1) return fail(OO_EINVAL, "step must be >= 1, got %d", cfg->step);
  if (!(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f))
    return fail(OO_EINVAL, "beta1 and beta2 must be in [0, 1)");
  if (!(cfg->eps >= 0.0f) || !(cfg->lr >= 0.0f)) return fail(OO_EINVAL, "lr and eps must be >= 0");
  if (cfg->work_dtype != OO_F32 && cfg->work_dtype != OO_F16 && cfg->work_dtype != OO_BF16)
    return fail(OO_EINVAL, "unknown work_dtype");
  if (n_segs == 0) return OO_OK;
  if (!segs) return fail(OO_EINVAL, "segments is NULL");
  AdamArgs A;
  A.n_segs = n_segs;
  A.first[0] = 0;
  for (int s = 0; s < n_segs; ++s) {
    const oo_adam_segment& S = segs[s];
    if (S.n < 0) return fail(OO_EINVAL, "segment %d: n must be >= 0", s);
    if (S.n > 0 && (!S.param || !S.grad || !S.m || !S.v))
      return fail(OO_EINVAL, "segment %d: param, grad, m and v are required", s);
    if (S.touched && (S.block <= 0 || S.block % 4))
      return fail(OO_EINVAL, "segment %d: block must be a positive multiple of 4 with touched flags", s);
    const size_t wa = cfg->work_dtype == OO_F32 ? 16 : 8;
    const bool vec = ((uintptr_t)S.param | (uintptr_t)S.grad | (uintptr_t)S.m | (uintptr_t)S.v) % 16 == 0 &&
                     (uintptr_t)S.work % wa == 0;
    A.seg[s] = AdamSeg{S.param, S.grad, S.m, S.v, S.work, S.n, S.touched, S.block, vec ? 1 : 0};
    A.first[s + 1] = A.first[s] + (S.n + 3) / 4;
  }
  A.lr = cfg->lr;
  A.b1 = cfg->beta1;
  A.b2 = cfg->beta2;
  A.eps = cfg->eps;
  A.inv_c1 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta1, (double)cfg->step)));
  A.inv_c2 = (float)(1.0 / (1.0 - std::pow((double)cfg->beta2, (double)cfg->step)));
  return hip_status(launch_adam(A, cfg->work_dtype, stream), "adam launch");
}

int oo_touched_nodes(const oo_tree* tree, const oo_mlp* mlp, const oo_residual_batch* batch, const void* workspace,
                     size_t workspace_bytes, uint32_t* touched, hipStream_t stream) {
  g_err[0] = 0;
  TreeArgs T;
  MlpArgs M;
  ResidualArgs A;
  int rc = check_tree(tree, T);
  if (rc) return rc;
  if ((rc = check_mlp(mlp, tree->n_levels * tree->C, M))) return rc;
  if ((rc = check_pair(tree, mlp))) return rc;
  if ((rc = check_batch(batch, A))) return rc;
  DispArgs G;
  if ((rc = check_disparity(tree, G, false))) return rc;
  if (!workspace) return fail(OO_EINVAL, "workspace is required");
  const Workspace w = workspace_layout(M, mlp->dtype, batch, tree);
  if (workspace_bytes < w.total)
    return fail(OO_EINVAL, "workspace of %zu bytes is smaller than the %zu this problem needs", workspace_bytes,
                w.total);
  if (w.Qb == 0) return OO_OK;
  if (!touched) return fail(OO_EINVAL, "touched is required");
  const char* ws = static_cast<const char*>(workspace);
  return hip_status(launch_touched(reinterpret_cast<const int32_t*>(ws + w.nidx), w.Qb, (int64_t)tree->n_levels * w.K,
                                   tree->level_offset[tree->n_levels], touched, stream),
                    "touched nodes launch");
}

int oo_cast_params(const float* src, void* dst, oo_dtype dst_dtype, int64_t n, hipStream_t stream) {
  g_err[0] = 0;
  if (n < 0) return fail(OO_EINVAL, "n must be >= 0");
  if (dst_dtype != OO_F32 && dst_dtype != OO_F16 && dst_dtype != OO_BF16) return fail(OO_EINVAL, "unknown dtype");
  if (n == 0) return OO_OK;
  if (!src || !dst) return fail(OO_EINVAL, "src and dst are required");
  ProfScope ps(OO_PROF_CAST, stream);
  return hip_status(launch_cast(src, dst, dst_dtype, n, stream), "cast launch");
}

}  // extern "C"
