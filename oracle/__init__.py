"""FP64 CPU oracle for the OctaOctree query and the neural-radiosity residual step.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. It loads
``liboo_oracle.so`` (built from ``octaoctree_oracle.c`` by ``oracle.build``),
which shares no code with the HIP library.

Arrays go in as numpy (FP32 for inputs and parameters, as the GPU path gets
them) and come back as FP64 numpy arrays. Each wrapper names the paper passage
its C function follows; the C file states the readings taken where the paper
is silent.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

MAX_LEVELS = 16
MAX_LAYERS = 7
_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the mutation test point the wrapper at a deliberately
# broken build of the same source.
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboo_oracle.so")


class _MLP(C.Structure):
    _fields_ = [
        ("n_layers", C.c_int32),
        ("dims", C.c_int32 * (MAX_LAYERS + 1)),
        ("W", C.c_void_p * MAX_LAYERS),
        ("b", C.c_void_p * MAX_LAYERS),
    ]


HASH_MAX_LEVELS = 16


class _Disparity(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32),
        ("F", C.c_int32),
        ("log2_T", C.c_int32),
        ("res", C.c_int32 * HASH_MAX_LEVELS),
        ("tables", C.c_void_p),
        ("mlp", _MLP),
    ]


class _Tree(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32),
        ("C", C.c_int32),
        ("res", C.c_int32 * MAX_LEVELS),
        ("level_offset", C.c_int64 * (MAX_LEVELS + 1)),
        ("nodes", C.c_void_p),
        ("feat", C.c_void_p * MAX_LEVELS),
        ("interp", C.c_int32),
        ("disp", C.POINTER(_Disparity)),
    ]


# Level-feature interpolation schemes.
INTERP_NODE_BILINEAR = 0  # containing node, bilinear on R x R texels
INTERP_PAPER = 1          # 8-cell trilinear (renormalised), barycentric on (R+1)^2 vertices


class _Batch(C.Structure):
    _fields_ = [
        ("B", C.c_int64),
        ("N", C.c_int32),
        ("x", C.c_void_p), ("dir", C.c_void_p), ("n", C.c_void_p), ("wo", C.c_void_p),
        ("albedo", C.c_void_p), ("Le", C.c_void_p),
        ("rough", C.c_void_p),
        ("x2", C.c_void_p), ("dir2", C.c_void_p), ("wi", C.c_void_p),
        ("pdf", C.c_void_p),
        ("target_override", C.c_void_p),
        ("F0", C.c_double),
        ("loss_kind", C.c_int32),
        ("eps", C.c_double),
        ("grad_through_rhs", C.c_int32),
        ("attr", C.c_void_p), ("attr2", C.c_void_p),
    ]


_lib = None


def lib():
    """Load the oracle library (built by ``oracle.build.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH}; run oracle.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.ora_build_octree.argtypes = [vp, i64, i32, i32, vp, i64, vp, vp]
        L.ora_build_octree.restype = C.c_int
        L.ora_quantize.argtypes = [vp, i64, i32, vp]
        L.ora_descend.argtypes = [vp, vp, i64, vp]
        L.ora_octa.argtypes = [vp, i64, vp]
        L.ora_octa_decode.argtypes = [vp, i64, vp]
        L.ora_taps.argtypes = [vp, i64, i32, vp, vp]
        L.ora_encode.argtypes = [vp, vp, vp, i64, vp, vp]
        L.ora_mlp_fwd.argtypes = [vp, vp, i64, vp]
        L.ora_query_fwd.argtypes = [vp, vp, vp, vp, vp, i64, vp, i32]
        L.ora_bsdf_weight.argtypes = [vp, vp]
        L.ora_residual_fwd.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32]
        L.ora_residual_fwd.restype = C.c_int
        L.ora_residual_bwd.argtypes = [vp, vp, vp, C.c_double, vp, vp, vp, vp, vp, vp, vp, i32]
        L.ora_hash_encode.argtypes = [vp, vp, i64, vp, vp, vp]
        L.ora_disparity_fwd.argtypes = [vp, vp, vp, i64, vp]
        L.ora_residual_bwd.restype = C.c_int
        L.ora_map_entries.argtypes = [i32, i32]
        L.ora_map_entries.restype = C.c_int64
        L.ora_bary.argtypes = [vp, i64, i32, vp, vp, vp]
        L.ora_neighbours.argtypes = [vp, vp, i64, i32, vp, vp, vp]
        L.ora_adam.argtypes = [vp, vp, vp, vp, i64, vp, i64, i32, C.c_double, C.c_double, C.c_double, C.c_double]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Disparity:
    """The disparity predictor (Sec. 3.3, Sec. 3.5): hash-grid tables
    [n_levels][2^log2_T][F] FP32 with N_i cells per side at level i, and
    an MLP on [encoding, unit(w_r), 0] with one output."""

    res: list                         # N_i per hash level
    F: int
    log2_T: int
    tables: np.ndarray
    W: list
    b: list

    def _struct(self):
        g = _Disparity()
        g.n_levels = len(self.res)
        g.F = int(self.F)
        g.log2_T = int(self.log2_T)
        for i, n in enumerate(self.res):
            g.res[i] = int(n)
        self._tables = _f32(self.tables)
        g.tables = self._tables.ctypes.data
        self._mlp = MLP(self.W, self.b)
        g.mlp = self._mlp._struct()
        return g


@dataclass
class Tree:
    """Octree + FP32 master feature tables, as the oracle reads them."""

    nodes: np.ndarray                 # uint32 [n_nodes]
    level_offset: np.ndarray          # int64 [L + 1]
    res: list                         # R_l per level
    C: int
    feat: list = field(default_factory=list)  # float32 [n_l][R_l][R_l][C] per level
    # INTERP_PAPER: feat[l] is [n_l][R_l + 1][R_l + 1][C] (map vertices)
    interp: int = INTERP_NODE_BILINEAR
    disp: "Disparity | None" = None   # INTERP_PAPER only: shifts each cell's lookup direction

    @property
    def n_levels(self):
        return len(self.res)

    def _struct(self):
        t = _Tree()
        t.n_levels = self.n_levels
        t.C = self.C
        for l, R in enumerate(self.res):
            t.res[l] = int(R)
        for l in range(self.n_levels + 1):
            t.level_offset[l] = int(self.level_offset[l])
        self._nodes = np.ascontiguousarray(self.nodes, dtype=np.uint32)
        t.nodes = self._nodes.ctypes.data
        self._feat = [_f32(f) for f in self.feat]
        for l, f in enumerate(self._feat):
            t.feat[l] = f.ctypes.data
        t.interp = int(self.interp)
        if self.disp is not None:
            self._disp = self.disp._struct()
            t.disp = C.pointer(self._disp)
        return t


@dataclass
class MLP:
    W: list   # float32 [out][in] per layer
    b: list   # float32 [out] per layer

    def _struct(self):
        m = _MLP()
        m.n_layers = len(self.W)
        self._W = [_f32(w) for w in self.W]
        self._b = [_f32(b) for b in self.b]
        m.dims[0] = self._W[0].shape[1]
        for i, w in enumerate(self._W):
            m.dims[i + 1] = w.shape[0]
            m.W[i] = w.ctypes.data
            m.b[i] = self._b[i].ctypes.data
        return m


def _batch_struct(bt: dict, keep: list):
    s = _Batch()
    s.B = int(bt["x"].shape[0])
    s.N = int(bt.get("N", 0))
    for name in ("x", "dir", "n", "wo", "albedo", "Le", "rough", "x2", "dir2", "wi", "pdf",
                 "target_override", "attr", "attr2"):
        a = bt.get(name)
        if a is not None:
            a = _f32(a)
            keep.append(a)
            setattr(s, name, a.ctypes.data)
    s.F0 = float(bt.get("F0", 0.04))
    s.loss_kind = int(bt.get("loss_kind", 0))
    s.eps = float(bt.get("eps", 1e-2))
    s.grad_through_rhs = int(bt.get("grad_through_rhs", 0))
    return s


# --------------------------------------------------------------------------
# Wrappers
# --------------------------------------------------------------------------

def build_octree(samples, D, tau):
    """Sparse octree from surface samples (Sec. 3.4 non-empty cells; Sec. 4.1
    o-cnn-style octree). Returns (nodes uint32, level_offset int64 [D+2])."""
    s = _f32(samples).reshape(-1, 3)
    lo = np.zeros(D + 2, np.int64)
    nn = np.zeros(1, np.int64)
    rc = lib().ora_build_octree(_p(s), s.shape[0], D, tau, None, 0, _p(lo), _p(nn))
    if rc != 0:
        raise RuntimeError(f"ora_build_octree size query failed: {rc}")
    nodes = np.zeros(int(nn[0]), np.uint32)
    rc = lib().ora_build_octree(_p(s), s.shape[0], D, tau, _p(nodes), nodes.size, _p(lo), _p(nn))
    if rc != 0:
        raise RuntimeError(f"ora_build_octree failed: {rc}")
    return nodes, lo


def quantize(x, D):
    x = _f32(x).reshape(-1, 3)
    q = np.zeros((x.shape[0], 3), np.int64)
    lib().ora_quantize(_p(x), x.shape[0], D, _p(q))
    return q


def descend(tree: Tree, x):
    """Containing node per level, -1 where absent. int32 [B][L]."""
    x = _f32(x).reshape(-1, 3)
    out = np.zeros((x.shape[0], tree.n_levels), np.int32)
    ts = tree._struct()
    lib().ora_descend(C.byref(ts), _p(x), x.shape[0], _p(out))
    return out


def octa(d):
    """Octahedral projection + fold (Sec. 3.3), as (s, t) in [0,1]^2."""
    d = _f32(d).reshape(-1, 3)
    st = np.zeros((d.shape[0], 2), np.float64)
    lib().ora_octa(_p(d), d.shape[0], _p(st))
    return st


def octa_decode(st):
    st = _f64(st).reshape(-1, 2)
    d = np.zeros((st.shape[0], 3), np.float64)
    lib().ora_octa_decode(_p(st), st.shape[0], _p(d))
    return d


def taps(st, R):
    """Bilinear taps with seam wrap: (ij int32 [B][4][2], w float64 [B][4])."""
    st = _f64(st).reshape(-1, 2)
    ij = np.zeros((st.shape[0], 4, 2), np.int32)
    w = np.zeros((st.shape[0], 4), np.float64)
    lib().ora_taps(_p(st), st.shape[0], int(R), _p(ij), _p(w))
    return ij, w


def map_entries(R, interp):
    """Entries of one node's map: R^2 texels, or (R + 1)^2 vertices for the
    paper's scheme (Sec. 4.1: features stored at map vertices)."""
    return int(lib().ora_map_entries(int(R), int(interp)))


def bary(st, R):
    """Barycentric vertex lookup (Sec. 3.3): vertices (i, j) [B][3][2] as
    found on the unfolded grid, weights [B][3], storage slots after the
    seam identification [B][3]."""
    st = _f64(st).reshape(-1, 2)
    B = st.shape[0]
    ij = np.zeros((B, 3, 2), np.int32)
    w = np.zeros((B, 3), np.float64)
    v = np.zeros((B, 3), np.int32)
    lib().ora_bary(_p(st), B, int(R), _p(ij), _p(w), _p(v))
    return ij, w, v


def neighbours(tree: Tree, x, l):
    """The 8 cells around x at level l (Sec. 3.4): node indices [B][8] (-1
    empty), cell coordinates [B][8][3], renormalised trilinear weights
    [B][8]."""
    x = _f32(x).reshape(-1, 3)
    B = x.shape[0]
    idx = np.zeros((B, 8), np.int32)
    cells = np.zeros((B, 8, 3), np.int64)
    w = np.zeros((B, 8), np.float64)
    ts = tree._struct()
    lib().ora_neighbours(C.byref(ts), _p(x), B, int(l), _p(idx), _p(cells), _p(w))
    return idx, cells, w


def encode(tree: Tree, x, d):
    """Concatenated level features h [B][L*C] and node indices [B][L] (Sec. 3.4)."""
    x = _f32(x).reshape(-1, 3)
    d = _f32(d).reshape(-1, 3)
    B = x.shape[0]
    h = np.zeros((B, tree.n_levels * tree.C), np.float64)
    idx = np.zeros((B, tree.n_levels), np.int32)
    ts = tree._struct()
    lib().ora_encode(C.byref(ts), _p(x), _p(d), B, _p(h), _p(idx))
    return h, idx


def mlp_fwd(mlp: MLP, h):
    """Decoder MLP (Sec. 3.5) on FP64 features."""
    h = _f64(h)
    ms = mlp._struct()
    out = np.zeros((h.shape[0], ms.dims[ms.n_layers]), np.float64)
    lib().ora_mlp_fwd(C.byref(ms), _p(h), h.shape[0], _p(out))
    return out


def query_fwd(tree: Tree, mlp: MLP, x, d, nthreads=0, attr=None):
    """Encode + decode: RGB radiance [B][3]. attr: [B][E] decoder attributes
    appended after h (Sec. 3.5), when the MLP's input is wider than L*C."""
    x = _f32(x).reshape(-1, 3)
    d = _f32(d).reshape(-1, 3)
    e = None if attr is None else _f32(attr).reshape(x.shape[0], -1)
    ts, ms = tree._struct(), mlp._struct()
    out = np.zeros((x.shape[0], 3), np.float64)
    lib().ora_query_fwd(C.byref(ts), C.byref(ms), _p(x), _p(d), _p(e), x.shape[0], _p(out), int(nthreads))
    return out


def bsdf_weight(batch: dict):
    """Per-sample weight f_r |n . wi| / pdf, [B][N][3] (Sec. 3.2)."""
    keep = []
    bs = _batch_struct(batch, keep)
    w = np.zeros((bs.B, bs.N, 3), np.float64)
    lib().ora_bsdf_weight(C.byref(bs), _p(w))
    return w


def residual_fwd(tree: Tree, mlp: MLP, batch: dict, nthreads=0):
    """Returns (lhs, rhs, resid) [B][3] and the loss (Sec. 3.2, 3.6)."""
    keep = []
    bs = _batch_struct(batch, keep)
    ts, ms = tree._struct(), mlp._struct()
    lhs = np.zeros((bs.B, 3))
    rhs = np.zeros((bs.B, 3))
    res = np.zeros((bs.B, 3))
    loss = np.zeros(1)
    rc = lib().ora_residual_fwd(C.byref(ts), C.byref(ms), C.byref(bs), _p(lhs), _p(rhs), _p(res),
                                _p(loss), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"ora_residual_fwd failed: {rc}")
    return lhs, rhs, res, float(loss[0])


def residual_bwd(tree: Tree, mlp: MLP, batch: dict, grad_loss=1.0, nthreads=0, disp_out=None):
    """FP64 gradients (dfeat per level, dW, db) of the loss times grad_loss.
    With a disparity predictor on the tree, its gradients (keys "tables",
    "W", "b") and dL/d disparity per backward query ("dd") go into the dict
    disp_out when given."""
    keep = []
    bs = _batch_struct(batch, keep)
    ts, ms = tree._struct(), mlp._struct()
    dfeat = [np.zeros(np.shape(f), np.float64) for f in tree.feat]
    dW = [np.zeros(np.shape(w), np.float64) for w in mlp.W]
    db = [np.zeros(np.shape(b), np.float64) for b in mlp.b]
    arr = lambda lst: (C.c_void_p * max(1, len(lst)))(*[a.ctypes.data for a in lst])
    gt = gW = gb = dd = None
    if tree.disp is not None and tree.interp == INTERP_PAPER:
        g = tree.disp
        gt = np.zeros(np.shape(g.tables), np.float64)
        gW = [np.zeros(np.shape(w), np.float64) for w in g.W]
        gb = [np.zeros(np.shape(b), np.float64) for b in g.b]
        full = batch.get("grad_through_rhs", 0) and batch.get("target_override") is None and bs.N > 0
        dd = np.zeros(bs.B * (1 + bs.N) if full else bs.B, np.float64)
    rc = lib().ora_residual_bwd(C.byref(ts), C.byref(ms), C.byref(bs), float(grad_loss),
                                arr(dfeat), arr(dW), arr(db), _p(gt), None if gW is None else arr(gW),
                                None if gb is None else arr(gb), _p(dd), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"ora_residual_bwd failed: {rc}")
    if disp_out is not None and gt is not None:
        disp_out.update(tables=gt, W=gW, b=gb, dd=dd)
    return dfeat, dW, db


def hash_encode(disp: Disparity, x):
    """Hash encoding of x (Sec. 3.5, Instant-NGP style): (enc [B][L F],
    vertex entries [B][L][8], trilinear weights [B][L][8])."""
    x = _f32(x).reshape(-1, 3)
    B, L = x.shape[0], len(disp.res)
    enc = np.zeros((B, L * disp.F), np.float64)
    idx = np.zeros((B, L, 8), np.int64)
    w = np.zeros((B, L, 8), np.float64)
    gs = disp._struct()
    lib().ora_hash_encode(C.byref(gs), _p(x), B, _p(enc), _p(idx), _p(w))
    return enc, idx, w


def disparity(disp: Disparity, x, d):
    """Predicted disparity d(x, w_r) per query [B] (Sec. 3.3)."""
    x = _f32(x).reshape(-1, 3)
    d = _f32(d).reshape(-1, 3)
    out = np.zeros(x.shape[0], np.float64)
    gs = disp._struct()
    lib().ora_disparity_fwd(C.byref(gs), _p(x), _p(d), x.shape[0], _p(out))
    return out


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.99, eps=1e-15, touched=None, block=1):
    """One Adam step (Kingma and Ba, Algorithm 1) on copies of FP32 arrays:
    returns (p, m, v) as FP32. touched: per-block flags (uint32) that limit
    the update to blocks of `block` entries some query read."""
    p, m, v = _f32(p).copy(), _f32(m).copy(), _f32(v).copy()
    g = _f32(g)
    tf = None if touched is None else np.ascontiguousarray(touched, dtype=np.uint32)
    lib().ora_adam(_p(p), _p(g), _p(m), _p(v), p.size, _p(tf), int(block), int(t), float(lr), float(b1),
                   float(b2), float(eps))
    return p, m, v
