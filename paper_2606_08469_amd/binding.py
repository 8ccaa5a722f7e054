"""Python binding of liboctaoctree (ctypes + torch for device memory/streams).

Argument marshalling only: every step runs in the library's HIP kernels. There
is no CPU fallback; a missing library or a failing call raises.

Entry points mirror include/octaoctree.h: build_octree, encode_query,
mlp_fwd, query_fwd, residual_workspace_bytes, residual_fwd, residual_bwd,
cast_params. ``OctaOctree`` bundles an octree, its FP32 master tables and MLP
(plus 16-bit working copies), and ``RadiosityResidual`` is the
torch.autograd.Function of the residual step (Sec. 3.2 / 3.6: the target is
detached).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

MAX_LEVELS = 16
MAX_LAYERS = 7
HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboctaoctree.so")

F32, F16, BF16 = 0, 1, 2
DTYPE_CODE = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
CODE_DTYPE = {v: k for k, v in DTYPE_CODE.items()}


class OOError(RuntimeError):
    pass


HASH_MAX_LEVELS = 16


class _Disparity(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("F", C.c_int32), ("log2_T", C.c_int32),
                ("res", C.c_int32 * HASH_MAX_LEVELS), ("tables", C.c_void_p), ("n_layers", C.c_int32),
                ("dims", C.c_int32 * 5), ("W", C.c_void_p * 4), ("b", C.c_void_p * 4),
                ("dtables", C.c_void_p), ("dW", C.c_void_p * 4), ("db", C.c_void_p * 4)]


class _Tree(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("C", C.c_int32), ("res", C.c_int32 * MAX_LEVELS),
                ("level_offset", C.c_int64 * (MAX_LEVELS + 1)), ("nodes", C.c_void_p),
                ("feat_dtype", C.c_int32), ("feat", C.c_void_p * MAX_LEVELS), ("interp", C.c_int32),
                ("disparity", C.POINTER(_Disparity))]


# Level-feature interpolation schemes (oo_tree.interp).
INTERP_NODE_BILINEAR = 0  # containing node, bilinear on R x R texels
INTERP_PAPER = 1          # 8 cells trilinear (renormalised), barycentric on (R+1)^2 vertices


class _MLP(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", C.c_int32 * (MAX_LAYERS + 1)), ("dtype", C.c_int32),
                ("W", C.c_void_p * MAX_LAYERS), ("b", C.c_void_p * MAX_LAYERS)]


class _Batch(C.Structure):
    _fields_ = [("B", C.c_int64), ("N", C.c_int32),
                ("x", C.c_void_p), ("dir", C.c_void_p), ("n", C.c_void_p), ("wo", C.c_void_p),
                ("albedo", C.c_void_p), ("Le", C.c_void_p), ("rough", C.c_void_p),
                ("x2", C.c_void_p), ("dir2", C.c_void_p), ("wi", C.c_void_p), ("pdf", C.c_void_p),
                ("target_override", C.c_void_p), ("F0", C.c_float), ("loss_kind", C.c_int32),
                ("eps", C.c_float), ("grad_through_rhs", C.c_int32), ("attr", C.c_void_p), ("attr2", C.c_void_p)]


class _AdamCfg(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int32), ("work_dtype", C.c_int32)]


class _AdamSeg(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("work", C.c_void_p), ("n", C.c_int64), ("touched", C.c_void_p), ("block", C.c_int64)]


ADAM_MAX_SEGMENTS = 32

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OOError(f"liboctaoctree.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.oo_build_octree.argtypes = [vp, i64, i32, i32, vp, i64, vp, vp]
        L.oo_encode_query.argtypes = [vp, vp, vp, i64, vp, i32, vp, vp]
        L.oo_mlp_fwd.argtypes = [vp, vp, i32, i64, vp, vp]
        L.oo_query_fwd.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.oo_residual_workspace_bytes.argtypes = [vp, vp, vp, C.POINTER(C.c_size_t)]
        sz = C.c_size_t
        L.oo_radiosity_residual_fwd.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.oo_radiosity_residual_bwd.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.oo_cast_params.argtypes = [vp, vp, i32, i64, vp]
        L.oo_residual_node_indices.argtypes = [vp, vp, vp, vp, sz, vp, vp]
        L.oo_dot_f64.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.oo_dot_f64_noalloc.argtypes = [vp, vp, vp, i32, vp, vp]
        L.oo_adam_step.argtypes = [vp, vp, i32, vp]
        L.oo_touched_nodes.argtypes = [vp, vp, vp, vp, sz, vp, vp]
        L.oo_profile_begin.argtypes = [i32]
        L.oo_profile_end.argtypes = [vp, vp]
        L.oo_profile_kind_name.argtypes = [i32]
        L.oo_profile_kind_name.restype = C.c_char_p
        L.oo_last_error.restype = C.c_char_p
        for f in ("oo_build_octree", "oo_encode_query", "oo_mlp_fwd", "oo_query_fwd",
                  "oo_residual_workspace_bytes", "oo_radiosity_residual_fwd", "oo_radiosity_residual_bwd",
                  "oo_cast_params", "oo_profile_begin", "oo_profile_end", "oo_residual_node_indices",
                  "oo_dot_f64", "oo_dot_f64_noalloc", "oo_adam_step", "oo_touched_nodes"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise OOError(f"{what} failed ({rc}): {lib().oo_last_error().decode()}")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def _dev(t, dtype=torch.float32):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    return t.to(device="cuda", dtype=dtype).contiguous()


# ---------------------------------------------------------------------------
# Host octree construction
# ---------------------------------------------------------------------------

def build_octree(samples, max_depth: int, split_threshold: int):
    """Sparse octree from FP32 surface samples (host, synchronous).
    Returns (nodes uint32 [n_nodes], level_offset int64 [max_depth + 2])."""
    s = np.ascontiguousarray(samples, dtype=np.float32).reshape(-1, 3)
    lo = np.zeros(max_depth + 2, np.int64)
    nn = np.zeros(1, np.int64)
    L = lib()
    _check(L.oo_build_octree(s.ctypes.data, s.shape[0], max_depth, split_threshold, None, 0,
                             lo.ctypes.data, nn.ctypes.data), "oo_build_octree (size)")
    nodes = np.zeros(int(nn[0]), np.uint32)
    _check(L.oo_build_octree(s.ctypes.data, s.shape[0], max_depth, split_threshold, nodes.ctypes.data,
                             nodes.size, lo.ctypes.data, nn.ctypes.data), "oo_build_octree")
    return nodes, lo


# ---------------------------------------------------------------------------
# Device-side descriptions
# ---------------------------------------------------------------------------

class Disparity:
    """The disparity predictor on the device (FP32): hash tables
    [16][2^log2_T][2] with res[i] cells per side at level i, and an MLP on
    [encoding, unit(w_r), 0] (hidden width 64, one output). grads: optional
    (dtables, dW list, db list) accumulators for the residual backward."""

    def __init__(self, res, log2_T, tables, W, b):
        self.res = [int(r) for r in res]
        self.log2_T = int(log2_T)
        self.tables = tables if isinstance(tables, torch.Tensor) else _dev(tables)
        self.W = [w if isinstance(w, torch.Tensor) else _dev(w) for w in W]
        self.b = [v if isinstance(v, torch.Tensor) else _dev(v) for v in b]

    def struct(self, grads=None):
        g = _Disparity()
        g.n_levels = len(self.res)
        g.F = int(self.tables.shape[-1])
        g.log2_T = self.log2_T
        for i, n in enumerate(self.res):
            g.res[i] = n
        g.tables = self.tables.data_ptr()
        g.n_layers = len(self.W)
        g.dims[0] = self.W[0].shape[1]
        for i, w in enumerate(self.W):
            g.dims[i + 1] = w.shape[0]
            g.W[i] = w.data_ptr()
            g.b[i] = self.b[i].data_ptr()
        if grads is not None:
            dt, dW, db = grads
            g.dtables = dt.data_ptr()
            for i in range(len(self.W)):
                g.dW[i] = dW[i].data_ptr()
                g.db[i] = db[i].data_ptr()
        return g


class Tree:
    """Octree on the device plus one feature table per level; with the
    paper's scheme optionally the disparity predictor that shifts each
    cell's lookup direction."""

    def __init__(self, nodes, level_offset, res, C_, feat, interp=INTERP_NODE_BILINEAR, disparity=None):
        self.nodes = torch.from_numpy(np.asarray(nodes, np.uint32).view(np.int32)).cuda()
        self.level_offset = [int(v) for v in level_offset]
        self.res = [int(r) for r in res]
        self.C = int(C_)
        self.interp = int(interp)
        self.feat = [f if isinstance(f, torch.Tensor) else _dev(f) for f in feat]
        self.disparity = disparity
        self.disp_grads = None  # (dtables, dW, db) the next struct() passes to a backward

    @property
    def corners(self):
        """Node indices per level of one query: 1, or the 8 neighbouring
        cells in the paper's scheme."""
        return 8 if self.interp == INTERP_PAPER else 1

    @property
    def n_levels(self):
        return len(self.res)

    def struct(self, feat=None):
        feat = self.feat if feat is None else feat
        t = _Tree()
        t.n_levels = self.n_levels
        t.C = self.C
        for l, R in enumerate(self.res):
            t.res[l] = R
        for l in range(self.n_levels + 1):
            t.level_offset[l] = self.level_offset[l]
        t.nodes = self.nodes.data_ptr()
        t.feat_dtype = DTYPE_CODE[feat[0].dtype]
        for l, f in enumerate(feat):
            t.feat[l] = f.data_ptr() if f.numel() else None
        t.interp = self.interp
        if self.disparity is not None:
            self._disp_struct = self.disparity.struct(self.disp_grads)
            t.disparity = C.pointer(self._disp_struct)
        return t


class MLP:
    def __init__(self, W, b):
        self.W = [w if isinstance(w, torch.Tensor) else _dev(w) for w in W]
        self.b = [v if isinstance(v, torch.Tensor) else _dev(v) for v in b]

    def struct(self, W=None):
        W = self.W if W is None else W
        m = _MLP()
        m.n_layers = len(W)
        m.dims[0] = W[0].shape[1]
        for i, w in enumerate(W):
            m.dims[i + 1] = w.shape[0]
            m.W[i] = w.data_ptr()
            m.b[i] = self.b[i].data_ptr()
        m.dtype = DTYPE_CODE[W[0].dtype]
        return m


_BATCH_ARRAYS = ("x", "dir", "n", "wo", "albedo", "Le", "rough", "x2", "dir2", "wi", "pdf", "target_override",
                 "attr", "attr2")


def device_batch(batch: dict) -> dict:
    """Copies a host batch (numpy arrays + scalars) to device FP32 tensors."""
    out = {k: v for k, v in batch.items() if k not in _BATCH_ARRAYS}
    for k in _BATCH_ARRAYS:
        out[k] = _dev(batch.get(k))
    return out


def batch_struct(b: dict):
    s = _Batch()
    s.B = int(b["x"].shape[0])
    s.N = int(b.get("N", 0))
    for k in _BATCH_ARRAYS:
        setattr(s, k, _ptr(b.get(k)))
    s.F0 = float(b.get("F0", 0.04))
    s.loss_kind = int(b.get("loss_kind", 0))
    s.eps = float(b.get("eps", 1e-2))
    s.grad_through_rhs = int(b.get("grad_through_rhs", 0))
    return s


# ---------------------------------------------------------------------------
# Entry points
# ---------------------------------------------------------------------------

def encode_query(tree: Tree, x, d, h_dtype=torch.float32, with_idx=True, feat=None):
    B = x.shape[0]
    h = torch.empty((B, tree.n_levels * tree.C), dtype=h_dtype, device="cuda")
    shape = (B, tree.n_levels) if tree.corners == 1 else (B, tree.n_levels, tree.corners)
    idx = torch.empty(shape, dtype=torch.int32, device="cuda") if with_idx else None
    ts = tree.struct(feat)
    _check(lib().oo_encode_query(C.byref(ts), _ptr(x), _ptr(d), B, _ptr(h), DTYPE_CODE[h_dtype], _ptr(idx),
                                 _stream()), "oo_encode_query")
    return h, idx


def mlp_fwd(mlp: MLP, h, W=None):
    B = h.shape[0]
    rgb = torch.empty((B, 3), dtype=torch.float32, device="cuda")
    ms = mlp.struct(W)
    _check(lib().oo_mlp_fwd(C.byref(ms), _ptr(h), DTYPE_CODE[h.dtype], B, _ptr(rgb), _stream()), "oo_mlp_fwd")
    return rgb


def query_fwd(tree: Tree, mlp: MLP, x, d, feat=None, W=None, out=None, attr=None):
    """attr: [B][E] FP32 surface attributes when the decoder reads them."""
    B = x.shape[0]
    rgb = torch.empty((B, 3), dtype=torch.float32, device="cuda") if out is None else out
    ts, ms = tree.struct(feat), mlp.struct(W)
    _check(lib().oo_query_fwd(C.byref(ts), C.byref(ms), _ptr(x), _ptr(d), _ptr(attr), B, _ptr(rgb), _stream()),
           "oo_query_fwd")
    return rgb


def residual_workspace_bytes(tree: Tree, mlp: MLP, batch: dict, feat=None, W=None) -> int:
    ts, ms, bs = tree.struct(feat), mlp.struct(W), batch_struct(batch)
    n = C.c_size_t(0)
    _check(lib().oo_residual_workspace_bytes(C.byref(ts), C.byref(ms), C.byref(bs), C.byref(n)),
           "oo_residual_workspace_bytes")
    return int(n.value)


def residual_fwd(tree: Tree, mlp: MLP, batch: dict, workspace, feat=None, W=None, outs=None):
    """Returns (lhs, rhs, resid) [B][3] FP32 and the loss (0-dim FP64 device tensor)."""
    B = batch["x"].shape[0]
    if outs is None:
        outs = tuple(torch.empty((B, 3), dtype=torch.float32, device="cuda") for _ in range(3)) + (
            torch.empty((), dtype=torch.float64, device="cuda"),)
    lhs, rhs, res, loss = outs
    ts, ms, bs = tree.struct(feat), mlp.struct(W), batch_struct(batch)
    _check(lib().oo_radiosity_residual_fwd(C.byref(ts), C.byref(ms), C.byref(bs), _ptr(lhs), _ptr(rhs), _ptr(res),
                                           _ptr(loss), _ptr(workspace), _nbytes(workspace), _stream()),
           "oo_radiosity_residual_fwd")
    return lhs, rhs, res, loss


def residual_bwd(tree: Tree, mlp: MLP, batch: dict, resid, rhs, grad_loss, dfeat, dW, db, workspace, feat=None,
                 W=None, disp_grads=None):
    """Accumulates (+=) FP32 gradients into dfeat / dW / db, and with a
    disparity predictor into disp_grads = (dtables, dW list, db list)."""
    tree.disp_grads = disp_grads
    try:
        ts = tree.struct(feat)
    finally:
        tree.disp_grads = None
    ms, bs = mlp.struct(W), batch_struct(batch)
    arr = lambda ts_: (C.c_void_p * max(1, len(ts_)))(*[t.data_ptr() if t.numel() else None for t in ts_])
    g = grad_loss.to(device="cuda", dtype=torch.float64).contiguous().reshape(())
    _check(lib().oo_radiosity_residual_bwd(C.byref(ts), C.byref(ms), C.byref(bs), _ptr(resid), _ptr(rhs), _ptr(g),
                                           arr(dfeat), arr(dW), arr(db), _ptr(workspace), _nbytes(workspace),
                                           _stream()),
           "oo_radiosity_residual_bwd")


def residual_node_indices(tree: Tree, mlp: MLP, batch: dict, workspace, feat=None, W=None):
    """Node index per level of every backward query, as the forward stored
    it in the workspace: int32 [Qb][L] (paper's scheme: [Qb][L][8]) in the
    caller's query order."""
    ts, ms, bs = tree.struct(feat), mlp.struct(W), batch_struct(batch)
    B, N = int(bs.B), int(bs.N)
    full = bs.grad_through_rhs and batch.get("target_override") is None and N > 0
    Qb = B * (1 + N) if full else B
    shape = (Qb, tree.n_levels) if tree.corners == 1 else (Qb, tree.n_levels, tree.corners)
    out = torch.full(shape, -2, dtype=torch.int32, device="cuda")
    _check(lib().oo_residual_node_indices(C.byref(ts), C.byref(ms), C.byref(bs), _ptr(workspace), _nbytes(workspace),
                                          _ptr(out), _stream()), "oo_residual_node_indices")
    return out


DOT_MAX_GROUPS, DOT_BLOCKS = 64, 256


def dot_f64(a, b=None):
    """FP64 inner products <a[g], b[g]> of lists of FP32 device tensors
    (b None: squared norms), summed on the GPU in a fixed order. Returns a
    FP64 device tensor [len(a)]."""
    a = [t.contiguous() for t in a]
    b = None if b is None else [t.contiguous() for t in b]
    G = len(a)
    if G > DOT_MAX_GROUPS:
        raise OOError(f"at most {DOT_MAX_GROUPS} groups")
    for i, t in enumerate(a):
        if t.dtype != torch.float32 or (b is not None and (b[i].dtype != torch.float32 or b[i].numel() != t.numel())):
            raise OOError("dot_f64 takes FP32 tensors of matching sizes")
    out = torch.empty(max(G, 1), dtype=torch.float64, device="cuda")
    part = torch.empty(max(G, 1) * DOT_BLOCKS, dtype=torch.float64, device="cuda")
    pa = (C.c_void_p * max(G, 1))(*[t.data_ptr() if t.numel() else None for t in a])
    pb = None if b is None else (C.c_void_p * max(G, 1))(*[t.data_ptr() if t.numel() else None for t in b])
    n = (C.c_int64 * max(G, 1))(*[t.numel() for t in a])
    _check(lib().oo_dot_f64(pa, pb, n, G, _ptr(out), _ptr(part), _stream()), "oo_dot_f64")
    return out[:G]


def dot_f64_noalloc(a, b=None, out=None):
    """dot_f64 through the entry point that allocates nothing: its partial
    sums live in the library's own per-device array. `out` (FP64 device
    tensor of at least len(a) elements) may be passed in, so that the call
    itself needs no allocation either."""
    a = [t.contiguous() for t in a]
    b = None if b is None else [t.contiguous() for t in b]
    G = len(a)
    for i, t in enumerate(a):
        if t.dtype != torch.float32 or (b is not None and (b[i].dtype != torch.float32 or b[i].numel() != t.numel())):
            raise OOError("dot_f64_noalloc takes FP32 tensors of matching sizes")
    if out is None:
        out = torch.empty(max(G, 1), dtype=torch.float64, device="cuda")
    if out.dtype != torch.float64 or out.numel() < G or not out.is_contiguous():
        raise OOError("out must be a contiguous FP64 tensor of at least len(a) elements")
    pa = (C.c_void_p * max(G, 1))(*[t.data_ptr() if t.numel() else None for t in a])
    pb = None if b is None else (C.c_void_p * max(G, 1))(*[t.data_ptr() if t.numel() else None for t in b])
    n = (C.c_int64 * max(G, 1))(*[t.numel() for t in a])
    _check(lib().oo_dot_f64_noalloc(pa, pb, n, G, _ptr(out), _stream()), "oo_dot_f64_noalloc")
    return out[:G]


def touched_nodes(tree: Tree, mlp: MLP, batch: dict, workspace, touched, feat=None, W=None):
    """Sets touched[node] = 1 (uint32 device tensor [n_nodes], cleared by
    the caller) for every node the forward's backward queries read."""
    ts, ms, bs = tree.struct(feat), mlp.struct(W), batch_struct(batch)
    assert touched.dtype == torch.int32 and touched.numel() == tree.level_offset[-1]
    _check(lib().oo_touched_nodes(C.byref(ts), C.byref(ms), C.byref(bs), _ptr(workspace), _nbytes(workspace),
                                  _ptr(touched), _stream()), "oo_touched_nodes")
    return touched


def adam_step(segments, step, lr=1e-3, beta1=0.9, beta2=0.99, eps=1e-15, work_dtype=torch.float32):
    """One fused Adam step. segments: list of dicts with FP32 device tensors
    param, grad, m, v, optional work (working copy) and optional touched
    (int32 per-block flags, block entries each)."""
    if len(segments) > ADAM_MAX_SEGMENTS:
        raise OOError(f"at most {ADAM_MAX_SEGMENTS} segments")
    arr = (_AdamSeg * max(1, len(segments)))()
    for i, sg in enumerate(segments):
        for k in ("param", "grad", "m", "v"):
            t = sg[k]
            if t.dtype != torch.float32 or not t.is_contiguous():
                raise OOError(f"segment {i}: {k} must be a contiguous FP32 tensor")
        arr[i].param, arr[i].grad = sg["param"].data_ptr(), sg["grad"].data_ptr()
        arr[i].m, arr[i].v = sg["m"].data_ptr(), sg["v"].data_ptr()
        arr[i].work = sg["work"].data_ptr() if sg.get("work") is not None else None
        arr[i].n = sg["param"].numel()
        arr[i].touched = sg["touched"].data_ptr() if sg.get("touched") is not None else None
        arr[i].block = int(sg.get("block", 0))
    cfg = _AdamCfg(float(lr), float(beta1), float(beta2), float(eps), int(step), DTYPE_CODE[work_dtype])
    _check(lib().oo_adam_step(C.byref(cfg), arr, len(segments), _stream()), "oo_adam_step")


PROF_KINDS = 11


def profile_begin(capacity: int = 4096):
    """Starts the library's launch timing (events around each kernel group)."""
    _check(lib().oo_profile_begin(int(capacity)), "oo_profile_begin")


def profile_end() -> dict:
    """Stops launch timing: {kind: (summed ms, timed launches)} for the kinds
    that ran."""
    ms = (C.c_double * PROF_KINDS)()
    n = (C.c_int64 * PROF_KINDS)()
    _check(lib().oo_profile_end(ms, n), "oo_profile_end")
    return {lib().oo_profile_kind_name(k).decode(): (ms[k], int(n[k])) for k in range(PROF_KINDS) if n[k]}


def cast_params(src, dst):
    assert src.dtype == torch.float32 and src.numel() == dst.numel()
    _check(lib().oo_cast_params(_ptr(src), _ptr(dst), DTYPE_CODE[dst.dtype], src.numel(), _stream()),
           "oo_cast_params")
    return dst


# ---------------------------------------------------------------------------
# Module and autograd
# ---------------------------------------------------------------------------

def _flat_layout(shapes, align=8):
    """Element offsets of tensors packed one after another in a flat buffer,
    each starting on a multiple of `align` elements (16 B for 16-bit
    elements, the tables' alignment requirement). Returns (offsets, total)."""
    offs, o = [], 0
    for sh in shapes:
        offs.append(o)
        n = int(np.prod(sh)) if len(sh) else 1
        o += (n + align - 1) // align * align
    return offs, max(o, align)


class OctaOctree(torch.nn.Module):
    """FP32 master feature tables and MLP weights as Parameters, with 16-bit
    working copies (refreshed by ``refresh()``) when ``dtype`` is FP16/BF16.

    Masters and working copies each live in one flat buffer with the same
    aligned layout, so a refresh is a single cast launch over the buffer."""

    def __init__(self, nodes, level_offset, res, C_, feat, W, b, dtype=torch.float32, interp=INTERP_NODE_BILINEAR,
                 disparity=None):
        """disparity: the paper's scheme only; dict(res, log2_T, tables, W, b)
        of the disparity predictor, kept as FP32 Parameters (no working copy:
        the predictor runs in FP32)."""
        super().__init__()
        self.dtype = dtype
        shapes = [tuple(np.shape(f)) for f in feat] + [tuple(np.shape(w)) for w in W]
        self._offs, total = _flat_layout(shapes)
        self._master = torch.zeros(total, dtype=torch.float32, device="cuda")
        views = []
        for src, sh, o in zip(list(feat) + list(W), shapes, self._offs):
            n = int(np.prod(sh)) if len(sh) else 1
            v = self._master[o:o + n].view(sh)
            v.copy_(_dev(src))
            views.append(torch.nn.Parameter(v))
        nf = len(feat)
        self.feat = torch.nn.ParameterList(views[:nf])
        self.W = torch.nn.ParameterList(views[nf:])
        self.b = torch.nn.ParameterList([torch.nn.Parameter(_dev(v)) for v in b])
        self.tree = Tree(nodes, level_offset, res, C_, list(self.feat), interp=interp)
        self.mlp = MLP(list(self.W), list(self.b))
        self.disp_params = []
        if disparity is not None:
            self.disp_tables = torch.nn.Parameter(_dev(disparity["tables"]))
            self.disp_W = torch.nn.ParameterList([torch.nn.Parameter(_dev(w)) for w in disparity["W"]])
            self.disp_b = torch.nn.ParameterList([torch.nn.Parameter(_dev(v)) for v in disparity["b"]])
            self.tree.disparity = Disparity(disparity["res"], disparity["log2_T"], self.disp_tables,
                                            list(self.disp_W), list(self.disp_b))
            self.disp_params = [self.disp_tables] + list(self.disp_W) + list(self.disp_b)
        self._ws = None
        self._work = None
        self._gen = 0
        self.work_feat, self.work_W = None, None
        self.refresh()

    def refresh(self):
        """Re-derive the working copies from the FP32 masters."""
        self._gen += 1  # a residual forward recorded before this refresh can no longer be differentiated
        with torch.no_grad():
            if self.dtype == torch.float32:
                self.work_feat, self.work_W = list(self.feat), list(self.W)
                return
            if self._work is None:
                self._work = torch.empty(self._master.numel(), dtype=self.dtype, device="cuda")
                views = [self._work[o:o + p.numel()].view(p.shape)
                         for p, o in zip(list(self.feat) + list(self.W), self._offs)]
                nf = len(self.feat)
                self.work_feat, self.work_W = views[:nf], views[nf:]
            cast_params(self._master, self._work)

    def forward(self, x, d, attr=None):
        """Radiance at (x, d) [B][3] (inference; no autograd); attr: the
        decoder's surface attributes [B][E] when it reads them."""
        return query_fwd(self.tree, self.mlp, x, d, feat=self.work_feat, W=self.work_W, attr=attr)

    def workspace(self, batch):
        """A workspace for explicit residual_fwd / residual_bwd calls on this
        batch: one buffer kept by the model and grown as needed, so a later
        call may overwrite what an earlier one left there."""
        n = residual_workspace_bytes(self.tree, self.mlp, batch, feat=self.work_feat, W=self.work_W)
        if self._ws is None or self._ws.numel() < n:
            self._ws = torch.empty(max(n, 256), dtype=torch.uint8, device="cuda")
        return self._ws

    def new_workspace(self, batch):
        """A workspace of its own for one forward/backward pair."""
        n = residual_workspace_bytes(self.tree, self.mlp, batch, feat=self.work_feat, W=self.work_W)
        return torch.empty(max(n, 256), dtype=torch.uint8, device="cuda")

    def residual(self, batch):
        """Loss of the residual step (0-dim FP64) with autograd to the masters."""
        return RadiosityResidual.apply(self, batch, *self.feat, *self.W, *self.b, *self.disp_params)

    def adam_segments(self, grads, state, touched=None):
        """oo_adam_step segments for this model's tables and layers: each
        level's table lazy over its nodes' flags (touched: int32 [n_nodes],
        or None for a dense step), weights and biases dense. grads and
        state['m'] / state['v']: lists shaped like feat + W + b."""
        params = list(self.feat) + list(self.W) + list(self.b) + self.disp_params
        works = (list(self.work_feat) + list(self.work_W) if self.dtype != torch.float32
                 else [None] * (len(self.feat) + len(self.W))) + [None] * (len(self.b) + len(self.disp_params))
        lo = self.tree.level_offset
        segs = []
        for i, p in enumerate(params):
            sg = dict(param=p.data.view(-1), grad=grads[i].view(-1), m=state["m"][i].view(-1),
                      v=state["v"][i].view(-1), work=None if works[i] is None else works[i].view(-1))
            if i < len(self.feat) and touched is not None and lo[i + 1] > lo[i]:
                sg.update(touched=touched[lo[i]:lo[i + 1]], block=p.numel() // (lo[i + 1] - lo[i]))
            segs.append(sg)
        return segs

    def new_adam_state(self):
        params = list(self.feat) + list(self.W) + list(self.b) + self.disp_params
        return {"m": [torch.zeros_like(p.data) for p in params], "v": [torch.zeros_like(p.data) for p in params],
                "t": 0}


class RadiosityResidual(torch.autograd.Function):
    """Neural-radiosity residual loss. Forward evaluates LHS and RHS queries
    and the FP64 loss; backward recomputes the LHS encoding, runs the decoder
    backward on matrix cores and scatters feature gradients with FP32
    atomics. Gradients w.r.t. the 16-bit working copies are returned for the
    FP32 masters.

    Each forward owns its workspace (the bucketed order, node indices and
    octahedral coordinates its backward reads), so several forwards may be
    summed before one backward. The backward refuses to run when the
    parameters it would differentiate changed after the forward: the FP32
    masters are saved tensors (an in-place update bumps their version), and
    a refresh of the 16-bit working copies bumps the model's generation."""

    @staticmethod
    def forward(ctx, model: OctaOctree, batch: dict, *params):
        ws = model.new_workspace(batch)
        lhs, rhs, res, loss = residual_fwd(model.tree, model.mlp, batch, ws, feat=model.work_feat,
                                           W=model.work_W)
        ctx.model, ctx.batch, ctx.ws, ctx.gen = model, batch, ws, model._gen
        ctx.save_for_backward(res, rhs, *params)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        model, batch = ctx.model, ctx.batch
        res, rhs = ctx.saved_tensors[:2]  # unpacking checks the masters' versions
        if model._gen != ctx.gen:
            raise OOError("RadiosityResidual: the working copies were refreshed after this forward")
        dfeat = [torch.zeros(f.shape, dtype=torch.float32, device="cuda") for f in model.feat]
        dW = [torch.zeros(w.shape, dtype=torch.float32, device="cuda") for w in model.W]
        db = [torch.zeros(v.shape, dtype=torch.float32, device="cuda") for v in model.b]
        dg = [torch.zeros(p.shape, dtype=torch.float32, device="cuda") for p in model.disp_params]
        nw = (len(dg) - 1) // 2
        residual_bwd(model.tree, model.mlp, batch, res, rhs, grad_loss, dfeat, dW, db, ctx.ws,
                     feat=model.work_feat, W=model.work_W,
                     disp_grads=(dg[0], dg[1:1 + nw], dg[1 + nw:]) if dg else None)
        return (None, None, *dfeat, *dW, *db, *dg)
