"""Host-side checks of liboctaoctree (no GPU needed): every symbol declared in
include/octaoctree.h is exported, the host octree builder is bit-identical to
the oracle's independent builder, and argument validation rejects bad input
before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2606_08469_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(binding.LIB_PATH):
        from paper_2606_08469_amd import build as pbuild
        pbuild.build()
    return binding.lib()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "octaoctree.h")).read()
    names = set(re.findall(r"^\s*(?:int|const char\*)\s+(oo_\w+)\s*\(", hdr, re.M))
    assert len(names) == 17, names
    for n in sorted(names):
        assert hasattr(L, n), n


@pytest.mark.parametrize("D,tau,n,seed", [(0, 4, 10, 0), (1, 2, 50, 1), (4, 32, 20000, 2), (6, 3, 3000, 3),
                                          (10, 8, 5000, 4), (15, 1, 300, 5)])
def test_builder_matches_oracle(L, D, tau, n, seed):
    g = np.random.default_rng(seed)
    x = (g.uniform(0, 1, (n, 3)) ** 2).astype(np.float32)
    x[: n // 10] = g.choice([0.0, 0.5, 1.0, -0.25, 1.5], (n // 10, 3))
    nodes, lo = binding.build_octree(x, D, tau)
    onodes, olo = oracle.build_octree(x, D, tau)
    np.testing.assert_array_equal(lo, olo)
    np.testing.assert_array_equal(nodes, onodes)


def test_builder_matches_oracle_config1(L):
    cfg = synth.CONFIGS[1]
    s = synth.tree_samples(cfg)
    nodes, lo = binding.build_octree(s, cfg.D, cfg.tau)
    onodes, olo = oracle.build_octree(s, cfg.D, cfg.tau)
    np.testing.assert_array_equal(nodes, onodes)
    np.testing.assert_array_equal(lo, olo)


def test_builder_size_query_and_capacity(L):
    x = np.random.default_rng(0).uniform(0, 1, (500, 3)).astype(np.float32)
    lo = np.zeros(5, np.int64)
    nn = np.zeros(1, np.int64)
    assert L.oo_build_octree(x.ctypes.data, 500, 3, 4, None, 0, lo.ctypes.data, nn.ctypes.data) == 0
    need = int(nn[0])
    small = np.zeros(need - 1, np.uint32)
    rc = L.oo_build_octree(x.ctypes.data, 500, 3, 4, small.ctypes.data, need - 1, lo.ctypes.data, nn.ctypes.data)
    assert rc == -2 and int(nn[0]) == need and b"capacity" in L.oo_last_error()
    assert L.oo_build_octree(x.ctypes.data, 500, -1, 4, None, 0, lo.ctypes.data, nn.ctypes.data) == -1
    assert L.oo_build_octree(x.ctypes.data, 500, 16, 4, None, 0, lo.ctypes.data, nn.ctypes.data) == -1


def _tree(n_levels=3, C_=8, res=(4, 4, 2), dtype=binding.F16):
    t = binding._Tree()
    t.n_levels, t.C = n_levels, C_
    for l, r in enumerate(res):
        t.res[l] = r
    for l in range(n_levels + 1):
        t.level_offset[l] = min(l, 1) + max(0, l - 1) * 2
    t.nodes = 0x1000
    t.feat_dtype = dtype
    for l in range(n_levels):
        t.feat[l] = 0x10000 * (l + 1)
    return t


def _mlp(K0=24, H=64, n_layers=3, dtype=binding.F16):
    m = binding._MLP()
    m.n_layers = n_layers
    m.dims[0] = K0
    for i in range(1, n_layers):
        m.dims[i] = H
    m.dims[n_layers] = 3
    m.dtype = dtype
    for i in range(n_layers):
        m.W[i] = 0x2000 * (i + 1)
        m.b[i] = 0x3000 * (i + 1)
    return m


def test_validation_errors(L):
    t, m = _tree(), _mlp()
    stream = None
    x = C.c_void_p(0x4000)
    # B = 0 is a no-op
    assert L.oo_query_fwd(C.byref(t), C.byref(m), x, x, None, 0, x, stream) == 0
    bad = _tree()
    bad.C = 5
    assert L.oo_query_fwd(C.byref(bad), C.byref(m), x, x, None, 16, x, stream) == -1
    bad = _tree()
    bad.res[1] = 3
    assert L.oo_query_fwd(C.byref(bad), C.byref(m), x, x, None, 16, x, stream) == -1
    bad = _tree()
    bad.res[0] = 128  # texel maps stop at 64 per side, vertex maps at 512
    assert L.oo_query_fwd(C.byref(bad), C.byref(m), x, x, None, 16, x, stream) == -1
    bad.interp, bad.res[0] = 1, 1024
    assert L.oo_query_fwd(C.byref(bad), C.byref(m), x, x, None, 16, x, stream) == -1
    assert b"512" in L.oo_last_error()
    bad = _tree()
    bad.feat[1] = 0x10008  # not 16-byte aligned
    assert L.oo_query_fwd(C.byref(bad), C.byref(m), x, x, None, 16, x, stream) == -1
    bad = _tree()
    bad.n_levels = 0
    assert L.oo_encode_query(C.byref(bad), x, x, 4, x, 0, None, stream) == -1
    assert L.oo_query_fwd(C.byref(t), C.byref(_mlp(K0=20)), x, x, None, 16, x, stream) == -1     # dims[0] != L*C
    assert L.oo_query_fwd(C.byref(t), C.byref(_mlp(H=96)), x, x, None, 16, x, stream) == -4      # width unsupported
    assert L.oo_query_fwd(C.byref(t), C.byref(_mlp(H=128, n_layers=6)), x, x, None, 16, x, stream) == -4  # > 5 layers
    assert L.oo_query_fwd(C.byref(t), C.byref(_mlp(dtype=binding.BF16)), x, x, None, 16, x, stream) == -4  # dtype pair
    assert L.oo_query_fwd(C.byref(t), C.byref(m), x, x, None, -1, x, stream) == -1
    assert L.oo_cast_params(x, x, 7, 4, stream) == -1
    assert L.oo_cast_params(x, x, 1, -2, stream) == -1
    assert b"" != L.oo_last_error()


def test_profile_host_paths(L):
    """Launch timing: argument checks and kind names (host only; enabling it
    creates HIP events, which needs a device)."""
    L.oo_profile_kind_name.restype = C.c_char_p
    assert L.oo_profile_end(None, None) == -1          # not enabled
    assert b"not enabled" in L.oo_last_error()
    assert L.oo_profile_begin(0) == -1
    assert L.oo_profile_begin(1 << 21) == -1
    names = [L.oo_profile_kind_name(k) for k in range(binding.PROF_KINDS)]
    assert names[1] == b"query" and names[5] == b"backward" and names[6] == b"scatter"
    assert len(set(names)) == binding.PROF_KINDS and all(names)
    assert L.oo_profile_kind_name(binding.PROF_KINDS) == b"" and L.oo_profile_kind_name(-1) == b""
    hdr = open(os.path.join(ROOT, "include", "octaoctree.h")).read()
    assert f"#define OO_PROF_KINDS {binding.PROF_KINDS}" in hdr


def test_residual_batch_validation(L):
    t, m = _tree(), _mlp()
    b = binding._Batch()
    b.B, b.N = 8, 2
    b.x = b.dir = b.Le = 0x5000
    n = C.c_size_t(0)
    assert L.oo_residual_workspace_bytes(C.byref(t), C.byref(m), C.byref(b), C.byref(n)) == -1  # x2 etc missing
    b.n = b.wo = b.albedo = b.rough = b.x2 = b.dir2 = b.wi = 0x5000
    b.loss_kind = 3
    assert L.oo_residual_workspace_bytes(C.byref(t), C.byref(m), C.byref(b), C.byref(n)) == -1
    b.loss_kind = 0
    b.N = -1
    assert L.oo_residual_workspace_bytes(C.byref(t), C.byref(m), C.byref(b), C.byref(n)) == -1


def test_residual_rejects_small_workspace(L):
    """A workspace smaller than oo_residual_workspace_bytes reports is
    refused before anything is launched (the pointers here are never
    dereferenced)."""
    t, m = _tree(), _mlp()
    b = binding._Batch()
    b.B, b.N = 8, 2
    b.x = b.dir = b.Le = b.n = b.wo = b.albedo = b.rough = b.x2 = b.dir2 = b.wi = 0x5000
    n = C.c_size_t(0)
    assert L.oo_residual_workspace_bytes(C.byref(t), C.byref(m), C.byref(b), C.byref(n)) == 0
    need = n.value
    assert need > 0
    p = C.c_void_p(0x5000)
    rc = L.oo_radiosity_residual_fwd(C.byref(t), C.byref(m), C.byref(b), p, p, p, p, p, need - 1, None)
    assert rc == -1 and b"workspace" in L.oo_last_error()
    ptrs = (C.c_void_p * 8)(*([0x5000] * 8))
    rc = L.oo_radiosity_residual_bwd(C.byref(t), C.byref(m), C.byref(b), p, p, p, ptrs, ptrs, ptrs, p, need - 1,
                                     None)
    assert rc == -1 and b"workspace" in L.oo_last_error()
    rc = L.oo_residual_node_indices(C.byref(t), C.byref(m), C.byref(b), p, need - 1, p, None)
    assert rc == -1 and b"workspace" in L.oo_last_error()


def test_surface_attribute_validation(L):
    """A decoder wider than the level features reads E = dims[0] - L C
    surface attributes per query: the query and residual calls refuse a
    missing attr (and attr2 when the RHS is estimated) before any device
    work, and an input width that is not a multiple of 4."""
    t = _tree()
    x = C.c_void_p(0x4000)
    wide = _mlp(K0=24 + 16)
    assert L.oo_query_fwd(C.byref(t), C.byref(wide), x, x, None, 16, x, None) == -1
    assert b"attr" in L.oo_last_error()
    assert L.oo_query_fwd(C.byref(t), C.byref(_mlp(K0=24 + 13)), x, x, x, 16, x, None) == -4  # not a multiple of 4
    assert b"multiple of 4" in L.oo_last_error()
    assert L.oo_query_fwd(C.byref(t), C.byref(_mlp(K0=132)), x, x, x, 16, x, None) == -4      # wider than 128
    b = binding._Batch()
    b.B, b.N = 8, 2
    b.x = b.dir = b.Le = b.n = b.wo = b.albedo = b.rough = b.x2 = b.dir2 = b.wi = 0x5000
    n = C.c_size_t(0)
    assert L.oo_residual_workspace_bytes(C.byref(t), C.byref(wide), C.byref(b), C.byref(n)) == 0
    p = C.c_void_p(0x5000)
    ptrs = (C.c_void_p * 8)(*([0x5000] * 8))
    for attr, attr2, word in ((0, 0, b"attr is"), (0x5000, 0, b"attr2")):
        b.attr, b.attr2 = attr, attr2
        rc = L.oo_radiosity_residual_fwd(C.byref(t), C.byref(wide), C.byref(b), p, p, p, p, p, n.value, None)
        assert rc == -1 and word in L.oo_last_error()
        rc = L.oo_radiosity_residual_bwd(C.byref(t), C.byref(wide), C.byref(b), p, p, p, ptrs, ptrs, ptrs, p,
                                         n.value, None)
        assert rc == -1 and word in L.oo_last_error()
    # with the target frozen no secondary query is made: attr2 is not needed
    b.target_override = 0x5000
    b.attr, b.attr2 = 0x5000, 0
    rc = L.oo_radiosity_residual_fwd(C.byref(t), C.byref(wide), C.byref(b), p, p, p, p, None, n.value, None)
    assert rc == -1 and b"loss_out" in L.oo_last_error()


def _disp(n_levels=16, F=2, n_layers=3, hidden=64, log2_T=10):
    g = binding._Disparity()
    g.n_levels, g.F, g.log2_T = n_levels, F, log2_T
    for i in range(n_levels):
        g.res[i] = 16 + i
    g.tables = 0x8000
    g.n_layers = n_layers
    g.dims[0] = n_levels * F + 4
    for i in range(1, n_layers):
        g.dims[i] = hidden
    g.dims[n_layers] = 1
    for i in range(n_layers):
        g.W[i], g.b[i] = 0x9000 + 0x100 * i, 0xa000 + 0x100 * i
    return g


def test_disparity_validation(L):
    """The disparity predictor: only with the paper's scheme, only the GPU
    shape (16 hash levels of 2 features, hidden width 64, 1 or 2 hidden
    layers), and the residual backward needs its gradient accumulators; all
    refused before any device work."""
    x = C.c_void_p(0x4000)
    m = _mlp()

    def tree_with(g, interp=1):
        t = _tree()
        t.interp = interp
        t.disparity = C.pointer(g)
        return t

    cases = [(tree_with(_disp(), interp=0), -1, b"OO_INTERP_PAPER"),
             (tree_with(_disp(n_levels=8)), -4, b"n_levels"),
             (tree_with(_disp(F=4)), -4, b"F must"),
             (tree_with(_disp(hidden=32)), -4, b"hidden"),
             (tree_with(_disp(n_layers=4)), -4, b"n_layers"),
             (tree_with(_disp(log2_T=30)), -1, b"log2_T")]
    for t, rc, word in cases:
        assert L.oo_query_fwd(C.byref(t), C.byref(m), x, x, None, 16, x, None) == rc
        assert word in L.oo_last_error(), L.oo_last_error()
    g = _disp()
    g.tables = 0x8004  # not 8-byte aligned
    assert L.oo_query_fwd(C.byref(tree_with(g)), C.byref(m), x, x, None, 16, x, None) == -1
    # the backward needs the gradient accumulators
    t = tree_with(_disp())
    b = binding._Batch()
    b.B, b.N = 8, 0
    b.x = b.dir = b.Le = 0x5000
    n = C.c_size_t(0)
    assert L.oo_residual_workspace_bytes(C.byref(t), C.byref(m), C.byref(b), C.byref(n)) == 0
    p = C.c_void_p(0x5000)
    ptrs = (C.c_void_p * 8)(*([0x5000] * 8))
    rc = L.oo_radiosity_residual_bwd(C.byref(t), C.byref(m), C.byref(b), p, p, p, ptrs, ptrs, ptrs, p, n.value, None)
    assert rc == -1 and b"disparity dW" in L.oo_last_error()
    # and its buffers are part of the workspace
    plain = _tree()
    plain.interp = 1
    n0 = C.c_size_t(0)
    assert L.oo_residual_workspace_bytes(C.byref(plain), C.byref(m), C.byref(b), C.byref(n0)) == 0
    assert n.value > n0.value


def test_dot_and_node_readback_validation(L):
    """Argument checks of oo_dot_f64 and oo_residual_node_indices that fail
    before any device work."""
    vp = C.c_void_p
    out = vp(16)
    assert L.oo_dot_f64(None, None, None, 0, None, None, None) == 0           # no groups: no-op
    assert L.oo_dot_f64(None, None, None, -1, out, out, None) == -1
    assert L.oo_dot_f64(None, None, None, binding.DOT_MAX_GROUPS + 1, out, out, None) == -1
    n = (C.c_int64 * 1)(5)
    a = (vp * 1)(None)
    assert L.oo_dot_f64(a, None, n, 1, out, out, None) == -1                 # NULL array with n > 0
    assert b"a[0]" in L.oo_last_error()
    n[0] = -3
    a[0] = 16
    assert L.oo_dot_f64(a, None, n, 1, out, out, None) == -1                 # negative size


def test_interp_scheme_validation_and_workspace(L):
    """An unknown interpolation scheme is refused before any device work;
    the paper's scheme stores eight corner nodes and a position per backward
    query, and uses no pair buffers, which the workspace size reflects."""
    t, m = _tree(), _mlp()
    x = C.c_void_p(0x4000)
    bad = _tree()
    bad.interp = 2
    assert L.oo_encode_query(C.byref(bad), x, x, 4, x, 0, None, None) == -1
    assert b"interp" in L.oo_last_error()
    assert L.oo_query_fwd(C.byref(bad), C.byref(m), x, x, None, 16, x, None) == -1
    b = binding._Batch()
    b.B, b.N = 1000, 0
    b.x = b.dir = b.Le = 0x5000
    n0, n1 = C.c_size_t(0), C.c_size_t(0)
    assert L.oo_residual_workspace_bytes(C.byref(t), C.byref(m), C.byref(b), C.byref(n0)) == 0
    paper = _tree()
    paper.interp = 1
    assert L.oo_residual_workspace_bytes(C.byref(paper), C.byref(m), C.byref(b), C.byref(n1)) == 0
    # 7 more node indices per level (3 levels, int32) and 16 B of position per query, 256-byte rounding aside
    extra = 1000 * (3 * 7 * 4 + 16)
    assert extra - 512 <= n1.value - n0.value <= extra + 512, (n0.value, n1.value)


def test_adam_validation(L):
    """oo_adam_step refuses bad hyper-parameters and segments before any
    launch."""
    cfg = binding._AdamCfg(1e-3, 0.9, 0.99, 1e-15, 1, binding.F16)
    segs = (binding._AdamSeg * 2)()
    for sg in segs:
        sg.param = sg.grad = sg.m = sg.v = 0x1000
        sg.n = 64
    assert L.oo_adam_step(C.byref(cfg), segs, 0, None) == 0                       # nothing to do
    assert L.oo_adam_step(C.byref(cfg), segs, binding.ADAM_MAX_SEGMENTS + 1, None) == -1
    bad = binding._AdamCfg(1e-3, 0.9, 0.99, 1e-15, 0, binding.F16)
    assert L.oo_adam_step(C.byref(bad), segs, 2, None) == -1 and b"step" in L.oo_last_error()
    bad = binding._AdamCfg(1e-3, 1.0, 0.99, 1e-15, 1, binding.F16)
    assert L.oo_adam_step(C.byref(bad), segs, 2, None) == -1
    segs[1].touched, segs[1].block = 0x2000, 6                                     # block not a multiple of 4
    assert L.oo_adam_step(C.byref(cfg), segs, 2, None) == -1 and b"block" in L.oo_last_error()
    segs[1].touched, segs[1].param = None, None
    assert L.oo_adam_step(C.byref(cfg), segs, 2, None) == -1 and b"required" in L.oo_last_error()
