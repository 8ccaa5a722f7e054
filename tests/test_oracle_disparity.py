"""Pins for the oracle's disparity-shifted lookup (Sec. 3.3: the predicted
disparity d, the virtual point y = x + w_r / d and, per neighbouring cell
with centre c_j, the lookup direction along (x - c_j) d + w_r; Sec. 3.5: the
predictor is a multi-resolution hash encoding followed by a small MLP).

What fixes each part independently of the oracle's code:
 - hash encoding: at a grid vertex the encoding reads that vertex's entry
   alone, so a one-hot table shows which entry each vertex uses: a dense
   level is a bijection onto its (N+1)^3 vertices, a hashed level follows
   the published spatial hash (per-axis primes, xor, modulo the table),
   and between vertices the encoding is the trilinear hat (partition of
   unity, continuity across cell faces);
 - predictor: the MLP written out in numpy on [encoding, unit(w_r), 0];
 - shift: with maps that hold each vertex's point on the octahedron, every
   cell returns the octahedron point of its own shifted direction, so the
   level feature is sum_j w_j v_j / |v_j|_1 with v_j = (x - c_j) d + w_r /
   |w_r| from the geometry; d = 0 gives back the unshifted lookup;
 - adjoint: FP64 central differences of the loss for hash-table entries,
   the predictor's weights, vertex entries and the decoder.
"""
import numpy as np
import pytest

import oracle
from test_oracle_paper_interp import full_tree, octa_point, paper_problem, vertex_table

PAPER = oracle.INTERP_PAPER


def make_disp(seed, n_levels=4, F=2, log2_T=9, n_min=2, growth=1.7, widths=(16, 16), const=None, scale=0.5):
    g = np.random.default_rng(seed)
    res = [int(np.floor(n_min * growth ** i)) for i in range(n_levels)]
    tables = g.uniform(-scale, scale, (n_levels, 1 << log2_T, F)).astype(np.float32)
    dims = (n_levels * F + 4,) + tuple(widths) + (1,)
    W = [(g.uniform(-1, 1, (o, i)) * np.sqrt(6 / (i + o))).astype(np.float32) for i, o in zip(dims[:-1], dims[1:])]
    b = [(0.1 * g.normal(size=o)).astype(np.float32) for o in dims[1:]]
    if const is not None:
        W[-1][:] = 0.0
        b[-1][:] = const
    return oracle.Disparity(res, F, log2_T, tables, W, b)


def with_disp(tree, disp):
    return oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, tree.feat, interp=PAPER, disp=disp)


# ------------------------------ hash encoding ------------------------------

def vertices(N):
    i, j, k = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], 1)


def test_dense_level_is_a_bijection_and_reads_the_vertex():
    """A level whose vertices fit in the table: the entries read at the
    (N+1)^3 grid vertices are all different, and a query exactly at a
    vertex reads that entry with weight 1."""
    disp = make_disp(0, n_levels=3, F=1, log2_T=9, n_min=2, growth=2.0)  # N = 2, 4, 8: 27, 125, 729 vertices
    disp = oracle.Disparity(disp.res[:2], 1, 9, disp.tables[:2], disp.W, disp.b)
    for lvl, N in enumerate(disp.res):
        assert (N + 1) ** 3 <= 1 << disp.log2_T
        v = vertices(N)
        x = (v / N).astype(np.float32)
        assert np.all(x.astype(np.float64) * N == v)  # exact grid positions
        _, idx, w = oracle.hash_encode(disp, x)
        slot = idx[:, lvl][np.arange(len(v)), np.argmax(w[:, lvl], axis=1)]
        assert np.all(w[:, lvl].max(1) == 1.0)
        assert len(np.unique(slot)) == len(v)
        assert slot.max() < (N + 1) ** 3


def test_hashed_level_follows_the_spatial_hash():
    """A level with more vertices than entries: the entry of vertex (a, b, c)
    is (a * 1) xor (b * 2654435761) xor (c * 805459861) mod 2^32, then mod
    the table size; checked on each axis alone (where it reduces to one
    product) and on their xor."""
    disp = make_disp(1, n_levels=1, F=1, log2_T=6, n_min=32)
    N, T = disp.res[0], 1 << disp.log2_T
    assert (N + 1) ** 3 > T
    g = np.random.default_rng(3)
    v = np.concatenate([np.stack([np.arange(N + 1), np.zeros(N + 1, int), np.zeros(N + 1, int)], 1),
                        np.stack([np.zeros(N + 1, int), np.arange(N + 1), np.zeros(N + 1, int)], 1),
                        np.stack([np.zeros(N + 1, int), np.zeros(N + 1, int), np.arange(N + 1)], 1),
                        g.integers(0, N + 1, (300, 3))])
    x = (v / N).astype(np.float32)
    _, idx, w = oracle.hash_encode(disp, x)
    got = idx[:, 0][np.arange(len(v)), np.argmax(w[:, 0], axis=1)]
    primes = (1, 2654435761, 805459861)
    per_axis = [(v[:, a].astype(np.uint64) * primes[a]) % (1 << 32) for a in range(3)]
    want = (per_axis[0] ^ per_axis[1] ^ per_axis[2]) % T
    np.testing.assert_array_equal(got, want.astype(np.int64))
    # along the first axis alone the hash is the coordinate itself
    np.testing.assert_array_equal(got[:N + 1], np.arange(N + 1) % T)


def test_hash_encoding_is_the_trilinear_hat():
    """All-ones tables give 1 everywhere (weights sum to 1, also with
    collisions); the encoding is continuous across cell faces; between the
    vertices of a dense level it is the trilinear interpolation of the
    vertex values read there."""
    disp = make_disp(2, n_levels=3, F=2, log2_T=7, n_min=2, growth=2.0)  # N = 2, 4 dense; 8 hashed
    g = np.random.default_rng(4)
    x = g.uniform(0, 1, (500, 3)).astype(np.float32)
    ones = oracle.Disparity(disp.res, disp.F, disp.log2_T, np.ones_like(disp.tables), disp.W, disp.b)
    np.testing.assert_allclose(oracle.hash_encode(ones, x)[0], 1.0, atol=1e-14)
    for lvl, N in enumerate(disp.res):
        # a face between two cells, approached from both sides
        xf = x.copy()
        xf[:, 0] = (np.floor(x[:, 0] * N).clip(1, N - 1) / N).astype(np.float32)
        lo, hi = xf.copy(), xf.copy()
        lo[:, 0] = np.nextafter(xf[:, 0], np.float32(0))
        hi[:, 0] = np.nextafter(xf[:, 0], np.float32(1))
        e_lo, e_hi = oracle.hash_encode(disp, lo)[0], oracle.hash_encode(disp, hi)[0]
        sl = slice(lvl * disp.F, (lvl + 1) * disp.F)
        np.testing.assert_allclose(e_lo[:, sl], e_hi[:, sl], atol=1e-5)
    # dense level 0: interpolate the values read at the cell's 8 vertices
    N = disp.res[0]
    enc = oracle.hash_encode(disp, x)[0][:, :disp.F]
    p = np.clip(x.astype(np.float64), 0, 1) * N
    base = np.minimum(np.floor(p), N - 1)
    f = p - base
    want = np.zeros_like(enc)
    for d in range(8):
        bits = np.array([(d >> a) & 1 for a in range(3)])
        corner = ((base + bits) / N).astype(np.float32)
        val = oracle.hash_encode(disp, corner)[0][:, :disp.F]
        wd = np.prod(np.where(bits, f, 1 - f), axis=1)
        want += wd[:, None] * val
    np.testing.assert_allclose(enc, want, rtol=1e-12, atol=1e-13)


def test_predictor_is_the_mlp_of_encoding_and_unit_direction():
    disp = make_disp(5)
    g = np.random.default_rng(6)
    x = g.uniform(-0.1, 1.1, (200, 3)).astype(np.float32)
    d = (g.normal(size=(200, 3)) * g.uniform(0.1, 5, (200, 1))).astype(np.float32)
    enc = oracle.hash_encode(disp, x)[0]
    u = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)
    a = np.concatenate([enc, u, np.zeros((200, 1))], 1)
    for i, (W, b) in enumerate(zip(disp.W, disp.b)):
        a = a @ W.astype(np.float64).T + b
        if i < len(disp.W) - 1:
            a = np.maximum(a, 0.0)
    np.testing.assert_allclose(oracle.disparity(disp, x, d), a[:, 0], rtol=1e-12, atol=1e-13)


# ---------------------------------- shift ----------------------------------

def octahedron_tree(res):
    """A complete tree whose every vertex map holds the vertex's point on
    the octahedron |x| + |y| + |z| = 1."""
    D = len(res) - 1
    nodes, lo = full_tree(D)
    feat = []
    for l, R in enumerate(res):
        tab = vertex_table(R, lambda i, j: np.concatenate([octa_point(i / R, j / R), [0.0]]), garbage=0.0)
        n = int(lo[l + 1] - lo[l])
        feat.append(np.broadcast_to(tab.reshape(1, R + 1, R + 1, 4), (n, R + 1, R + 1, 4)).astype(np.float32))
    return oracle.Tree(nodes, lo, list(res), 4, feat, interp=PAPER)


@pytest.mark.parametrize("d0", [0.0, 0.7, 3.0, -1.5])
def test_shifted_lookup_closed_form(d0):
    """Every cell returns the octahedron point of its own direction
    v_j = (x - c_j) d + unit(w_r), c_j its centre (cell + 1/2) / 2^l, so
    the level feature is sum_j w_j v_j / |v_j|_1 with the (pinned) cells and
    renormalised weights of the neighbour search."""
    res = [8, 8, 4, 4]
    tree = with_disp(octahedron_tree(res), make_disp(7, const=d0))
    g = np.random.default_rng(8)
    x = g.uniform(0, 1, (400, 3)).astype(np.float32)
    w_r = (g.normal(size=(400, 3)) * 3.0).astype(np.float32)
    np.testing.assert_allclose(oracle.disparity(tree.disp, x, w_r), d0, atol=1e-15)
    h, _ = oracle.encode(tree, x, w_r)
    u = w_r.astype(np.float64) / np.linalg.norm(w_r.astype(np.float64), axis=1, keepdims=True)
    xc = np.clip(x.astype(np.float64), 0, 1)
    for l in range(len(res)):
        _, cells, wn = oracle.neighbours(tree, x, l)
        want = np.zeros((len(x), 3))
        for d in range(8):
            c = (cells[:, d].astype(np.float64) + 0.5) / 2 ** l
            v = (xc - c) * d0 + u
            want += wn[:, d, None] * v / np.abs(v).sum(1, keepdims=True)
        # the maps hold FP32-rounded octahedron points
        np.testing.assert_allclose(h[:, 4 * l:4 * l + 3], want, atol=2e-7)


def test_zero_disparity_is_the_unshifted_lookup():
    """d = 0 reads every cell along w_r: the residual and the feature
    gradients equal those of the tree without a predictor, and no gradient
    reaches the predictor's hash tables."""
    tree, mlp, batch = paper_problem(30, D=3, res=(4, 4, 2, 2), N=3, B=24, bias_scale=0.1)
    shifted = with_disp(tree, make_disp(9, const=0.0))
    for a, b in zip(oracle.residual_fwd(shifted, mlp, batch)[:3], oracle.residual_fwd(tree, mlp, batch)[:3]):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
    out = {}
    df_s, dW_s, _ = oracle.residual_bwd(shifted, mlp, batch, disp_out=out)
    df_t, dW_t, _ = oracle.residual_bwd(tree, mlp, batch)
    for a, b in zip(df_s, df_t):
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-15)
    # the output layer's weights are zero here: nothing flows below them
    assert np.all(out["tables"] == 0.0) and np.all(out["W"][0] == 0.0)
    assert np.abs(out["b"][-1]).max() > 0.0


# --------------------------------- adjoint ---------------------------------

def _loss(tree, mlp, batch):
    return oracle.residual_fwd(tree, mlp, batch)[3]


def _steps(theta, h):
    up, dn = np.float32(theta + h), np.float32(theta - h)
    return up, dn, float(up) - float(dn)


def _disp_with(disp, tables=None, W=None, b=None):
    return oracle.Disparity(disp.res, disp.F, disp.log2_T, disp.tables if tables is None else tables,
                            disp.W if W is None else W, disp.b if b is None else b)


@pytest.mark.parametrize("full", [0, 1])
def test_disparity_adjoint_matches_central_differences(full):
    """FP64 central differences of the loss against the adjoint for
    hash-table entries the batch reads, every layer of the predictor, vertex
    entries and decoder weights (target frozen in the detached mode)."""
    tree, mlp, batch = paper_problem(31, D=3, res=(4, 4, 2, 2), N=3, B=24, bias_scale=0.1)
    disp = make_disp(10, n_levels=3, F=2, log2_T=8, n_min=2, growth=2.0, scale=1.0)
    tree = with_disp(tree, disp)
    batch = dict(batch, grad_through_rhs=full)
    if not full:
        _, T, _, _ = oracle.residual_fwd(tree, mlp, batch)
        batch = dict(batch, target_override=T.astype(np.float32))
    out = {}
    dfeat, dW, _ = oracle.residual_bwd(tree, mlp, batch, disp_out=out)
    # the output bias enters d directly: its gradient is the sum of dL/dd
    np.testing.assert_allclose(out["b"][-1][0], out["dd"].sum(), rtol=1e-12, atol=1e-18)
    assert len(out["dd"]) == len(batch["x"]) * (1 + (batch["N"] if full else 0))
    g = np.random.default_rng(11)
    # small enough that no step crosses a ReLU kink of either network (the
    # closest hidden pre-activation of the predictor sits 3.6e-5 from zero)
    h = 1e-5
    got, want = [], []
    # hash entries read by the LHS queries
    _, hidx, hw = oracle.hash_encode(disp, batch["x"])
    for _ in range(16):
        b = int(g.integers(len(batch["x"])))
        i, d, e = int(g.integers(disp.res.__len__())), int(g.integers(8)), int(g.integers(disp.F))
        flat = (i * (1 << disp.log2_T) + hidx[b, i, d]) * disp.F + e
        up, dn, step = _steps(disp.tables.reshape(-1)[flat], h)

        def at(v):
            t = disp.tables.copy()
            t.reshape(-1)[flat] = v
            return _loss(with_disp(tree, _disp_with(disp, tables=t)), mlp, batch)
        got.append(out["tables"].reshape(-1)[flat])
        want.append((at(up) - at(dn)) / step)
    # the predictor's weights and biases
    for li in range(len(disp.W)):
        for which in ("W", "b"):
            src = (disp.W if which == "W" else disp.b)[li]
            flat = int(g.integers(src.size))
            up, dn, step = _steps(src.reshape(-1)[flat], h)

            def at(v):
                Ws, bs = [w.copy() for w in disp.W], [v_.copy() for v_ in disp.b]
                (Ws if which == "W" else bs)[li].reshape(-1)[flat] = v
                return _loss(with_disp(tree, _disp_with(disp, W=Ws, b=bs)), mlp, batch)
            got.append(out[which][li].reshape(-1)[flat])
            want.append((at(up) - at(dn)) / step)
    # vertex entries and the decoder's first layer
    for _ in range(8):
        l = int(g.integers(tree.n_levels))
        nz = np.flatnonzero(dfeat[l])
        flat = int(nz[g.integers(len(nz))])
        up, dn, step = _steps(tree.feat[l].reshape(-1)[flat], h)

        def at(v):
            feat = [f.copy() for f in tree.feat]
            feat[l].reshape(-1)[flat] = v
            return _loss(oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, feat, interp=PAPER, disp=disp),
                         mlp, batch)
        got.append(dfeat[l].reshape(-1)[flat])
        want.append((at(up) - at(dn)) / step)
    got, want = np.array(got), np.array(want)
    assert np.abs(want).max() > 0
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err < 1e-5, (err, [(i, a, b) for i, (a, b) in enumerate(zip(got, want)) if abs(a - b) > 1e-6 * abs(b) + 1e-12])
