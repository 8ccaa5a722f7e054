"""Pins for the oracle's version of the paper's own interpolation: barycentric
lookup on vertex-stored octahedral maps (Sec. 3.3) and the blend of the 8
neighbouring octree cells, trilinear and renormalised over the non-empty
ones (Sec. 3.4, level-feature equation).

What fixes each part independently of the oracle's code:
 - map size: the paper's count of stored entries for its 8-level
   configuration (Sec. 4.3, Table 2 and the per-level statistics);
 - triangle choice and barycentric weights: every octahedron face is affine
   in map coordinates, so a map holding each vertex's point on the
   octahedron |x| + |y| + |z| = 1 must return the query direction's own
   octahedron point exactly; a triangle that straddles a face edge fails;
 - the seam: border vertices that are one direction share one slot, so the
   lookup is continuous across the folded seams and at the pole even when
   the unused slots hold garbage;
 - neighbour search: brute force over every node's cell;
 - trilinear weights: on a complete tree, maps that hold an affine function
   of the node's cell centre reproduce it at any interior point; the
   renormalisation: constant maps give the constant even next to empty cells.
"""
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = oracle.INTERP_PAPER


def read_table2():
    levels, extra = [], {}
    for line in open(os.path.join(HERE, "golden", "table2_vertex_entries.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        parts = line.split()
        if parts[0].isdigit():
            levels.append(tuple(int(v) for v in parts))
        else:
            extra[parts[0]] = int(parts[1])
    return levels, extra


def test_table2_entry_count():
    levels, extra = read_table2()
    total = sum(n * oracle.map_entries(vres - 1, PAPER) for _, _, vres, n in levels)
    assert total == extra["total_entries"]
    assert round(total * 4 * 4 / 2 ** 20) == extra["storage_MB"]
    # a texel map of R x R entries does not give the paper's count
    assert sum(n * oracle.map_entries(vres - 1, oracle.INTERP_NODE_BILINEAR) for _, _, vres, n in levels) != total
    # spatial and directional resolution run in opposite directions
    assert all(s * (v - 1) == 1024 for _, s, v, _ in levels)


def octa_point(s, t):
    """Point of the octahedron |x| + |y| + |z| = 1 at map coordinate (s, t):
    inside the diamond the upper hemisphere, outside it the folded lower
    one (the inverse of the fold, written independently of the oracle)."""
    u, v = 2.0 * s - 1.0, 2.0 * t - 1.0
    z = 1.0 - abs(u) - abs(v)
    if z >= 0.0:
        return np.array([u, v, z])
    su, sv = (1.0 if u >= 0 else -1.0), (1.0 if v >= 0 else -1.0)
    return np.array([su * (1.0 - abs(v)), sv * (1.0 - abs(u)), z])


def vertex_table(R, fill, garbage=None, seed=0):
    """(R+1)^2 slots; fill(i, j) at each vertex's canonical slot (found by
    asking the oracle which slot a query exactly at that vertex reads);
    slots never read hold `garbage` (NaN by default)."""
    g = np.random.default_rng(seed)
    C = len(fill(0, 0))
    tab = np.full(((R + 1) ** 2, C), np.nan if garbage is None else garbage, np.float64)
    for j in range(R + 1):
        for i in range(R + 1):
            st = np.array([[min(i / R, 1.0), min(j / R, 1.0)]])
            ij, w, v = oracle.bary(st, R)
            k = int(np.argmax(w[0]))
            tab[v[0, k]] = fill(i, j)
    return tab


def lookup(tab, st, R):
    _, w, v = oracle.bary(st, R)
    return np.einsum("bk,bkc->bc", w, tab[v])


@pytest.mark.parametrize("R", [2, 4, 8, 16, 64])
def test_bary_weights_and_position(R):
    g = np.random.default_rng(R)
    st = g.uniform(0, 1, (4000, 2))
    st[:100] = np.round(st[:100] * R) / R  # on grid lines and vertices
    ij, w, _ = oracle.bary(st, R)
    assert np.all(w >= -1e-15) and np.allclose(w.sum(1), 1.0, atol=1e-14)
    pos = np.einsum("bk,bka->ba", w, ij.astype(np.float64)) / R
    np.testing.assert_allclose(pos, st, atol=1e-13)
    # the three vertices form a right isosceles triangle of one grid cell
    lo = ij.min(axis=1)
    assert np.all(ij.max(axis=1) - lo == 1)
    assert np.all((0 <= ij) & (ij <= R))


@pytest.mark.parametrize("R", [2, 4, 8, 32])
def test_bary_reproduces_octahedron(R):
    """Vertices hold their octahedron points; every query returns its own."""
    tab = vertex_table(R, lambda i, j: octa_point(i / R, j / R))
    g = np.random.default_rng(R + 1)
    d = g.normal(size=(5000, 3))
    d[:200, 2] = 0.0                          # equator
    d[200:400, 0] = 0.0                       # seams of the lower hemisphere
    d[200:300, 2] = -np.abs(d[200:300, 2])
    d[400:500, 1] = 0.0
    d[400:500, 2] = -np.abs(d[400:500, 2])
    d = d.astype(np.float32)
    st = oracle.octa(d)
    got = lookup(tab, st, R)
    d64 = d.astype(np.float64)
    want = d64 / np.abs(d64).sum(1, keepdims=True)
    np.testing.assert_allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("R", [2, 4, 16])
def test_bary_seam_and_pole_continuity(R):
    """Random vertex maps (unused slots NaN): the value is continuous across
    the folded seams (w_x = 0 or w_y = 0 below the equator), across the
    equator, and at the -z pole."""
    g = np.random.default_rng(3 * R)
    vals = g.normal(size=((R + 1) ** 2, 4))
    tab = vertex_table(R, lambda i, j: vals[j * (R + 1) + i])
    assert np.isnan(tab).any() or R < 2
    for delta in (1e-3, 1e-5):
        base = g.normal(size=(500, 3))
        for axis, lower in ((0, True), (1, True), (2, False)):
            p = base.copy()
            p[:, axis] = 0.0
            if lower:
                p[:, 2] = -np.abs(p[:, 2]) - 0.1
            a, b = p.copy(), p.copy()
            a[:, axis] += delta
            b[:, axis] -= delta
            va = lookup(tab, oracle.octa(a.astype(np.float32)), R)
            vb = lookup(tab, oracle.octa(b.astype(np.float32)), R)
            assert np.all(np.isfinite(va)) and np.all(np.isfinite(vb))
            assert np.max(np.abs(va - vb)) < 50 * R * delta * np.abs(vals).max(), (axis, delta)
    pole = np.array([[1e-6, 2e-6, -1.0], [-1e-6, 1e-6, -1.0], [1e-6, -3e-6, -1.0], [-2e-6, -1e-6, -1.0]],
                    np.float32)
    vp = lookup(tab, oracle.octa(pole), R)
    assert np.max(np.abs(vp - vp[0])) < 1e-3


def full_tree(D):
    """Every cell of every level exists (samples at every finest cell
    centre, refine at more than 0 samples)."""
    n = 2 ** D
    c = (np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) / n
    return oracle.build_octree(c.astype(np.float32), D, 0)


def node_cells(nodes, lo):
    """Integer cell of every node, recovered by walking child masks."""
    cells = np.zeros((int(lo[-1]), 3), np.int64)
    for l in range(len(lo) - 2):
        for v in range(lo[l], lo[l + 1]):
            w = int(nodes[v])
            mask, first = w & 0xFF, w >> 8
            k = 0
            for o in range(8):
                if (mask >> o) & 1:
                    cells[first + k] = 2 * cells[v] + [(o >> a) & 1 for a in range(3)]
                    k += 1
    return cells


def sparse_tree(seed=0, D=4, n=400, tau=3):
    g = np.random.default_rng(seed)
    s = (g.uniform(0, 1, (n, 3)) ** 2).astype(np.float32)
    return oracle.build_octree(s, D, tau)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_neighbours_brute_force(seed):
    nodes, lo = sparse_tree(seed)
    D = len(lo) - 2
    cells = node_cells(nodes, lo)
    tree = oracle.Tree(nodes, lo, [2] * (D + 1), 4, [np.zeros((int(lo[l + 1] - lo[l]), 3, 3, 4), np.float32)
                                                    for l in range(D + 1)], interp=PAPER)
    g = np.random.default_rng(seed + 10)
    x = g.uniform(0, 1, (300, 3)).astype(np.float32)
    x[:20] = np.array([0.0, 1.0, 0.5], np.float32)[g.integers(3, size=(20, 3))]
    for l in range(D + 1):
        idx, cc, w = oracle.neighbours(tree, x, l)
        lookup_ = {tuple(c): v for v, c in zip(range(lo[l], lo[l + 1]), cells[lo[l]:lo[l + 1]])}
        for b in range(len(x)):
            xc = np.clip(x[b].astype(np.float64), 0, 1) * 2 ** l - 0.5
            lo_c = np.floor(xc).astype(np.int64)
            for d in range(8):
                want_c = lo_c + [(d >> a) & 1 for a in range(3)]
                assert tuple(cc[b, d]) == tuple(want_c)
                assert idx[b, d] == lookup_.get(tuple(want_c), -1)
            assert np.isclose(w[b].sum(), 1.0) or (w[b].sum() == 0 and np.all(idx[b] < 0))
            assert np.all(w[b][idx[b] < 0] == 0)


def paper_tree(nodes, lo, res, C, fill_level):
    feat = [fill_level(l, int(lo[l + 1] - lo[l]), R) for l, R in enumerate(res)]
    return oracle.Tree(nodes, lo, list(res), C, feat, interp=PAPER)


def test_trilinear_reproduces_affine_on_full_tree():
    D = 3
    nodes, lo = full_tree(D)
    cells = node_cells(nodes, lo)
    res = [4, 4, 2, 2]
    a, c0 = np.array([0.7, -1.3, 2.1]), 0.25

    def fill(l, n, R):
        centre = (cells[lo[l]:lo[l + 1]] + 0.5) / 2 ** l
        f = centre @ a + c0
        return np.repeat(f[:, None, None, None], (R + 1) ** 2 * 4, axis=1).reshape(n, R + 1, R + 1, 4).astype(np.float64)

    tree = paper_tree(nodes, lo, res, 4, lambda l, n, R: fill(l, n, R).astype(np.float32))
    g = np.random.default_rng(4)
    x = g.uniform(0, 1, (2000, 3)).astype(np.float32)
    dirs = g.normal(size=(2000, 3)).astype(np.float32)
    h, _ = oracle.encode(tree, x, dirs)
    # level 0 has one cell: the blend is its value wherever x is
    np.testing.assert_allclose(h[:, 0], np.float32(0.5 * a.sum() + c0), rtol=1e-7)
    for l in range(1, D + 1):
        # between the outermost cell centres all 8 neighbours exist; the
        # maps hold FP32-rounded values, hence the tolerance
        inner = np.all((x >= 0.5 / 2 ** l) & (x <= 1 - 0.5 / 2 ** l), axis=1)
        assert inner.sum() > 100
        want = x[inner].astype(np.float64) @ a + c0
        np.testing.assert_allclose(h[inner, 4 * l], want, atol=2e-6)
        # outside it the missing cells are dropped: no longer affine in x
        assert np.max(np.abs(h[~inner, 4 * l] - (x[~inner].astype(np.float64) @ a + c0))) > 1e-2


@pytest.mark.parametrize("seed", [0, 1])
def test_renormalised_constant_next_to_empty_cells(seed):
    nodes, lo = sparse_tree(seed)
    D = len(lo) - 2
    res = [4] * (D + 1)
    tree = paper_tree(nodes, lo, res, 4,
                      lambda l, n, R: np.full((n, R + 1, R + 1, 4), 0.75 + l, np.float32))
    g = np.random.default_rng(seed)
    x = g.uniform(0, 1, (400, 3)).astype(np.float32)
    d = g.normal(size=(400, 3)).astype(np.float32)
    h, _ = oracle.encode(tree, x, d)
    partial = 0
    for l in range(D + 1):
        idx, _, _ = oracle.neighbours(tree, x, l)
        any_ = (idx >= 0).any(1)
        partial += int((any_ & (idx < 0).any(1)).sum())
        np.testing.assert_allclose(h[any_, 4 * l], 0.75 + l, rtol=1e-14)
        assert np.all(h[~any_, 4 * l] == 0.0)
    assert partial > 50  # many queries blend across empty cells


def test_encode_is_the_neighbour_vertex_blend():
    """One-hot vertex maps: the feature equals the product of the node's
    renormalised trilinear weight and the vertex's barycentric weight,
    summed over the reads that hit the planted entry."""
    nodes, lo = sparse_tree(5, D=3)
    D = len(lo) - 2
    res = [4, 2, 2, 2][:D + 1]
    g = np.random.default_rng(7)
    x = g.uniform(0, 1, (300, 3)).astype(np.float32)
    d = g.normal(size=(300, 3)).astype(np.float32)
    st = oracle.octa(d)
    for l in range(D + 1):
        n_l = int(lo[l + 1] - lo[l])
        node = int(g.integers(n_l))
        R = res[l]
        slot = int(g.integers((R + 1) ** 2))
        feat = [np.zeros((int(lo[k + 1] - lo[k]), res[k] + 1, res[k] + 1, 4), np.float32) for k in range(D + 1)]
        feat[l].reshape(n_l, -1, 4)[node, slot, 2] = 1.0
        tree = oracle.Tree(nodes, lo, list(res), 4, feat, interp=PAPER)
        h, _ = oracle.encode(tree, x, d)
        idx, _, wn = oracle.neighbours(tree, x, l)
        _, wv, v = oracle.bary(st, R)
        want = ((idx == lo[l] + node) * wn).sum(1) * ((v == slot) * wv).sum(1)
        np.testing.assert_allclose(h[:, 4 * l + 2], want, atol=1e-15)
        assert np.all(np.delete(h, 4 * l + 2, axis=1) == 0.0)


# -------------------------------- adjoint ---------------------------------

def paper_problem(seed, **kw):
    """The tiny residual problem of the bilinear pins with vertex maps."""
    from _tiny import tiny_problem
    tree, mlp, batch = tiny_problem(seed=seed, **kw)
    g = np.random.default_rng(seed + 100)
    feat = [g.normal(0, 0.1, (int(tree.level_offset[l + 1] - tree.level_offset[l]), R + 1, R + 1, tree.C))
            .astype(np.float32) for l, R in enumerate(tree.res)]
    return oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, feat, interp=PAPER), mlp, batch


def _with_feat(tree, feat):
    return oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, feat, interp=tree.interp)


def _frozen(tree, mlp, batch):
    _, T, _, _ = oracle.residual_fwd(tree, mlp, batch)
    return dict(batch, target_override=T.astype(np.float32))


def _read_entries(tree, batch, g, k):
    """Entries the batch's LHS queries read: (level, flat index)."""
    st = oracle.octa(batch["dir"])
    out = []
    while len(out) < k:
        b = int(g.integers(len(batch["x"])))
        l = int(g.integers(tree.n_levels))
        idx, _, wn = oracle.neighbours(tree, batch["x"][b:b + 1], l)
        d = int(g.integers(8))
        if idx[0, d] < 0 or wn[0, d] == 0:
            continue
        _, _, v = oracle.bary(st[b:b + 1], tree.res[l])
        slot = int(v[0, g.integers(3)])
        node = idx[0, d] - tree.level_offset[l]
        out.append((l, int((node * (tree.res[l] + 1) ** 2 + slot) * tree.C + g.integers(tree.C))))
    return out


@pytest.mark.parametrize("full", [0, 1])
def test_paper_adjoint_matches_central_differences(full):
    """FP64 central differences of the loss against the adjoint, for vertex
    entries the batch reads through any of the 8 neighbouring cells and for
    every layer's weights (target frozen in the detached mode)."""
    tree, mlp, batch = paper_problem(20, D=3, res=(4, 4, 2, 2), N=3, B=24, bias_scale=0.1)
    batch = dict(batch, grad_through_rhs=full)
    fb = batch if full else _frozen(tree, mlp, batch)
    dfeat, dW, db = oracle.residual_bwd(tree, mlp, fb)
    g = np.random.default_rng(2)
    h = 1e-5
    got, want = [], []
    for l, flat in _read_entries(tree, batch, g, 24):
        v0 = tree.feat[l].reshape(-1)[flat]
        up, dn = np.float32(v0 + h), np.float32(v0 - h)
        lv = []
        for v in (up, dn):
            feat = [f.copy() for f in tree.feat]
            feat[l].reshape(-1)[flat] = v
            lv.append(oracle.residual_fwd(_with_feat(tree, feat), mlp, fb)[3])
        got.append(dfeat[l].reshape(-1)[flat])
        want.append((lv[0] - lv[1]) / (float(up) - float(dn)))
    for i in range(len(mlp.W)):
        flat = int(g.integers(mlp.W[i].size))
        v0 = mlp.W[i].reshape(-1)[flat]
        up, dn = np.float32(v0 + h), np.float32(v0 - h)
        lv = []
        for v in (up, dn):
            W = [w.copy() for w in mlp.W]
            W[i].reshape(-1)[flat] = v
            lv.append(oracle.residual_fwd(tree, oracle.MLP(W, mlp.b), fb)[3])
        got.append(dW[i].reshape(-1)[flat])
        want.append((lv[0] - lv[1]) / (float(up) - float(dn)))
    got, want = np.array(got), np.array(want)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-6
    assert np.all(np.abs(got) > 0)


def test_paper_scatter_conservation_uniform_shift():
    """A shift of every entry of level l, channel c moves h_l[c] by the shift
    wherever some neighbouring cell exists (renormalised weights and
    barycentric weights both sum to 1): the level's gradient sums to the
    derivative of that shift."""
    tree, mlp, batch = paper_problem(21, D=3, res=(4, 4, 2, 2), N=2, B=32, bias_scale=0.1)
    q = [np.round(f * 2.0 ** 20).astype(np.float32) / np.float32(2.0 ** 20) for f in tree.feat]
    tree = _with_feat(tree, q)
    e = 2.0 ** -16
    fb = _frozen(tree, mlp, batch)
    dfeat, _, _ = oracle.residual_bwd(tree, mlp, fb)
    for l in range(tree.n_levels):
        for c in range(tree.C):
            lv = []
            for s in (e, -e):
                feat = [f.copy() for f in tree.feat]
                feat[l][..., c] += np.float32(s)
                lv.append(oracle.residual_fwd(_with_feat(tree, feat), mlp, fb)[3])
            fd = (lv[0] - lv[1]) / (2 * e)
            assert abs(dfeat[l][..., c].sum() - fd) <= 2e-6 * max(1e-3, abs(fd)), (l, c)


def test_paper_gradient_lands_on_neighbouring_cells():
    """Node n of level l gets a gradient exactly when it is one of the 8
    cells around some LHS point with a non-zero renormalised weight; cells
    from the geometry, node cells from the child masks."""
    tree, mlp, batch = paper_problem(22, D=4, res=(4, 4, 2, 2, 2), N=2, B=60, n_samples=3000, tau=3,
                                     bias_scale=0.1)
    dfeat, _, _ = oracle.residual_bwd(tree, mlp, batch)
    coord = node_cells(tree.nodes, tree.level_offset)
    x = np.clip(batch["x"].astype(np.float64), 0, 1)
    checked = 0
    for l in range(tree.n_levels):
        lo_, hi = tree.level_offset[l], tree.level_offset[l + 1]
        pos = {tuple(c): i for i, c in enumerate(coord[lo_:hi])}
        base = np.floor(x * 2 ** l - 0.5).astype(np.int64)
        frac = x * 2 ** l - 0.5 - base
        want = set()
        for b in range(len(x)):
            for d in range(8):
                bits = np.array([(d >> a) & 1 for a in range(3)])
                if np.any(np.where(bits == 1, frac[b], 1 - frac[b]) == 0):
                    continue  # zero trilinear weight
                c = tuple(base[b] + bits)
                if c in pos:
                    want.add(pos[c])
        touched = set(np.nonzero(np.abs(dfeat[l]).reshape(hi - lo_, -1).sum(1) > 0)[0].tolist())
        assert touched == want, l
        checked += len(want)
    assert checked > 100
