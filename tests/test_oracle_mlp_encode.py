"""Pins for the oracle's level features (Sec. 3.4: per-level maps read at the
containing node and concatenated level by level) and decoder MLP (Sec. 3.5)."""
import numpy as np

import oracle
from _tiny import tiny_problem
from test_oracle_octree import cells, node_cells


def test_mlp_matches_dense_layers():
    g = np.random.default_rng(0)
    dims = [20, 64, 64, 3]
    W = [g.normal(size=(o, i)).astype(np.float32) for i, o in zip(dims[:-1], dims[1:])]
    b = [g.normal(size=o).astype(np.float32) for o in dims[1:]]
    h = g.normal(size=(50, 20))
    a = h
    for i in range(3):
        z = a @ W[i].astype(np.float64).T + b[i]
        a = np.maximum(z, 0) if i < 2 else z
    np.testing.assert_allclose(oracle.mlp_fwd(oracle.MLP(W, b), h), a, rtol=1e-12, atol=1e-12)


def test_mlp_single_layer_is_affine():
    g = np.random.default_rng(1)
    W = [g.normal(size=(3, 7)).astype(np.float32)]
    b = [g.normal(size=3).astype(np.float32)]
    h = g.normal(size=(9, 7))
    np.testing.assert_allclose(oracle.mlp_fwd(oracle.MLP(W, b), h), h @ W[0].T.astype(np.float64) + b[0],
                               rtol=1e-13, atol=1e-13)


def test_encode_one_hot_texels_give_tap_weights():
    tree, mlp, batch = tiny_problem(seed=3)
    x, d = batch["x"], batch["dir"]
    idx = oracle.descend(tree, x)
    st = oracle.octa(d)
    C = tree.C
    for l in range(tree.n_levels):
        R = tree.res[l]
        ij, w = oracle.taps(st, R)
        for c in (0, C - 1):
            feat = [np.zeros_like(f) for f in tree.feat]
            # one-hot in channel c of every texel of every node, scaled by texel id
            tid = np.arange(R * R, dtype=np.float32).reshape(R, R) + 1
            feat[l][..., c] = tid[None]
            t1 = oracle.Tree(tree.nodes, tree.level_offset, tree.res, C, feat)
            h, _ = oracle.encode(t1, x, d)
            want = (w * tid[ij[..., 1], ij[..., 0]]).sum(1) * (idx[:, l] >= 0)
            np.testing.assert_allclose(h[:, l * C + c], want, atol=1e-12)
            others = np.delete(h, l * C + c, axis=1)
            assert np.all(others == 0)


def test_encode_linear_in_tables_and_missing_levels_zero():
    tree, mlp, batch = tiny_problem(seed=4)
    x, d = batch["x"], batch["dir"]
    h1, idx = oracle.encode(tree, x, d)
    t2 = oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, [2 * f for f in tree.feat])
    h2, _ = oracle.encode(t2, x, d)
    np.testing.assert_allclose(h2, 2 * h1, rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(idx, oracle.descend(tree, x))
    C = tree.C
    for l in range(tree.n_levels):
        miss = idx[:, l] < 0
        assert np.all(h1[miss, l * C:(l + 1) * C] == 0)
    assert (idx < 0).any() and (idx >= 0).all(0).any()


def test_query_is_encode_then_mlp_and_thread_invariant():
    tree, mlp, batch = tiny_problem(seed=5)
    h, _ = oracle.encode(tree, batch["x"], batch["dir"])
    q1 = oracle.query_fwd(tree, mlp, batch["x"], batch["dir"], nthreads=1)
    q4 = oracle.query_fwd(tree, mlp, batch["x"], batch["dir"], nthreads=4)
    np.testing.assert_array_equal(q1, oracle.mlp_fwd(mlp, h))
    np.testing.assert_array_equal(q1, q4)


def test_encode_reads_the_map_of_the_cell_holding_x():
    """Which node's map a level reads (Sec. 3.4: level j reads the map of the
    cell c_j that holds x). Every node gets a constant map that spells out its
    own cell coordinates and level, so the bilinear fetch returns exactly
    those values and h_l names the node that was read. The cell is found here
    from the geometry alone, floor(x 2^l) clamped to the cube, and the node
    cells by walking the child masks from the root; a level whose cell holds
    no node must read zeros."""
    for seed in (21, 22):
        tree, mlp, batch = tiny_problem(seed=seed, D=4, res=(4, 4, 2, 2, 2), B=400, n_samples=3000, tau=3)
        x, d = batch["x"], batch["dir"]
        coord = node_cells(tree.nodes, tree.level_offset)
        feat = []
        for l in range(tree.n_levels):
            lo, hi = tree.level_offset[l], tree.level_offset[l + 1]
            R = tree.res[l]
            val = np.concatenate([coord[lo:hi] + 1, np.full((hi - lo, 1), l + 1)], axis=1).astype(np.float32)
            feat.append(np.ascontiguousarray(np.broadcast_to(val[:, None, None, :], (hi - lo, R, R, 4))))
        t1 = oracle.Tree(tree.nodes, tree.level_offset, tree.res, 4, feat)
        h, _ = oracle.encode(t1, x, d)
        deep = 0
        for l in range(tree.n_levels):
            lo, hi = tree.level_offset[l], tree.level_offset[l + 1]
            have = {tuple(c) for c in coord[lo:hi]}
            c = cells(x, l)
            exists = np.array([tuple(v) in have for v in c])
            want = np.where(exists[:, None], np.concatenate([c + 1, np.full((len(x), 1), l + 1)], axis=1), 0)
            np.testing.assert_allclose(h[:, 4 * l:4 * l + 4], want, rtol=0, atol=1e-12, err_msg=f"level {l}")
            if l >= 2 and hi - lo > 8:
                deep += int(exists.sum())
        assert deep > 100  # many queries read deep levels with many nodes
