"""Pins for the oracle's level features (Sec. 3.4: per-level maps read at the
containing node and concatenated level by level) and decoder MLP (Sec. 3.5)."""
import numpy as np

import oracle
from _tiny import tiny_problem


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
