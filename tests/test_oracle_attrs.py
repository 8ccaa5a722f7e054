"""Pins for the decoder's surface attributes (Sec. 3.5: the prediction is the
decoder applied to the level features h followed by g = [x, w_r, n, a,
alpha]): where the oracle places them, which query's attributes each
decoder evaluation reads, and their share of the adjoint."""
import numpy as np
import pytest

import oracle
from _tiny import tiny_problem
from test_oracle_residual import _frozen, _fd_w, _touched, _fd_feat

E = 13


def dense_decoder(mlp, a):
    """The decoder written out with numpy in FP64: ReLU hidden layers, a
    linear output layer."""
    a = np.asarray(a, np.float64)
    for i, (W, b) in enumerate(zip(mlp.W, mlp.b)):
        a = a @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        if i < len(mlp.W) - 1:
            a = np.maximum(a, 0.0)
    return a


def test_query_reads_features_then_attributes():
    """The decoder input is [h, g]: h from the (separately pinned) encoding,
    then the query's own attributes in their order."""
    tree, mlp, batch = tiny_problem(seed=3, N=0, B=48, bias_scale=0.1, n_attr=E)
    x, d, g = batch["x"], batch["dir"], batch["attr"]
    h, _ = oracle.encode(tree, x, d)
    want = dense_decoder(mlp, np.concatenate([h, g], axis=1))
    got = oracle.query_fwd(tree, mlp, x, d, attr=g)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    # the attributes matter: reversing their order changes the result
    assert np.abs(oracle.query_fwd(tree, mlp, x, d, attr=g[:, ::-1]) - got).max() > 1e-3


def test_residual_reads_lhs_and_secondary_attributes():
    """LHS queries read attr, secondary queries attr2 ([B][N][E]): the
    residual's L and T against the decoder written out and the pinned BSDF
    weights."""
    tree, mlp, batch = tiny_problem(seed=4, N=3, B=32, bias_scale=0.1, n_attr=E)
    lhs, T, r, _ = oracle.residual_fwd(tree, mlp, batch)
    h, _ = oracle.encode(tree, batch["x"], batch["dir"])
    want_lhs = dense_decoder(mlp, np.concatenate([h, batch["attr"]], axis=1))
    B, N = 32, 3
    h2, _ = oracle.encode(tree, batch["x2"].reshape(-1, 3), batch["dir2"].reshape(-1, 3))
    L2 = dense_decoder(mlp, np.concatenate([h2, batch["attr2"].reshape(B * N, E)], axis=1)).reshape(B, N, 3)
    w = oracle.bsdf_weight(batch)
    want_T = batch["Le"].astype(np.float64) + (w * L2).mean(axis=1)
    np.testing.assert_allclose(lhs, want_lhs, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(T, want_T, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r, lhs - T, rtol=0, atol=0)


def test_zero_attribute_weights_reduce_to_features_only():
    """With the attribute columns of W_0 zero the decoder is the features-
    only decoder: same outputs and same feature gradients."""
    tree, mlp, batch = tiny_problem(seed=5, N=3, B=32, bias_scale=0.1, n_attr=E)
    LC = tree.n_levels * tree.C
    W0 = mlp.W[0].copy()
    W0[:, LC:] = 0.0
    wide = oracle.MLP([W0] + list(mlp.W[1:]), mlp.b)
    narrow = oracle.MLP([W0[:, :LC].copy()] + list(mlp.W[1:]), mlp.b)
    plain = {k: v for k, v in batch.items() if k not in ("attr", "attr2")}
    for a, b_ in zip(oracle.residual_fwd(tree, wide, batch)[:3], oracle.residual_fwd(tree, narrow, plain)[:3]):
        np.testing.assert_array_equal(a, b_)
    for full in (0, 1):
        fw = dict(batch, grad_through_rhs=full)
        fn = dict(plain, grad_through_rhs=full)
        df_w, dW_w, _ = oracle.residual_bwd(tree, wide, fw)
        df_n, dW_n, _ = oracle.residual_bwd(tree, narrow, fn)
        for a, b_ in zip(df_w, df_n):
            np.testing.assert_allclose(a, b_, rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(dW_w[0][:, :LC], dW_n[0], rtol=1e-13, atol=1e-16)


def test_zero_padded_attributes_get_zero_gradient():
    """Zero attribute columns (the padding that keeps the input width a
    multiple of 4) contribute nothing and receive an exactly zero dW."""
    tree, mlp, batch = tiny_problem(seed=6, N=3, B=32, bias_scale=0.1, n_attr=16)
    batch = dict(batch, grad_through_rhs=1)
    batch["attr"][:, E:] = 0.0
    batch["attr2"][:, :, E:] = 0.0
    _, dW, _ = oracle.residual_bwd(tree, mlp, batch)
    LC = tree.n_levels * tree.C
    assert np.all(dW[0][:, LC + E:] == 0.0)
    assert np.abs(dW[0][:, LC:LC + E]).max() > 0.0


@pytest.mark.parametrize("full", [0, 1])
def test_attribute_adjoint_matches_central_differences(full):
    """FP64 central differences of the loss against the adjoint for W_0's
    attribute columns, the other layers and touched feature entries, with
    the target detached (frozen) or differentiated (the RHS queries then
    carry their own attributes)."""
    tree, mlp, batch = tiny_problem(seed=11, N=3, B=24, bias_scale=0.1, n_attr=E)
    batch = dict(batch, grad_through_rhs=full)
    fb = batch if full else _frozen(tree, mlp, batch)
    dfeat, dW, db = oracle.residual_bwd(tree, mlp, fb, grad_loss=1.0)
    g = np.random.default_rng(2)
    LC = tree.n_levels * tree.C
    h = 1e-5
    got, want = [], []
    for _ in range(12):  # W_0 entries in the attribute columns
        o, k = int(g.integers(mlp.W[0].shape[0])), LC + int(g.integers(E))
        flat = o * mlp.W[0].shape[1] + k
        got.append(dW[0].reshape(-1)[flat])
        want.append(_fd_w(tree, mlp, fb, 0, flat, "W", h))
    for i in range(1, len(mlp.W)):
        flat = int(g.integers(mlp.W[i].size))
        got.append(dW[i].reshape(-1)[flat])
        want.append(_fd_w(tree, mlp, fb, i, flat, "W", h))
    for l, flat in _touched(tree, batch, g, 12):
        got.append(dfeat[l].reshape(-1)[flat])
        want.append(_fd_feat(tree, mlp, fb, l, flat, h))
    got, want = np.array(got), np.array(want)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err < 1e-6, err
    assert np.abs(got - want).max() < 1e-6 * np.abs(want).max() + 1e-12
