"""Pins for the oracle's BSDF weight, residual and adjoint (Sec. 3.2 Monte-Carlo
right-hand side; Sec. 3.6 detached target and loss)."""
import math

import numpy as np
import pytest

import oracle
from _tiny import tiny_problem


def one_sample(n, wo, wi, albedo, alpha, F0=0.04, pdf=1.0):
    b = dict(x=np.zeros((1, 3), np.float32), n=np.array([n], np.float32), wo=np.array([wo], np.float32),
             wi=np.array([[wi]], np.float32), albedo=np.array([albedo], np.float32),
             rough=np.array([alpha], np.float32), pdf=np.array([[pdf]], np.float32), N=1, F0=F0)
    return oracle.bsdf_weight(b)[0, 0]


def unit(v):
    v = np.asarray(v, np.float64)
    return (v / np.linalg.norm(v)).astype(np.float32)


@pytest.mark.parametrize("alpha", [0.05, 0.3, 1.0])
@pytest.mark.parametrize("F0", [0.04, 0.5, 1.0])
def test_normal_incidence_closed_form(alpha, F0):
    # wi = wo = n: h = n, D = 1/(pi a^2), G = 1, F = F0, cos = 1
    a32 = float(np.float32(alpha))
    w = one_sample([0, 0, 1], [0, 0, 1], [0, 0, 1], [0.2, 0.5, 0.8], alpha, F0)
    want = np.array([0.2, 0.5, 0.8], np.float32).astype(np.float64) / math.pi + F0 / (4 * math.pi * a32 ** 2)
    np.testing.assert_allclose(w, want, rtol=1e-12)


def test_alpha_one_closed_form_any_angle():
    # alpha = 1: D = 1/pi everywhere, G1(c) = 2c/(c+1); with F0 = 1 the
    # specular term is 1 / (pi (cos_i + 1)(cos_o + 1)).
    g = np.random.default_rng(2)
    for _ in range(50):
        wi, wo = unit(g.normal(size=3)), unit(g.normal(size=3))
        wi[2], wo[2] = abs(wi[2]), abs(wo[2])
        n = np.array([0, 0, 1], np.float32)
        ci = float(wi[2]) / np.linalg.norm(wi.astype(np.float64))
        co = float(wo[2]) / np.linalg.norm(wo.astype(np.float64))
        w = one_sample(n, wo, wi, [0, 0, 0], 1.0, F0=1.0)
        np.testing.assert_allclose(w, ci / (math.pi * (ci + 1) * (co + 1)), rtol=1e-11)
        # with F0 = 0 Schlick's term is (1 - wi.h)^5 at any angle
        u = lambda v: v.astype(np.float64) / np.linalg.norm(v.astype(np.float64))
        hv = u(u(wi) + u(wo))
        fres = (1.0 - float(np.dot(u(wi), hv))) ** 5
        w0 = one_sample(n, wo, wi, [0, 0, 0], 1.0, F0=0.0)
        np.testing.assert_allclose(w0, ci * fres / (math.pi * (ci + 1) * (co + 1)), rtol=1e-9, atol=1e-15)


def test_reciprocity_horizon_albedo_and_pdf():
    g = np.random.default_rng(3)
    for _ in range(50):
        n = unit(g.normal(size=3))
        wi, wo = unit(g.normal(size=3)), unit(g.normal(size=3))
        if np.dot(wi, n) <= 0:
            wi = -wi
        if np.dot(wo, n) <= 0:
            wo = -wo
        a = float(g.uniform(0.02, 1))
        alb = g.uniform(0, 1, 3).astype(np.float32)
        un = lambda v: v.astype(np.float64) / np.linalg.norm(v.astype(np.float64))
        ci, co = float(np.dot(un(wi), un(n))), float(np.dot(un(wo), un(n)))
        f_io = one_sample(n, wo, wi, alb, a) / ci
        f_oi = one_sample(n, wi, wo, alb, a) / co
        np.testing.assert_allclose(f_io, f_oi, rtol=1e-12)  # reciprocity
        diff = one_sample(n, wo, wi, alb, a) - one_sample(n, wo, wi, [0, 0, 0], a)
        np.testing.assert_allclose(diff, alb.astype(np.float64) / math.pi * ci, rtol=1e-10, atol=1e-15)
        np.testing.assert_allclose(one_sample(n, wo, wi, alb, a, pdf=0.25),
                                   4 * one_sample(n, wo, wi, alb, a), rtol=1e-14)
        assert np.all(one_sample(n, wo, -wi, alb, a) == 0)                     # below horizon
        assert np.all(one_sample(n, -wo, wi, alb, a) == 0)


def constant_field(mlp, c):
    W = [w.copy() for w in mlp.W]
    b = [v.copy() for v in mlp.b]
    W[-1][:] = 0
    b[-1][:] = np.asarray(c, np.float32)
    return oracle.MLP(W, b)


def test_constant_radiance_closed_form():
    """With a zero last layer and bias c the field is c everywhere, so
    r = c - L_e - c * mean_k w_k and the loss is sum r^2 / (3B)."""
    tree, mlp, batch = tiny_problem(seed=6, N=4, B=40)
    c = np.array([0.7, 1.3, 0.4], np.float32)
    m = constant_field(mlp, c)
    lhs, T, r, loss = oracle.residual_fwd(tree, m, batch)
    w = oracle.bsdf_weight(batch)
    want_T = batch["Le"] + c * w.mean(1)
    np.testing.assert_allclose(lhs, np.broadcast_to(c, lhs.shape), rtol=0, atol=0)
    np.testing.assert_allclose(T, want_T, rtol=1e-14)
    np.testing.assert_allclose(r, c - want_T, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(loss, (r ** 2).sum() / (3 * 40), rtol=1e-13)


def test_lambertian_cosine_sampling_closed_form():
    """Pure diffuse (zero specular via albedo-only difference): with cosine
    sampling each weight is the albedo, so T = L_e + c * a."""
    tree, mlp, batch = tiny_problem(seed=7, N=3, B=30)
    c = np.array([0.5, 0.5, 0.5], np.float32)
    m = constant_field(mlp, c)
    w_full = oracle.bsdf_weight(batch)
    b0 = dict(batch, albedo=np.zeros_like(batch["albedo"]))
    w_spec = oracle.bsdf_weight(b0)
    # cosine pdf = cos/pi, so the diffuse part of every weight is the albedo
    # (up to FP32 rounding of the stored pdf and directions)
    np.testing.assert_allclose(w_full - w_spec, np.broadcast_to(batch["albedo"][:, None], w_full.shape),
                               rtol=1e-6)
    _, T, _, _ = oracle.residual_fwd(tree, m, batch)
    _, T0, _, _ = oracle.residual_fwd(tree, m, b0)
    np.testing.assert_allclose(T - T0, c * batch["albedo"], rtol=1e-6)


def test_no_samples_and_override():
    tree, mlp, batch = tiny_problem(seed=8, N=0, B=25)
    lhs, T, r, loss = oracle.residual_fwd(tree, mlp, batch)
    np.testing.assert_array_equal(T, batch["Le"].astype(np.float64))
    ov = np.random.default_rng(0).uniform(0, 1, (25, 3)).astype(np.float32)
    lhs2, T2, r2, loss2 = oracle.residual_fwd(tree, mlp, dict(batch, target_override=ov))
    np.testing.assert_array_equal(T2, ov.astype(np.float64))
    np.testing.assert_allclose(loss2, ((lhs - ov) ** 2).mean(), rtol=1e-13)
    assert oracle.residual_fwd(tree, mlp, dict(batch, x=batch["x"][:0], dir=batch["dir"][:0],
                                               n=batch["n"][:0], wo=batch["wo"][:0],
                                               albedo=batch["albedo"][:0], rough=batch["rough"][:0],
                                               Le=batch["Le"][:0]))[3] == 0.0


def test_relative_loss():
    tree, mlp, batch = tiny_problem(seed=9, N=2, B=20)
    lhs, T, r, l2 = oracle.residual_fwd(tree, mlp, batch)
    _, _, _, lr = oracle.residual_fwd(tree, mlp, dict(batch, loss_kind=1, eps=0.01))
    rho = np.maximum(lhs + T, 0) + 0.01
    np.testing.assert_allclose(lr, ((r / rho) ** 2).mean(), rtol=1e-13)


# -------------------------------- adjoint ---------------------------------

def _loss(tree, mlp, batch):
    return oracle.residual_fwd(tree, mlp, batch)[3]


def _steps(theta, h):
    """FP32 parameters: the perturbed values are rounded to FP32, so the
    difference quotient divides by the step actually taken."""
    up, dn = np.float32(theta + h), np.float32(theta - h)
    return up, dn, float(up) - float(dn)


def _fd_feat(tree, mlp, batch, l, flat, h):
    up, dn, step = _steps(tree.feat[l].reshape(-1)[flat], h)

    def at(v):
        feat = [f.copy() for f in tree.feat]
        feat[l].reshape(-1)[flat] = v
        return _loss(oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, feat), mlp, batch)
    return (at(up) - at(dn)) / step


def _fd_w(tree, mlp, batch, i, flat, which, h):
    src = (mlp.W if which == "W" else mlp.b)[i].reshape(-1)
    up, dn, step = _steps(src[flat], h)

    def at(v):
        W = [w.copy() for w in mlp.W]
        b = [v_.copy() for v_ in mlp.b]
        (W if which == "W" else b)[i].reshape(-1)[flat] = v
        return _loss(tree, oracle.MLP(W, b), batch)
    return (at(up) - at(dn)) / step


def _frozen(tree, mlp, batch):
    """Detached-target semantics: freeze T at the current parameters."""
    _, T, _, _ = oracle.residual_fwd(tree, mlp, batch)
    return dict(batch, target_override=T.astype(np.float32))


def _touched(tree, batch, g, k):
    idx = oracle.descend(tree, batch["x"])
    st = oracle.octa(batch["dir"])
    out = []
    for _ in range(k):
        b = int(g.integers(len(batch["x"])))
        l = int(g.integers(tree.n_levels))
        if idx[b, l] < 0:
            continue
        ij, _ = oracle.taps(st[b:b + 1], tree.res[l])
        i, j = ij[0, int(g.integers(4))]
        R = tree.res[l]
        node = idx[b, l] - tree.level_offset[l]
        out.append((l, int(((node * R + j) * R + i) * tree.C + g.integers(tree.C))))
    return out


@pytest.mark.parametrize("full", [0, 1])
def test_adjoint_matches_central_differences(full):
    """FP64 central differences of the oracle loss against its adjoint, for
    feature entries the batch touches and for every layer's W and b. In the
    detached mode the target is frozen (as the adjoint assumes); in full mode
    the gradient also flows through the RHS queries."""
    tree, mlp, batch = tiny_problem(seed=10, N=3, B=24, bias_scale=0.1)
    batch = dict(batch, grad_through_rhs=full)
    g = np.random.default_rng(1)
    fb = batch if full else _frozen(tree, mlp, batch)
    dfeat, dW, db = oracle.residual_bwd(tree, mlp, fb, grad_loss=1.0)
    h = 1e-5
    got, want = [], []
    for l, flat in _touched(tree, batch, g, 24):
        got.append(dfeat[l].reshape(-1)[flat])
        want.append(_fd_feat(tree, mlp, fb, l, flat, h))
    for i in range(len(mlp.W)):
        for _ in range(6):
            flat = int(g.integers(mlp.W[i].size))
            got.append(dW[i].reshape(-1)[flat])
            want.append(_fd_w(tree, mlp, fb, i, flat, "W", h))
        flat = int(g.integers(mlp.b[i].size))
        got.append(db[i][flat])
        want.append(_fd_w(tree, mlp, fb, i, flat, "b", h))
    got, want = np.array(got), np.array(want)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err < 1e-6, err
    assert np.abs(got - want).max() < 1e-6 * np.abs(want).max() + 1e-12


def test_adjoint_scales_with_grad_loss_and_relative_mode():
    """grad_loss scales every gradient; the relative loss divides each
    element's seed by its squared (detached) normaliser. With a zero last
    layer the prediction is exactly the bias, so the last layer's gradient
    separates the three channels: dW_last[c] = seed_c * a and
    db_last[c] = seed_c for a single point."""
    tree, mlp, batch = tiny_problem(seed=11, N=2, B=1, bias_scale=0.1)
    c = np.array([0.3, 0.9, 0.05], np.float32)
    m = constant_field(mlp, c)
    ov = (c + np.array([0.25, -0.5, 0.125], np.float32))[None]
    b1 = dict(batch, target_override=ov)
    _, W1, b1g = oracle.residual_bwd(tree, m, b1, 1.0)
    _, W3, b3g = oracle.residual_bwd(tree, m, b1, 3.0)
    _, Wr, brg = oracle.residual_bwd(tree, m, dict(b1, loss_kind=1, eps=0.01), 1.0)
    for a, b_ in zip(W1 + b1g, W3 + b3g):
        np.testing.assert_allclose(b_, 3 * a, rtol=1e-13, atol=1e-16)
    rho = np.maximum(c.astype(np.float64) + ov[0], 0) + 0.01
    r = c.astype(np.float64) - ov[0]
    np.testing.assert_allclose(b1g[-1], 2 * r / 3, rtol=1e-14)
    np.testing.assert_allclose(brg[-1], 2 * r / 3 / rho ** 2, rtol=1e-14)
    np.testing.assert_allclose(Wr[-1], W1[-1] / rho[:, None] ** 2, rtol=1e-14)


def test_scatter_conservation_uniform_shift():
    """Adding e to channel c of every texel of level l shifts h_l[c] by e for
    every query with a node there (weights sum to 1), so the sum of the
    level's feature gradient equals the derivative of that shift."""
    tree, mlp, batch = tiny_problem(seed=12, N=2, B=32, bias_scale=0.1)
    # tables on a 2^-20 grid so that a shift by 2^-16 is exact in FP32
    q = [np.round(f * 2.0 ** 20).astype(np.float32) / np.float32(2.0 ** 20) for f in tree.feat]
    tree = oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, q)
    e = 2.0 ** -16  # loss is piecewise quadratic in a shift: central differences are exact off kinks
    fb = _frozen(tree, mlp, batch)
    dfeat, _, _ = oracle.residual_bwd(tree, mlp, fb)
    for l in range(tree.n_levels):
        for c in range(tree.C):
            def at(e):
                feat = [f.copy() for f in tree.feat]
                feat[l][..., c] += e
                return _loss(oracle.Tree(tree.nodes, tree.level_offset, tree.res, tree.C, feat), mlp, fb)
            fd = (at(np.float32(e)) - at(np.float32(-e))) / (2 * e)
            s = dfeat[l][..., c].sum()
            assert abs(s - fd) <= 2e-6 * max(1e-3, abs(fd)), (l, c, s, fd)


def test_feature_gradient_lands_on_the_nodes_holding_the_points():
    """The adjoint of the level features (Sec. 3.4, 3.6) changes only the maps
    the forward read: with the target detached, node n of level l receives a
    gradient exactly when some LHS point of the batch lies in n's cell. Cells
    come from the geometry (floor(x 2^l), clamped) and the node cells from
    walking the child masks, independently of the descent."""
    from test_oracle_octree import cells, node_cells
    tree, mlp, batch = tiny_problem(seed=13, D=4, res=(4, 4, 2, 2, 2), N=2, B=60, n_samples=3000, tau=3,
                                    bias_scale=0.1)
    dfeat, _, _ = oracle.residual_bwd(tree, mlp, batch)
    coord = node_cells(tree.nodes, tree.level_offset)
    checked = 0
    for l in range(tree.n_levels):
        lo, hi = tree.level_offset[l], tree.level_offset[l + 1]
        pos = {tuple(c): i for i, c in enumerate(coord[lo:hi])}
        visited = {pos[tuple(c)] for c in cells(batch["x"], l) if tuple(c) in pos}
        touched = set(np.nonzero(np.abs(dfeat[l]).reshape(hi - lo, -1).sum(1) > 0)[0].tolist())
        assert touched == visited, (l, sorted(touched), sorted(visited))
        checked += len(visited)
    assert checked > 60
