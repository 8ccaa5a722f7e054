"""Pins for the oracle's bilinear taps on the octahedral map: texel-centred
bilinear weights and the seam identification that keeps the lookup
continuous over the sphere (Sec. 3.3: edge samples are shared by adjacent
faces, so interpolation is continuous across the spherical domain)."""
import numpy as np
import pytest

import oracle


def interp(table, st, R):
    """Value of an R x R scalar map at (s, t) through the oracle's taps."""
    ij, w = oracle.taps(st, R)
    return (w * table[ij[..., 1], ij[..., 0]]).sum(1)


@pytest.mark.parametrize("R", [2, 4, 16, 64])
def test_weights_partition_of_unity_and_indices_in_range(R):
    g = np.random.default_rng(R)
    st = g.uniform(0, 1, (20000, 2))
    st[:50] = g.integers(0, 2, (50, 2))  # exact corners and edges
    ij, w = oracle.taps(st, R)
    assert np.all(w >= 0)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-15)
    assert ij.min() >= 0 and ij.max() < R


@pytest.mark.parametrize("R", [2, 8, 32])
def test_texel_centre_returns_texel(R):
    g = np.random.default_rng(100 + R)
    T = g.normal(size=(R, R))
    i, j = np.meshgrid(np.arange(R), np.arange(R))
    st = np.stack([(i.ravel() + 0.5) / R, (j.ravel() + 0.5) / R], 1)
    np.testing.assert_allclose(interp(T, st, R), T[j.ravel(), i.ravel()], atol=1e-15)


@pytest.mark.parametrize("R", [4, 16])
def test_constant_and_affine_reproduction(R):
    g = np.random.default_rng(7)
    st = g.uniform(0, 1, (5000, 2))
    np.testing.assert_allclose(interp(np.full((R, R), 3.25), st, R), 3.25, atol=1e-14)
    # affine in the texel-centre coordinates is reproduced where no tap wraps
    c = (np.arange(R) + 0.5) / R
    T = 0.3 + 1.7 * c[None, :] - 0.9 * c[:, None]
    inner = st[(st.min(1) >= 0.5 / R) & (st.max(1) <= 1 - 0.5 / R)]
    np.testing.assert_allclose(interp(T, inner, R), 0.3 + 1.7 * inner[:, 0] - 0.9 * inner[:, 1],
                               atol=1e-13)


def lookup_dir(T, d, R):
    return interp(T, oracle.octa(np.asarray(d, np.float32)), R)


@pytest.mark.parametrize("R", [2, 4, 16])
def test_continuity_across_lower_hemisphere_seams(R):
    """Directions just either side of the planes w_x = 0 and w_y = 0 in the
    lower hemisphere land on opposite halves of one map edge; the values must
    still agree as the gap closes."""
    g = np.random.default_rng(200 + R)
    T = g.normal(size=(R, R))
    m = 400
    a = g.uniform(0.05, 0.95, m)
    z = -np.sqrt(1 - a * a)
    for delta in (1e-3, 1e-5):
        for axis in (0, 1):
            other = g.choice([-1.0, 1.0], m) * a
            plus = np.zeros((m, 3))
            minus = np.zeros((m, 3))
            plus[:, axis], minus[:, axis] = delta, -delta
            plus[:, 1 - axis] = minus[:, 1 - axis] = other
            plus[:, 2] = minus[:, 2] = z
            jump = np.abs(lookup_dir(T, plus, R) - lookup_dir(T, minus, R))
            # Lipschitz bound: the map moves O(delta) and a tap changes at
            # most |T| range * R per unit of (s, t)
            assert jump.max() <= 8 * R * delta * np.ptp(T) + 1e-6


@pytest.mark.parametrize("R", [2, 8])
def test_continuity_across_equator(R):
    g = np.random.default_rng(300 + R)
    T = g.normal(size=(R, R))
    phi = g.uniform(0, 2 * np.pi, 500)
    for delta in (1e-3, 1e-5):
        up = np.stack([np.cos(phi), np.sin(phi), np.full_like(phi, delta)], 1)
        dn = np.stack([np.cos(phi), np.sin(phi), np.full_like(phi, -delta)], 1)
        jump = np.abs(lookup_dir(T, up, R) - lookup_dir(T, dn, R))
        assert jump.max() <= 8 * R * delta * np.ptp(T) + 1e-6


@pytest.mark.parametrize("R", [2, 4, 32])
def test_pole_averages_four_corners(R):
    g = np.random.default_rng(400 + R)
    T = g.normal(size=(R, R))
    v = lookup_dir(T, [[0, 0, -1]], R)[0]
    corners = T[0, 0] + T[0, R - 1] + T[R - 1, 0] + T[R - 1, R - 1]
    assert abs(v - corners / 4) < 1e-14


def test_wrong_seam_mirror_would_break_continuity():
    """Self-check of the continuity test: a seam rule that does not mirror
    the other coordinate produces a visible jump at the same tolerance."""
    R = 8
    g = np.random.default_rng(5)
    T = g.normal(size=(R, R))

    def bad_interp(st):
        pu, pv = st[:, 0] * R - 0.5, st[:, 1] * R - 0.5
        i0, j0 = np.floor(pu).astype(int), np.floor(pv).astype(int)
        fu, fv = pu - i0, pv - j0
        out = 0
        for a in (0, 1):
            for b in (0, 1):
                i, j = np.clip(i0 + a, 0, R - 1), np.clip(j0 + b, 0, R - 1)  # clamp, no seam
                out = out + (fu if a else 1 - fu) * (fv if b else 1 - fv) * T[j, i]
        return out

    a = np.linspace(0.1, 0.9, 50)
    z = -np.sqrt(1 - a * a)
    plus = np.stack([np.full_like(a, 1e-6), a, z], 1).astype(np.float32)
    minus = np.stack([np.full_like(a, -1e-6), a, z], 1).astype(np.float32)
    bad = np.abs(bad_interp(oracle.octa(plus)) - bad_interp(oracle.octa(minus))).max()
    good = np.abs(lookup_dir(T, plus, R) - lookup_dir(T, minus, R)).max()
    assert bad > 1e-2 and good < 1e-3
