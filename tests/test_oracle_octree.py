"""Pins for the oracle's octree build and descent (Sec. 3.4: a sparse octree
whose non-empty cells carry maps; Sec. 4.1: o-cnn-style octree). Expected
trees are rebuilt here from cell sets (which cells hold samples, which
parents hold more than tau), and descents are checked against brute-force
point-in-cell search over every node."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle


def cells(x, l):
    """Cell of each point at level l (half-open cells, x == 1 clamped)."""
    x = np.asarray(x, np.float64)
    return np.clip(np.floor(x * 2.0 ** l), 0, 2 ** l - 1).astype(np.int64)


def morton(c, l):
    key = np.zeros(len(c), np.int64)
    for bit in range(l):
        for a in range(3):
            key |= ((c[:, a] >> bit) & 1) << (3 * bit + a)
    return key


def expected_tree(x, D, tau):
    """Node words from the definition: level l+1 holds every non-empty cell
    whose parent is a node holding more than tau samples; nodes are in
    breadth-first order and, inside a level, in Morton order."""
    levels = [np.zeros((1, 3), np.int64)]
    counts = [np.array([len(x)])]
    for l in range(D):
        par = levels[-1]
        split = {tuple(p) for p, n in zip(par, counts[-1]) if n > tau}
        c = cells(x, l + 1)
        ok = np.array([tuple(v >> 1) in split for v in c], bool) if len(c) else np.zeros(0, bool)
        uniq, cnt = np.unique(c[ok], axis=0, return_counts=True) if ok.any() else (np.zeros((0, 3), np.int64), np.zeros(0, np.int64))
        order = np.argsort(morton(uniq, l + 1), kind="stable")
        levels.append(uniq[order])
        counts.append(cnt[order])
    offsets = np.cumsum([0] + [len(v) for v in levels])
    words = []
    for l, lv in enumerate(levels):
        nxt = {tuple(v): i + (offsets[l + 1] if l + 1 < len(levels) else 0)
               for i, v in enumerate(levels[l + 1])} if l + 1 < len(levels) else {}
        for v in lv:
            mask, first = 0, None
            for o in range(8):
                child = (2 * v[0] + (o & 1), 2 * v[1] + ((o >> 1) & 1), 2 * v[2] + ((o >> 2) & 1))
                if child in nxt:
                    mask |= 1 << o
                    first = nxt[child] if first is None else first
            words.append(0 if mask == 0 else (first << 8) | mask)
    return np.array(words, np.uint32), offsets, levels, counts


def node_cells(nodes, offsets):
    """Cell coordinates of every node, walking child masks from the root."""
    coord = np.zeros((len(nodes), 3), np.int64)
    for v in range(len(nodes)):
        w = int(nodes[v])
        mask, first = w & 0xFF, w >> 8
        k = 0
        for o in range(8):
            if mask >> o & 1:
                coord[first + k] = 2 * coord[v] + np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1])
                k += 1
    return coord


def brute_descent(nodes, offsets, x, L):
    coord = node_cells(nodes, offsets)
    out = np.full((len(x), L), -1, np.int32)
    for l in range(L):
        lo, hi = offsets[l], offsets[l + 1]
        c = cells(x, l)
        for b in range(len(x)):
            hit = np.nonzero((coord[lo:hi] == c[b]).all(1))[0]
            assert len(hit) <= 1
            if len(hit):
                out[b, l] = lo + hit[0]
    return out


def make_tree(nodes, lo, D):
    return oracle.Tree(nodes, lo, [2] * (D + 1), 4, [])


@pytest.mark.parametrize("D,tau,n", [(0, 4, 50), (1, 4, 50), (3, 2, 300), (4, 8, 2000), (5, 3, 500)])
def test_build_matches_definition(D, tau, n):
    g = np.random.default_rng(D * 100 + n)
    x = g.uniform(0, 1, (n, 3)).astype(np.float32)
    x[: n // 10] = g.choice([0.0, 0.5, 1.0], (n // 10, 3))  # cell boundaries and x == 1
    nodes, lo = oracle.build_octree(x, D, tau)
    ew, eo, _, _ = expected_tree(x, D, tau)
    np.testing.assert_array_equal(lo, eo)
    np.testing.assert_array_equal(nodes, ew)


def test_build_clustered_samples_refine_deeper():
    g = np.random.default_rng(3)
    x = np.concatenate([g.uniform(0, 1, (200, 3)), 0.3 + 0.01 * g.uniform(0, 1, (400, 3))]).astype(np.float32)
    nodes, lo = oracle.build_octree(x, 6, 16)
    ew, eo, levels, counts = expected_tree(x, 6, 16)
    np.testing.assert_array_equal(nodes, ew)
    # invariants: children partition the parent's samples; leaves hold <= tau
    # samples unless at depth D
    for l in range(6):
        for i, w in enumerate(nodes[lo[l]:lo[l + 1]]):
            n_here = counts[l][i]
            if w == 0:
                assert n_here <= 16
            else:
                first, mask = int(w) >> 8, int(w) & 0xFF
                kids = counts[l + 1][first - lo[l + 1]: first - lo[l + 1] + bin(mask).count("1")]
                assert kids.sum() == n_here


def test_empty_and_root_only():
    nodes, lo = oracle.build_octree(np.zeros((0, 3), np.float32), 3, 4)
    assert list(nodes) == [0] and list(lo) == [0, 1, 1, 1, 1]
    nodes, lo = oracle.build_octree(np.full((4, 3), 0.5, np.float32), 3, 4)
    assert list(nodes) == [0]  # 4 samples do not exceed tau = 4
    # 5 coincident samples refine one chain down to depth D
    nodes, lo = oracle.build_octree(np.full((5, 3), 0.5, np.float32), 3, 4)
    assert list(lo) == [0, 1, 2, 3, 4]
    assert list(nodes) == [(1 << 8) | 0x80, (2 << 8) | 0x01, (3 << 8) | 0x01, 0]


@pytest.mark.parametrize("D,tau,n", [(2, 2, 80), (4, 4, 600), (5, 2, 300)])
def test_descent_matches_brute_force(D, tau, n):
    g = np.random.default_rng(1 + D)
    x = g.uniform(0, 1, (n, 3)).astype(np.float32)
    nodes, lo = oracle.build_octree(x, D, tau)
    q = np.concatenate([x[:100], g.uniform(0, 1, (200, 3)), g.choice([0.0, 0.25, 0.5, 1.0], (40, 3)),
                        g.uniform(-0.5, 1.5, (40, 3))]).astype(np.float32)  # outside the cube: clamped
    got = oracle.descend(make_tree(nodes, lo, D), q)
    np.testing.assert_array_equal(got, brute_descent(nodes, lo, q, D + 1))
    # a sample point always finds a node at every level its cell was refined to
    assert np.all(got[:100, 0] == 0)


@settings(max_examples=30, deadline=None)
@given(st.integers(0, 5), st.integers(0, 6), st.integers(1, 200), st.integers(0, 2 ** 31 - 1))
def test_descent_property(D, tau, n, seed):
    g = np.random.default_rng(seed)
    x = (g.uniform(0, 1, (n, 3)) ** 2).astype(np.float32)
    nodes, lo = oracle.build_octree(x, D, tau)
    ew, eo, _, _ = expected_tree(x, D, tau)
    np.testing.assert_array_equal(nodes, ew)
    q = np.concatenate([x[:20], g.uniform(0, 1, (20, 3))]).astype(np.float32)
    np.testing.assert_array_equal(oracle.descend(make_tree(nodes, lo, D), q),
                                  brute_descent(nodes, lo, q, D + 1))


def test_quantize_exact_dyadic():
    x = np.array([[0.0, 0.5, 1.0], [0.999999940395, 0.25, 0.75], [-1.0, 2.0, 0.5]], np.float32)
    q = oracle.quantize(x, 10)
    assert q.tolist() == [[0, 512, 1023], [1023, 256, 768], [0, 1023, 512]]
