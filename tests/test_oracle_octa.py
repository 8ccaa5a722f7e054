"""Pins for the oracle's octahedral map (Sec. 3.3 projection and fold)."""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "octa_hand_vectors.txt")


def test_hand_vectors():
    rows = np.loadtxt(GOLD)
    d = rows[:, :3].astype(np.float32)
    st = oracle.octa(d)
    # inputs are FP32, so the expected values hold to FP32 input rounding
    np.testing.assert_allclose(st, rows[:, 3:], atol=2e-7, rtol=0)


def test_fold_uses_unfolded_coordinates():
    # (1, 2, -2)/3: a sequential in-place fold would give t = 0.7, not 0.9.
    st = oracle.octa(np.array([[1, 2, -2]], np.float32))
    assert abs(st[0, 1] - 0.9) < 1e-7


def test_round_trip_random_directions():
    g = np.random.default_rng(11)
    d = g.normal(size=(20000, 3)).astype(np.float32)
    back = oracle.octa_decode(oracle.octa(d))
    dd = d.astype(np.float64)
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    assert np.abs(back - dd).max() < 1e-14


def test_hemispheres_land_inside_and_outside_diamond():
    g = np.random.default_rng(12)
    d = g.normal(size=(5000, 3)).astype(np.float32)
    st = oracle.octa(d)
    l1 = np.abs(st[:, 0] - 0.5) + np.abs(st[:, 1] - 0.5)
    up = d[:, 2] > 0
    assert np.all(l1[up] <= 0.5 + 1e-15)
    assert np.all(l1[~up] >= 0.5 - 1e-15)
    assert np.all((st >= 0) & (st <= 1))


def test_scale_invariance():
    g = np.random.default_rng(13)
    d = g.normal(size=(1000, 3)).astype(np.float32)
    np.testing.assert_allclose(oracle.octa(d), oracle.octa(d * np.float32(4.0)), atol=0, rtol=0)


def test_zero_vector_maps_to_centre():
    st = oracle.octa(np.zeros((1, 3), np.float32))
    assert st[0, 0] == 0.5 and st[0, 1] == 0.5


def test_decode_then_encode_interior():
    g = np.random.default_rng(14)
    st = g.uniform(0.001, 0.999, size=(5000, 2))
    d = oracle.octa_decode(st).astype(np.float32)
    # FP32 rounding of the decoded direction bounds the agreement
    np.testing.assert_allclose(oracle.octa(d), st, atol=2e-7)
