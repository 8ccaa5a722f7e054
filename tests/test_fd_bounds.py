"""CPU check of the finite-difference bounds used by the GPU adjoint test
(tests/_fd.py): on the FP64 oracle, where rounding noise is negligible, the
difference quotient at the chosen step must equal the oracle's adjoint to
FP64 accuracy once the computed kink term tau is allowed for (Sec. 3.6,
detached target). The steps (0.05 for a texel entry, 1e-3 for a weight)
cross ReLU branches of some queries; the computed shift must account for
them exactly."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2606_08469_amd import synth

import _fd


@pytest.fixture(scope="module")
def setup():
    cfg = dataclasses.replace(synth.CONFIGS[3], B=4096)
    s = synth.tree_samples(synth.CONFIGS[cfg.tree_cfg])
    nodes, lo = oracle.build_octree(s, cfg.D, cfg.tau)
    feat = synth.init_tables(cfg, np.diff(lo))
    W, b = synth.init_mlp(cfg)
    batch = synth.train_batch(cfg)
    otree, omlp = oracle.Tree(nodes, lo, list(cfg.res), cfg.C, feat), oracle.MLP(W, b)
    _, rhs, _, _ = oracle.residual_fwd(otree, omlp, batch)
    T = rhs.astype(np.float32)
    frozen = dict(batch, target_override=T)
    dfeat, dW, _ = oracle.residual_bwd(otree, omlp, frozen)
    prob = _fd.Problem(cfg, otree, W, b, batch["x"], batch["dir"], T.astype(np.float64))
    return cfg, otree, omlp, frozen, dfeat, dW, prob, feat, W, b


def _fp64_floor(loss, step):
    """Rounding of the FP64 loss sums (12,288 terms) in the two evaluations,
    divided by the step."""
    return 2.0 * 12288 * 2.0 ** -53 * abs(loss) / step


def _loss(cfg, otree, feat, W, b, frozen):
    t = oracle.Tree(otree.nodes, otree.level_offset, list(otree.res), otree.C, feat)
    return oracle.residual_fwd(t, oracle.MLP(W, b), frozen)[3]


def test_feature_steps_are_exact(setup):
    cfg, otree, omlp, frozen, dfeat, dW, prob, feat, W, b = setup
    g = np.random.default_rng(5)
    checked = kinks = 0
    while checked < 12:
        q = int(g.integers(len(frozen["x"])))
        l = int(g.integers(cfg.D + 1))
        if prob.idx[q, l] < 0:
            continue
        ij, _ = oracle.taps(prob.st[q:q + 1], cfg.res[l])
        i, j = ij[0, int(g.integers(4))]
        node = prob.idx[q, l] - otree.level_offset[l]
        flat = int(((node * cfg.res[l] + j) * cfg.res[l] + i) * cfg.C + g.integers(cfg.C))
        v0 = float(np.asarray(feat[l]).reshape(-1)[flat])
        e = prob.entry("feat", l, flat, v0)
        lv = []
        for v in (e["up"], e["dn"]):
            f2 = [np.array(f, np.float32) for f in feat]
            f2[l].reshape(-1)[flat] = v
            lv.append(_loss(cfg, otree, f2, W, b, frozen))
        fd = (lv[0] - lv[1]) / (e["up"] - e["dn"])
        adj = dfeat[l].reshape(-1)[flat]
        assert abs(fd - e["shift"] - adj) <= 1e-9 * abs(adj) + _fp64_floor(lv[0], e["up"] - e["dn"]), (l, fd, adj, e)
        kinks += e["kinks"]
        checked += 1
    assert kinks > 0  # the kink correction was exercised


def test_weight_steps_kink_term(setup):
    cfg, otree, omlp, frozen, dfeat, dW, prob, feat, W, b = setup
    g = np.random.default_rng(6)
    kinks = 0
    for _ in range(12):
        li = int(g.integers(len(W)))
        flat = int(g.integers(np.size(W[li])))
        v0 = float(np.asarray(W[li]).reshape(-1)[flat])
        e = prob.entry("W", li, flat, v0)
        lv = []
        for v in (e["up"], e["dn"]):
            W2 = [np.array(w, np.float32) for w in W]
            W2[li].reshape(-1)[flat] = v
            lv.append(_loss(cfg, otree, feat, W2, b, frozen))
        fd = (lv[0] - lv[1]) / (e["up"] - e["dn"])
        adj = dW[li].reshape(-1)[flat]
        assert abs(fd - e["shift"] - adj) <= 1e-9 * abs(adj) + _fp64_floor(lv[0], e["up"] - e["dn"]), (li, fd, adj, e)
        kinks += e["kinks"]
    assert kinks > 0  # the kink correction was exercised


def test_noise_floor_model_is_small_for_texel_steps(setup):
    """The rounding floor of a texel step stays well below the 1e-2
    relative bar for most entries (otherwise the GPU check would be
    vacuous)."""
    cfg, otree, omlp, frozen, dfeat, dW, prob, feat, W, b = setup
    g = np.random.default_rng(7)
    ratios = []
    while len(ratios) < 20:
        q = int(g.integers(len(frozen["x"])))
        l = int(g.integers(cfg.D + 1))
        if prob.idx[q, l] < 0:
            continue
        ij, _ = oracle.taps(prob.st[q:q + 1], cfg.res[l])
        i, j = ij[0, 0]
        node = prob.idx[q, l] - otree.level_offset[l]
        flat = int(((node * cfg.res[l] + j) * cfg.res[l] + i) * cfg.C)
        v0 = float(np.asarray(feat[l]).reshape(-1)[flat])
        e = prob.entry("feat", l, flat, v0)
        adj = dfeat[l].reshape(-1)[flat]
        if adj != 0.0:
            ratios.append(e["nu"] / abs(adj))
    print(f"[fd-bounds] median nu / |adj| over 20 texel entries: {np.median(ratios):.2e}")
    assert np.median(ratios) < 1e-2, ratios
