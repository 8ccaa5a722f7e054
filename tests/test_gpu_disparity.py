"""GPU parity of the disparity-shifted lookup (Sec. 3.3: each of the eight
neighbouring cells read along (x - c_j) d + w_r / |w_r| with d from the
hash-grid predictor of Sec. 3.5) against the FP64 oracle, through the C-ABI:
the encoding, the fused query, the residual step's outputs and every
gradient group, the predictor's hash tables and MLP included.

Where the lookup's derivative with respect to d jumps (a shifted direction on
a triangle edge or a grid line of its map, on the equator or a fold of the
lower hemisphere), FP32 and FP64 can take different sides; so can a ReLU of
either network near zero. The FP32 gradient checks drop the few queries
within a stated band of any of these, computed in FP64 from the oracle's
geometry, and report how many."""
import dataclasses
import functools

import numpy as np
import pytest
import torch

import oracle
from paper_2606_08469_amd import binding, synth
from _gpu import (cosine, kink_margin_ok_tree, map_res_tol, oracle_tree_for, rel_l2, report, subset_batch, to_np,
                  tree_for)
from test_gpu_paper import compare_grads, dev, oracle_corners, run_residual

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
MIX_TOL = 1e-2
MIX_COS = 0.999
CI = 6
PAPER = binding.INTERP_PAPER


@functools.lru_cache(maxsize=None)
def params(log2_T=14, scale=0.5, d0=1.5):
    """FP32 masters of config 6 (vertex maps, decoder with attributes) and a
    predictor whose tables are large enough that the disparity varies."""
    cfg = synth.CONFIGS[CI]
    _, lo = oracle_tree_for(cfg.tree_cfg)
    feat = synth.init_tables(cfg, np.diff(lo), vertices=True)
    W, b = synth.init_mlp(cfg)
    disp = synth.init_disparity(cfg, log2_T=log2_T, table_scale=scale, d0=d0)
    return feat, W, b, disp


def models(dtype=torch.float32, disp=None):
    cfg = synth.CONFIGS[CI]
    feat, W, b, d = params()
    d = d if disp is None else disp
    _, nodes, lo = tree_for(cfg.tree_cfg)
    onodes, olo = oracle_tree_for(cfg.tree_cfg)
    gpu = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=dtype, interp=PAPER, disparity=d)
    od = oracle.Disparity(d["res"], synth.HASH_F, d["log2_T"], d["tables"], d["W"], d["b"])
    otree = oracle.Tree(onodes, olo, list(cfg.res), cfg.C, feat, interp=PAPER, disp=od)
    return gpu, otree, oracle.MLP(W, b)


@functools.lru_cache(maxsize=None)
def batch(B, N=None):
    cfg = synth.CONFIGS[CI]
    return synth.train_batch(dataclasses.replace(cfg, B=B, N=cfg.N if N is None else N))


def octa64(v):
    """Octahedral map in FP64 (for the kink filter only)."""
    S = np.abs(v).sum(1)
    u = v[:, :2] / np.where(S > 0, S, 1.0)[:, None]
    low = v[:, 2] < 0
    sx, sy = np.where(u[:, 0] < 0, -1.0, 1.0), np.where(u[:, 1] < 0, -1.0, 1.0)
    fu = np.where(low, (1 - np.abs(u[:, 1])) * sx, u[:, 0])
    fv = np.where(low, (1 - np.abs(u[:, 0])) * sy, u[:, 1])
    return 0.5 * (fu + 1), 0.5 * (fv + 1)


def shift_kink_ok(otree, x, d, band=2e-4):
    """Per query: no shifted lookup with non-zero cell weight within `band`
    (map cells, or relative to |v|_1 for the folds) of a place where its
    derivative with respect to the disparity jumps."""
    dh = oracle.disparity(otree.disp, x, d)
    d64 = d.astype(np.float64)
    u = d64 / np.linalg.norm(d64, axis=1, keepdims=True)
    xc = np.clip(x.astype(np.float64), 0, 1)
    ok = np.ones(len(x), bool)
    for l, R in enumerate(otree.res):
        _, cells, wn = oracle.neighbours(otree, x, l)
        for c in range(8):
            v = (xc - (cells[:, c] + 0.5) / 2 ** l) * dh[:, None] + u
            S = np.abs(v).sum(1)
            near = np.abs(v[:, 2]) < band * S
            near |= (v[:, 2] < 0) & ((np.abs(v[:, 0]) < band * S) | (np.abs(v[:, 1]) < band * S))
            s, t = octa64(v)
            pu, pv = s * R, t * R
            i, j = np.clip(np.floor(pu), 0, R - 1), np.clip(np.floor(pv), 0, R - 1)
            fu, fv = pu - i, pv - j
            same = (2 * i >= R) == (2 * j >= R)
            diag = np.where(same, np.abs(fu + fv - 1), np.abs(fu - fv))
            near |= np.minimum.reduce([fu, 1 - fu, fv, 1 - fv, diag]) < band
            ok &= ~(near & (wn[:, c] > 0))
    return ok


def predictor_kink_ok(disp, x, d, band=1e-5):
    """Per query: every hidden pre-activation of the predictor is at least
    band * (sum |w a| + |b|) from zero (FP64 from the oracle's encoding)."""
    enc = oracle.hash_encode(disp, x)[0]
    d64 = d.astype(np.float64)
    a = np.concatenate([enc, d64 / np.linalg.norm(d64, axis=1, keepdims=True), np.zeros((len(x), 1))], 1)
    ok = np.ones(len(x), bool)
    for W, b in zip(disp.W[:-1], disp.b[:-1]):
        W64, b64 = W.astype(np.float64), b.astype(np.float64)
        z = a @ W64.T + b64
        ok &= (np.abs(z) / (np.abs(a) @ np.abs(W64).T + np.abs(b64) + 1e-300)).min(1) >= band
        a = np.maximum(z, 0.0)
    return ok


def kink_safe(otree, W, b, bt, full):
    def ok_of(x, d, g):
        return (shift_kink_ok(otree, x, d) & predictor_kink_ok(otree.disp, x, d) &
                kink_margin_ok_tree(otree, W, b, x, d, attr=g))
    ok = ok_of(bt["x"], bt["dir"], bt["attr"])
    N = int(bt["N"])
    if full:
        ok &= ok_of(bt["x2"].reshape(-1, 3), bt["dir2"].reshape(-1, 3),
                    bt["attr2"].reshape(-1, synth.G_WIDTH)).reshape(-1, N).all(1)
    return subset_batch(bt, np.nonzero(ok)[0]), int((~ok).sum())


def disp_grads_of(model):
    """The predictor's gradients from the model's Parameters' .grad."""
    return [to_np(p.grad) for p in model.disp_params]


def compare_disp_grads(name, got, otree, mlp, bt, tol=None, cos=None):
    """The predictor's gradients against the oracle's. With tol, the FP32 bar
    is derived: dL/dd of a query sums its lookups' weight derivatives, which
    are proportional to R (their FP32 error scales with the largest map as
    for the features, map_res_tol), and every predictor gradient is a sum
    over queries of dL/dd times the predictor's own derivatives; where those
    sums cancel (in full mode the LHS and RHS seeds of a point have
    opposite signs) their relative FP32 error grows by the cancellation
    ratio kappa = sum |dL/dd| / |sum dL/dd| (from the oracle's per-query
    dL/dd; the output bias's gradient is exactly that sum)."""
    out = {}
    oracle.residual_bwd(otree, mlp, bt, disp_out=out)
    want = [out["tables"]] + list(out["W"]) + list(out["b"])
    if tol is not None:
        kappa = float(np.abs(out["dd"]).sum() / max(abs(out["dd"].sum()), 1e-300))
        tol = max(map_res_tol(otree.res, base=tol)) * max(1.0, kappa)
        report(f"{name} predictor bar", kappa=kappa, tol=tol)
    names = ["tables"] + [f"W[{i}]" for i in range(len(out["W"]))] + [f"b[{i}]" for i in range(len(out["b"]))]
    bad = []
    for nm, g, w in zip(names, got, want):
        e, c = rel_l2(g, w), cosine(g, w)
        report(f"{name} predictor {nm}", rel_l2=e, cos=c)
        if (tol is not None and e > tol) or (cos is not None and c < cos):
            bad.append((nm, e, c))
    assert not bad, bad


def test_shifted_encode_matches_oracle():
    """Features of the shifted lookup (FP32) and the eight corner nodes per
    level (bit-exact; they do not depend on the direction); 16-bit features
    of the shifted encoding are refused."""
    bt = batch(2048, 2)
    x = np.concatenate([bt["x"], bt["x2"].reshape(-1, 3)])
    d = np.concatenate([bt["dir"], bt["dir2"].reshape(-1, 3)])
    gpu, otree, _ = models()
    print(f"[case] shifted encode B={len(x)}", flush=True)
    h, idx = binding.encode_query(gpu.tree, dev(x), dev(d), torch.float32)
    want_h, _ = oracle.encode(otree, x, d)
    disp = oracle.disparity(otree.disp, x, d)
    C = otree.C
    for l, tl in enumerate(map_res_tol(otree.res)):
        e = rel_l2(to_np(h)[:, l * C:(l + 1) * C], want_h[:, l * C:(l + 1) * C])
        report(f"shifted encode level {l}", R=otree.res[l], h_rel_l2=e)
        assert e <= tl
    report("shifted encode", B=len(x), h_rel_l2=rel_l2(to_np(h), want_h), disparity_min=float(disp.min()),
           disparity_max=float(disp.max()))
    assert disp.max() - disp.min() > 0.3  # the shift really varies across queries
    np.testing.assert_array_equal(idx.cpu().numpy(), oracle_corners(otree, x))
    with pytest.raises(binding.OOError, match="FP32"):
        binding.encode_query(gpu.tree, dev(x), dev(d), torch.float16)


@pytest.mark.parametrize("dtype,tol", [(torch.float32, FP32_TOL), (torch.float16, MIX_TOL),
                                       (torch.bfloat16, MIX_TOL)])
def test_shifted_query_fwd(dtype, tol):
    bt = batch(1024, 4)
    x = np.concatenate([bt["x"], bt["x2"].reshape(-1, 3)])
    d = np.concatenate([bt["dir"], bt["dir2"].reshape(-1, 3)])
    g = np.concatenate([bt["attr"], bt["attr2"].reshape(-1, synth.G_WIDTH)])
    gpu, otree, omlp = models(dtype)
    print(f"[case] shifted query {dtype} B={len(x)}", flush=True)
    got = to_np(gpu(dev(x), dev(d), attr=dev(g)))
    want = oracle.query_fwd(otree, omlp, x, d, attr=g)
    e = rel_l2(got, want)
    report(f"shifted query {dtype}", B=len(x), rel_l2=e)
    assert e <= tol


def test_zero_disparity_matches_unshifted_gpu_path():
    """A predictor that outputs 0 reads every cell along w_r: the fused
    query equals the unshifted paper scheme's on the GPU."""
    feat, W, b, d = params()
    zero = dict(d, W=[w.copy() for w in d["W"]], b=[v.copy() for v in d["b"]])
    zero["W"][-1][:] = 0.0
    zero["b"][-1][:] = 0.0
    shifted, _, _ = models(disp=zero)
    cfg = synth.CONFIGS[CI]
    _, nodes, lo = tree_for(cfg.tree_cfg)
    plain = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, interp=PAPER)
    bt = batch(1024, 4)
    print("[case] zero disparity", flush=True)
    a = to_np(shifted(dev(bt["x"]), dev(bt["dir"]), attr=dev(bt["attr"])))
    p = to_np(plain(dev(bt["x"]), dev(bt["dir"]), attr=dev(bt["attr"])))
    e = rel_l2(a, p)
    report("zero disparity vs unshifted", rel_l2=e)
    assert e <= 1e-6


@pytest.mark.parametrize("B,N,full", [(512, 8, 0), (256, 4, 1)])
def test_shifted_residual_fp32(B, N, full):
    """Residual outputs, loss and every gradient group, the predictor's
    hash tables and MLP included, element-wise within 1e-5 (the batch
    without the points the kink filter drops)."""
    bt = dict(batch(B, N), grad_through_rhs=full)
    gpu, otree, omlp = models()
    _, W, b, _ = params()
    bt, dropped = kink_safe(otree, W, b, bt, full)
    print(f"[case] shifted residual fp32 B={len(bt['x'])} N={N} full={full} (kink-dropped {dropped})", flush=True)
    got = run_residual(gpu, bt)
    gd = disp_grads_of(gpu)
    lhs, rhs, res, loss = oracle.residual_fwd(otree, omlp, bt)
    for k, w in (("lhs", lhs), ("rhs", rhs), ("resid", res)):
        e = rel_l2(got[k], w)
        report(f"shifted residual {k}", rel_l2=e)
        assert e <= FP32_TOL
    el = abs(got["loss"] - loss) / abs(loss)
    report("shifted residual loss", rel=el)
    assert el <= FP32_TOL
    compare_disp_grads(f"shifted full={full}", gd, otree, omlp, bt, tol=FP32_TOL, cos=0.999999)
    compare_grads(f"shifted full={full}", got, otree, omlp, bt, tol=FP32_TOL, level_tol=map_res_tol(otree.res))


def test_shifted_paper_config_fp16():
    """The paper's configuration with the predictor, FP16 maps and decoder,
    4096 LHS points x 32 samples: radiance and loss within 1e-2, every
    gradient group (the predictor's too) at cosine >= 0.999."""
    bt = batch(4096)
    gpu, otree, omlp = models(torch.float16)
    print(f"[case] shifted paper config fp16 B=4096 N={bt['N']}", flush=True)
    got = run_residual(gpu, bt)
    gd = disp_grads_of(gpu)
    lhs, rhs, _, loss = oracle.residual_fwd(otree, omlp, bt)
    e1, e2, el = rel_l2(got["lhs"], lhs), rel_l2(got["rhs"], rhs), abs(got["loss"] - loss) / abs(loss)
    report("shifted paper config fp16", lhs_rel=e1, rhs_rel=e2, loss_rel=el)
    assert max(e1, e2, el) <= MIX_TOL
    compare_disp_grads("shifted paper config fp16", gd, otree, omlp, bt, cos=MIX_COS)
    compare_grads("shifted paper config fp16", got, otree, omlp, bt, cos=MIX_COS)


def test_predictor_backward_two_row_passes():
    """The predictor's backward runs at most 262,144 queries per pass through
    its row buffer. With the gradient through the target, 8,192 points x 32
    samples give 270,336 backward queries: two passes, the second starting
    at sorted position 262,144 and adding its parameter sums to the first's.
    Every predictor gradient group against the oracle at cosine >= 0.9999
    (FP32, no kink filter: a pass that overwrote instead of adding, or read
    another pass's rows, would lose about 3% of the queries' share)."""
    B, N = 8192, 32
    assert B * (1 + N) > 262144, "two passes of the predictor's row buffer"
    bt = dict(batch(B, N), grad_through_rhs=1)
    gpu, otree, omlp = models()
    print(f"[case] predictor backward two row passes B={B} N={N} full", flush=True)
    run_residual(gpu, bt)
    gd = disp_grads_of(gpu)
    compare_disp_grads("predictor two row passes", gd, otree, omlp, bt, cos=0.9999)
