"""GPU parity of the optimiser step (Adam, Kingma and Ba, Algorithm 1, fused
with the working-copy refresh and the gradient clear, lazy over feature-map
blocks no query read) against the oracle, and of the touched-node marking
against the nodes the oracle's descent and neighbour search find."""
import numpy as np
import pytest
import torch

import oracle
from paper_2606_08469_amd import binding, synth
from _gpu import gpu_models, oracle_models, report, to_np, train_batch

pytestmark = pytest.mark.gpu


def _rand(g, n, scale=1.0):
    return (g.normal(size=n) * scale).astype(np.float32)


@pytest.mark.parametrize("work", [torch.float16, torch.bfloat16, torch.float32])
def test_adam_step_matches_oracle(work):
    """Several segments (lazy ones with per-block flags, dense ones with
    ragged lengths) over two consecutive steps: parameters and moments
    within FP32 rounding of the oracle's FP64 step, the working copy the
    round-to-nearest-even of the new parameters, gradients cleared where
    updated, and untouched blocks not written at all."""
    g = np.random.default_rng(3)
    # (n, block, touched fraction, offset): a non-zero offset places the
    # segment's arrays one element past an aligned address, which takes the
    # kernel's per-element path instead of its vector path
    specs = [(64 * 37, 64, 0.5, 0), (81 * 8 * 13, 81 * 8, 0.3, 0), (128 * 88 + 3, 0, 0, 0), (5, 0, 0, 0),
             (1, 0, 0, 0), (4 * 4 * 4 * 1000, 64, 0.05, 0), (64 * 21, 64, 0.5, 1), (1003, 0, 0, 1)]

    def placed(a, off, dtype=None):
        buf = torch.zeros(len(a) + off, dtype=torch.float32 if dtype is None else dtype, device="cuda")
        view = buf[off:]
        view.copy_(torch.from_numpy(a) if dtype is None else torch.from_numpy(a).to(dtype))
        return view

    segs, host = [], []
    for n, block, frac, off in specs:
        p, gr = _rand(g, n), _rand(g, n, 1e-3)
        m, v = _rand(g, n, 1e-4), np.abs(_rand(g, n, 1e-6))
        flags = (g.uniform(size=n // block) < frac).astype(np.int32) if block else None
        t = {k: placed(a.copy(), off) for k, a in (("param", p), ("grad", gr), ("m", m), ("v", v))}
        t["work"] = placed(np.full(n, 7.0, np.float32), off, work) if work != torch.float32 else None
        if block:
            t["touched"], t["block"] = torch.from_numpy(flags).cuda(), block
        segs.append(t)
        host.append(dict(p=p, g=gr, m=m, v=v, flags=flags, block=block))
    # the library takes its hyper-parameters in FP32: the oracle gets those
    # same values, so that 1 - beta is the same number on both sides
    hp = {k: float(np.float32(v)) for k, v in dict(lr=2e-3, beta1=0.9, beta2=0.99, eps=1e-15).items()}
    for step in (1, 2):
        print(f"[case] adam step {step} work={work} segments={len(segs)}", flush=True)
        binding.adam_step(segs, step, lr=hp["lr"], beta1=hp["beta1"], beta2=hp["beta2"], eps=hp["eps"],
                          work_dtype=work)
        torch.cuda.synchronize()
        for i, (t, h) in enumerate(zip(segs, host)):
            flags = None if h["flags"] is None else h["flags"].astype(np.uint32)
            p1, m1, v1 = oracle.adam(h["p"], h["g"], h["m"], h["v"], t=step, lr=hp["lr"], b1=hp["beta1"],
                                     b2=hp["beta2"], eps=hp["eps"], touched=flags, block=max(h["block"], 1))
            on = np.ones(len(p1), bool) if flags is None else np.repeat(flags.astype(bool), h["block"])
            gp, gm, gv, gg = (to_np(t[k]) for k in ("param", "m", "v", "grad"))
            step_size = np.abs(p1.astype(np.float64) - h["p"])
            dp = np.abs(gp.astype(np.float64) - p1)
            bar = 2.0 ** -22 * np.abs(p1) + 1e-5 * step_size
            report(f"adam seg {i} step {step}", n=len(p1), updated=int(on.sum()),
                   worst_p_over_bar=float((dp / np.maximum(bar, 1e-300)).max()),
                   m_rel=float(np.abs(gm - m1).max() / (np.abs(m1).max() + 1e-30)))
            assert np.all(dp <= bar)
            # each moment is a two-term blend computed in FP32: a few units
            # in the last place of the larger term bound it, also where the
            # two terms cancel
            b1, b2 = hp["beta1"], hp["beta2"]
            g64 = h["g"].astype(np.float64)
            m_bar = 2.0 ** -21 * (b1 * np.abs(h["m"]) + (1 - b1) * np.abs(g64)) + 1e-38
            v_bar = 2.0 ** -21 * (b2 * np.abs(h["v"]) + (1 - b2) * g64 * g64) + 1e-44
            assert np.all(np.abs(gm[on].astype(np.float64) - m1[on]) <= m_bar[on])
            assert np.all(np.abs(gv[on].astype(np.float64) - v1[on]) <= v_bar[on])
            # untouched blocks are not written at all
            np.testing.assert_array_equal(gp[~on], h["p"][~on])
            np.testing.assert_array_equal(gm[~on], h["m"][~on])
            np.testing.assert_array_equal(gg[~on], h["g"][~on])
            assert np.all(gg[on] == 0.0)
            if t["work"] is not None:
                w = t["work"].float().cpu().numpy()
                want = torch.from_numpy(gp).to(work).float().numpy()
                np.testing.assert_array_equal(w[on], want[on])
                assert np.all(w[~on] == 7.0)
            # the next step starts from the GPU's state, with fresh gradients
            h.update(p=gp.copy(), m=gm.copy(), v=gv.copy())
            newg = _rand(g, len(gp), 1e-3)
            h["g"] = np.where(on, newg, gg).astype(np.float32)
            t["grad"].copy_(torch.from_numpy(h["g"]))


@pytest.mark.parametrize("interp,full", [(0, 0), (0, 1), (1, 0)])
def test_touched_nodes_match_oracle(interp, full):
    """The nodes marked after a residual forward are exactly those the
    oracle finds for the backward queries: the node per level (bilinear
    scheme) or the eight corner cells' nodes (paper's scheme), of the LHS
    queries, and of the secondary queries too with the gradient through the
    target."""
    ci = 3
    cfg = synth.CONFIGS[ci]
    batch = dict(train_batch(ci, 4096))
    batch["grad_through_rhs"] = full
    if interp:
        from test_gpu_paper import paper_gpu, paper_oracle
        model, (otree, _) = paper_gpu(ci), paper_oracle(ci)
    else:
        model, (otree, _) = gpu_models(ci), oracle_models(ci)
    b = binding.device_batch(batch)
    ws = model.new_workspace(b)
    binding.residual_fwd(model.tree, model.mlp, b, ws)
    n_nodes = model.tree.level_offset[-1]
    touched = torch.zeros(n_nodes, dtype=torch.int32, device="cuda")
    print(f"[case] touched nodes interp={interp} full={full}", flush=True)
    binding.touched_nodes(model.tree, model.mlp, b, ws, touched)
    got = touched.cpu().numpy().astype(bool)
    xs = [batch["x"]] + ([batch["x2"].reshape(-1, 3)] if full else [])
    want = np.zeros(n_nodes, bool)
    for x in xs:
        if interp:
            for l in range(otree.n_levels):
                idx = oracle.neighbours(otree, x, l)[0]
                want[idx[idx >= 0]] = True
        else:
            idx = oracle.descend(otree, x)
            want[idx[idx >= 0]] = True
    report(f"touched interp={interp} full={full}", marked=int(got.sum()), expected=int(want.sum()),
           mismatches=int((got != want).sum()))
    np.testing.assert_array_equal(got, want)


def test_adam_segments_of_a_model_after_backward():
    """A full training iteration on the FP16 model: residual forward and
    backward, touched nodes, one lazy Adam step through the model's
    segments. Untouched nodes' maps keep their parameters, every touched
    block's gradient is cleared, and the working copy equals the cast of
    the updated masters."""
    ci = 3
    model = gpu_models(ci, torch.float16)
    batch = binding.device_batch(train_batch(ci, 4096))
    for p in model.parameters():
        p.grad = None
    print("[case] model adam step after backward", flush=True)
    before = [p.detach().clone() for p in model.feat]
    loss = model.residual(batch)
    loss.backward()
    ws = model.new_workspace(batch)
    binding.residual_fwd(model.tree, model.mlp, batch, ws, feat=model.work_feat, W=model.work_W)
    touched = torch.zeros(model.tree.level_offset[-1], dtype=torch.int32, device="cuda")
    binding.touched_nodes(model.tree, model.mlp, batch, ws, touched, feat=model.work_feat, W=model.work_W)
    grads = [p.grad.contiguous() for p in model.parameters()]
    state = model.new_adam_state()
    binding.adam_step(model.adam_segments(grads, state, touched), 1, lr=1e-3, work_dtype=torch.float16)
    torch.cuda.synchronize()
    lo = model.tree.level_offset
    t = touched.cpu().numpy().astype(bool)
    moved = 0
    for l, (p, p0, w, gr) in enumerate(zip(model.feat, before, model.work_feat, grads)):
        n_l = lo[l + 1] - lo[l]
        on = t[lo[l]:lo[l + 1]]
        a, a0 = to_np(p).reshape(n_l, -1), to_np(p0).reshape(n_l, -1)
        np.testing.assert_array_equal(a[~on], a0[~on])
        assert np.all(to_np(gr).reshape(n_l, -1)[on] == 0.0)
        np.testing.assert_array_equal(w.float().cpu().numpy().reshape(n_l, -1)[on],
                                      p.detach().half().float().cpu().numpy().reshape(n_l, -1)[on])
        moved += int((a[on] != a0[on]).sum())
    report("model adam step", touched=int(t.sum()), entries_moved=moved)
    assert moved > 0
