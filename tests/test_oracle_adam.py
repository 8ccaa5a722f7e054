"""Pins for the oracle's optimiser step (Adam, Kingma and Ba, Algorithm 1)
over FP32 masters, with the lazy treatment of feature-map blocks no query
read: torch.optim.Adam in FP64 as an independent implementation, the
first-step closed form, and the untouched blocks left bit-identical."""
import numpy as np
import pytest
import torch

import oracle


def test_first_step_closed_form():
    """From zero moments, the bias-corrected moments are g and g^2, so the
    first step moves each entry by lr g / (|g| + eps)."""
    g = np.random.default_rng(0)
    p0 = g.normal(size=1000).astype(np.float32)
    gr = (g.normal(size=1000) * 10.0 ** g.uniform(-8, 0, 1000)).astype(np.float32)
    lr, eps = 1e-2, 1e-8
    p1, m1, v1 = oracle.adam(p0, gr, np.zeros(1000), np.zeros(1000), t=1, lr=lr, b1=0.9, b2=0.99, eps=eps)
    g64 = gr.astype(np.float64)
    want = (p0.astype(np.float64) - lr * g64 / (np.abs(g64) + eps)).astype(np.float32)
    np.testing.assert_array_equal(p1, want)
    np.testing.assert_array_equal(m1, (0.1 * g64).astype(np.float32))
    np.testing.assert_array_equal(v1, (0.01 * g64 * g64).astype(np.float32))


@pytest.mark.parametrize("b1,b2,eps", [(0.9, 0.99, 1e-15), (0.8, 0.999, 1e-8)])
def test_matches_torch_adam_over_steps(b1, b2, eps):
    """Five steps against torch.optim.Adam on FP64 tensors (the oracle keeps
    FP32 state, hence the tolerance)."""
    g = np.random.default_rng(1)
    n = 4000
    p = g.normal(size=n).astype(np.float32)
    m, v = np.zeros(n, np.float32), np.zeros(n, np.float32)
    tp = torch.tensor(p.astype(np.float64), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(b1, b2), eps=eps)
    for t in range(1, 6):
        gr = (g.normal(size=n) * 1e-3).astype(np.float32)
        p, m, v = oracle.adam(p, gr, m, v, t=t, lr=3e-3, b1=b1, b2=b2, eps=eps)
        tp.grad = torch.tensor(gr.astype(np.float64))
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-6, atol=1e-9)


def test_untouched_blocks_unchanged():
    """Blocks whose flag is zero keep parameters and moments bit-identical;
    flagged blocks get the dense update."""
    g = np.random.default_rng(2)
    block, nb = 32, 50
    n = block * nb
    p = g.normal(size=n).astype(np.float32)
    m = (g.normal(size=n) * 1e-3).astype(np.float32)
    v = (g.uniform(size=n) * 1e-6).astype(np.float32)
    gr = (g.normal(size=n) * 1e-3).astype(np.float32)
    flags = (g.uniform(size=nb) < 0.4).astype(np.uint32)
    lp, lm, lv = oracle.adam(p, gr, m, v, t=7, touched=flags, block=block)
    dp, dm, dv = oracle.adam(p, gr, m, v, t=7)
    on = np.repeat(flags.astype(bool), block)
    for got, dense, old in ((lp, dp, p), (lm, dm, m), (lv, dv, v)):
        np.testing.assert_array_equal(got[on], dense[on])
        np.testing.assert_array_equal(got[~on], old[~on])
    assert on.any() and (~on).any()
