"""Small seeded problems shared by the oracle pins and the GPU parity tests."""
import math

import numpy as np

import oracle
from paper_2606_08469_amd import synth


def tiny_problem(seed=0, D=3, res=(4, 4, 2, 2), C=4, widths=(64, 64), B=64, N=3, tau=4,
                 n_samples=600, bias_scale=0.0, n_attr=0):
    """n_attr > 0: the decoder also reads that many surface attributes per
    query (drawn from a generator of their own, so the rest of the problem
    is the same as without them)."""
    g = np.random.default_rng(seed)
    samples = (g.uniform(0, 1, (n_samples, 3)) ** 1.5).astype(np.float32)
    nodes, lo = oracle.build_octree(samples, D, tau)
    counts = np.diff(lo)
    feat = [g.normal(0, 0.1, (int(n), R, R, C)).astype(np.float32) for n, R in zip(counts, res)]
    dims = (len(res) * C + n_attr,) + tuple(widths) + (3,)
    W = [g.uniform(-1, 1, (o, i)).astype(np.float32) * np.float32(math.sqrt(6 / (i + o)))
         for i, o in zip(dims[:-1], dims[1:])]
    b = [(bias_scale * g.normal(size=o)).astype(np.float32) for o in dims[1:]]
    x = np.concatenate([samples[:B // 2], g.uniform(0, 1, (B - B // 2, 3))]).astype(np.float32)
    n = synth.uniform_sphere(B, g)
    wo, _ = synth.cosine_hemisphere(n, g, 1)
    wo = wo[:, 0]
    batch = dict(x=x, dir=wo.astype(np.float32), n=n.astype(np.float32), wo=wo.astype(np.float32),
                 albedo=g.uniform(0.05, 0.95, (B, 3)).astype(np.float32),
                 rough=g.uniform(0.05, 1.0, B).astype(np.float32),
                 Le=np.where(g.uniform(size=(B, 1)) < 0.2, g.uniform(1, 10, (B, 3)), 0).astype(np.float32),
                 N=N, F0=0.04, loss_kind=0, eps=1e-2, grad_through_rhs=0, target_override=None)
    if N > 0:
        wi, cos = synth.cosine_hemisphere(n, g, N)
        batch["wi"] = wi.astype(np.float32)
        batch["pdf"] = (cos / math.pi).astype(np.float32)
        batch["x2"] = g.uniform(0, 1, (B, N, 3)).astype(np.float32)
        batch["dir2"] = (-wi).astype(np.float32)
    else:
        batch["wi"] = batch["pdf"] = batch["x2"] = batch["dir2"] = None
    if n_attr:
        ga = np.random.default_rng(seed + 7919)
        batch["attr"] = ga.uniform(-1, 1, (B, n_attr)).astype(np.float32)
        if N > 0:
            batch["attr2"] = ga.uniform(-1, 1, (B, N, n_attr)).astype(np.float32)
    tree = oracle.Tree(nodes, lo, list(res), C, feat)
    mlp = oracle.MLP(W, b)
    return tree, mlp, batch
