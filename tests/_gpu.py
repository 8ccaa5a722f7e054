"""Shared setup for the GPU parity tests: seeded workloads built once per
session. The GPU side runs on the library's tree, the oracle on the tree its
own builder makes from the same samples (the two are checked bit-identical
separately); both read the same FP32 masters."""
import dataclasses
import functools
import math

import numpy as np
import torch

import oracle
from paper_2606_08469_amd import binding, synth


def rel_l2(got, want):
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    den = np.linalg.norm(want)
    return float(np.linalg.norm(got - want) / (den if den > 0 else 1.0))


def cosine(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


def report(name, **kv):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kv.items()),
          flush=True)


@functools.lru_cache(maxsize=None)
def tree_for(tree_cfg: int):
    """(samples, nodes, level_offset) of a config's tree, library-built."""
    cfg = synth.CONFIGS[tree_cfg]
    s = synth.tree_samples(cfg)
    nodes, lo = binding.build_octree(s, cfg.D, cfg.tau)
    return s, nodes, lo


@functools.lru_cache(maxsize=None)
def oracle_tree_for(tree_cfg: int):
    cfg = synth.CONFIGS[tree_cfg]
    return oracle.build_octree(synth.tree_samples(cfg), cfg.D, cfg.tau)


@functools.lru_cache(maxsize=None)
def params_for(ci: int):
    """FP32 masters, sized by the oracle's tree (the library's tree has the
    same level sizes, or its parity tests fail)."""
    cfg = synth.CONFIGS[ci]
    _, lo = oracle_tree_for(cfg.tree_cfg)
    feat = synth.init_tables(cfg, np.diff(lo))
    W, b = synth.init_mlp(cfg)
    return feat, W, b


def oracle_models(ci: int):
    """The oracle's view of config ci: its own tree and the FP32 masters."""
    cfg = synth.CONFIGS[ci]
    nodes, lo = oracle_tree_for(cfg.tree_cfg)
    feat, W, b = params_for(ci)
    return oracle.Tree(nodes, lo, list(cfg.res), cfg.C, feat), oracle.MLP(W, b)


def gpu_models(ci: int, dtype=torch.float32):
    cfg = synth.CONFIGS[ci]
    _, nodes, lo = tree_for(cfg.tree_cfg)
    feat, W, b = params_for(ci)
    return binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=dtype)


@functools.lru_cache(maxsize=None)
def render_queries(ci: int):
    return synth.render_queries(synth.CONFIGS[ci])


@functools.lru_cache(maxsize=None)
def train_batch(ci: int, B: int | None = None):
    cfg = synth.CONFIGS[ci]
    if B is not None:
        cfg = dataclasses.replace(cfg, B=B)
    return synth.train_batch(cfg)


def subset_batch(batch: dict, idx) -> dict:
    out = {}
    for k, v in batch.items():
        out[k] = v[idx] if isinstance(v, np.ndarray) else v
    return out


def to_np(t):
    return t.detach().float().cpu().numpy() if t.dtype != torch.float64 else t.detach().cpu().numpy()


def map_res_tol(res, base=1e-5, r_ref=64):
    """FP32 bar per level for quantities read through a level's maps. A
    lookup's weights are affine in (s R, t R); FP32 rounds s and t to about
    2^-24, so the weights, and the features and gradients formed from them,
    carry an error proportional to R. The FP32 bar of the workload
    definitions (1e-5) was set for maps of at most 64 per side; a level
    with R > 64 (the paper's 2^8 + 1 vertices) gets it scaled by R / 64."""
    return [base * max(1.0, R / r_ref) for R in res]


# Relative distance of a hidden pre-activation from zero below which FP32
# evaluation (operands rounded to 2^-24, sums of up to 128 products) can put
# it on the other side of the ReLU kink than the FP64 oracle does.
KINK_BAND = 1e-5


def kink_margin_ok(ci: int, x, d, band=KINK_BAND):
    """True per query when every hidden pre-activation z of the decoder, in
    FP64, satisfies |z| >= band * (sum of |w a| + |b|): a path whose rounding
    of z stays below that band takes the oracle's ReLU derivative branch."""
    otree, _ = oracle_models(ci)
    _, W, b = params_for(ci)
    return kink_margin_ok_tree(otree, W, b, x, d, band)


def kink_margin_ok_tree(otree, W, b, x, d, band=KINK_BAND, attr=None):
    """attr: [B][E] surface attributes the decoder reads after h."""
    a = oracle.encode(otree, x, d)[0].astype(np.float64)
    if attr is not None:
        a = np.concatenate([a, np.asarray(attr, np.float64).reshape(len(a), -1)], axis=1)
    ok = np.ones(len(a), bool)
    for i in range(len(W) - 1):
        Wi, bi = np.asarray(W[i], np.float64), np.asarray(b[i], np.float64)
        z = a @ Wi.T + bi
        scale = np.abs(a) @ np.abs(Wi).T + np.abs(bi) + 1e-300
        ok &= (np.abs(z) / scale).min(axis=1) >= band
        a = np.maximum(z, 0.0)
    return ok


def kink_safe_batch(ci: int, batch: dict, full: bool, band=KINK_BAND):
    """The batch without the points whose differentiated queries (the LHS
    query; with the gradient through the target also its secondary queries)
    sit within `band` (relative rounding of the path) of a ReLU kink.
    Returns (batch, dropped)."""
    ok = kink_margin_ok(ci, batch["x"], batch["dir"], band)
    N = int(batch.get("N", 0))
    if full and N > 0:
        ok2 = kink_margin_ok(ci, batch["x2"].reshape(-1, 3), batch["dir2"].reshape(-1, 3), band)
        ok &= ok2.reshape(-1, N).all(axis=1)
    return subset_batch(batch, np.nonzero(ok)[0]), int((~ok).sum())
