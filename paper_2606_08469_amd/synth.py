"""Seeded synthetic workloads shaped like the paper's scenes.

The paper trains and renders Mitsuba scenes (Bathroom, Cornell-box, Kitchen,
Living-room, Veach-ajar) at 1024x1024 and 1280x720 (Sec. 4.1-4.2). None of them
is available, so these generators stand in for them: spheres, boxes, a floor
and a closed room inside the unit cube, area-weighted surface samples for the
octree, pinhole-camera primary hits for render queries, and cosine-sampled
secondary rays traced against the same primitives for the training step.

This module holds no part of the method's arithmetic (no octree, encoding,
network or residual). It only produces FP32 inputs and FP32 initial
parameters, identical for the GPU library and the CPU oracle. All randomness
comes from ``numpy.random.default_rng(1000 * config + k)`` with k = 0 scene,
1 tree samples, 2 queries, 3 feature tables, 4 BSDF inputs and targets,
5 MLP weights, 6 index subsets, 7 materials of rendered pixels, 8 the
disparity predictor's tables and weights.

Configs with ``gbuf`` feed the decoder the paper's surface attributes
g = [x, w_r, n, a, alpha] (Sec. 3.5) after the level features: 13 values per
query, stored with 3 zero columns (``G_WIDTH``) so that the decoder's input
width stays a multiple of 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ROOM_LO, ROOM_HI = 0.01, 0.99


@dataclass(frozen=True)
class Config:
    idx: int
    name: str
    scene: str               # "floor3" or "room16"
    tree_cfg: int            # which config's tree/scene this one uses
    D: int                   # max octree depth; levels 0..D
    res: tuple               # octahedral map resolution per level
    C: int                   # features per texel
    tau: int                 # refine a node holding more than tau samples
    n_tree_samples: int
    obj_fraction: float      # share of tree samples placed on objects (room scenes)
    mlp: tuple               # layer widths, input first
    kind: str                # "train" or "render"
    B: int                   # LHS points (train) or pixels (render)
    N: int = 0               # secondary hits per LHS point
    width: int = 0
    height: int = 0
    rough: tuple = (0.05, 1.0)
    table_dtype: str = "f32"
    mlp_dtype: str = "f32"
    hot: float = 1.0         # extra sample density on four detailed objects
    gbuf: bool = False       # decoder also reads the surface attributes g
    lookup: str = "wo"       # lookup direction: "wo" (outgoing) or "mirror" (w_r)
    loss_kind: int = 0       # 0 mean L2, 1 relative L2
    interp: int = 0          # 0 node + bilinear texels, 1 the paper's (8 cells, vertex maps)


CONFIGS = {
    1: Config(1, "tiny-fwd-bwd-fp32", "floor3", 1, 4, (16, 16, 8, 8, 4), 4, 32, 20_000, 0.0,
              (20, 64, 64, 3), "train", 4096, 0),
    2: Config(2, "render-1280x720", "room16", 2, 8, (32, 32, 16, 16, 8, 8, 4, 4, 2), 8, 32,
              2_000_000, 0.5, (72, 64, 64, 64, 3), "render", 1280 * 720, width=1280, height=720,
              table_dtype="f16", mlp_dtype="f16"),
    3: Config(3, "train-step-fp32", "room16", 2, 8, (32, 32, 16, 16, 8, 8, 4, 4, 2), 8, 32,
              2_000_000, 0.5, (72, 64, 64, 64, 3), "train", 1 << 18, 4, rough=(0.05, 1.0)),
    4: Config(4, "render-1024x1024-glossy", "room16", 4, 10,
              (64, 64, 64, 32, 32, 32, 16, 8, 4, 2, 2), 8, 32, 9_500_000, 0.7,
              (88, 128, 128, 3), "render", 1024 * 1024, width=1024, height=1024,
              table_dtype="bf16", mlp_dtype="bf16", hot=8.0),
    5: Config(5, "train-step-large-mixed", "room16", 4, 10,
              (64, 64, 64, 32, 32, 32, 16, 8, 4, 2, 2), 8, 32, 9_500_000, 0.7,
              (88, 128, 128, 3), "train", 1 << 20, 8, rough=(0.02, 0.2),
              table_dtype="f16", mlp_dtype="f16", hot=8.0),
    # The paper's network and loss (Sec. 3.5, Sec. 3.6, Sec. 4 implementation
    # details): 8 levels of 4 channels with vertex maps from 257^2 down to
    # 3^2, the 13 surface attributes, four hidden layers of width 128,
    # relative L2, lookup along the mirror direction, 65536 LHS points with
    # 32 secondary samples each (the first quarter of its schedule).
    6: Config(6, "train-paper-decoder", "room16", 6, 7, (256, 128, 64, 32, 16, 8, 4, 2), 4, 32,
              9_500_000, 0.7, (8 * 4 + 16, 128, 128, 128, 128, 3), "train", 1 << 16, 32, rough=(0.02, 0.2),
              table_dtype="f16", mlp_dtype="f16", hot=8.0, gbuf=True, lookup="mirror", loss_kind=1, interp=1),
}

G_ATTRS = 13   # x, w_r, n, albedo, roughness
G_WIDTH = 16   # stored width: the attributes, then zeros

# The paper's batch schedule (Sec. 4): every quarter of training halves the
# LHS points and doubles the secondary samples per point.
PAPER_SCHEDULE = ((1 << 16, 32), (1 << 15, 64), (1 << 14, 128), (1 << 13, 256))


def rng(cfg: int, k: int) -> np.random.Generator:
    return np.random.default_rng(1000 * cfg + k)


# --------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------

@dataclass
class Scene:
    spheres: np.ndarray      # [ns][4] centre xyz, radius
    boxes: np.ndarray        # [nb][6] centre xyz, half extents xyz
    floor_z: float | None    # square z = floor_z over [0,1]^2, normal +z
    room: bool               # closed room [ROOM_LO, ROOM_HI]^3, inward normals


def make_scene(cfg: Config) -> Scene:
    g = rng(cfg.tree_cfg, 0)
    if cfg.scene == "floor3":
        r = g.uniform(0.1, 0.3, 3)
        c = g.uniform(r[:, None], 1.0 - r[:, None], (3, 3))
        return Scene(np.concatenate([c, r[:, None]], 1), np.zeros((0, 6)), 0.05, False)
    # 8 spheres and 8 boxes inside a closed room; the front band y < 0.25
    # stays free for the camera.
    r = g.uniform(0.05, 0.15, 8)
    lo = np.stack([ROOM_LO + 0.02 + r, 0.25 + r, ROOM_LO + 0.02 + r], 1)
    hi = np.stack([ROOM_HI - 0.02 - r] * 3, 1)
    cs = g.uniform(lo, hi)
    he = g.uniform(0.03, 0.12, (8, 3))
    lo = np.stack([ROOM_LO + 0.02 + he[:, 0], 0.25 + he[:, 1], ROOM_LO + he[:, 2]], 1)
    hi = ROOM_HI - 0.02 - he
    cb = g.uniform(lo, hi)
    return Scene(np.concatenate([cs, r[:, None]], 1), np.concatenate([cb, he], 1), None, True)


def _sphere_areas(s):
    return 4.0 * math.pi * s[:, 3] ** 2


def _box_face_table(b):
    """Per box face: (box, axis, side, area)."""
    rows = []
    for i, (cx, cy, cz, hx, hy, hz) in enumerate(b):
        h = (hx, hy, hz)
        for axis in range(3):
            u, v = [a for a in range(3) if a != axis]
            for side in (-1.0, 1.0):
                rows.append((i, axis, side, 4.0 * h[u] * h[v]))
    return rows


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _sample_spheres(s, m, g, density=None):
    if m == 0:
        return np.zeros((0, 3)), np.zeros((0, 3))
    p = _sphere_areas(s) * (1.0 if density is None else density)
    k = g.choice(len(s), size=m, p=p / p.sum())
    n = _unit(g.normal(size=(m, 3)))
    return s[k, :3] + s[k, 3:4] * n, n


def _sample_box_faces(rows, centres, half, m, g, inward=False, density=None):
    if m == 0:
        return np.zeros((0, 3)), np.zeros((0, 3))
    a = np.array([r[3] for r in rows])
    if density is not None:
        a = a * density[np.array([r[0] for r in rows])]
    k = g.choice(len(rows), size=m, p=a / a.sum())
    box = np.array([r[0] for r in rows])[k]
    axis = np.array([r[1] for r in rows])[k]
    side = np.array([r[2] for r in rows])[k]
    c, h = centres[box], half[box]
    x = c + h * g.uniform(-1.0, 1.0, (m, 3))
    ar = np.arange(m)
    x[ar, axis] = c[ar, axis] + side * h[ar, axis]
    n = np.zeros((m, 3))
    n[ar, axis] = -side if inward else side
    return x, n


def _room_rows():
    half = 0.5 * (ROOM_HI - ROOM_LO)
    return _box_face_table(np.array([[0.5, 0.5, 0.5, half, half, half]]))


def sample_surfaces(scene: Scene, m: int, g: np.random.Generator, obj_fraction: float | None = None,
                    hot: float = 1.0):
    """Area-weighted points and normals on the scene's surfaces. With
    obj_fraction set (room scenes), that share of the points goes to the
    objects and the rest to the room walls. Within the objects the first two
    spheres and first two boxes are sampled ``hot`` times more densely per
    unit area (finely detailed objects refine deeper)."""
    ds = np.where(np.arange(len(scene.spheres)) < 2, hot, 1.0)
    db = np.where(np.arange(len(scene.boxes)) < 2, hot, 1.0)
    sph_a = (_sphere_areas(scene.spheres) * ds).sum() if len(scene.spheres) else 0.0
    box_rows = _box_face_table(scene.boxes) if len(scene.boxes) else []
    box_a = sum(r[3] * db[r[0]] for r in box_rows)
    obj_a = sph_a + box_a
    wall_a = (6 * (ROOM_HI - ROOM_LO) ** 2 if scene.room else 0.0) + (1.0 if scene.floor_z is not None else 0.0)
    if obj_fraction is None:
        m_obj = g.binomial(m, obj_a / (obj_a + wall_a))
    else:
        m_obj = int(round(m * obj_fraction))
    m_wall = m - m_obj
    m_sph = g.binomial(m_obj, sph_a / obj_a) if obj_a > 0 else 0
    m_box = m_obj - m_sph
    parts = [_sample_spheres(scene.spheres, m_sph, g, ds)]
    if m_box:
        parts.append(_sample_box_faces(box_rows, scene.boxes[:, :3], scene.boxes[:, 3:], m_box, g,
                                       density=db))
    if scene.room:
        half = 0.5 * (ROOM_HI - ROOM_LO)
        parts.append(_sample_box_faces(_room_rows(), np.array([[0.5] * 3]), np.array([[half] * 3]),
                                       m_wall, g, inward=True))
    elif scene.floor_z is not None and m_wall:
        xy = g.uniform(0.0, 1.0, (m_wall, 2))
        parts.append((np.concatenate([xy, np.full((m_wall, 1), scene.floor_z)], 1),
                      np.tile([0.0, 0.0, 1.0], (m_wall, 1))))
    x = np.concatenate([p[0] for p in parts], 0)
    n = np.concatenate([p[1] for p in parts], 0)
    perm = g.permutation(m)
    return np.clip(x[perm], 0.0, 1.0), n[perm]


# --------------------------------------------------------------------------
# Ray casting against the primitives (nearest hit, t > t_min)
# --------------------------------------------------------------------------

def _hit_spheres(s, o, d, t_min, best_t, best_n):
    for cx, cy, cz, r in s:
        oc = o - np.array([cx, cy, cz])
        b = np.einsum("ij,ij->i", oc, d)
        cc = np.einsum("ij,ij->i", oc, oc) - r * r
        disc = b * b - cc
        ok = disc >= 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t1, t2 = -b - sq, -b + sq
        t = np.where(t1 > t_min, t1, np.where(t2 > t_min, t2, np.inf))
        t = np.where(ok, t, np.inf)
        upd = t < best_t
        if upd.any():
            best_t[upd] = t[upd]
            p = o[upd] + t[upd, None] * d[upd]
            best_n[upd] = (p - np.array([cx, cy, cz])) / r


def _hit_boxes(bx, o, d, t_min, best_t, best_n):
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
    for cx, cy, cz, hx, hy, hz in bx:
        lo = np.array([cx - hx, cy - hy, cz - hz])
        hi = np.array([cx + hx, cy + hy, cz + hz])
        with np.errstate(invalid="ignore"):
            ta, tb = (lo - o) * inv, (hi - o) * inv
        tn, tf = np.minimum(ta, tb), np.maximum(ta, tb)
        tn = np.nan_to_num(tn, nan=-np.inf)
        tf = np.nan_to_num(tf, nan=np.inf)
        tmin, tmax = tn.max(1), tf.min(1)
        ok = (tmax >= tmin) & (tmax > t_min)
        enter = tmin > t_min
        t = np.where(ok, np.where(enter, tmin, tmax), np.inf)
        upd = t < best_t
        if upd.any():
            ax = np.where(enter, tn.argmax(1), tf.argmin(1))[upd]
            sgn = np.where(enter[upd], -np.sign(d[upd, ax]), np.sign(d[upd, ax]))
            nn = np.zeros((int(upd.sum()), 3))
            nn[np.arange(len(ax)), ax] = sgn
            best_t[upd] = t[upd]
            best_n[upd] = nn


def _hit_room(o, d, best_t, best_n):
    with np.errstate(divide="ignore", invalid="ignore"):
        tb = np.where(d > 0, (ROOM_HI - o) / d, np.where(d < 0, (ROOM_LO - o) / d, np.inf))
    ax = tb.argmin(1)
    t = tb[np.arange(len(o)), ax]
    upd = t < best_t
    if upd.any():
        nn = np.zeros((int(upd.sum()), 3))
        nn[np.arange(nn.shape[0]), ax[upd]] = -np.sign(d[upd, ax[upd]])
        best_t[upd] = t[upd]
        best_n[upd] = nn


def cast(scene: Scene, o, d, t_min=1e-6, chunk=1 << 20):
    """Nearest hit along unit rays: (hit point, normal, t). Inside the closed
    room every ray hits."""
    out_p = np.empty_like(o)
    out_n = np.empty_like(o)
    out_t = np.empty(len(o))
    for s in range(0, len(o), chunk):
        oo, dd = o[s:s + chunk], d[s:s + chunk]
        bt = np.full(len(oo), np.inf)
        bn = np.zeros_like(oo)
        _hit_spheres(scene.spheres, oo, dd, t_min, bt, bn)
        _hit_boxes(scene.boxes, oo, dd, t_min, bt, bn)
        if scene.room:
            _hit_room(oo, dd, bt, bn)
        out_t[s:s + chunk] = bt
        out_p[s:s + chunk] = oo + np.where(np.isfinite(bt), bt, 0.0)[:, None] * dd
        out_n[s:s + chunk] = bn
    return out_p, out_n, out_t


# --------------------------------------------------------------------------
# Directions
# --------------------------------------------------------------------------

def uniform_sphere(m, g):
    return _unit(g.normal(size=(m, 3)))


def _frame(n):
    a = np.where(np.abs(n[:, :1]) > 0.9, np.array([[0.0, 1.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    t = _unit(np.cross(a, n))
    return t, np.cross(n, t)


def cosine_hemisphere(n, g, k=1):
    """k cosine-distributed directions about each normal: ([m][k][3], cos [m][k])."""
    m = len(n)
    u1, u2 = g.uniform(size=(m, k)), g.uniform(size=(m, k))
    r, phi = np.sqrt(u1), 2.0 * math.pi * u2
    lx, ly, lz = r * np.cos(phi), r * np.sin(phi), np.sqrt(np.maximum(0.0, 1.0 - u1))
    t, b = _frame(n)
    w = lx[..., None] * t[:, None] + ly[..., None] * b[:, None] + lz[..., None] * n[:, None]
    return _unit(w), lz


def reflect(wo, n):
    return 2.0 * np.einsum("ij,ij->i", wo, n)[:, None] * n - wo


def gbuffer(x, wr, n, albedo, rough):
    """Surface attributes [x, w_r, n, a, alpha] per query, FP32 [m][G_WIDTH]
    (the last G_WIDTH - G_ATTRS columns zero)."""
    m = len(x)
    g = np.zeros((m, G_WIDTH), np.float32)
    g[:, 0:3], g[:, 3:6], g[:, 6:9] = x, wr, n
    g[:, 9:12], g[:, 12] = albedo, np.asarray(rough).reshape(m)
    return g


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def tree_samples(cfg: Config) -> np.ndarray:
    """FP32 surface samples from which the octree is built."""
    tc = CONFIGS[cfg.tree_cfg]
    x, _ = sample_surfaces(make_scene(tc), tc.n_tree_samples, rng(tc.idx, 1),
                           tc.obj_fraction if tc.scene == "room16" else None, tc.hot)
    return x.astype(np.float32)


def camera_rays(width, height, eye, target, vfov_deg=60.0):
    """Pinhole rays in scanline order (row 0 at the top)."""
    fwd = _unit(np.asarray(target, float) - np.asarray(eye, float))
    right = _unit(np.cross(fwd, [0.0, 0.0, 1.0]))
    up = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2)
    i = (np.arange(width) + 0.5) / width * 2 - 1
    j = 1 - (np.arange(height) + 0.5) / height * 2
    I, J = np.meshgrid(i * th * width / height, j * th)
    d = fwd + I.reshape(-1, 1) * right + J.reshape(-1, 1) * up
    return _unit(d)


def render_queries(cfg: Config):
    """One query per pixel: x = primary hit, d = mirror reflection of the view
    direction about the hit normal. FP32 [W*H][3] each."""
    scene = make_scene(CONFIGS[cfg.tree_cfg])
    eye = np.array([0.5, 0.06, 0.45])
    d = camera_rays(cfg.width, cfg.height, eye, [0.5, 0.9, 0.4])
    o = np.tile(eye, (len(d), 1))
    p, n, t = cast(scene, o, d)
    assert np.isfinite(t).all()
    wr = _unit(reflect(-d, n))
    return np.clip(p, 0.0, 1.0).astype(np.float32), wr.astype(np.float32)


def render_gbuffer(cfg: Config):
    """Queries and surface attributes of the rendered pixels: (x, w_r, g),
    with a seeded albedo and roughness per pixel."""
    scene = make_scene(CONFIGS[cfg.tree_cfg])
    eye = np.array([0.5, 0.06, 0.45])
    d = camera_rays(cfg.width, cfg.height, eye, [0.5, 0.9, 0.4])
    p, n, t = cast(scene, np.tile(eye, (len(d), 1)), d)
    assert np.isfinite(t).all()
    x = np.clip(p, 0.0, 1.0).astype(np.float32)
    wr = _unit(reflect(-d, n)).astype(np.float32)
    gm = rng(cfg.idx, 7)
    albedo = gm.uniform(0.05, 0.95, (len(x), 3))
    rough = gm.uniform(cfg.rough[0], cfg.rough[1], len(x))
    return x, wr, gbuffer(x, wr, n, albedo, rough)


def train_batch(cfg: Config):
    """Neural-radiosity training batch: LHS points with BSDF inputs and, when
    N > 0, N cosine-sampled secondary hits each; config 1 instead carries
    U[0,1] targets and uniform directions."""
    scene = make_scene(CONFIGS[cfg.tree_cfg])
    g = rng(cfg.idx, 2)
    x, n = sample_surfaces(scene, cfg.B, g, None)
    gb = rng(cfg.idx, 4)
    B, N = cfg.B, cfg.N
    if N == 0:
        d = uniform_sphere(B, g)
        wo = d
    else:
        wo, _ = cosine_hemisphere(n, g, 1)
        wo = wo[:, 0]
        d = _unit(reflect(wo, n)) if cfg.lookup == "mirror" else wo
    out = dict(x=x.astype(np.float32), dir=d.astype(np.float32), n=n.astype(np.float32),
               wo=wo.astype(np.float32), N=N, F0=0.04, loss_kind=cfg.loss_kind, eps=1e-2, grad_through_rhs=0)
    out["albedo"] = gb.uniform(0.05, 0.95, (B, 3)).astype(np.float32)
    out["rough"] = gb.uniform(cfg.rough[0], cfg.rough[1], B).astype(np.float32)
    le = np.zeros((B, 3))
    em = gb.uniform(size=B) < 0.02
    le[em] = gb.uniform(1.0, 10.0, (int(em.sum()), 3))
    out["Le"] = le.astype(np.float32)
    if N == 0:
        out["target_override"] = gb.uniform(0.0, 1.0, (B, 3)).astype(np.float32)
        out["x2"] = out["dir2"] = out["wi"] = out["pdf"] = None
        if cfg.gbuf:
            out["attr"] = gbuffer(x, d, n, out["albedo"], out["rough"])
        return out
    wi, cos = cosine_hemisphere(n, g, N)                       # [B][N][3]
    o = np.repeat(x + 1e-4 * n, N, axis=0)
    p, n2, t = cast(scene, o, wi.reshape(-1, 3))
    assert np.isfinite(t).all()
    x2 = np.clip(p, 0.0, 1.0)
    # at the hit the outgoing direction points back along the sample
    wo2 = -wi.reshape(-1, 3)
    d2 = _unit(reflect(wo2, n2)) if cfg.lookup == "mirror" else wo2
    out["x2"] = x2.reshape(B, N, 3).astype(np.float32)
    out["dir2"] = d2.reshape(B, N, 3).astype(np.float32)
    out["wi"] = wi.astype(np.float32)
    out["pdf"] = (cos / math.pi).astype(np.float32)
    out["target_override"] = None
    if cfg.gbuf:
        albedo2 = gb.uniform(0.05, 0.95, (B * N, 3))
        rough2 = gb.uniform(cfg.rough[0], cfg.rough[1], B * N)
        out["attr"] = gbuffer(x, d, n, out["albedo"], out["rough"])
        out["attr2"] = gbuffer(x2, d2, n2, albedo2, rough2).reshape(B, N, -1)
    return out


def init_tables(cfg: Config, level_counts, vertices: bool = False):
    """FP32 feature tables N(0, 0.1), [n_l][R_l][R_l][C] per level, or
    [n_l][R_l + 1][R_l + 1][C] for vertex-stored maps."""
    g = rng(cfg.idx, 3)
    e = 1 if vertices else 0
    return [g.normal(0.0, 0.1, (int(n), R + e, R + e, cfg.C)).astype(np.float32)
            for n, R in zip(level_counts, cfg.res)]


def init_mlp(cfg: Config):
    """Glorot-uniform weights [out][in] and zero biases, FP32."""
    g = rng(cfg.idx, 5)
    W, b = [], []
    for fin, fout in zip(cfg.mlp[:-1], cfg.mlp[1:]):
        lim = math.sqrt(6.0 / (fin + fout))
        W.append(g.uniform(-lim, lim, (fout, fin)).astype(np.float32))
        b.append(np.zeros(fout, np.float32))
    return W, b


# The disparity predictor (Sec. 3.3, Sec. 3.5): Instant-NGP's hash grid
# shape (16 levels of 2 features, resolutions growing geometrically from
# 16 to 2048 cells per side) and two hidden layers of 64 (Sec. 4).
HASH_LEVELS, HASH_F, HASH_NMIN, HASH_NMAX = 16, 2, 16, 2048


def hash_resolutions(n_levels=HASH_LEVELS, n_min=HASH_NMIN, n_max=HASH_NMAX):
    """N_i = floor(n_min b^i) with b = (n_max / n_min)^(1 / (n_levels - 1))."""
    b = math.exp((math.log(n_max) - math.log(n_min)) / (n_levels - 1))
    return [int(math.floor(n_min * b ** i)) for i in range(n_levels)]


def init_disparity(cfg: Config, log2_T=19, table_scale=1e-4, d0=1.0, widths=(64, 64)):
    """FP32 predictor: hash tables U(-table_scale, table_scale), Glorot MLP on
    [encoding, unit(w_r), 0] -> 1 with zero biases except the output's, d0
    (the disparity it starts from)."""
    g = rng(cfg.idx, 8)
    tables = g.uniform(-table_scale, table_scale, (HASH_LEVELS, 1 << log2_T, HASH_F)).astype(np.float32)
    dims = (HASH_LEVELS * HASH_F + 4,) + tuple(widths) + (1,)
    W, b = [], []
    for fin, fout in zip(dims[:-1], dims[1:]):
        lim = math.sqrt(6.0 / (fin + fout))
        W.append(g.uniform(-lim, lim, (fout, fin)).astype(np.float32))
        b.append(np.zeros(fout, np.float32))
    b[-1][:] = d0
    return dict(res=hash_resolutions(), log2_T=log2_T, tables=tables, W=W, b=b)


def subset(n_total, m, cfg_idx, k=6):
    """Seeded sorted subset of query indices (for oracle checks on big runs)."""
    return np.sort(rng(cfg_idx, k).choice(n_total, size=min(m, n_total), replace=False))
