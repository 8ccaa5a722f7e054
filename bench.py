"""Throughput of the OctaOctree neural-radiosity hot path on one MI355X.

One step = one neural-radiosity training step over one batch of synthetic
input, every stage of the hot path included: FP32 -> FP16 refresh of the
working tables and weights, zeroing of the FP32 gradients, the residual
forward (octree descent, octahedral bilinear fetch per level, decoder MLP for
the B LHS and B*N secondary queries, GGX-weighted Monte-Carlo target, FP64
loss) and the residual backward (recomputed LHS encoding, decoder backward on
matrix cores, FP32 atomic scatter into the feature tables, dW/db reduction).

Workload (the largest configuration, all stages): 2^20 LHS points x (1 + 8)
queries on a depth-10 octree (~0.98M nodes), 11 levels x 8 FP16 channels,
decoder 88-128-128-3 on FP16 matrix cores with FP32 accumulation. The same
batch also runs on the FP32 plain path, and the render forwards at 1280x720
(FP32 unfused and FP16 fused) and 1024x1024 (BF16 fused) are timed alongside.

Prints one JSON line.
"""
import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32 step and render forwards")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the legs of the paper's interpolation and configuration (shorter profiled runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the hot path has no multi-GPU component in this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_08469_amd import binding, synth

    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calib_copy:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE under the
        # profiler give the scale between counter readings and bytes moved.
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    # ---------------- workload --------------------------------------------
    cfg = synth.CONFIGS[5]
    t0 = time.time()
    samples = synth.tree_samples(cfg)
    nodes, lo = binding.build_octree(samples, cfg.D, cfg.tau)
    counts = np.diff(lo)
    feat = synth.init_tables(cfg, counts)
    W, b = synth.init_mlp(cfg)
    batch_np = synth.train_batch(cfg)
    log(f"workload built in {time.time() - t0:.1f}s: nodes={len(nodes)} levels={counts.tolist()}")
    B, N = cfg.B, cfg.N
    Q = B * (1 + N)

    mixed = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=torch.float16)
    batch = binding.device_batch(batch_np)
    outs = tuple(torch.empty((B, 3), dtype=torch.float32, device=dev) for _ in range(3)) + (
        torch.empty((), dtype=torch.float64, device=dev),)
    gl = torch.ones((), dtype=torch.float64, device=dev)
    grad_bufs = {}

    def grads_for(model):
        """FP32 gradient accumulators of a model in one flat buffer (aligned
        views), zeroed with a single fill per step."""
        key = id(model)
        if key not in grad_bufs:
            params = list(model.feat) + list(model.W) + list(model.b) + list(model.disp_params)
            gshapes = [tuple(t.shape) for t in params]
            goffs, gtotal = binding._flat_layout(gshapes)
            gflat = torch.zeros(gtotal, dtype=torch.float32, device=dev)
            gviews = [gflat[o:o + int(np.prod(sh))].view(sh) for sh, o in zip(gshapes, goffs)]
            nf, nw, nb = len(model.feat), len(model.W), len(model.b)
            grad_bufs.clear()  # one model's buffers at a time
            gd = gviews[nf + nw + nb:]
            nd = (len(gd) - 1) // 2
            grad_bufs[key] = (gflat, {"dfeat": gviews[:nf], "dW": gviews[nf:nf + nw], "db": gviews[nf + nw:nf + nw + nb],
                                      "disp": (gd[0], gd[1:1 + nd], gd[1 + nd:]) if gd else None})
        return grad_bufs[key]

    def step(model, ev=None, bt=None, o=None):
        bt = batch if bt is None else bt
        o = outs if o is None else o
        gflat, grads = grads_for(model)
        if ev:
            ev[3].record()
        model.refresh()
        gflat.zero_()
        if ev:
            ev[0].record()
        ws = model.workspace(bt)  # sized for this model's dtypes
        lhs, rhs, res, loss = binding.residual_fwd(model.tree, model.mlp, bt, ws, feat=model.work_feat,
                                                   W=model.work_W, outs=o)
        if ev:
            ev[1].record()
        binding.residual_bwd(model.tree, model.mlp, bt, res, rhs, gl, grads["dfeat"], grads["dW"], grads["db"],
                             ws, feat=model.work_feat, W=model.work_W, disp_grads=grads["disp"])
        if ev:
            ev[2].record()
            ev[4].record()
        return loss

    def timed(model, steps, warmup, kernels=False, bt=None, o=None):
        """Wall time per step over the timed steps, their mean forward and
        backward event times, and (kernels=True) the library's own per-launch
        event timings of every kernel group in the timed region."""
        for _ in range(warmup):
            step(model, bt=bt, o=o)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
        if kernels:
            binding.profile_begin(64 * steps)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            step(model, evs[i], bt=bt, o=o)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps
        per = None
        if kernels:  # kind -> (ms per launch, launches per step)
            per = {k: (v[0] / v[1], v[1] / steps) for k, v in binding.profile_end().items()}
        fwd = [e[0].elapsed_time(e[1]) for e in evs]
        bwd = [e[1].elapsed_time(e[2]) for e in evs]
        tot = np.array([e[3].elapsed_time(e[4]) for e in evs])
        stats = {"median": float(np.median(tot)), "p10": float(np.percentile(tot, 10)),
                 "p90": float(np.percentile(tot, 90)), "mean": float(tot.mean())}
        return wall * 1e3, float(np.mean(fwd)), float(np.mean(bwd)), per, stats

    log("timing mixed step")
    ms, fwd_ms, bwd_ms, per_kernel, st_mixed = timed(mixed, args.steps, args.warmup, kernels=True)
    loss_mixed = float(outs[3].item())
    log(f"mixed: {ms:.3f} ms/step (fwd {fwd_ms:.3f} ms, bwd {bwd_ms:.3f} ms); step events median "
        f"{st_mixed['median']:.3f} p10 {st_mixed['p10']:.3f} p90 {st_mixed['p90']:.3f} ms")
    log("per launch (ms): " + ", ".join(f"{k} {v[0]:.4f}" for k, v in per_kernel.items()))

    # ---------------- optimiser step (NEXT to the hot path) ------------------
    # the last timed step's gradients: mark the nodes the batch read, then
    # one lazy fused Adam step (refresh of the working copy and clear of the
    # gradients included), as a training loop would run after the backward
    opt = optimizer_bench(torch, binding, mixed, batch, grads_for(mixed)[1], args)

    # ---------------- algorithmic bytes / FLOPs ----------------------------
    # Levels present per query: the descent stops at the first missing child.
    xq = torch.cat([batch["x"], batch["x2"].reshape(-1, 3)])
    dq = torch.cat([batch["dir"], batch["dir2"].reshape(-1, 3)])
    _, idx = binding.encode_query(mixed.tree, xq, dq, torch.float16, feat=mixed.work_feat)
    present = (idx >= 0).sum(1).to(torch.float64)
    lv_all = float(present.sum().item())
    lv_lhs = float(present[:B].sum().item())
    # scatter requests to the atomic units: per LHS query and present level,
    # two footprint rows of 2 texels, each one 64-byte chunk when it starts on
    # an even texel and two otherwise (1.5 on average); a 2x2 map is 2 chunks,
    # and so is a level whose gradients go through the library's pair buffers
    per_level = (idx[:B] >= 0).sum(0).to(torch.float64).cpu().numpy()
    paired = pair_buffered_levels(cfg, np.diff(lo))
    atomic_req = float(sum(n * (2.0 if (r == 2 or l in paired) else 3.0)
                           for l, (n, r) in enumerate(zip(per_level, cfg.res))))
    del xq, dq, idx, present
    kern = kernel_rooflines(cfg, B, Q, lv_all, lv_lhs, per_kernel)
    if "scatter" in kern:
        k = kern["scatter"]
        req = atomic_req / k["launches_per_step"]
        rate = req / (k["ms_per_launch"] * 1e-3) / 1e9
        k.update(atomic_requests=int(req), atomic_Greq_s=round(rate, 2), atomic_ceiling_Greq_s=ATOMIC_GREQ_S,
                 frac_of_atomic_ceiling=round(rate / ATOMIC_GREQ_S, 4))
    # the dominant kernel: most launch time per step on the caller's stream
    # (the scatter runs beside the decoder backward on a second stream, so
    # it is reported in `kernels` but not chosen here)
    dom = max((k for k in kern if k != "scatter"), key=lambda k: kern[k]["ms_per_step"])
    roof = {"kernel": dom, **kern[dom], "kernels": kern,
            "traffic_source": ("profiles/traffic_train_step_cfg5.txt" if kern[dom]["traffic"] is not None
                               else "no counter summary for the current kernels")}
    for k, v in kern.items():
        log(f"{k}: {v['ms_per_launch']:.4f} ms/launch, {v['achieved']:.1f} {v['unit']} ({100 * v['frac']:.1f}% of "
            f"{v['bound']} peak); MFMA {100 * v['mfma_frac']:.2f}%")

    # ---------------- FP32 plain step and render forwards -------------------
    extra = {}
    if not args.no_extra:
        fp32 = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=torch.float32)
        log("timing FP32 plain step")
        ms32, f32, b32, _, st32 = timed(fp32, max(3, args.steps // 4), 2)
        loss32 = float(outs[3].item())
        extra["fp32_plain_step"] = {"ms_per_step": round(ms32, 4), "fwd_ms": round(f32, 4), "bwd_ms": round(b32, 4),
                                    "step_event_ms": {k: round(v, 4) for k, v in st32.items()},
                                    "value": round(Q / (ms32 * 1e-3) / 1e6, 2), "unit": "Mqueries/s"}
        extra["speedup_mixed_vs_fp32"] = round(ms32 / ms, 3)
        extra["loss_mixed_vs_fp32_rel"] = abs(loss_mixed - loss32) / abs(loss32)
        del fp32
        torch.cuda.empty_cache()
        extra["render"] = render_bench(torch, binding, synth, args)
    if not args.no_extra and not args.no_paper:
        # the paper's interpolation (8-cell trilinear blend over barycentric
        # vertex maps) on the same tree, batch and decoder
        del mixed
        grad_bufs.clear()
        torch.cuda.empty_cache()
        vfeat = synth.init_tables(cfg, counts, vertices=True)
        paper = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, vfeat, W, b, dtype=torch.float16,
                                   interp=binding.INTERP_PAPER)
        log("timing paper-scheme mixed step")
        msp, fp_, bp_, perp, stp = timed(paper, max(5, args.steps // 4), 2, kernels=True)
        extra["paper_scheme"] = {
            "workload": "same training step with the paper's level feature: 8 neighbouring cells (trilinear, "
                        "renormalised) x 3 barycentric vertices per level, (R+1)^2-vertex FP16 maps",
            "ms_per_step": round(msp, 4), "fwd_ms": round(fp_, 4), "bwd_ms": round(bp_, 4),
            "step_event_ms": {k: round(v, 4) for k, v in stp.items()},
            "value": round(Q / (msp * 1e-3) / 1e6, 2), "unit": "Mqueries/s",
            "ms_per_launch": {k: round(v[0], 4) for k, v in perp.items()},
            "launches_per_step": {k: round(v[1], 2) for k, v in perp.items()}}
        log(f"paper scheme: {msp:.3f} ms/step (fwd {fp_:.3f}, bwd {bp_:.3f})")
        del paper
        grad_bufs.clear()
        torch.cuda.empty_cache()
        extra["paper_scheme"]["render"] = render_bench(torch, binding, synth, args, interp=binding.INTERP_PAPER)
        extra["paper_config"] = paper_config_bench(torch, binding, synth, args, timed, grad_bufs)

    # ---------------- CPU baseline (oracle) --------------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(batch_np, nodes, lo, cfg, feat, W, b)

    value = Q / (ms * 1e-3) / 1e6
    line = {
        "metric": "Mqueries/s encode+MLP fwd and fwd+bwd, mixed vs FP32 at <=1e-2 err; % HBM/MFMA peak",
        "value": round(value, 2),
        "unit": "Mqueries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {
            "workload": "neural-radiosity training step: 2^20 LHS points x (1+8) queries, fwd+bwd, "
                        "depth-10 octree (%d nodes), 11 levels x 8 FP16 channels, MLP 88-128-128-3 "
                        "FP16 MFMA, FP32 atomics" % len(nodes),
            "queries_per_step": Q, "lhs_points_per_step": B,
            "lhs_points_per_s_M": round(B / (ms * 1e-3) / 1e6, 3),
            "fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4),
            "step_event_ms": {k: round(v, 4) for k, v in st_mixed.items()},
            "ms_per_launch": {k: round(v[0], 4) for k, v in per_kernel.items()},
            "launches_per_step": {k: round(v[1], 2) for k, v in per_kernel.items()},
        },
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    line["optimizer_step"] = opt
    line.update(extra)
    print(json.dumps(line), flush=True)


def paper_config_bench(torch, binding, synth, args, timed, grad_bufs):
    """The paper's network and loss on its batch schedule: 8 levels x 4 FP16
    channels on vertex maps (257^2 .. 3^2), eight-cell blend along the
    disparity-shifted directions (hash-grid predictor, 16 levels x 2, MLP
    36-64-64-1 with FP32 parameters, its forward on split BF16 operands),
    the 13 surface attributes (+3 zero columns), four
    hidden layers of width 128, relative L2, mirror-direction lookup. One
    timed training step (forward and backward, the predictor's included) per
    schedule stage (B LHS points x M samples), and the first stage without
    the shift for comparison."""
    cfg = synth.CONFIGS[6]
    t0 = time.time()
    nodes, lo = binding.build_octree(synth.tree_samples(cfg), cfg.D, cfg.tau)
    counts = np.diff(lo)
    feat = synth.init_tables(cfg, counts, vertices=True)
    W, b = synth.init_mlp(cfg)
    disp = synth.init_disparity(cfg)
    model = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=torch.float16,
                               interp=binding.INTERP_PAPER, disparity=disp)
    out = {"workload": "paper network and loss: depth-7 octree (%d nodes), 8 levels x 4 FP16 channels on "
                       "(R+1)^2 vertex maps R = 256..2 read along disparity-shifted directions (hash grid "
                       "16 x 2^19 x 2 + MLP 36-64-64-1, FP32 parameters, split-BF16 forward), 13 surface attributes (+3 zero), decoder "
                       "48-128-128-128-128-3 FP16 MFMA, relative L2, detached target" % len(nodes),
           "stages": []}
    log(f"paper config: tree built in {time.time() - t0:.1f}s, nodes={len(nodes)} levels={counts.tolist()}")
    for B, N in synth.PAPER_SCHEDULE:
        bt_np = synth.train_batch(dataclasses.replace(cfg, B=B, N=N))
        bt = binding.device_batch(bt_np)
        del bt_np
        o = tuple(torch.empty((B, 3), dtype=torch.float32, device="cuda") for _ in range(3)) + (
            torch.empty((), dtype=torch.float64, device="cuda"),)
        grad_bufs.clear()
        msc, fc, bc, perc, stc = timed(model, max(5, args.steps // 5), 2, kernels=True, bt=bt, o=o)
        Q = B * (1 + N)
        out["stages"].append({
            "lhs_points": B, "samples_per_point": N, "queries_per_step": Q, "ms_per_step": round(msc, 4),
            "fwd_ms": round(fc, 4), "bwd_ms": round(bc, 4), "value": round(Q / (msc * 1e-3) / 1e6, 2),
            "unit": "Mqueries/s", "step_event_ms": {k: round(v, 4) for k, v in stc.items()},
            "ms_per_launch": {k: round(v[0], 4) for k, v in perc.items()},
            "launches_per_step": {k: round(v[1], 2) for k, v in perc.items()}})
        log(f"paper config B={B} M={N}: {msc:.3f} ms/step (fwd {fc:.3f}, bwd {bc:.3f}), "
            f"{Q / (msc * 1e-3) / 1e6:.1f} Mqueries/s")
        if (B, N) == synth.PAPER_SCHEDULE[0]:
            # the same stage without the shift (every cell reads the unshifted direction)
            plain = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=torch.float16,
                                       interp=binding.INTERP_PAPER)
            grad_bufs.clear()
            msn, fn, bn, _, _ = timed(plain, max(5, args.steps // 5), 2, bt=bt, o=o)
            out["no_shift_first_stage"] = {"ms_per_step": round(msn, 4), "fwd_ms": round(fn, 4),
                                           "bwd_ms": round(bn, 4)}
            log(f"paper config without the shift, B={B} M={N}: {msn:.3f} ms/step")
            del plain
            grad_bufs.clear()
        del bt, o
        torch.cuda.empty_cache()
    del model
    grad_bufs.clear()
    torch.cuda.empty_cache()
    return out


def optimizer_bench(torch, binding, model, batch, grads, args):
    """Times the node marking and the fused lazy Adam step (FP16 working
    copy) on the gradients of one backward, and reports the share of the
    feature tables it touched and the bytes it moved (per updated element:
    parameter, gradient, both moments read; parameter and moments written,
    the working copy written, the gradient cleared)."""
    ws = model.workspace(batch)
    n_nodes = model.tree.level_offset[-1]
    touched = torch.zeros(n_nodes, dtype=torch.int32, device="cuda")
    flat = [grads["dfeat"][i] for i in range(len(model.feat))] + list(grads["dW"]) + list(grads["db"])
    state = model.new_adam_state()
    reps = max(5, args.steps // 5)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for i in range(reps):
        evs[i][0].record()
        touched.zero_()
        binding.touched_nodes(model.tree, model.mlp, batch, ws, touched, feat=model.work_feat, W=model.work_W)
        evs[i][1].record()
        binding.adam_step(model.adam_segments(flat, state, touched), i + 1, lr=1e-3, work_dtype=model.dtype)
        evs[i][2].record()
    torch.cuda.synchronize()
    mark = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    step = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    lo = model.tree.level_offset
    t = touched.cpu().numpy().astype(bool)
    upd = sum(int(t[lo[l]:lo[l + 1]].sum()) * (p.numel() // max(lo[l + 1] - lo[l], 1))
              for l, p in enumerate(model.feat)) + sum(w.numel() for w in model.W) + sum(v.numel() for v in model.b)
    total = sum(p.numel() for p in model.parameters())
    nbytes = upd * (16 + 12 + 2 + 4)
    log(f"optimizer: mark {mark:.4f} ms, lazy Adam {step:.4f} ms over {upd} of {total} elements "
        f"({nbytes / (step * 1e-3) / 1e9:.0f} GB/s)")
    return {"mark_touched_ms": round(mark, 4), "adam_ms": round(step, 4), "updated_elements": upd,
            "total_elements": total, "touched_nodes": int(t.sum()), "nodes": int(n_nodes),
            "bytes_moved": int(nbytes), "achieved_GBs": round(nbytes / (step * 1e-3) / 1e9, 1),
            "frac_of_hbm_peak": round(nbytes / (step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "lazy Adam (untouched nodes' maps skipped) fused with the FP16 refresh and gradient clear; "
                    "in a training loop it replaces the full refresh and the full gradient clear of the step"}


def _event_times(torch, run, reps):
    """Per-call event times (ms) of `run` over `reps` calls after 3 warm-ups;
    returns (median, p10, p90, last output)."""
    for _ in range(3):
        out_ = run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record()
        out_ = run()
        e1.record()
    torch.cuda.synchronize()
    t = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    return float(np.median(t)), float(np.percentile(t, 10)), float(np.percentile(t, 90)), out_


def render_bench(torch, binding, synth, args, interp=0):
    """Render-query forwards (one query per pixel) on the FP32 plain path
    (encode to memory + decoder kernel) and the 16-bit fused path, with the
    fused path's roofline; and (bilinear scheme only) the standalone 16-bit
    decoder (oo_mlp_fwd on materialised features) at config 4's
    88-128-128-3, the one place where the decoder alone can approach the
    matrix cores' peak. interp selects the level-feature scheme."""
    out = {}
    reps = max(20, args.steps)
    for ci, dtypes in ((2, (torch.float32, torch.float16)), (4, (torch.float32, torch.bfloat16))):
        cfg = synth.CONFIGS[ci]
        s = synth.tree_samples(cfg)
        nodes, lo = binding.build_octree(s, cfg.D, cfg.tau)
        feat = synth.init_tables(cfg, np.diff(lo), vertices=bool(interp))
        W, b = synth.init_mlp(cfg)
        x, d = synth.render_queries(cfg)
        xt = torch.from_numpy(x).cuda()
        dt = torch.from_numpy(d).cuda()
        res = {}
        ref = None
        lv = None
        for dtype in dtypes:
            m = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=dtype, interp=interp)
            if dtype == torch.float32:
                def run():
                    h, _ = binding.encode_query(m.tree, xt, dt, torch.float32, with_idx=False)
                    return binding.mlp_fwd(m.mlp, h)
                name = "fp32_plain_unfused"
                _, idx = binding.encode_query(m.tree, xt, dt, torch.float32)
                # node words read and map entries gathered: one word and 4 texels
                # per present level, or one word and 3 vertices per present corner
                lv = float((idx >= 0).sum().item())
                entries = lv * (3 if interp else 4)
                del idx
            else:
                run = lambda: m(xt, dt)
                name = f"{str(dtype).split('.')[-1]}_fused"
            med, p10, p90, out_ = _event_times(torch, run, reps)
            if ref is None:
                ref = out_.clone()
            err = float(((out_ - ref).norm() / ref.norm()).item())
            rec = {"ms": round(med, 4), "p10_ms": round(p10, 4), "p90_ms": round(p90, 4),
                   "Mqueries_s": round(len(x) / (med * 1e-3) / 1e6, 1), "rel_l2_vs_fp32": err}
            if dtype != torch.float32:
                rec["roofline"] = render_roofline(cfg, len(x), entries, lv, med, 2)
            res[name] = rec
            log(f"render cfg{ci} {name}: {med:.4f} ms (p10 {p10:.4f}, p90 {p90:.4f}), "
                f"{len(x) / (med * 1e-3) / 1e6:.0f} Mq/s, err {err:.2e}")
            if ci == 4 and dtype == torch.float32 and not interp:
                # standalone decoder on materialised 16-bit features
                for hd in (torch.float16, torch.bfloat16):
                    m16 = binding.OctaOctree(nodes, lo, list(cfg.res), cfg.C, feat, W, b, dtype=hd)
                    h16, _ = binding.encode_query(m.tree, xt, dt, hd, with_idx=False)
                    med_m, p10_m, p90_m, _ = _event_times(torch, lambda: binding.mlp_fwd(m16.mlp, h16, W=m16.work_W),
                                                          reps)
                    K0, Hd = cfg.mlp[0], cfg.mlp[1]
                    flop = len(x) * 2 * (K0 * Hd + (len(cfg.mlp) - 3) * Hd * Hd + Hd * 3)
                    nb = len(x) * (K0 * 2 + 12)
                    tsec = med_m * 1e-3
                    key = f"mlp_fwd_{str(hd).split('.')[-1]}"
                    res[key] = {"ms": round(med_m, 4), "p10_ms": round(p10_m, 4), "p90_ms": round(p90_m, 4),
                                "Mqueries_s": round(len(x) / tsec / 1e6, 1),
                                "roofline": {"bound": "mfma", "achieved": round(flop / tsec / 1e12, 1),
                                             "peak": MFMA_F16_PEAK_TFS, "unit": "TFLOP/s",
                                             "frac": round(flop / tsec / 1e12 / MFMA_F16_PEAK_TFS, 4),
                                             "hbm_GBs": round(nb / tsec / 1e9, 1)}}
                    log(f"mlp_fwd cfg4 {key}: {med_m:.4f} ms, {flop / tsec / 1e12:.1f} TFLOP/s "
                        f"({100 * flop / tsec / 1e12 / MFMA_F16_PEAK_TFS:.1f}% of MFMA peak)")
                    del m16, h16
            del m
        out[f"cfg{ci}_{cfg.width}x{cfg.height}"] = res
        torch.cuda.empty_cache()
    return out


HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
# Sustained rate of global FP32 atomic-add requests (one per 64-byte chunk an
# instruction touches) measured on MI355X with a plain atomic kernel.
ATOMIC_GREQ_S = 21.0
MFMA_F16_PEAK_TFS = 2500.0  # MI355X dense FP16 matrix cores


def kernel_rooflines(cfg, B, Q, lv_all, lv_lhs, per_kernel):
    """Algorithmic bytes and FLOPs per launch of the three dominant kernels of
    the step, against their launch times measured in the timed region (the
    backward and the scatter run in several launches per step, each over its
    share of the queries).

    Algorithmic bytes are the method's own work (lv = sum over queries of
    the levels that have a node, FP16 texels):
     - query, per query: 4 taps x C channels x 2 B per present level + a 4 B
       node word per present level + 24 B (x, dir) + 12 B radiance out;
     - backward, per LHS point: the recomputed LHS query (as above) + the
       12 B residual seed;
     - scatter, per LHS point and present level: 4 taps x C FP32 atomic adds
       of 4 B.
    Traffic that only this implementation's split causes is listed apart as
    implementation_bytes: the bucketed order (4 B per query) and the node
    indices and octahedral coordinates the forward keeps for the backward
    (4 B per level + 8 B per LHS query); in the backward those indices and
    coordinates, the order entry, and the FP32 dh it hands to the scatter
    (K0 x 4 B per LHS query); in the scatter the dh, node index and
    coordinates it reads back."""
    C, L, K0 = cfg.C, len(cfg.res), cfg.mlp[0]
    H = cfg.mlp[1]
    mlp_flop = 2 * (K0 * H + (len(cfg.mlp) - 3) * H * H + H * 3)
    gather = 4 * C * 2 + 4
    out = {}
    spec = {
        "query": (lv_all * gather + Q * (24 + 12), Q * 4 + B * (L * 4 + 8), Q * mlp_flop),
        "backward": (lv_lhs * gather + B * (24 + 12 + 12), B * (8 + 4 + K0 * 4), B * 3 * mlp_flop),
        "scatter": (lv_lhs * 4 * C * 4, lv_lhs * (C * 4 + 4) + B * 8, 0),
    }
    counters = counter_traffic()
    for k, (nbytes, impl, flop) in spec.items():
        if k not in per_kernel:
            continue
        # the backward runs in chunks: per-launch work is the step's share
        per_step = per_kernel[k][1]
        nbytes, impl, flop = nbytes / per_step, impl / per_step, flop / per_step
        t = per_kernel[k][0] * 1e-3
        gbs = nbytes / t / 1e9
        rec = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(gbs / HBM_PEAK_GBS, 4), "ms_per_launch": round(per_kernel[k][0], 4),
               "launches_per_step": round(per_step, 2), "ms_per_step": round(per_kernel[k][0] * per_step, 4),
               "algorithmic_bytes": int(nbytes), "implementation_bytes": int(impl), "mlp_flop": int(flop),
               "mfma_frac": round(flop / t / 1e12 / MFMA_F16_PEAK_TFS, 4)}
        if k in counters:
            hb = counters[k]
            rec.update(traffic=hb, measured_GBs=round(hb / t / 1e9, 1),
                       measured_frac=round(hb / t / 1e9 / HBM_PEAK_GBS, 4))
        else:
            rec["traffic"] = None
        out[k] = rec
    return out


def render_roofline(cfg, n_queries, entries, words, ms, elem_bytes):
    """Algorithmic bytes of the fused render forward (C x element size per
    map entry gathered, 4 B per node word read, 24 B position and direction
    and 12 B radiance per query) and its decoder FLOPs, against the measured
    time."""
    C, K0, H = cfg.C, cfg.mlp[0], cfg.mlp[1]
    mlp_flop = 2 * (K0 * H + (len(cfg.mlp) - 3) * H * H + H * 3)
    nbytes = entries * C * elem_bytes + words * 4 + n_queries * 36
    t = ms * 1e-3
    return {"bound": "hbm", "achieved": round(nbytes / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes),
            "mlp_flop": int(n_queries * mlp_flop), "mfma_frac": round(n_queries * mlp_flop / t / 1e12 / MFMA_F16_PEAK_TFS, 4)}


def pair_buffered_levels(cfg, nodes_per_level):
    """Levels whose feature gradients the library accumulates in pair
    buffers: with C = 8, the leading levels with maps of at least 8x8 texels
    whose buffers (per node R + 2 rows of R + 1 pairs of two C-float texels)
    fit in 64 MiB together."""
    out, total = set(), 0
    if cfg.C != 8:
        return out
    for l, (R, n) in enumerate(zip(cfg.res, nodes_per_level)):
        f = int(n) * (R + 2) * (R + 1) * 2 * cfg.C * 4
        if R < 8 or total + f > (64 << 20):
            break
        out.add(l)
        total += f
    return out


def source_digest():
    """SHA-256 over the library sources: a stored counter reading is only
    used while the kernels it measured are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_08469_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "octaoctree.h"), "rb").read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per launch of each kernel in the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by the copy calibration), or {}
    when the summary is missing or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_train_step_cfg5.txt")
    if not os.path.exists(path):
        return {}
    rec = json.load(open(path))
    if rec.get("source_sha256") != source_digest():
        return {}
    return {k: int(v["hbm_bytes_per_launch"]) for k, v in rec.get("kernels", {}).items()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch_np, nodes, lo, cfg, feat, W, b):
    """The FP64 oracle as it stands, on bounded samples of the same batch:
    the first S LHS points with their N secondary queries, residual forward
    plus backward (both spread over T threads). T is every core this
    process may use, within the OMP_NUM_THREADS share when that is set, and
    then T = 1 on a smaller sample."""
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        from oracle import build as obuild
        obuild.build()
    ot, om = oracle.Tree(nodes, lo, list(cfg.res), cfg.C, feat), oracle.MLP(W, b)
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    nt = min(usable, share) if share > 0 else usable
    runs = {}
    for S, T in ((1 << 18, nt), (1 << 14, 1)):
        sb = {k: (v[:S] if isinstance(v, np.ndarray) else v) for k, v in batch_np.items()}
        t = time.perf_counter()
        oracle.residual_fwd(ot, om, sb, nthreads=T)
        oracle.residual_bwd(ot, om, sb, nthreads=T)
        dt = time.perf_counter() - t
        q = S * (1 + cfg.N)
        runs[T] = (q / dt / 1e6, dt, S, q)
        log(f"oracle: {dt:.2f}s for {S} points on {T} thread(s)")
    v, dt, S, q = runs[nt]
    v1, dt1, S1, q1 = runs[1]
    return {"value": round(v, 6), "unit": "Mqueries/s", "cores": nt, "kind": "oracle",
            "sample": f"first {S} of 2^20 LHS points with their {cfg.N} secondary queries each ({q} queries), "
                      f"residual fwd + bwd in FP64 on {nt} threads: {dt:.2f} s",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(), "usable_cores": usable,
            "omp_share": share or None,
            "single_thread": {"value": round(v1, 6), "unit": "Mqueries/s", "cores": 1,
                              "sample": f"first {S1} LHS points ({q1} queries): {dt1:.2f} s"}}


if __name__ == "__main__":
    main()
