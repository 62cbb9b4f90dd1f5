"""Throughput of the whole mapping-loss step on one MI355X.

One step = forward render (RGB + depth + 16-d feature) of every view, the L1
loss gradient of Eq. (1) (without D-SSIM), and the full backward to the
Gaussian parameters and the pose twists (lgs_forward + lgs_backward_l1, all
stages in the library's HIP kernels) on device-resident inputs.  The same
step with the D-SSIM term of the photometric loss (lam = 0.2, lgs_loss
before the backward) and the loss kernel alone are reported beside it.  Metric: Mpixel/s = sum over views of W x H per step
/ step time.

Default workload: the batched configuration (500k Gaussians in a 6x6x3 m
room, 8 keyframes: 4 at 640x480 and 4 at 320x240 on a 2 m circle looking
inward, colours and features stored in BF16, FP32 arithmetic), with tile size
and work chunking picked by the library's autotuner.  The plain FP32
single-view form (300k Gaussians, 640x480) is measured beside it.  Inputs are
seeded synthetic scenes shaped like the paper's indoor RGB-D workloads.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s fwd+bwd (RGB+D+16-d feat), BF16 batched vs FP32 plain; HBM GB/s"
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (256 CUs, 2.4 GHz, dual-issue)
PEAK_HBM_GBS = 8000.0

# Algorithmic FP32 operations of the compositing kernels, per (pixel, list
# entry) unit, counted from the per-pixel definition (FMA = 2):
#   evaluation  : offsets 2, quadratic form 8, exp argument 1, exp 1,
#                 alpha 2, the two cut tests 2                      = 16
#   forward contribution : T' 2, stop test 1, weight 1, 20 FMAs 40   = 44
#   backward contribution: 1 - alpha, 1/(1-alpha), T_prev, weight 4,
#                 g.y 40, dL/dalpha 4, running sum 2, dL/dalpha alpha 1,
#                 its five moments over the pixel offsets 5, opacity 1,
#                 20 colour partials 20, sum of the 26 partials over
#                 pixels 26                                         = 103
#   (the factor -1/2 of dL/dm2 and the conic's entries multiply the summed
#   moments once per Gaussian, in the projection backward, not per pixel;
#   dL/dalpha has no transmittance-upstream term in the fused L1 step)
FLOPS_EVAL = 16
FLOPS_FWD_CONTRIB = 44
FLOPS_BWD_CONTRIB = 103


# Algorithmic FP32 operations per evaluated (pixel, list entry) unit in the
# scope table's own count (forward 52 + exp; backward 140 + exp + rcp), reported
# beside the count above.
FLOPS_FWD_EVAL_ALT = 52
FLOPS_BWD_EVAL_ALT = 140


# (tile, chunk, order) of the committed counter summaries
PROFILED_SETTINGS = (32, 4, 2)


def measured_traffic(kernel, settings, workload, mode, field="bytes_per_launch"):
    """HBM bytes per launch of `kernel` (or per step: kernel == "step") from
    the committed counter summary, or None when the kernel sources changed
    since, or the settings, mode or workload differ from the profiled ones.
    field "bytes_per_launch": two rocprofv3 passes, FETCH_SIZE then
    WRITE_SIZE, each scaled against a kernel of known traffic;
    "request_size_bytes": the reads counted by request size (32/64/128 B
    requests at the L2's memory side) plus WRITE_SIZE."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_compositing_batched_c4.md")
    if not os.path.exists(path) or workload != "batched":
        return None
    src = os.path.join(ROOT, "paper_2511_16144_amd", "csrc")
    if kernel == "step":
        h = hashlib.sha256(b"".join(open(os.path.join(src, f), "rb").read()
                                    for f in sorted(os.listdir(src)))).hexdigest()
    else:
        h = hashlib.sha256(open(os.path.join(src, "raster.hip"), "rb").read() +
                           open(os.path.join(src, "lgs_internal.h"), "rb").read()).hexdigest()
    want = {"tile": str(settings["tile"]), "chunk": str(settings["chunk"]), "order": str(settings["order"]),
            "mode": mode, "source_sha256": h}
    for line in open(path):
        f = line.split()
        if len(f) >= 3 and f[0] == "traffic" and f[1] == kernel:
            kv = dict(x.split("=", 1) for x in f[2:] if "=" in x)
            if all(kv.get(k) == v for k, v in want.items()):
                return float(kv[field]) if field in kv else None
    return None


def algorithmic_bytes(wl, c):
    """HBM bytes one step must move by the method's own accounting (the scope
    table's per-unit figures, with the units counted by the kernels):
    compulsory: every Gaussian's geometry (44 B) and appearance (38 B BF16 /
    76 B FP32; read once per step, every Gaussian of the batched workload is
    visible in some view), the images written (RGB, depth, 16 features, T and
    the last contributor: 88 B/px), the fused L1 gradient's reads (rendered and
    target images, 80 + 80 B/px), the gradients written (120 B/Gaussian);
    method: the depth-hoisted sort (4 passes over the visible (view, Gaussian)
    ids and 2 over the pairs, 16 B per element per pass), every visited list
    entry's records in the forward and the backward (32 B geometry + 40 B BF16
    / 80 B FP32 appearance), and the backward's partial records (104 B written
    and read once each)."""
    n, px = wl.scene.n, wl.pixels
    app = 38 if wl.scene.dtype == "bf16" else 76
    rec = 32 + (40 if wl.scene.dtype == "bf16" else 80)
    parts = {
        "compulsory": n * (44 + app) + px * 88 + px * 160 + n * 120,
        "sort": 4 * 16 * c["n_visible"] + 2 * 16 * c["n_pairs"],
        "records": rec * (c["fwd_entries"] + c["bwd_entries"]),
        "partials": 2 * 104 * c["bwd_written"],
    }
    parts["total"] = sum(parts.values())
    return parts


def copy_bandwidth(dev, mib=1024, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time), median of
    `reps` copies of `mib` MiB timed with HIP events."""
    import torch
    a = torch.empty(mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    del a, b
    return 2.0 * (mib << 20) / (ts[len(ts) // 2] / 1e3) / 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_workload(ctx, wl, steps, warmup, dev, tune, settings):
    """Time `steps` whole steps (forward of every view, fused L1 gradient,
    backward) after `warmup` untimed ones; the library records HIP events
    around each stage on the launching stream (settings.profile)."""
    import torch
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    dt = torch.bfloat16 if wl.scene.dtype == "bf16" else torch.float32
    s = wl.scene
    params = P.params_from_arrays(s.means, s.log_scales, s.quats, s.logits, s.rgb, s.feat, device=dev,
                                  appearance_dtype=dt)
    V = len(wl.cams)
    D = wl.scene.feat.shape[1]
    outs = [{"rgb": torch.empty((3, c.height, c.width), device=dev),
             "depth": torch.empty((c.height, c.width), device=dev),
             "feat": torch.empty((D, c.height, c.width), device=dev),
             "T": torch.empty((c.height, c.width), device=dev)} for c in wl.cams]
    tgts = [{"rgb": torch.as_tensor(t.rgb).to(dev), "depth": torch.as_tensor(t.depth).to(dev),
             "feat": torch.as_tensor(t.feat).to(dev)} for t in wl.targets]
    grads = B._grad_buffers(s.n, V, dev, wl.scene.feat.shape[1])
    st = settings
    if tune:
        shapes = [(c.height, c.width) for c in wl.cams]
        g = B.gaussians_c(params["means"], params["log_scales"], params["quats"], params["logits"],
                          params["rgb"], params["feat"])
        cams = (B.lgs_camera * V)(*[B.camera_c(c) for c in wl.cams])
        best = B.lgs_settings()
        sc = settings.to_c()
        rc = B.lib().lgs_autotune(ctx._h, C.byref(sc), C.byref(g), V, cams, B._images_c(tgts, shapes, False),
                                  (C.c_float * 3)(*wl.loss_w), B._images_c(outs, shapes, True),
                                  C.byref(grads[1]), 0, C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  None, C.byref(best))
        if rc != 0:
            raise B.LgsError(rc, B.lib().lgs_last_error(ctx._h).decode())
        st = B.Settings.from_c(best)
        st.profile = settings.profile

    def step(record):
        o, state = ctx.forward(params, wl.cams, st, out=outs)
        ctx.backward_l1(state, params, outs, tgts, wl.loss_w, grads=grads)
        if record is not None:
            record.append(state.stage_ms())
        state.release()

    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    stages = [] if st.profile & B.PROFILE_EVENTS else None
    t0 = time.perf_counter()
    e0.record()
    for a, b in ev:
        a.record()
        step(stages)
        b.record()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_mean = e0.elapsed_time(e1) / steps
    per = sorted(a.elapsed_time(b) for a, b in ev)
    ms = per[len(per) // 2]
    # the work counts come from one more step with the compositing kernels'
    # counting variants (the timed steps run the variants that do not count)
    cs = B.Settings.from_c(st.to_c())
    cs.profile = B.PROFILE_COUNTS
    o, state = ctx.forward(params, wl.cams, cs, out=outs)
    ctx.backward_l1(state, params, outs, tgts, wl.loss_w, grads=grads)
    counts = state.counts()
    state.release()
    med_st = [sorted(x[i] for x in stages)[len(stages) // 2] for i in range(5)] if stages else None
    return {"ms": ms, "ms_mean": ms_mean, "wall_s": wall, "counts": counts, "stages": med_st,
            "settings": {"tile": st.tile, "chunk": st.chunk, "order": st.order}}


def featdim_sweep(ctx, steps, warmup, dev, settings, dims=(8, 16, 32, 64, 128)):
    """The batched step (graph mode, fixed settings) for several language-
    feature dimensions D: step time, the D-dependent arrays the caller holds
    (BF16 features, rendered and target feature images, feature gradients)
    and the D-dependent part of the library's workspace (one appearance
    record per Gaussian and 16-channel group beyond the first; for D > 16 the
    per-group partial sums and scratch images), both counted from sizes."""
    import math
    import scenes
    out = []
    for D in dims:
        wl = scenes.make_workload(4, feat_dim=D)
        r = time_workload_graph(ctx, wl, steps, warmup, dev, False, settings)
        n, V, G = wl.scene.n, len(wl.cams), (D + 15) // 16
        n_rid = V << max(0, math.ceil(math.log2(max(n, 1))))
        caller = n * D * 2 + wl.pixels * D * 4 * 2 + n * D * 4
        work = (G - 1) * n * 40 + ((9 * 4 * wl.pixels + 32 * 4 * n_rid) if G > 1 else 0)
        out.append({"feat_dim": D, "ms_per_step": round(r["ms"], 4),
                    "Mpixel/s": round(wl.pixels / (r["ms"] / 1e3) / 1e6, 3),
                    "feature_arrays_MB": round(caller / 1e6, 1), "extra_workspace_MB": round(work / 1e6, 1)})
        log(f"[bench] feat_dim {D}: {out[-1]}")
        del wl
    return out


def time_workload_graph(ctx, wl, steps, warmup, dev, tune, settings, ssim_lambda=0.0):
    """Same step as `time_workload`, captured once as a hipGraph by the
    library (lgs_graph_create) and replayed: one launch per step."""
    import torch
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    dt = torch.bfloat16 if wl.scene.dtype == "bf16" else torch.float32
    s = wl.scene
    params = P.params_from_arrays(s.means, s.log_scales, s.quats, s.logits, s.rgb, s.feat, device=dev,
                                  appearance_dtype=dt)
    V = len(wl.cams)
    shapes = [(c.height, c.width) for c in wl.cams]
    D = wl.scene.feat.shape[1]
    outs = [{"rgb": torch.empty((3, c.height, c.width), device=dev),
             "depth": torch.empty((c.height, c.width), device=dev),
             "feat": torch.empty((D, c.height, c.width), device=dev),
             "T": torch.empty((c.height, c.width), device=dev)} for c in wl.cams]
    tgts = [{"rgb": torch.as_tensor(t.rgb).to(dev), "depth": torch.as_tensor(t.depth).to(dev),
             "feat": torch.as_tensor(t.feat).to(dev)} for t in wl.targets]
    grads = B._grad_buffers(s.n, V, dev, wl.scene.feat.shape[1])
    g = B.gaussians_c(params["means"], params["log_scales"], params["quats"], params["logits"],
                      params["rgb"], params["feat"])
    cams = (B.lgs_camera * V)(*[B.camera_c(c) for c in wl.cams])
    im, ti = B._images_c(outs, shapes, True), B._images_c(tgts, shapes, False)
    lw = (C.c_float * 3)(*wl.loss_w)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = settings.to_c()
    if tune:
        best = B.lgs_settings()
        rc = B.lib().lgs_autotune(ctx._h, C.byref(st), C.byref(g), V, cams, ti, lw, im, C.byref(grads[1]), 0,
                                  stream, None, C.byref(best))
        if rc != 0:
            raise B.LgsError(rc, B.lib().lgs_last_error(ctx._h).decode())
        st = best
    st.profile = 0     # one graph for the whole step; stage times come from the eager form
    h = C.c_void_p()
    rc = B.lib().lgs_graph_create(ctx._h, C.byref(st), C.byref(g), V, cams, ti, lw, C.c_float(ssim_lambda), im, C.byref(grads[1]), 0,
                                  stream, C.byref(h))
    if rc != 0:
        raise B.LgsError(rc, B.lib().lgs_last_error(ctx._h).decode())

    def launch():
        rc = B.lib().lgs_graph_launch(h, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        if rc != 0:
            raise RuntimeError(f"graph launch failed: {rc}")
    try:
        for _ in range(warmup):
            launch()
        torch.cuda.synchronize()
        if B.lib().lgs_graph_status(h) != 0:
            raise RuntimeError(B.lib().lgs_last_error(ctx._h).decode())
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for a, b in ev:
            a.record()
            launch()
            b.record()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_mean = e0.elapsed_time(e1) / steps
        per = sorted(a.elapsed_time(b) for a, b in ev)
        ms = per[len(per) // 2]
        cnt = B.lgs_counts()
        B.lib().lgs_graph_counts(h, C.byref(cnt))
        counts = {k: getattr(cnt, k) for k, _ in B.lgs_counts._fields_}
        stages = None
    finally:
        torch.cuda.synchronize()
        B.lib().lgs_graph_destroy(h)
    return {"ms": ms, "ms_mean": ms_mean, "wall_s": wall, "counts": counts, "stages": stages,
            "settings": {"tile": st.tile, "chunk": st.chunk, "order": st.order}}


# Algorithmic HBM bytes of the loss kernel per pixel: rendered and observed
# RGB read (12 + 12), RGB gradient written (12); depth read 4 + 4, written 4;
# features read 64 + 64, written 64.
LOSS_BYTES_PER_PIXEL = 240


def time_loss(ctx, wl, dev, settings, lam, reps=50, warmup=5):
    """Median time of one lgs_loss call (D-SSIM + L1 terms and dL/dY of every
    view) on the workload's rendered images: HIP events on the launching
    stream around each call (the call also copies its small view table to
    the device)."""
    import torch
    import paper_2511_16144_amd as P
    dt = torch.bfloat16 if wl.scene.dtype == "bf16" else torch.float32
    s = wl.scene
    params = P.params_from_arrays(s.means, s.log_scales, s.quats, s.logits, s.rgb, s.feat, device=dev,
                                  appearance_dtype=dt)
    outs, state = ctx.forward(params, wl.cams, settings)
    torch.cuda.synchronize()
    state.release()
    ims = [{k: o[k] for k in ("rgb", "depth", "feat")} for o in outs]
    tgts = [{"rgb": torch.as_tensor(t.rgb).to(dev), "depth": torch.as_tensor(t.depth).to(dev),
             "feat": torch.as_tensor(t.feat).to(dev)} for t in wl.targets]
    grad = [{"rgb": torch.empty((3, c.height, c.width), device=dev),
             "depth": torch.empty((c.height, c.width), device=dev),
             "feat": torch.empty((wl.scene.feat.shape[1], c.height, c.width), device=dev)} for c in wl.cams]
    for _ in range(warmup):
        ctx.loss(wl.cams, ims, tgts, wl.loss_w, lam, grad=grad)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        _, terms = ctx.loss(wl.cams, ims, tgts, wl.loss_w, lam, grad=grad)
        e1.record()
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return ts[len(ts) // 2], terms.cpu().numpy()


# Algorithmic HBM bytes of the decoder loss per pixel at C output channels:
# targets read (2 C in BF16), feature map read (64), its gradient written (64).
def decoder_bytes_per_pixel(C):
    return 2 * C + 128


def time_decoder(ctx, wl, dev, C=512, reps=20, warmup=3):
    """Median times of the feature-decoder loss over every view of the
    workload (one decoder shared by the views, BF16 targets of C channels),
    HIP events on the launching stream: (one lgs_decoder_l1_views call over
    all views, one lgs_decoder_l1 call per view)."""
    import torch
    import scenes
    _, Wm, b, _ = scenes.decoder_inputs(99, 1, 1, C)
    tw, tb = torch.as_tensor(Wm).to(dev), torch.as_tensor(b).to(dev)
    feats, tgts = [], []
    for v, c in enumerate(wl.cams):
        F, _, _, G = scenes.decoder_inputs(100 + v, c.width, c.height, C)
        feats.append(torch.as_tensor(F).to(dev))
        tgts.append(torch.as_tensor(G).to(torch.bfloat16).to(dev))
    out_all = (torch.empty(1, device=dev), [torch.empty_like(f) for f in feats], torch.empty_like(tw),
               torch.empty_like(tb))
    outs = [(torch.empty(1, device=dev), torch.empty_like(f), torch.empty_like(tw), torch.empty_like(tb))
            for f in feats]

    def batched():
        ctx.decoder_l1_views(feats, tw, tb, tgts, 1.0, out=out_all)

    def per_view():
        for f, g, o in zip(feats, tgts, outs):
            ctx.decoder_l1(f, tw, tb, g, 1.0, out=o)

    def median(run):
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            run()
            e1.record()
        torch.cuda.synchronize()
        ts = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        return ts[len(ts) // 2]
    return median(batched), median(per_view)


def time_prune(ctx, dev, reps=10, warmup=2):
    """Median time of lgs_prune (grid keys, sort, K-nearest search with the
    similarity test, geometric criteria, mask) on the batched workload's 500k
    Gaussians with object-coherent features; each call synchronises."""
    import torch
    import scenes
    import paper_2511_16144_amd as P
    sc = scenes.prune_scene(0)
    prm = P.params_from_arrays(sc.means, sc.log_scales, sc.quats, sc.logits, sc.rgb, sc.feat, device=dev,
                               appearance_dtype=torch.bfloat16)
    mask = torch.empty(sc.n, dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        _, counts = ctx.prune(prm, mask=mask)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, counts = ctx.prune(prm, mask=mask)
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return ts[len(ts) // 2], counts, sc.n


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 oracle (forward + autodiff backward) on a bounded sample of
    the same workload: 64x64 crops of the first view, until about `budget_s`
    seconds of work are done (cycling over up to 64 seeded crops), with every host core."""
    import numpy as np
    import torch
    import scenes
    from oracle import raster_fp64 as R
    torch.set_num_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    cam = wl.cams[0]
    wins = scenes.crop_windows(11, cam, k=64, size=64)
    done_px = 0
    t0 = time.perf_counter()
    n_crops = 0
    for i in range(1000):
        w = wins[i % len(wins)]
        rects = [[w]] + [[] for _ in wl.cams[1:]]
        ups = scenes.random_upstream(2, [cam], windows=[[w]])
        R.render(wl.scene, [cam], R.Settings(), rects=[[w]], want_margin=False)
        R.vjp(wl.scene, [cam], ups, R.Settings(), rects=[[w]])
        done_px += w[2] * w[3]
        n_crops += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done_px / dt / 1e6, "unit": "Mpixel/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n_crops} crop(s) of 64x64 px of view 0 (forward + backward, FP64, "
                      f"whole-scene projection included), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="batched", choices=["batched", "plain", "precision", "differentiation"])
    ap.add_argument("--no-tune", action="store_true",
                    help="plain FP32 leg: library defaults instead of the autotuner")
    ap.add_argument("--tune", action="store_true",
                    help="batched step: the autotuner's settings instead of the profiled ones")
    ap.add_argument("--mode", default="graph", choices=["eager", "graph"],
                    help="eager: lgs_forward + lgs_backward_l1 per step; graph: one captured launch per step")
    ap.add_argument("--tile", type=int, default=None, help="fix the tile size (skips the autotuner)")
    ap.add_argument("--chunk", type=int, default=None)
    ap.add_argument("--order", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--featdim-sweep", action="store_true",
                    help="also time the batched step for language-feature dimensions 8, 16, 32, 64, 128")
    ap.add_argument("--no-prune", action="store_true",
                    help="skip the language-guided pruning timing (500k Gaussians)")
    ap.add_argument("--no-decoder", action="store_true",
                    help="skip the feature-decoder loss timing (1x1 conv 16 -> 512, BF16 targets)")
    ap.add_argument("--no-dssim", action="store_true",
                    help="skip the step with the D-SSIM loss term (lam = 0.2) and the loss-kernel timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times: a kernel of known HBM traffic "
                         "against which rocprofv3 FETCH_SIZE / WRITE_SIZE counts are scaled")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import scenes
    import paper_2511_16144_amd as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    cfg = {"batched": 4, "plain": 2, "precision": 3, "differentiation": 5}[args.workload]
    log(f"[bench] building workload C{cfg}")
    wl = scenes.make_workload(cfg)
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.rand(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 2.0, out=b)      # one elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written, x3")
        del a, b
    ctx = P.Context(0)
    settings = P.Settings(profile=1)
    # The batched step runs at the settings its committed rocprofv3 counters
    # were taken at (the autotuner's pick among them moves between boxes
    # within timing noise, and measured traffic is only valid for the
    # profiled settings); --tune lets the autotuner choose, any of --tile /
    # --chunk / --order fixes the rest at the library defaults.
    if not args.tune and all(x is None for x in (args.tile, args.chunk, args.order)):
        args.tile, args.chunk, args.order = PROFILED_SETTINGS
    fixed = any(x is not None for x in (args.tile, args.chunk, args.order))
    if args.tile is not None:
        settings.tile = args.tile
    if args.chunk is not None:
        settings.chunk = args.chunk
    if args.order is not None:
        settings.order = args.order
    log(f"[bench] timing C{cfg}: {wl.scene.n} Gaussians, {len(wl.cams)} views, {wl.pixels} px")
    timer = time_workload_graph if args.mode == "graph" else time_workload
    r = timer(ctx, wl, args.steps, args.warmup, dev, args.tune and not fixed, settings)
    mpx = wl.pixels / (r["ms"] / 1e3) / 1e6
    c = r["counts"]
    st = r["stages"]
    if args.mode == "graph":
        # per-stage times come from the eager form of the same step with the
        # same settings: HIP events on the launching stream around each kernel
        fixed_st = P.Settings(profile=1, **r["settings"])
        re = time_workload(ctx, wl, args.steps, args.warmup, dev, False, fixed_st)
        st = re["stages"]
        c = re["counts"]
    if st and min(st) <= 0.0:
        st = None
    names = ["project+depth sort+scans", "pair emission+tile sort", "forward compositing",
             "backward compositing", "gradient reduction+projection backward"]
    stages = {n: round(v, 4) for n, v in zip(names, st)} if st else None
    # dominant kernel: backward compositing (a single kernel between its events)
    fl = FLOPS_EVAL * c["bwd_evals"] + FLOPS_BWD_CONTRIB * c["bwd_contrib"]
    fl_alt = FLOPS_BWD_EVAL_ALT * c["bwd_evals"]
    kms = st[3] if st else None
    achieved = fl / (kms / 1e3) / 1e12 if kms else None
    achieved_alt = fl_alt / (kms / 1e3) / 1e12 if kms else None
    mode = args.mode
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": (achieved / PEAK_FP32_TFLOPS) if achieved else None,
            "traffic": measured_traffic("k_raster_bwd", r["settings"], args.workload, mode),
            "traffic_by_request_size": measured_traffic("k_raster_bwd", r["settings"], args.workload, mode,
                                                        "request_size_bytes"),
            "kernel": "k_raster_bwd", "kernel_ms": kms,
            "units": {"bwd_evals": c["bwd_evals"], "bwd_contrib": c["bwd_contrib"]},
            "flops_per_unit": {"eval": FLOPS_EVAL, "contrib": FLOPS_BWD_CONTRIB},
            "alt_count": {"flops_per_eval": FLOPS_BWD_EVAL_ALT, "achieved": achieved_alt,
                          "frac": (achieved_alt / PEAK_FP32_TFLOPS) if achieved_alt else None},
            "frac_of_unpacked_fp32": (achieved / (PEAK_FP32_TFLOPS / 2)) if achieved else None}
    fwd_fl = FLOPS_EVAL * c["fwd_evals"] + FLOPS_FWD_CONTRIB * c["fwd_contrib"]
    fwd_tf = fwd_fl / (st[2] / 1e3) / 1e12 if st else None
    fwd_tf_alt = FLOPS_FWD_EVAL_ALT * c["fwd_evals"] / (st[2] / 1e3) / 1e12 if st else None
    eager_ms = re["ms"] if args.mode == "graph" else None
    log("[bench] measuring device-copy bandwidth")
    copy_gbs = copy_bandwidth(dev)
    # the step's algorithmic bytes over its time, against the HBM peak and
    # against the measured copy bandwidth
    ab = algorithmic_bytes(wl, c)
    ab_gbs = ab["total"] / (r["ms"] / 1e3) / 1e9
    # whole-step HBM traffic (both counter passes, every kernel, same mode and
    # settings) over the step time
    step_bytes = measured_traffic("step", r["settings"], args.workload, mode)
    step_bytes_rs = measured_traffic("step", r["settings"], args.workload, mode, "request_size_bytes")
    hbm = {"algorithmic_bytes_per_step": ab, "algorithmic_GB/s": round(ab_gbs, 1),
           "algorithmic_frac": round(ab_gbs / PEAK_HBM_GBS, 4),
           "algorithmic_frac_of_copy": round(ab_gbs / copy_gbs, 4),
           "peak": PEAK_HBM_GBS, "copy_GB/s": round(copy_gbs, 1)}
    if step_bytes is not None:
        gbs = step_bytes / (r["ms"] / 1e3) / 1e9
        hbm.update({"measured_bytes_per_step": step_bytes, "measured_GB/s": round(gbs, 1),
                    "measured_frac": round(gbs / PEAK_HBM_GBS, 4), "measured_frac_of_copy": round(gbs / copy_gbs, 4),
                    "source": "profiles/hbm_traffic_compositing_batched_c4.md (FETCH_SIZE + WRITE_SIZE, calibrated)"})
    if step_bytes_rs is not None:
        gbs = step_bytes_rs / (r["ms"] / 1e3) / 1e9
        hbm.update({"measured_bytes_per_step_by_request_size": step_bytes_rs,
                    "measured_GB/s_by_request_size": round(gbs, 1),
                    "measured_frac_by_request_size": round(gbs / PEAK_HBM_GBS, 4)})
    out = {"metric": METRIC, "value": round(mpx, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(r["ms"], 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if wl.scene.dtype == "bf16" else "f32",
           "data": "synthetic (seeded room-surface scenes shaped like indoor RGB-D keyframes)",
           "config": {"workload": wl.name, "gaussians": wl.scene.n,
                      "views": [f"{cc.width}x{cc.height}" for cc in wl.cams],
                      "appearance_storage": wl.scene.dtype,
                      "arithmetic": "fp32 accumulation and transmittance; fp64 projection; bf16 matrix-core "
                                    "operands split exactly where the appearance is bf16",
                      "loss_w": list(wl.loss_w), "mode": args.mode,
                      **r["settings"],
                      "settings_from": "autotuner" if args.tune and not fixed else
                                       ("profiled settings" if tuple(r["settings"][k] for k in ("tile", "chunk", "order"))
                                        == PROFILED_SETTINGS else "command line"),
                      "parallelism": "single GPU"},
           "timing": {"ms_per_step": "median of the timed steps (HIP events around each step)",
                      "ms_per_step_mean": round(r["ms_mean"], 4)},
           "roofline": roof, "stages_ms": stages,
           "forward_compositing": {"TFLOP/s": fwd_tf, "frac": fwd_tf / PEAK_FP32_TFLOPS if fwd_tf else None,
                                   "alt_count_TFLOP/s": fwd_tf_alt},
           "hbm": hbm,
           "counts": c}
    if eager_ms is not None:
        out["eager_ms_per_step"] = round(eager_ms, 4)
    if not args.no_dssim:
        lam = 0.2
        log(f"[bench] timing the step with the D-SSIM loss term (lam = {lam}) and the loss kernel")
        fixed_st = P.Settings(**r["settings"])
        rd = time_workload_graph(ctx, wl, args.steps, args.warmup, dev, False, fixed_st, ssim_lambda=lam)
        loss_ms, terms = time_loss(ctx, wl, dev, fixed_st, lam)
        lb = LOSS_BYTES_PER_PIXEL * wl.pixels
        out["dssim"] = {"ssim_lambda": lam, "graph_ms_per_step": round(rd["ms"], 4),
                        "Mpixel/s": round(wl.pixels / (rd["ms"] / 1e3) / 1e6, 3),
                        "loss_call_ms": round(loss_ms, 4), "loss_bytes": lb,
                        "loss_GB/s": round(lb / (loss_ms / 1e3) / 1e9, 1),
                        "loss_hbm_frac": round(lb / (loss_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                        "view0_terms": [round(float(x), 6) for x in terms[0]]}
    if not args.no_decoder:
        Cd = 512
        log(f"[bench] timing the feature-decoder loss (16 -> {Cd}, every view)")
        dms, dms_pv = time_decoder(ctx, wl, dev, Cd)
        db_ = decoder_bytes_per_pixel(Cd) * wl.pixels
        dfl = 6 * 16 * Cd * wl.pixels       # three products of 16 x C per pixel, FMA = 2
        out["decoder"] = {"out_dim": Cd, "target_dtype": "bf16", "call": "lgs_decoder_l1_views",
                          "ms": round(dms, 4), "ms_one_call_per_view": round(dms_pv, 4),
                          "Mpixel/s": round(wl.pixels / (dms / 1e3) / 1e6, 3),
                          "roofline": {"bound": "hbm", "achieved": round(db_ / (dms / 1e3) / 1e9, 1),
                                       "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                       "frac": round(db_ / (dms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                                       "bytes": db_},
                          "mfma_TFLOP/s": round(dfl / (dms / 1e3) / 1e12, 2)}
    if args.featdim_sweep:
        log("[bench] feature-dimension sweep (batched step, graph mode)")
        out["feat_dim_sweep"] = featdim_sweep(ctx, min(args.steps, 30), min(args.warmup, 5), dev,
                                              P.Settings(**r["settings"]))
    if not args.no_prune:
        log("[bench] timing language-guided pruning (500k Gaussians)")
        pms, pcounts, pn = time_prune(ctx, dev)
        out["prune"] = {"gaussians": pn, "ms": round(pms, 3), "Mgaussians/s": round(pn / (pms / 1e3) / 1e6, 2),
                        "redundant": pcounts[0], "geometric": pcounts[1], "pruned": pcounts[2],
                        "timing": "host wall clock per call (the call synchronises)"}
    if not args.no_plain and cfg != 2:
        log("[bench] timing the plain FP32 single-view form (C2)")
        wl2 = scenes.make_workload(2)
        r2 = timer(ctx, wl2, args.steps, args.warmup, dev, not args.no_tune, P.Settings())
        out["plain_fp32"] = {"workload": wl2.name, "Mpixel/s": round(wl2.pixels / (r2["ms"] / 1e3) / 1e6, 3),
                             "ms_per_step": round(r2["ms"], 4), **r2["settings"]}
        out["batched_bf16_over_plain_fp32"] = round(mpx / out["plain_fp32"]["Mpixel/s"], 3)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(wl)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
