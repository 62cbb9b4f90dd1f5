"""GPU tests of the captured whole-step graph (forward + fused L1 gradient +
backward), its capacity overflow path, the autotuner and multi-view batching,
all through the C ABI.  Where the oracle's loss gradient is compared, the
oracle forms it from its own render, and the targets are first moved away
from that render's values (by 1e-4 at least) so that no L1 residual changes
sign between FP32 and FP64."""
import ctypes as C
import json
import os
import sys

import numpy as np
import pytest
import torch

import scenes
from oracle import raster_fp64 as R
from gpu_helpers import GraphRun
from parity import (TOL_F32, ambiguous, forward_errors, fmt, gaussian_ambiguity, gpu_params, grad_errors,
                    grads_np, rel_err, separate_targets, to_np, upstream_tensors)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_16144_amd as P
    c = P.Context(0)
    yield c
    c.close()


def assert_close_groups(a, b, tol=1e-5):
    """The fused L1 backward multiplies the exact BF16 sign of the residual by
    the per-channel scale after the matrix-core product; an explicit upstream
    is split into two BF16 terms before it.  The two agree to rounding, not
    bitwise."""
    for k in a:
        l2, mx = rel_err(a[k], b[k])
        assert l2 <= tol and mx <= tol, (k, l2, mx)


def l1_upstream_f32(outs, wl):
    """dL/dY of the L1 loss, computed in FP32 exactly as the kernel does."""
    ups = []
    for o, t in zip(outs, wl.targets):
        H, W = t.depth.shape
        HW = np.float32(H * W)
        s = [np.float32(wl.loss_w[0]) / (np.float32(3.0) * HW), np.float32(wl.loss_w[1]) / HW,
             np.float32(wl.loss_w[2]) / (np.float32(16.0) * HW)]
        g = np.empty((20, H, W), np.float32)
        g[:3] = np.sign(o["rgb"] - t.rgb) * s[0]
        g[3] = np.sign(o["depth"] - t.depth) * s[1]
        g[4:] = np.sign(o["feat"] - t.feat) * s[2]
        ups.append(g)
    return ups


def test_graph_equals_eager_and_replays(ctx):
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(1)
    say("[case] C1 graph vs eager, 4 replays with eager work between")
    ref = R.render(wl.scene, wl.cams, R.Settings())
    wl.targets = separate_targets(ref, wl.targets)
    run = GraphRun(ctx, wl, P.Settings(tile=16))
    assert run.rc == 0, P.lib().lgs_last_error(ctx._h).decode()
    snaps = []
    for k in range(4):
        run.launch()
        assert run.status() == 0
        snaps.append(run.snapshot())
        # unrelated eager work between replays
        prm = gpu_params(scenes.make_workload(1, n=300, res_scale=0.5).scene)
        outs, st = ctx.forward(prm, scenes.make_workload(1, n=300, res_scale=0.5).cams, P.Settings(tile=8))
        torch.cuda.synchronize()
        st.release()
        x = torch.randn(1000, device="cuda").sum().item()
    for s in snaps[1:]:
        for a, b in zip(s[0], snaps[0][0]):
            for k in a:
                assert np.array_equal(a[k], b[k]), k
        for k in s[1]:
            assert np.array_equal(s[1][k], snaps[0][1][k]), k
    outs_g, grads_g = snaps[0]
    # eager forward with the same settings: bitwise equal images
    prm = gpu_params(wl.scene)
    outs_e, state = ctx.forward(prm, wl.cams, P.Settings(tile=16))
    outs_e = to_np(outs_e)
    for k in ("rgb", "depth", "feat", "T"):
        assert np.array_equal(outs_e[0][k], outs_g[0][k]), k
    # eager fused-L1 backward: bitwise equal gradients (same kernels)
    tg = [{"rgb": torch.as_tensor(t.rgb).cuda(), "depth": torch.as_tensor(t.depth).cuda(),
           "feat": torch.as_tensor(t.feat).cuda()} for t in wl.targets]
    outs_t = [{k: torch.as_tensor(v).cuda() for k, v in o.items() if k != "n"} for o in outs_e]
    gl = grads_np(ctx.backward_l1(state, prm, outs_t, tg, wl.loss_w))
    torch.cuda.synchronize()
    for k in gl:
        assert np.array_equal(gl[k], grads_g[k]), k
    # eager backward of the same L1 upstream given explicitly: equal to rounding
    ups = l1_upstream_f32(outs_e, wl)
    ge = grads_np(ctx.backward(state, prm, upstream_tensors(ups)))
    torch.cuda.synchronize()
    state.release()
    assert_close_groups(ge, grads_g)
    # and the oracle's gradient of the same loss on its own render
    gr = R.vjp(wl.scene, wl.cams, R.l1_upstream(ref, wl.targets, wl.loss_w), R.Settings())
    amb = ambiguous(ref[0]["margin"])
    err = grad_errors(grads_g, gr, gaussian_ambiguity(ref[0], amb, wl.scene.n))
    say("  graph grads vs oracle:", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)
    run.destroy()


def test_graph_capacity_overflow_and_recreate(ctx):
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(1)
    say("[case] C1 graph with pair capacity 64 -> LGS_ERR_CAPACITY, then auto capacity")
    run = GraphRun(ctx, wl, P.Settings(tile=8), capacity=64)
    assert run.rc == 0
    run.launch()
    assert run.status() == P.binding.LGS_ERR_CAPACITY
    outs, grads = run.snapshot()
    assert np.isfinite(grads["twist"]).all()        # overflow writes zero gradients, no garbage
    assert np.all(grads["means"] == 0)
    run.destroy()
    run = GraphRun(ctx, wl, P.Settings(tile=8, profile=P.binding.PROFILE_COUNTS), capacity=0)
    run.launch()
    assert run.status() == 0
    c = run.counts()
    assert c["n_pairs"] > 64 and c["fwd_evals"] > 0 and c["bwd_evals"] > 0
    run.destroy()


def test_graph_autotune_and_cache(ctx, tmp_path):
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    wl = scenes.make_workload(4, n=20000, res_scale=0.25)
    say("[case] autotune on a reduced batched scene")
    run = GraphRun(ctx, wl, P.Settings())
    assert run.rc == 0
    best = B.lgs_settings()
    cache = str(tmp_path / "tune.json")
    rc = B.lib().lgs_autotune(ctx._h, C.byref(run.st), C.byref(run.g), len(wl.cams), run.cams, run.tgts, run.lw,
                              run.imgs, C.byref(run.gr), 0, run.stream(), cache.encode(), C.byref(best))
    assert rc == 0, B.lib().lgs_last_error(ctx._h).decode()
    assert best.tile in (8, 16, 32) and best.chunk in (1, 2, 4) and best.order in (0, 1, 2)
    d = json.load(open(cache))
    assert len(d) == 1 and list(d.values())[0] == {"tile": best.tile, "chunk": best.chunk, "order": best.order}
    best2 = B.lgs_settings()
    rc = B.lib().lgs_autotune(ctx._h, C.byref(run.st), C.byref(run.g), len(wl.cams), run.cams, run.tgts, run.lw,
                              run.imgs, C.byref(run.gr), 0, run.stream(), cache.encode(), C.byref(best2))
    assert rc == 0 and (best2.tile, best2.chunk, best2.order) == (best.tile, best.chunk, best.order)
    run.destroy()


@pytest.mark.parametrize("order", [0, 1, 2])
def test_batched_views_equal_single_views(ctx, order):
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(4, n=40000, res_scale=0.25)
    say(f"[case] batched 8 views vs one view at a time, order={order}")
    prm = gpu_params(wl.scene)
    outs, st = ctx.forward(prm, wl.cams, P.Settings(tile=16, order=order), want_n=True)
    outs = to_np(outs)
    ups = scenes.random_upstream(4, wl.cams)
    gb = grads_np(ctx.backward(st, prm, upstream_tensors(ups)))
    torch.cuda.synchronize()
    st.release()
    gsum = None
    for v, cam in enumerate(wl.cams):
        o1, s1 = ctx.forward(prm, [cam], P.Settings(tile=16))
        o1 = to_np(o1)[0]
        for k in ("rgb", "depth", "feat", "T"):
            assert np.array_equal(o1[k], outs[v][k]), (v, k)
        g1 = grads_np(ctx.backward(s1, prm, upstream_tensors([ups[v]])))
        torch.cuda.synchronize()
        s1.release()
        assert np.allclose(g1["twist"][0], gb["twist"][v], rtol=1e-5, atol=1e-9)
        gsum = g1 if gsum is None else {k: gsum[k] + g1[k] for k in g1 if k != "twist"}
    for k in ("means", "log_scales", "quats", "logits", "rgb", "feat"):
        scale = np.abs(gb[k]).max()
        assert np.abs(gsum[k] - gb[k]).max() <= 1e-5 * scale, k


def test_eager_l1_step_vs_oracle(ctx):
    """forward + lgs_backward_l1: the fused L1 gradient equals the FP32 host
    gradient fed through lgs_backward to rounding, and the oracle's loss
    gradient within 1e-4."""
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(1)
    say("[case] C1 eager L1 step (fused) vs explicit upstream and oracle")
    ref = R.render(wl.scene, wl.cams, R.Settings())
    wl.targets = separate_targets(ref, wl.targets)
    prm = gpu_params(wl.scene)
    tg = [{"rgb": torch.as_tensor(t.rgb).cuda(), "depth": torch.as_tensor(t.depth).cuda(),
           "feat": torch.as_tensor(t.feat).cuda()} for t in wl.targets]
    outs, st = ctx.forward(prm, wl.cams, P.Settings(tile=16))
    gf = grads_np(ctx.backward_l1(st, prm, outs, tg, wl.loss_w))
    torch.cuda.synchronize()
    outs_np = to_np(outs)
    ups = l1_upstream_f32(outs_np, wl)
    ge = grads_np(ctx.backward(st, prm, upstream_tensors(ups)))
    torch.cuda.synchronize()
    st.release()
    assert_close_groups(ge, gf)
    gr = R.vjp(wl.scene, wl.cams, R.l1_upstream(ref, wl.targets, wl.loss_w), R.Settings())
    amb = ambiguous(ref[0]["margin"])
    err = grad_errors(gf, gr, gaussian_ambiguity(ref[0], amb, wl.scene.n))
    say("  fused L1 grads vs oracle:", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)


def test_eager_autotune_and_cache(ctx, tmp_path):
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    wl = scenes.make_workload(4, n=20000, res_scale=0.25)
    say("[case] eager autotune on a reduced batched scene")
    prm = gpu_params(wl.scene)
    V = len(wl.cams)
    g = B.gaussians_c(prm["means"], prm["log_scales"], prm["quats"], prm["logits"], prm["rgb"], prm["feat"])
    outs = [{"rgb": torch.empty((3, c.height, c.width), device="cuda"),
             "depth": torch.empty((c.height, c.width), device="cuda"),
             "feat": torch.empty((16, c.height, c.width), device="cuda"),
             "T": torch.empty((c.height, c.width), device="cuda")} for c in wl.cams]
    tg = [{"rgb": torch.as_tensor(t.rgb).cuda(), "depth": torch.as_tensor(t.depth).cuda(),
           "feat": torch.as_tensor(t.feat).cuda()} for t in wl.targets]
    shapes = [(c.height, c.width) for c in wl.cams]
    im = B._images_c(outs, shapes, True)
    ti = B._images_c(tg, shapes, False)
    _, gr = B._grad_buffers(wl.scene.n, V, "cuda")
    cams = (B.lgs_camera * V)(*[B.camera_c(c) for c in wl.cams])
    lw = (C.c_float * 3)(*wl.loss_w)
    st = P.Settings().to_c()
    best = B.lgs_settings()
    cache = str(tmp_path / "tune.json")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = B.lib().lgs_autotune(ctx._h, C.byref(st), C.byref(g), V, cams, ti, lw, im, C.byref(gr), 0, s,
                              cache.encode(), C.byref(best))
    assert rc == 0, B.lib().lgs_last_error(ctx._h).decode()
    assert best.tile in (8, 16, 32) and best.chunk in (1, 2, 4) and best.order in (0, 1, 2)
    d = json.load(open(cache))
    assert len(d) == 1 and list(d.values())[0] == {"tile": best.tile, "chunk": best.chunk, "order": best.order}
    best2 = B.lgs_settings()
    rc = B.lib().lgs_autotune(ctx._h, C.byref(st), C.byref(g), V, cams, ti, lw, im, C.byref(gr), 0, s,
                              cache.encode(), C.byref(best2))
    assert rc == 0 and (best2.tile, best2.chunk, best2.order) == (best.tile, best.chunk, best.order)


def test_profiled_graph_and_stage_times(ctx):
    """settings.profile = 1: the graph launches its five stages as five
    graphs with events between them; results equal the one-graph form bitwise
    and every stage time is positive.  The eager stage times too, also after
    a graph has been used and destroyed (no stale error leaks into it)."""
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    wl = scenes.make_workload(1)
    say("[case] C1 profiled graph vs one-graph form, stage times")
    snaps = []
    for prof in (0, 1):
        run = GraphRun(ctx, wl, P.Settings(tile=16, profile=prof))
        assert run.rc == 0, P.lib().lgs_last_error(ctx._h).decode()
        for _ in range(2):
            run.launch()
        assert run.status() == 0
        snaps.append(run.snapshot())
        if prof:
            ms = (C.c_float * 5)()
            assert B.lib().lgs_graph_stage_ms(run.h, ms) == 0
            say("  graph stage ms", list(ms))
            assert all(x > 0 for x in ms)
        run.destroy()
    for a, b in zip(snaps[0][0], snaps[1][0]):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    for k in snaps[0][1]:
        assert np.array_equal(snaps[0][1][k], snaps[1][1][k]), k
    prm = gpu_params(wl.scene)
    outs, state = ctx.forward(prm, wl.cams, P.Settings(tile=16, profile=1))
    ctx.backward(state, prm, upstream_tensors(scenes.random_upstream(1, wl.cams)))
    ms = state.stage_ms()
    state.release()
    say("  eager stage ms", ms)
    assert all(x > 0 for x in ms)
