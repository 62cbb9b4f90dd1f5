"""GPU parity of the configuration the throughput benchmark measures: the
batched workload at full size (500k Gaussians, 8 keyframes: 4 x 640x480 +
4 x 320x240, colours and features stored in BF16), binning tile 32, four
8x8 blocks per work-group, work queue ordered by list length, and whatever
setting the autotuner returns; plus tunable invariance of the BF16 path.

* eager forward + explicit-upstream backward at those settings against the
  FP64 oracle on four seeded 64x64 windows per view (the upstream vanishes
  outside them and at the oracle's ambiguous pixels): window pixels and
  every Gaussian's gradient, 1e-4;
* the captured whole-step graph (forward + fused L1 gradient + backward) at
  those settings: images and gradients bitwise equal to the eager forward +
  lgs_backward_l1, and its gradient against the oracle's gradient of the L1
  loss on the windows.  For that comparison the targets handed to the GPU
  equal the GPU's own eager render outside the windows and at ambiguous
  pixels (so sign(0) = 0 makes the loss gradient vanish there); inside the
  windows they are the workload's targets moved at least 1e-4 away from the
  oracle's rendered values.  The oracle only evaluates the windows, with the
  workload's targets: none of its inputs comes from the GPU;
* reduced batched BF16 scene: forward bitwise identical and gradients within
  1e-5 across tile {8, 16, 32} x chunk {1, 2, 4} x order {0, 1, 2}.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import scenes
from gpu_helpers import GraphRun
from oracle import raster_fp64 as R
from parity import (TOL_F32, ambiguous, fmt, gpu_params, grad_errors, grads_np, mask_upstream, rel_err,
                    separate_targets, to_np, upstream_tensors)

pytestmark = pytest.mark.gpu

BENCH = dict(tile=32, chunk=4, order=1)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_16144_amd as P
    c = P.Context(0)
    yield c
    c.close()


def crop_subscene(wl, wins):
    """Gaussians that can touch any window of any view (a superset, judged
    from the oracle's own projection), in their original order."""
    keep = np.zeros(wl.scene.n, bool)
    for v, cam in enumerate(wl.cams):
        o = R.render(wl.scene, [cam], R.Settings(), rects=[[]], want_margin=False)[0]
        mu, cov, vis = o["mu"], o["cov2d"], o["vis"]
        rx = 3.0 * np.sqrt(np.maximum(cov[:, 0], 0)) + 2.0
        ry = 3.0 * np.sqrt(np.maximum(cov[:, 2], 0)) + 2.0
        for (x0, y0, w, h) in wins[v]:
            keep |= vis & (mu[:, 0] + rx >= x0) & (mu[:, 0] - rx <= x0 + w - 1) & \
                (mu[:, 1] + ry >= y0) & (mu[:, 1] - ry <= y0 + h - 1)
    return np.nonzero(keep)[0]


def window_masks(wl, wins):
    ms = []
    for v, cam in enumerate(wl.cams):
        m = np.zeros((cam.height, cam.width), bool)
        for (x0, y0, w, h) in wins[v]:
            m[y0:y0 + h, x0:x0 + w] = True
        ms.append(m)
    return ms


def full_grads(sub_g, idx, n):
    g = {k: np.zeros((n,) + np.shape(v)[1:]) for k, v in sub_g.items() if k != "twist"}
    for k in g:
        g[k][idx] = sub_g[k]
    g["twist"] = sub_g["twist"]
    return g


@pytest.fixture(scope="module")
def c4():
    """The full-size batched workload, its windows and the oracle's render
    of the windows (on the Gaussians that can reach them)."""
    wl = scenes.make_workload(4)
    wins = [scenes.crop_windows(40 + v, c, k=4, size=64) for v, c in enumerate(wl.cams)]
    idx = crop_subscene(wl, wins)
    sub = wl.scene.subset(idx)
    say(f"[fixture] C4 full size: {wl.scene.n} Gaussians, 8 views, oracle sub-scene {len(idx)} Gaussians")
    ref = R.render(sub, wl.cams, R.Settings(), rects=wins)
    ambs = [ambiguous(r["margin"]) for r in ref]
    return {"wl": wl, "wins": wins, "idx": idx, "sub": sub, "ref": ref, "ambs": ambs,
            "masks": window_masks(wl, wins)}


def autotuned(ctx, wl):
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    run = GraphRun(ctx, wl, P.Settings(**BENCH))
    assert run.rc == 0, P.lib().lgs_last_error(ctx._h).decode()
    best = B.lgs_settings()
    rc = B.lib().lgs_autotune(ctx._h, C.byref(run.st), C.byref(run.g), len(wl.cams), run.cams, run.tgts, run.lw,
                              run.imgs, C.byref(run.gr), 0, run.stream(), None, C.byref(best))
    assert rc == 0, B.lib().lgs_last_error(ctx._h).decode()
    run.destroy()
    return dict(tile=best.tile, chunk=best.chunk, order=best.order)


@pytest.mark.parametrize("which", ["bench", "autotuned"])
def test_c4_full_size_at_bench_settings_vs_oracle(ctx, c4, which):
    import paper_2511_16144_amd as P
    wl, wins, idx, sub, ref, ambs = c4["wl"], c4["wins"], c4["idx"], c4["sub"], c4["ref"], c4["ambs"]
    st = BENCH if which == "bench" else autotuned(ctx, wl)
    say(f"[case] C4 full size BF16, explicit windowed upstream, settings {which}: {st}")
    ups = mask_upstream(scenes.random_upstream(44, wl.cams, windows=wins), ambs)
    prm = gpu_params(wl.scene)
    outs, state = ctx.forward(prm, wl.cams, P.Settings(**st), want_n=True)
    g = grads_np(ctx.backward(state, prm, upstream_tensors(ups)))
    torch.cuda.synchronize()
    counts = state.counts()
    state.release()
    say("  counts", counts)
    out = to_np(outs)
    worst = 0.0
    for v in range(len(wl.cams)):
        keep = c4["masks"][v] & ~ambs[v]
        res = {k: rel_err(out[v][k], ref[v][k], keep) for k in ("rgb", "depth", "feat", "T")}
        worst = max(worst, max(max(x) for x in res.values()))
        for k, (l2, mx) in res.items():
            assert l2 <= TOL_F32 and mx <= TOL_F32, (v, k, l2, mx)
        assert np.array_equal(out[v]["n"][keep], ref[v]["n"][keep]), v
    say(f"  forward, 8 views x 4 windows: worst rel error {worst:.2e}; ambiguous px "
        f"{sum(int((a & m).sum()) for a, m in zip(ambs, c4['masks']))}")
    gr = full_grads(R.vjp(sub, wl.cams, ups, R.Settings(), rects=wins), idx, wl.scene.n)
    outside = np.ones(wl.scene.n, bool)
    outside[idx] = False
    for k in ("means", "logits", "feat"):
        gk = g[k].T if g[k].ndim == 2 else g[k]
        assert np.all(gk[outside] == 0), k
    err = grad_errors(g, gr, np.zeros(wl.scene.n, bool))
    say("  backward, every Gaussian:", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)


def test_c4_graph_at_bench_settings(ctx, c4):
    import paper_2511_16144_amd as P
    wl, wins, idx, sub, ref, ambs = c4["wl"], c4["wins"], c4["idx"], c4["sub"], c4["ref"], c4["ambs"]
    say(f"[case] C4 full size BF16, captured graph (fused L1) at {BENCH}")
    prm = gpu_params(wl.scene)
    outs_e, state = ctx.forward(prm, wl.cams, P.Settings(**BENCH))
    oe = to_np(outs_e)
    # targets: the workload's (moved away from the oracle's values) inside
    # the windows, the GPU's own render elsewhere and at ambiguous pixels
    sep = separate_targets(ref, wl.targets)
    tg_np = []
    for v in range(len(wl.cams)):
        inside = c4["masks"][v] & ~ambs[v]
        t = {}
        for k in ("rgb", "depth", "feat"):
            a = np.array(oe[v][k], np.float32, copy=True)
            s = getattr(sep[v], k)
            a[..., inside] = s[..., inside]
            t[k] = a
        tg_np.append(scenes.Targets(t["rgb"], t["depth"], t["feat"]))
    wl_g = scenes.Workload(wl.name, wl.scene, wl.cams, tg_np, wl.loss_w)
    run = GraphRun(ctx, wl_g, P.Settings(**BENCH))
    assert run.rc == 0, P.lib().lgs_last_error(ctx._h).decode()
    for _ in range(2):
        run.launch()
    assert run.status() == 0
    outs_g, grads_g = run.snapshot()
    # forward in the graph: bitwise the eager forward
    for v in range(len(wl.cams)):
        for k in ("rgb", "depth", "feat", "T"):
            assert np.array_equal(outs_g[v][k], oe[v][k]), (v, k)
    # eager fused-L1 backward with the same targets: bitwise the graph's
    tg = [{k: torch.as_tensor(getattr(t, k)).cuda() for k in ("rgb", "depth", "feat")} for t in tg_np]
    gl = grads_np(ctx.backward_l1(state, prm, outs_e, tg, wl.loss_w))
    torch.cuda.synchronize()
    state.release()
    for k in gl:
        assert np.array_equal(gl[k], grads_g[k]), k
    run.destroy()
    # the oracle's gradient of the L1 loss over the windows (its own render,
    # the workload's targets moved away from it), zero at ambiguous pixels
    ups = R.l1_upstream(ref, sep, wl.loss_w)
    ups = mask_upstream([np.nan_to_num(u, nan=0.0) for u in ups], ambs)
    for u, m in zip(ups, c4["masks"]):
        u[:, ~m] = 0.0
    gr = full_grads(R.vjp(sub, wl.cams, ups, R.Settings(), rects=wins), idx, wl.scene.n)
    outside = np.ones(wl.scene.n, bool)
    outside[idx] = False
    for k in ("means", "logits", "feat"):
        gk = grads_g[k].T if grads_g[k].ndim == 2 else grads_g[k]
        assert np.all(gk[outside] == 0), k
    err = grad_errors(grads_g, gr, np.zeros(wl.scene.n, bool))
    say("  graph gradient vs oracle (every Gaussian):", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)


def test_bf16_tunable_invariance(ctx):
    """Reduced batched BF16 scene: every (tile, chunk, order) gives the same
    forward bit for bit (contributor lists, order and per-pixel arithmetic do
    not depend on the tunables) and the same gradients to rounding (the
    per-Gaussian sums are taken over 8x8-block slots in a fixed order, but
    the work-group that fills a slot depends on the tile size only through
    the list it walks)."""
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(4, n=100000, res_scale=0.3)
    say(f"[case] BF16 tunable invariance, 8 views, n={wl.scene.n}")
    prm = gpu_params(wl.scene)
    ups = upstream_tensors(scenes.random_upstream(45, wl.cams))
    tg = [{k: torch.as_tensor(getattr(t, k)).cuda() for k in ("rgb", "depth", "feat")} for t in wl.targets]
    base = None
    n_cases = 0
    worst = 0.0
    for tile in (8, 16, 32):
        for chunk in (1, 2, 4):
            for order in (0, 1, 2):
                st = P.Settings(tile=tile, chunk=chunk, order=order)
                outs, state = ctx.forward(prm, wl.cams, st, want_n=True)
                g = grads_np(ctx.backward(state, prm, ups))
                gl = grads_np(ctx.backward_l1(state, prm, outs, tg, wl.loss_w))
                torch.cuda.synchronize()
                state.release()
                o = to_np(outs)
                if base is None:
                    base = (o, g, gl)
                    continue
                for v in range(len(wl.cams)):
                    for k in ("rgb", "depth", "feat", "T", "n"):
                        assert np.array_equal(o[v][k], base[0][v][k]), (tile, chunk, order, v, k)
                for a, b in ((g, base[1]), (gl, base[2])):
                    for k in a:
                        l2, mx = rel_err(a[k], b[k])
                        worst = max(worst, mx)
                        assert l2 <= 1e-5 and mx <= 1e-5, (tile, chunk, order, k, l2, mx)
                n_cases += 1
    say(f"  {n_cases + 1} settings: forward bitwise equal, gradients within {worst:.1e}")
