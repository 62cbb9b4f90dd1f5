"""GPU parity for language-feature dimensions other than 16 (the
feature-dimension variants of the paper's ablation), through the C ABI.

The library renders the D feature channels in groups of 16 (8 for D = 8),
re-running the compositing kernels per group.  Checked here:

* the 2000-Gaussian 128x96 workload with D = 8, 32, 64 and 128: forward
  (every channel) and the backward of a seeded upstream (zeroed at
  ambiguous pixels) against the FP64 oracle, every Gaussian, 1e-4;
* the group mechanism bitwise: at D = 32 the RGB, depth, T and contributor
  counts equal the D = 16 render of the first 16 features, and feature
  channels 16..31 equal the D = 16 render of the last 16;
* the fused L1 step (lgs_backward_l1) equals the backward of the same L1
  upstream given explicitly, to rounding (1e-5), and the captured graph
  equals the eager fused step bitwise;
* BF16 storage at D = 32 on a reduced batched scene (8 views) against the
  oracle on the rounded inputs.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import scenes
from oracle import raster_fp64 as R
from parity import (TOL_F32, ambiguous, fmt, gpu_params, grad_errors, grads_np, mask_upstream, rel_err,
                    separate_targets, to_np, upstream_tensors)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_16144_amd as P
    c = P.Context(0)
    yield c
    c.close()


def check_forward(out, ref, label):
    amb = ambiguous(ref["margin"])
    keep = ~amb
    res = {k: rel_err(out[k], ref[k], keep) for k in ("rgb", "depth", "feat", "T")}
    say(f"  {label} forward ({int(amb.sum())} ambiguous px): {fmt(res)}")
    for k, (l2, mx) in res.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (label, k, l2, mx)
    assert np.array_equal(out["n"][keep], ref["n"][keep])
    return amb


@pytest.mark.parametrize("D", [8, 32, 64, 128])
def test_feature_dimension_vs_oracle(ctx, D):
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(1, feat_dim=D)
    say(f"[case] C1 with D = {D}")
    ref = R.render(wl.scene, wl.cams, R.Settings())
    prm = gpu_params(wl.scene)
    outs, st = ctx.forward(prm, wl.cams, P.Settings(tile=16), want_n=True)
    out = to_np(outs)[0]
    assert out["feat"].shape == (D, 96, 128)
    amb = check_forward(out, ref[0], f"D={D}")
    ups = mask_upstream(scenes.random_upstream(D, wl.cams, feat_dim=D), [amb])
    g = grads_np(ctx.backward(st, prm, upstream_tensors(ups)))
    torch.cuda.synchronize()
    st.release()
    assert g["feat"].shape == (D, wl.scene.n)
    gr = R.vjp(wl.scene, wl.cams, ups, R.Settings())
    err = grad_errors(g, gr, np.zeros(wl.scene.n, bool))
    say(f"  D={D} backward: {fmt(err)}")
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (D, k, l2, mx)


def test_groups_equal_separate_16d_renders_bitwise(ctx):
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(1, feat_dim=32)
    sc = wl.scene
    say("[case] D = 32 vs the two 16-d halves, bitwise")

    def render(feat):
        s = scenes.Scene(sc.means, sc.log_scales, sc.quats, sc.logits, sc.rgb, np.ascontiguousarray(feat), "f32")
        outs, st = ctx.forward(gpu_params(s), wl.cams, P.Settings(tile=16), want_n=True)
        torch.cuda.synchronize()
        st.release()
        return to_np(outs)[0]
    full, a, b = render(sc.feat), render(sc.feat[:, :16]), render(sc.feat[:, 16:])
    for k in ("rgb", "depth", "T", "n"):
        assert np.array_equal(full[k], a[k]), k
    assert np.array_equal(full["feat"][:16], a["feat"]) and np.array_equal(full["feat"][16:], b["feat"])


def test_fused_l1_step_and_graph_at_32(ctx):
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    from test_gpu_graph import GraphRun, assert_close_groups
    D = 32
    wl = scenes.make_workload(1, feat_dim=D)
    ref = R.render(wl.scene, wl.cams, R.Settings())
    wl.targets = separate_targets(ref, wl.targets)
    say("[case] D = 32: fused L1 (eager), explicit upstream, graph, oracle")
    prm = gpu_params(wl.scene)
    tg = [{"rgb": torch.as_tensor(t.rgb).cuda(), "depth": torch.as_tensor(t.depth).cuda(),
           "feat": torch.as_tensor(t.feat).cuda()} for t in wl.targets]
    st_ = P.Settings(tile=16)
    outs, st = ctx.forward(prm, wl.cams, st_)
    gf = grads_np(ctx.backward_l1(st, prm, outs, tg, wl.loss_w))
    torch.cuda.synchronize()
    o = to_np(outs)[0]
    H, W = 96, 128
    up = np.empty((4 + D, H, W), np.float32)
    t = wl.targets[0]
    up[:3] = np.sign(o["rgb"] - t.rgb) * np.float32(wl.loss_w[0] / (3 * H * W))
    up[3] = np.sign(o["depth"] - t.depth) * np.float32(wl.loss_w[1] / (H * W))
    up[4:] = np.sign(o["feat"] - t.feat) * np.float32(wl.loss_w[2] / (D * H * W))
    ge = grads_np(ctx.backward(st, prm, upstream_tensors([up])))
    torch.cuda.synchronize()
    st.release()
    assert_close_groups(ge, gf)
    gr = R.vjp(wl.scene, wl.cams, R.l1_upstream(ref, wl.targets, wl.loss_w), R.Settings())
    from parity import gaussian_ambiguity
    err = grad_errors(gf, gr, gaussian_ambiguity(ref[0], ambiguous(ref[0]["margin"]), wl.scene.n))
    say("  fused L1 vs oracle:", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)
    run = GraphRun(ctx, wl, st_)
    assert run.rc == 0, B.lib().lgs_last_error(ctx._h).decode()
    run.launch()
    assert run.status() == 0
    _, gg = run.snapshot()
    run.destroy()
    for k in gf:
        assert np.array_equal(gg[k], gf[k]), k


def test_bf16_batched_reduced_at_32(ctx):
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(4, n=60000, res_scale=0.25, feat_dim=32)
    say(f"[case] batched reduced, BF16, D = 32: {len(wl.cams)} views, n={wl.scene.n}")
    ref = R.render(wl.scene, wl.cams, R.Settings())
    prm = gpu_params(wl.scene)
    outs, st = ctx.forward(prm, wl.cams, P.Settings(tile=16, order=1), want_n=True)
    out = to_np(outs)
    ambs = [check_forward(out[v], ref[v], f"view {v}") for v in range(len(wl.cams))]
    ups = mask_upstream(scenes.random_upstream(32, wl.cams, feat_dim=32), ambs)
    g = grads_np(ctx.backward(st, prm, upstream_tensors(ups)))
    torch.cuda.synchronize()
    st.release()
    gr = R.vjp(wl.scene, wl.cams, ups, R.Settings())
    err = grad_errors(g, gr, np.zeros(wl.scene.n, bool))
    say("  backward:", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)


def test_dssim_step_at_32(ctx):
    """The captured step with the D-SSIM loss at D = 32 (colour gradient from
    the loss kernel, depth and the two feature groups' L1 gradients formed in
    the backward) equals the eager forward + lgs_loss + lgs_backward to
    rounding, and lgs_loss's feature term is a mean over the 32 planes."""
    import paper_2511_16144_amd as P
    from oracle import loss_fp64 as LF
    from test_gpu_graph import GraphRun
    D = 32
    wl = scenes.make_workload(1, feat_dim=D)
    ref = R.render(wl.scene, wl.cams, R.Settings())
    wl.targets = separate_targets(ref, wl.targets)
    say("[case] D = 32 with D-SSIM: graph vs eager, loss terms vs oracle")
    st_ = P.Settings(tile=16)
    run = GraphRun(ctx, wl, st_, ssim_lambda=0.2)
    assert run.rc == 0
    run.launch()
    assert run.status() == 0
    outs_g, gg = run.snapshot()
    run.destroy()
    prm = gpu_params(wl.scene)
    outs, st = ctx.forward(prm, wl.cams, st_)
    tg = [{"rgb": torch.as_tensor(t.rgb).cuda(), "depth": torch.as_tensor(t.depth).cuda(),
           "feat": torch.as_tensor(t.feat).cuda()} for t in wl.targets]
    ups, terms = ctx.loss(wl.cams, [{k: o[k] for k in ("rgb", "depth", "feat")} for o in outs], tg, wl.loss_w, 0.2)
    ge = grads_np(ctx.backward(st, prm, ups))
    torch.cuda.synchronize()
    st.release()
    for k in ge:
        l2, mx = rel_err(ge[k], gg[k])
        assert l2 <= 1e-5 and mx <= 1e-5, (k, l2, mx)
    o = to_np(outs)
    _, ref_terms, _ = LF.loss_and_upstream([{k: o[0][k] for k in ("rgb", "depth", "feat")}], wl.targets,
                                           wl.loss_w, 0.2)
    t = terms.cpu().numpy()[0]
    say("  terms gpu", t, "oracle (on the GPU's images)", np.round(ref_terms[0], 7))
    for i in range(4):
        assert abs(t[i] - ref_terms[0][i]) <= 1e-5 * max(1.0, abs(ref_terms[0][i]))
