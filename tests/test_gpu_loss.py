"""GPU parity of the mapping loss with its D-SSIM term (lgs_loss, through the
C ABI) against the FP64 loss oracle, and of the whole step with that loss
(captured graph and eager form) against the oracle's render, loss and
vector-Jacobian product.

Loss-only cases take seeded image pairs (``scenes.loss_images``): tiny and
ragged sizes (1x1, 3x2, images smaller than the 11 x 11 window, sides that
are not multiples of the 32-pixel tile), several views of different sizes
in one call, lam = 0 (L1 only), lam = 1, and the full sizes of the batched
and the differentiation workloads; every element of the gradient is
compared.  Tolerance: 1e-4 relative per channel group (rel_L2 and rel_max),
as for the rasterizer; the loss terms to 1e-5.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import scenes
from oracle import loss_fp64 as LF
from oracle import raster_fp64 as R
from parity import (TOL_F32, ambiguous, dilate, fmt, gaussian_ambiguity, gpu_params, grad_errors, grads_np,
                    rel_err, separate_targets, to_np)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_16144_amd as P
    c = P.Context(0)
    yield c
    c.close()


class _Cam:
    def __init__(self, W, H):
        self.width, self.height = W, H
        self.fx = self.fy = 1.0
        self.cx = self.cy = 0.0
        self.R_cw = np.eye(3)
        self.t_cw = np.zeros(3)


def _dev(ims):
    return [{k: torch.as_tensor(np.ascontiguousarray(v)).cuda() for k, v in d.items()} for d in ims]


def _tgt_dicts(tgts):
    return [{"rgb": t.rgb, "depth": t.depth, "feat": t.feat} for t in tgts]


def gpu_loss(ctx, sizes, outs, tgts, loss_w, lam):
    cams = [_Cam(W, H) for (W, H) in sizes]
    grad, terms = ctx.loss(cams, _dev(outs), _dev(_tgt_dicts(tgts)), loss_w, lam)
    torch.cuda.synchronize()
    g = [np.concatenate([d["rgb"].cpu().numpy(), d["depth"].cpu().numpy()[None], d["feat"].cpu().numpy()], 0)
         for d in grad]
    return g, terms.cpu().numpy()


def check_loss(g, terms, ref_terms, ref_ups, label, tol=TOL_F32):
    for v, (a, b) in enumerate(zip(g, ref_ups)):
        res = {"rgb": rel_err(a[:3], b[:3]), "depth": rel_err(a[3], b[3]), "feat": rel_err(a[4:], b[4:])}
        say(f"  {label} view {v} dL/dY:", fmt(res))
        for k, (l2, mx) in res.items():
            assert l2 <= tol and mx <= tol, (label, v, k, l2, mx)
        for i, name in enumerate(("l1_rgb", "dssim", "l1_depth", "l1_feat")):
            assert abs(terms[v, i] - ref_terms[v][i]) <= 1e-5 * max(1.0, abs(ref_terms[v][i])), \
                (label, v, name, terms[v, i], ref_terms[v][i])


CASES = [
    ("1x1", [(1, 1)], 0.2, (1.0, 1.0, 1.0), False),
    ("3x2", [(3, 2)], 0.2, (1.0, 1.0, 1.0), False),
    ("11x7 lam=1", [(11, 7)], 1.0, (1.0, 0.1, 1.0), False),
    ("33x31 ragged", [(33, 31)], 0.2, (1.0, 1.0, 1.0), False),
    ("3 views", [(70, 45), (32, 32), (5, 90)], 0.2, (0.5, 1.0, 2.0), False),
    ("128x96 lam=0", [(128, 96)], 0.0, (1.0, 1.0, 1.0), False),
    ("97x64 independent", [(97, 64)], 0.2, (1.0, 1.0, 1.0), True),
]


@pytest.mark.parametrize("label,sizes,lam,w,indep", CASES, ids=[c[0] for c in CASES])
def test_loss_vs_oracle(ctx, label, sizes, lam, w, indep):
    say(f"[case] loss {label}: sizes {sizes} lam {lam} w {w}")
    outs, tgts = scenes.loss_images(len(label), sizes, independent=indep)
    g, terms = gpu_loss(ctx, sizes, outs, tgts, w, lam)
    _, ref_terms, ref_ups = LF.loss_and_upstream(outs, tgts, w, lam)
    check_loss(g, terms, ref_terms, ref_ups, label)
    if lam == 0.0:
        assert np.all(terms[:, 1] == 0.0)


@pytest.mark.parametrize("cfg", [4, 5])
def test_loss_full_size_vs_oracle(ctx, cfg):
    """Every view of the batched workload (4 x 640x480 + 4 x 320x240) and the
    1296x968 view of the differentiation workload, all elements."""
    sizes = {4: [(640, 480), (320, 240)] * 4, 5: [(1296, 968)]}[cfg]
    w = {4: (1.0, 1.0, 1.0), 5: (1.0, 0.1, 1.0)}[cfg]
    say(f"[case] loss full size C{cfg}: {sizes}")
    outs, tgts = scenes.loss_images(100 + cfg, sizes)
    g, terms = gpu_loss(ctx, sizes, outs, tgts, w, 0.2)
    _, ref_terms, ref_ups = LF.loss_and_upstream(outs, tgts, w, 0.2)
    check_loss(g, terms, ref_terms, ref_ups, f"C{cfg}")


def test_loss_deterministic_and_rejects_bad_arguments(ctx):
    from paper_2511_16144_amd import binding as B
    sizes = [(50, 40), (20, 70)]
    outs, tgts = scenes.loss_images(3, sizes)
    g1, t1 = gpu_loss(ctx, sizes, outs, tgts, (1.0, 1.0, 1.0), 0.2)
    g2, t2 = gpu_loss(ctx, sizes, outs, tgts, (1.0, 1.0, 1.0), 0.2)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)
    assert np.array_equal(t1, t2)
    cams = [_Cam(W, H) for (W, H) in sizes]
    for lam in (-0.1, 1.5, float("nan")):
        with pytest.raises(B.LgsError) as e:
            ctx.loss(cams, _dev(outs), _dev(_tgt_dicts(tgts)), (1.0, 1.0, 1.0), lam)
        assert e.value.status == B.LGS_ERR_INVALID_ARG
    with pytest.raises(B.LgsError) as e:
        ctx.loss(cams, _dev(outs), _dev(_tgt_dicts(tgts)), (1.0, float("inf"), 1.0), 0.2)
    assert e.value.status == B.LGS_ERR_INVALID_ARG
    V = len(sizes)
    cc = (B.lgs_camera * V)(*[B.camera_c(c) for c in cams])
    im = B._images_c(_dev(outs), [(H, W) for (W, H) in sizes], False)
    lw = (C.c_float * 3)(1.0, 1.0, 1.0)
    assert B.lib().lgs_loss(ctx._h, V, cc, 16, im, im, lw, C.c_float(0.2), None, None, None) == B.LGS_ERR_INVALID_ARG
    assert B.lib().lgs_loss(ctx._h, V, cc, 16, im, im, None, C.c_float(0.2), im, None, None) == B.LGS_ERR_INVALID_ARG
    assert B.lib().lgs_loss(ctx._h, V, cc, 24, im, im, lw, C.c_float(0.2), im, None, None) == B.LGS_ERR_INVALID_ARG


def test_step_with_dssim_graph_eager_and_oracle(ctx):
    """Whole step with the D-SSIM loss (lam = 0.2) on the 2000-Gaussian
    128x96 workload: the captured graph replays bitwise; it equals the eager
    forward + lgs_loss + lgs_backward to rounding (1e-5: the graph's backward
    forms the depth and feature L1 gradients itself, as the sign times the
    scale after the matrix-core product, where the eager backward splits the
    given FP32 values into two BF16 terms); and it equals the oracle's render
    + loss + vector-Jacobian product within 1e-4 (Gaussians within the
    two-window reach, 10 px, of an ambiguous pixel are left out of
    rel_max)."""
    import paper_2511_16144_amd as P
    from test_gpu_graph import GraphRun
    wl = scenes.make_workload(1)
    say("[case] C1 step with D-SSIM: graph, eager, oracle")
    ref = R.render(wl.scene, wl.cams, R.Settings())
    wl.targets = separate_targets(ref, wl.targets)
    st = P.Settings(tile=16)
    run = GraphRun(ctx, wl, st, ssim_lambda=0.2)
    assert run.rc == 0, P.lib().lgs_last_error(ctx._h).decode()
    run.launch()
    assert run.status() == 0
    outs_g, grads_g = run.snapshot()
    run.launch()
    outs_g2, grads_g2 = run.snapshot()
    for k in grads_g:
        assert np.array_equal(grads_g[k], grads_g2[k]), k
    run.destroy()
    # eager: forward, lgs_loss, lgs_backward
    prm = gpu_params(wl.scene)
    outs, state = ctx.forward(prm, wl.cams, st)
    ups, terms = ctx.loss(wl.cams, [{k: o[k] for k in ("rgb", "depth", "feat")} for o in outs],
                          _dev(_tgt_dicts(wl.targets)), wl.loss_w, 0.2)
    ge = grads_np(ctx.backward(state, prm, ups))
    torch.cuda.synchronize()
    state.release()
    for k in ge:
        l2, mx = rel_err(ge[k], grads_g[k])
        assert l2 <= 1e-5 and mx <= 1e-5, (k, l2, mx)
    # oracle
    L, ref_terms, ref_ups = LF.loss_and_upstream(ref, wl.targets, wl.loss_w, 0.2)
    say("  loss terms gpu", terms.cpu().numpy()[0], "oracle", np.round(ref_terms[0], 7))
    gr = R.vjp(wl.scene, wl.cams, ref_ups, R.Settings())
    amb = ambiguous(ref[0]["margin"])
    reach = dilate(amb, 2 * LF.SSIM_RADIUS)
    err = grad_errors(grads_g, gr, gaussian_ambiguity(ref[0], reach, wl.scene.n))
    say(f"  step grads vs oracle ({int(amb.sum())} ambiguous px, {int(reach.sum())} within reach):", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)
