"""The torch.autograd path (RasterFn / render) on the GPU: render every view,
take the L1 mapping loss of Eq. (1) in torch, call .backward(), and compare
the .grad of every parameter leaf and of the pose-twist leaf with the FP64
oracle's gradient of the same loss (Sec. III-B.3 map optimisation, Sec.
III-B.2 pose refinement through the renderer).

Colours and features are stored in FP32, or in BF16 from FP32 master leaves
(the gradient is the library's FP32 gradient with respect to the stored
values; the oracle runs on the rounded values).  The targets are moved at
least 1e-4 away from the oracle's rendered values so that no L1 residual
changes sign between FP32 and FP64; Gaussians whose box covers an ambiguous
pixel are left out of the per-element comparison."""
import numpy as np
import pytest
import torch

import scenes
from oracle import raster_fp64 as R
from parity import TOL_F32, ambiguous, fmt, gaussian_ambiguity, grad_errors, separate_targets

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def bf16_scene(sc):
    return scenes.Scene(sc.means, sc.log_scales, sc.quats, sc.logits, scenes.round_bf16(sc.rgb),
                        scenes.round_bf16(sc.feat), "bf16", sc.rgb, sc.feat)


def leaves(sc, master_rgb, master_feat, dev="cuda"):
    def soa(a):
        return torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float32).T)).to(dev).requires_grad_(True)
    return {"means": soa(sc.means), "log_scales": soa(sc.log_scales), "quats": soa(sc.quats),
            "logits": torch.as_tensor(np.asarray(sc.logits, np.float32)).to(dev).requires_grad_(True),
            "rgb": soa(master_rgb), "feat": soa(master_feat)}


def torch_l1(outs, targets, loss_w):
    L = 0.0
    for o, t in zip(outs, targets):
        L = L + loss_w[0] * (o["rgb"] - t["rgb"]).abs().mean() + loss_w[1] * (o["depth"] - t["depth"]).abs().mean() \
            + loss_w[2] * (o["feat"] - t["feat"]).abs().mean()
    return L


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_rasterfn_l1_step_vs_oracle(storage):
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(1)
    sc = wl.scene if storage == "f32" else bf16_scene(wl.scene)
    say(f"[case] RasterFn on C1 ({sc.n} Gaussians, 128x96), {storage} appearance storage")
    ref = R.render(sc, wl.cams, R.Settings())
    targets = separate_targets(ref, wl.targets)
    ctx = P.Context(0)
    # FP32 masters: the unrounded values; BF16 storage rounds them (nearest even)
    lv = leaves(sc, sc.rgb_unrounded if storage == "bf16" else sc.rgb,
                sc.feat_unrounded if storage == "bf16" else sc.feat)
    twist = torch.zeros((1, 6), device="cuda", requires_grad=True)
    st = P.Settings(tile=16)
    outs = P.render(ctx, lv, wl.cams, st, twist=twist,
                    storage=torch.bfloat16 if storage == "bf16" else torch.float32)
    tg = [{k: torch.as_tensor(getattr(t, k)).cuda() for k in ("rgb", "depth", "feat")} for t in targets]
    seen = [{} for _ in outs]       # the upstream autograd hands to RasterFn, as it arrives
    for o, d in zip(outs, seen):
        for k in ("rgb", "depth", "feat"):
            o[k].register_hook(lambda gr, d=d, k=k: d.__setitem__(k, gr.detach().clone()))
    L = torch_l1(outs, tg, wl.loss_w)
    L.backward()
    torch.cuda.synchronize()
    for k, t in list(lv.items()) + [("twist", twist)]:
        assert t.grad is not None and t.grad.dtype == torch.float32, k
    g = {k: t.grad.detach().cpu().numpy() for k, t in lv.items()}
    g["twist"] = twist.grad.detach().cpu().numpy()
    # the same upstream through Context.backward: bitwise the autograd result
    prm = {k: t.detach() for k, t in lv.items()}
    if storage == "bf16":
        prm["rgb"] = prm["rgb"].to(torch.bfloat16).contiguous()
        prm["feat"] = prm["feat"].to(torch.bfloat16).contiguous()
    o2, state = ctx.forward(prm, wl.cams, st)
    for a, b in zip(o2, outs):
        for k in ("rgb", "depth", "feat", "T"):
            assert torch.equal(a[k], b[k].detach()), k
    gb = ctx.backward(state, prm, seen)
    torch.cuda.synchronize()
    state.release()
    for k in g:
        assert np.array_equal(gb[k].cpu().numpy(), g[k]), k
    # the oracle's gradient of the same loss on its own render
    gr = R.vjp(sc, wl.cams, R.l1_upstream(ref, targets, wl.loss_w), R.Settings())
    amb = ambiguous(ref[0]["margin"])
    bad = gaussian_ambiguity(ref[0], amb, sc.n)
    err = grad_errors(g, gr, bad)
    say(f"  .grad vs oracle ({int((~bad).sum())} Gaussians, {int(amb.sum())} ambiguous px):", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)
    # the loss value itself against the oracle's
    L_ref = R.l1_loss(ref, targets, wl.loss_w)
    say(f"  loss {float(L):.9f} vs oracle {L_ref:.9f}")
    assert abs(float(L) - L_ref) <= 1e-5 * abs(L_ref)
    ctx.close()


def test_rasterfn_two_views_and_unused_outputs():
    """Two views in one call, a loss that reads only some outputs (the
    others get zero upstream), the transmittance output in the loss (its
    upstream goes through the final_T plane), and a second backward through
    a fresh render: .grad accumulates across the two backward calls."""
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(4, n=3000, res_scale=0.2)
    cams = wl.cams[:2]
    say(f"[case] RasterFn, 2 views {[(c.width, c.height) for c in cams]}, n={wl.scene.n}")
    ref = R.render(wl.scene, cams, R.Settings())
    ctx = P.Context(0)
    lv = leaves(wl.scene, wl.scene.rgb, wl.scene.feat)
    st = P.Settings(tile=8)
    ambs = [ambiguous(r["margin"]) for r in ref]
    rng = np.random.Generator(np.random.PCG64(71))
    wT_np = [rng.normal(size=(c.height, c.width)).astype(np.float32) for c in cams]
    wF_np = [rng.normal(size=(16, c.height, c.width)).astype(np.float32) for c in cams]
    for a, t, f in zip(ambs, wT_np, wF_np):     # no upstream where FP32 cannot resolve a decision
        t[a] = 0.0
        f[:, a] = 0.0
    wT = [torch.as_tensor(t).cuda() for t in wT_np]
    wF = [torch.as_tensor(f).cuda() for f in wF_np]
    grads = []
    for rep in range(2):
        twist = torch.zeros((2, 6), device="cuda", requires_grad=True)
        outs = P.render(ctx, lv, cams, st, twist=twist)
        L = (outs[0]["T"] * wT[0]).sum() + (outs[1]["feat"] * wF[1]).sum()
        L.backward()
        torch.cuda.synchronize()
        grads.append({k: t.grad.detach().cpu().numpy().copy() for k, t in lv.items()})
        grads[-1]["twist"] = twist.grad.detach().cpu().numpy()
    for k in ("means", "log_scales", "quats", "logits", "rgb", "feat"):
        assert np.array_equal(grads[1][k], 2 * grads[0][k]), k       # accumulated, run-to-run identical
    assert np.array_equal(grads[1]["twist"], grads[0]["twist"])
    g = grads[0]
    ups = [np.zeros((20, c.height, c.width)) for c in cams]
    ups[1][4:] = wF_np[1]
    upT = [wT_np[0], np.zeros((cams[1].height, cams[1].width))]
    gr = R.vjp(wl.scene, cams, ups, R.Settings(), upstream_T=upT)
    err = grad_errors(g, gr, np.zeros(wl.scene.n, bool))
    say("  .grad vs oracle:", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)
    ctx.close()
