"""Central finite differences of the FP64 oracle's L1 loss at full image sizes
(test infrastructure).

A parameter of Gaussian i only changes the pixels of its own footprint, so
each evaluation renders only that footprint; the pose twist re-renders the
union of all footprints.  Each evaluation returns, per pixel, the loss
contribution and a digest of the renderer's decisions there (contributors,
their order, alpha-clamp sides).  At full resolution a perturbation of h
moves cut boundaries across a few pixels, where the rendered value jumps; the
difference quotient is therefore taken over the pixels whose digest is the
same in the base, +h and -h evaluations, and compared with the autodiff
gradient minus the autodiff contribution of the remaining (unstable) pixels.
The signs of each pixel's L1 residuals are part of its digest too: the loss
has a kink where one changes, and because the L1 gradient is a sum of +-w/n
terms that largely cancel, a few such crossings would shift a difference
quotient measurably.  A parameter whose +-h evaluations change a per-Gaussian
decision (cull, Jacobian clamp side) is excluded and counted.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from oracle import raster_fp64 as R

F64 = torch.float64
SHAPES = {"means": 3, "log_scales": 3, "quats": 4, "logits": 1, "rgb": 3, "feat": 16}


def local_eval(scene, cam, target, loss_w, rects, xi=None, block=64):
    """Per-pixel L1 loss terms (normalised by whole-image element counts)
    over `rects`, per-pixel decision digests, pixel coordinates, and the
    per-Gaussian decision bytes."""
    P = R._params(scene)
    with torch.no_grad():
        xi = torch.zeros(6, dtype=F64) if xi is None else torch.as_tensor(np.asarray(xi, np.float64))
        proj = R.project_view(P, cam, xi, R.Settings())
        y = R._y_of(P, proj)
        H, W = cam.height, cam.width
        Ls, Ds, XY = [], [], []
        for blk in R._blocks(cam, rects, block):
            x0, y0, x1, y1 = blk
            yy, xx = torch.meshgrid(torch.arange(y0, y1, dtype=F64), torch.arange(x0, x1, dtype=F64), indexing="ij")
            cand = R._candidates(proj, blk, R.Settings())
            sg = []
            Yb, _, _, _ = R.composite(xx.flatten(), yy.flatten(), proj["mu"][cand], proj["conic"][cand],
                                      proj["opac"][cand], proj["z"][cand], y[cand], cand, R.Settings(), sig=sg)
            Yb = Yb.numpy()                                         # [P, 20]
            ys, xs = yy.flatten().numpy().astype(int), xx.flatten().numpy().astype(int)
            l = (loss_w[0] / (3 * H * W)) * np.abs(Yb[:, :3] - target.rgb[:, ys, xs].T).sum(1) \
                + (loss_w[1] / (H * W)) * np.abs(Yb[:, 3] - target.depth[ys, xs]) \
                + (loss_w[2] / (16 * H * W)) * np.abs(Yb[:, 4:] - target.feat[:, ys, xs].T).sum(1)
            Ls.append(l)
            # the digest also carries the signs of the pixel's 20 L1 residuals
            # (a sign change is a kink of the loss at that pixel)
            sgn = np.concatenate([Yb[:, :3] > target.rgb[:, ys, xs].T, (Yb[:, 3] > target.depth[ys, xs])[:, None],
                                  Yb[:, 4:] > target.feat[:, ys, xs].T], 1)
            bits = (sgn.astype(np.int64) << np.arange(20, dtype=np.int64)[None, :]).sum(1)
            Ds.append(sg[0].numpy() * 1048583 + bits)
            XY.append(np.stack([xs, ys], 1))
        glob = (proj["vis"].numpy().tobytes() + proj["clampx"].numpy().tobytes()
                + proj["clampy"].numpy().tobytes())
        if not Ls:
            return np.zeros(0), np.zeros(0, np.int64), np.zeros((0, 2), int), glob
        return np.concatenate(Ls), np.concatenate(Ds), np.concatenate(XY), glob


def footprint_rects(scene, cam, margin=3):
    o = R.render(scene, [cam], R.Settings(), rects=[[]], want_margin=False)[0]
    rects = []
    for g in range(scene.n):
        if not o["vis"][g]:
            rects.append([])
            continue
        a, _, c = o["cov2d"][g]
        rx, ry = 3.0 * np.sqrt(a) + margin, 3.0 * np.sqrt(c) + margin
        x0 = int(max(0, np.floor(o["mu"][g, 0] - rx)))
        x1 = int(min(cam.width, np.ceil(o["mu"][g, 0] + rx) + 1))
        y0 = int(max(0, np.floor(o["mu"][g, 1] - ry)))
        y1 = int(min(cam.height, np.ceil(o["mu"][g, 1] + ry) + 1))
        rects.append([(x0, y0, x1 - x0, y1 - y0)] if x1 > x0 and y1 > y0 else [])
    return rects


def _unstable_vjp(scene, cam, ups_full, pixels):
    """Autodiff gradient of the loss restricted to `pixels` ([k, 2] x, y):
    the upstream gradient is zeroed everywhere else (blocks without upstream
    are skipped by the oracle's VJP)."""
    if len(pixels) == 0:
        return None
    m = np.zeros(ups_full.shape[1:], bool)
    m[pixels[:, 1], pixels[:, 0]] = True
    return R.vjp(scene, [cam], [ups_full * m[None]], R.Settings())


def base_gradient(scene, cam, target, loss_w):
    """The oracle's L1 upstream and autodiff gradient of the whole image."""
    outs = R.render(scene, [cam], R.Settings(), want_margin=False)
    ups = R.l1_upstream(outs, [target], loss_w)[0]
    return ups, R.vjp(scene, [cam], [ups], R.Settings())


def fd_check(scene, cam, target, loss_w, params, twist=True, h=1e-4, max_unstable=200000,
             twist_components=range(6), base_grad=None, richardson=False):
    """For each (key, gaussian, component) in `params` (and the twist
    components): (fd, ad) over the decision-stable pixels.  Returns a list of
    (name, fd, ad, n_unstable), the number of excluded parameters and the
    autodiff gradient.  `base_grad`: (ups, AD) from base_gradient, if already
    computed."""
    ups, AD = base_grad if base_grad is not None else base_gradient(scene, cam, target, loss_w)
    rects = footprint_rects(scene, cam)
    res, excluded = [], 0
    base = {}

    def compare(name, rect, perturb, ad_full, pick):
        nonlocal excluded
        if rect not in base:
            base[rect] = local_eval(scene, cam, target, loss_w, list(rect))
        l0, d0, xy, g0 = base[rect]
        steps = (1, 2) if richardson else (1,)
        ev = {(m, s): perturb(s * m) for m in steps for s in (+1, -1)}
        if any(e[3] != g0 for e in ev.values()):
            excluded += 1
            return
        stable = np.ones(len(d0), bool)
        for e in ev.values():
            stable &= e[1] == d0
        bad = xy[~stable]
        if len(bad) > max_unstable:
            excluded += 1
            return
        D = {m: ((ev[(m, 1)][0] - ev[(m, -1)][0])[stable]).sum() / (2 * m * h) for m in steps}
        # central difference, O(h^2); with richardson the extrapolation of the
        # h and 2h quotients, (4 D(h) - D(2h)) / 3, O(h^4)
        fd = (4.0 * D[1] - D[2]) / 3.0 if richardson else D[1]
        ad = ad_full
        corr = _unstable_vjp(scene, cam, ups, bad)
        if corr is not None:
            ad = ad - pick(corr)
        res.append((name, fd, ad, int(len(bad))))

    for (k, g, c) in params:
        if not rects[g]:
            continue
        rect = tuple(rects[g])

        def perturb(s, k=k, g=g, c=c):      # s: signed multiple of h
            sc = copy.copy(scene)
            arr = np.array(getattr(scene, k), np.float64)
            if arr.ndim == 1:
                arr[g] += s * h
            else:
                arr[g, c] += s * h
            setattr(sc, k, arr)
            return local_eval(sc, cam, target, loss_w, list(rect))

        pick = (lambda G, k=k, g=g, c=c: G[k][g] if np.ndim(G[k]) == 1 else G[k][g, c])
        compare(f"{k}[{g},{c}]", rect, perturb, pick(AD), pick)
        if (len(res) + excluded) % 30 == 0:
            print(f"    fd: {len(res) + excluded} parameters done", flush=True)
    if twist:   # the pose moves every footprint: evaluate the whole image (no pixel twice)
        rect = ((0, 0, cam.width, cam.height),)
        for j in twist_components:
            def perturb(s, j=j):
                xi = np.zeros(6)
                xi[j] = s * h
                return local_eval(scene, cam, target, loss_w, list(rect), xi)
            pick = (lambda G, j=j: G["twist"][0][j])
            compare(f"twist[{j}]", rect, perturb, pick(AD), pick)
            print(f"    fd: twist component {j} done", flush=True)
    return res, excluded, AD


def subscene_64(wl, seed=5, k=64):
    """k Gaussians drawn with `seed` among those visible in the first view
    whose mean projects inside the image."""
    o = R.render(wl.scene, wl.cams[:1], R.Settings(), rects=[[]], want_margin=False)[0]
    vis = np.nonzero(o["vis"] & (o["mu"][:, 0] >= 0) & (o["mu"][:, 0] < wl.cams[0].width)
                     & (o["mu"][:, 1] >= 0) & (o["mu"][:, 1] < wl.cams[0].height))[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = np.sort(rng.choice(vis, size=k, replace=False))
    return wl.scene.subset(idx), idx


# -- parallel driver (spawned worker processes; each rebuilds the inputs) ----
_FD = {}


def fd_worker_init(seed=5):
    import scenes
    torch.set_num_threads(1)
    wl = scenes.make_workload(5)
    sub, _ = subscene_64(wl, seed)
    cam, target, loss_w = wl.cams[0], wl.targets[0], wl.loss_w
    del wl
    _FD.update(sub=sub, cam=cam, target=target, loss_w=loss_w,
               base=base_gradient(sub, cam, target, loss_w))


def fd_worker_task(task):
    """task: ("gaussians", [indices]) or ("twist", component)."""
    kind, arg = task
    W = _FD
    if kind == "gaussians":
        params = [(k, g, c) for g in arg for k, cc in SHAPES.items() for c in range(cc)]
        res, excl, _ = fd_check(W["sub"], W["cam"], W["target"], W["loss_w"], params, twist=False,
                                base_grad=W["base"], richardson=True)
    else:
        res, excl, _ = fd_check(W["sub"], W["cam"], W["target"], W["loss_w"], [], twist=True,
                                twist_components=[arg], base_grad=W["base"], richardson=True)
    return res, excl
