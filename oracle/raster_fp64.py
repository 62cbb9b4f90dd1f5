"""Plain FP64 definition of the rasterizer (torch CPU float64 + autograd).

TEST INFRASTRUCTURE ONLY (see the package docstring): the product never
imports this file.

Definition followed (per pixel; Sec. III-B.1, the 3DGS rasterizer it builds on,
Sec. III-B.3 Eq. (1) for the depth channel and the loss).  Readings where the
paper is silent are marked [reading]:

  O1  s = exp(l); qh = q/|q| (culled if |q| = 0 or any input is non-finite);
      o = 1/(1+exp(-lambda)).
  O2  R(qh) for qh = (w, x, y, z), the unit-quaternion rotation matrix.
  O3  M = R(qh) diag(s); Sigma = M M^T.
  O4  x_c = R_cw p + t_cw; z = x_c[2]; culled if z <= z_near [reading: 0.2].
  O5  mu' = (fx x/z + cx, fy y/z + cy).
  O6  Jacobian of the pinhole projection with the view-angle clamp
      [reading: kappa = 1.3]: Lx = kappa max(cx + 1/2, W - 1/2 - cx)/fx,
      tx = z clip(x/z, -Lx, Lx) (same for y), J = [[fx/z, 0, -fx tx/z^2],
      [0, fy/z, -fy ty/z^2]].
  O7  EWA screen covariance Sigma' = J R_cw Sigma R_cw^T J^T + eps I
      [reading: eps = 0.3 px^2, no opacity compensation].
  O8  conic Q = Sigma'^{-1}.
  O9  pixel (i, j) is evaluated at its integer centre u = (i, j) [reading];
      m2 = (u-mu')^T Q (u-mu'); G = exp(-m2/2); alpha = min(alpha_max, o G).
  O10 contributors of a pixel: visible Gaussians with m2 <= 9 and
      alpha >= 1/255, ordered by (z, index) ascending [reading].
  O11 front to back: T' = T (1 - alpha); if T' < 1e-4 stop before this
      Gaussian [reading]; else w = alpha T, Y += w [c, z, f], T = T'.
      Y = [RGB (3), depth (1), feature (D)]; background 0; outputs Y, the
      final transmittance T and the contributor count n.
  O12 colour is per-Gaussian RGB (spherical-harmonics degree 0, no view
      dependence) [reading]; depth is the unnormalised sum w z [reading];
      features are the unnormalised sum w f [reading].
  O13 gradients: the exact piecewise derivative with every discrete decision
      (culls, cuts, order, termination, clamp sides) held fixed; the pose
      twist xi = (rho, phi) perturbs the world->camera pose on the left,
      T_cw(xi) = Exp(xi) T_cw, and is differentiated at xi = 0.

Evaluation strategy (not part of the definition): pixels are processed in
square blocks; a Gaussian is a candidate for a block when its m2 <= cutoff2
ellipse's axis-aligned box (half extents sqrt(cutoff2 Sigma'_xx),
sqrt(cutoff2 Sigma'_yy)), grown by one pixel, meets the block.  Every contributor of every pixel of the block is a
candidate, so the per-pixel result is the definition's.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np
import torch

F64 = torch.float64


@dataclass(frozen=True)
class Settings:
    z_near: float = 0.2
    eps2d: float = 0.3
    fov_clamp: float = 1.3
    alpha_max: float = 0.99
    alpha_min: float = 1.0 / 255.0
    T_eps: float = 1e-4
    cutoff2: float = 9.0


def _t(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------------------
# Projection (O1 - O8)
# ---------------------------------------------------------------------------
def quat_to_rotmat(qh: torch.Tensor) -> torch.Tensor:
    """O2: rotation matrix of unit quaternions (w, x, y, z), [N, 3, 3]."""
    w, x, y, z = qh.unbind(-1)
    rows = [
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ]
    return torch.stack(rows, -2)


def se3_exp(xi: torch.Tensor) -> torch.Tensor:
    """SE(3) exponential of the twist xi = (rho, phi): the matrix exponential
    of [[phi]_x, rho; 0, 0] (translation part first)."""
    rho, phi = xi[:3], xi[3:]
    z = torch.zeros((), dtype=F64)
    hat = torch.stack([
        torch.stack([z, -phi[2], phi[1], rho[0]]),
        torch.stack([phi[2], z, -phi[0], rho[1]]),
        torch.stack([-phi[1], phi[0], z, rho[2]]),
        torch.stack([z, z, z, z]),
    ])
    return torch.linalg.matrix_exp(hat)


def project_view(P: dict, cam, xi: torch.Tensor, st: Settings) -> dict:
    """Per-Gaussian screen-space quantities for one camera.

    P holds float64 tensors: means [N,3], log_scales [N,3], quats [N,4],
    logits [N], rgb [N,3], feat [N,D].  Returns mu [N,2], conic [N,3]
    (Q_xx, Q_xy, Q_yy), cov2d [N,3] (Sigma'_xx, Sigma'_xy, Sigma'_yy),
    opac [N], z [N], vis [N] bool (culling decision) and clampx/clampy [N]
    bool (Jacobian clamp sides, for decision signatures)."""
    means, log_s, quats, logits = P["means"], P["log_scales"], P["quats"], P["logits"]
    N = means.shape[0]
    finite = torch.ones(N, dtype=torch.bool)
    for k in ("means", "log_scales", "quats", "logits", "rgb", "feat"):
        a = P[k].detach()
        finite &= torch.isfinite(a.reshape(N, -1)).all(1)
    qn = torch.linalg.norm(torch.where(finite[:, None], quats, torch.ones_like(quats)), dim=1)
    ok = finite & (qn.detach() > 0)

    def safe(a, fill=0.0):
        return torch.where(ok.reshape((N,) + (1,) * (a.dim() - 1)), a, torch.full_like(a, fill))

    s = torch.exp(safe(log_s))                                   # O1
    qh = safe(quats, 1.0) / torch.where(ok, qn, torch.ones_like(qn))[:, None]
    o = torch.sigmoid(safe(logits))
    R = quat_to_rotmat(qh)                                       # O2
    M = R * s[:, None, :]                                        # O3: R diag(s)

    E = se3_exp(xi)
    Rcw = E[:3, :3] @ _t(cam.R_cw)
    tcw = E[:3, :3] @ _t(cam.t_cw) + E[:3, 3]
    xc = safe(means) @ Rcw.T + tcw                               # O4
    z = xc[:, 2]
    vis = ok & (z.detach() > st.z_near)
    zs = torch.where(vis, z, torch.ones_like(z))
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    W, H = int(cam.width), int(cam.height)
    u = xc[:, 0] / zs
    v = xc[:, 1] / zs
    mu = torch.stack([fx * u + cx, fy * v + cy], -1)            # O5
    Lx = st.fov_clamp * max(cx + 0.5, W - 0.5 - cx) / fx         # O6
    Ly = st.fov_clamp * max(cy + 0.5, H - 0.5 - cy) / fy
    tx = zs * torch.clamp(u, -Lx, Lx)
    ty = zs * torch.clamp(v, -Ly, Ly)
    zero = torch.zeros_like(zs)
    J = torch.stack([
        torch.stack([fx / zs, zero, -fx * tx / (zs * zs)], -1),
        torch.stack([zero, fy / zs, -fy * ty / (zs * zs)], -1),
    ], -2)                                                       # [N, 2, 3]
    m = J @ Rcw @ M                                              # rows m1, m2
    m1, m2 = m[:, 0, :], m[:, 1, :]
    a = (m1 * m1).sum(-1) + st.eps2d                             # O7
    c = (m2 * m2).sum(-1) + st.eps2d
    b = (m1 * m2).sum(-1)
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], -1)        # O8
    return {
        "mu": mu, "conic": conic, "cov2d": torch.stack([a, b, c], -1),
        "opac": o, "z": z, "vis": vis,
        "clampx": (u.detach().abs() > Lx), "clampy": (v.detach().abs() > Ly),
    }


# ---------------------------------------------------------------------------
# Per-pixel compositing (O9 - O11)
# ---------------------------------------------------------------------------
def composite(px: torch.Tensor, py: torch.Tensor, mu, conic, opac, z, y, ids,
              st: Settings, want_margin: bool = False, sig: list | None = None):
    """Composite K candidate Gaussians over P pixels.

    px, py [P] pixel centres; mu [K,2], conic [K,3], opac [K], z [K],
    y [K,C] = [rgb, z, feat] (C = 4 + the feature dimension); ids [K]
    Gaussian indices (tie-break).  Candidates may be in any order; they are
    sorted by (z, id) here.  Returns Y [P,C], T [P], n [P], and (want_margin) a dict of each
    pixel's smallest relative distance to every kind of discrete decision:
    "m2" (m2 vs cutoff2), "alpha" (alpha vs alpha_min), "clamp" (o G vs
    alpha_max), "T" (T' vs T_eps) over the candidates up to the one that ends
    the pixel, and "z" (relative depth gap between consecutive contributors,
    which decides their order)."""
    K = mu.shape[0]
    P = px.shape[0]
    if K == 0:
        Y = torch.zeros((P, y.shape[1]), dtype=F64)
        mg = {k: torch.full((P,), math.inf, dtype=F64) for k in ("m2", "alpha", "clamp", "T", "z")}
        if sig is not None:
            sig.append(torch.zeros(P, dtype=torch.int64))
        return Y, torch.ones(P, dtype=F64), torch.zeros(P, dtype=torch.int64), \
            (mg if want_margin else None)
    order = np.lexsort((ids.numpy(), z.detach().numpy()))          # (z, id)
    order = torch.as_tensor(order)
    mu, conic, opac, z, y = mu[order], conic[order], opac[order], z[order], y[order]
    dx = px[:, None] - mu[None, :, 0]
    dy = py[:, None] - mu[None, :, 1]
    m2 = conic[None, :, 0] * dx * dx + 2.0 * conic[None, :, 1] * dx * dy \
        + conic[None, :, 2] * dy * dy                                # O9
    G = torch.exp(-0.5 * m2)
    a_raw = opac[None, :] * G
    alpha = torch.minimum(a_raw, torch.full_like(a_raw, st.alpha_max))
    mask = (m2.detach() <= st.cutoff2) & (alpha.detach() >= st.alpha_min)   # O10
    one_m = torch.where(mask, 1.0 - alpha, torch.ones_like(alpha))
    cp = torch.cumprod(one_m.detach(), dim=1)                      # T after each
    incl = mask & (cp >= st.T_eps)                                 # O11 (break)
    keep = torch.where(incl, 1.0 - alpha, torch.ones_like(alpha))
    Tinc = torch.cumprod(keep, dim=1)
    Tbefore = torch.cat([torch.ones((P, 1), dtype=F64), Tinc[:, :-1]], 1)
    w = torch.where(incl, alpha * Tbefore, torch.zeros_like(alpha))
    Y = w @ y
    T = Tinc[:, -1]
    n = incl.sum(1)
    if sig is not None:
        # digest of every per-pixel decision: which candidates contribute, in
        # which order, and which of them sit on the alpha clamp
        with torch.no_grad():
            sid = ids[order].to(torch.int64) + 1
            pos = torch.cumsum(incl.to(torch.int64), 1)
            clamp = (a_raw > st.alpha_max) & incl
            d = (incl.to(torch.int64) * sid[None, :] * (pos * 7919 + 1)).sum(1) \
                + (clamp.to(torch.int64) * sid[None, :] * 104729).sum(1) + n * 15485863
            sig.append(d)
    margin = None
    if want_margin:
        with torch.no_grad():
            inf = torch.full_like(m2, math.inf)
            # decisions that matter: candidates up to and including the one
            # that terminates the pixel (all of them if none does)
            term = mask & (cp < st.T_eps)
            first_term = torch.where(term.any(1), term.float().argmax(1),
                                     torch.full((P,), K - 1, dtype=torch.int64))
            upto = torch.arange(K)[None, :] <= first_term[:, None]

            def mn(r):
                return torch.where(upto, r, inf).min(1).values
            margin = {
                "m2": mn((m2 - st.cutoff2).abs() / st.cutoff2),
                "alpha": mn(torch.where(m2 <= st.cutoff2,
                                        (alpha - st.alpha_min).abs() / st.alpha_min, inf)),
                "clamp": mn(torch.where(mask, (a_raw - st.alpha_max).abs() / st.alpha_max, inf)),
                "T": mn(torch.where(mask, (cp - st.T_eps).abs() / st.T_eps, inf)),
            }
            # depth order between consecutive contributors (and the one that
            # terminates the pixel)
            zz = z.detach()
            if K > 1:
                gap = (zz[1:] - zz[:-1]).abs() / zz[:-1].abs().clamp_min(1e-30)
                # consecutive masked candidates: next masked index after each
                idx = torch.arange(K)[None, :].expand(P, K)
                big = torch.full_like(idx, K)
                nxt = torch.where(mask, idx, big).flip(1).cummin(1).values.flip(1)
                nxt_after = torch.cat([nxt[:, 1:], torch.full((P, 1), K)], 1)
                ok = mask & upto & (nxt_after < K)
                zpad = torch.cat([zz, zz[-1:]])
                zn = zpad[nxt_after.clamp_max(K - 1)]
                gz = (zn - zz[None, :]).abs() / zz[None, :].abs().clamp_min(1e-30)
                margin["z"] = torch.where(ok, gz, inf).min(1).values
            else:
                margin["z"] = torch.full((P,), math.inf, dtype=F64)
    return Y, T, n, margin


# ---------------------------------------------------------------------------
# Whole-image drivers
# ---------------------------------------------------------------------------
def _params(scene, requires_grad=False) -> dict:
    P = {
        "means": _t(scene.means), "log_scales": _t(scene.log_scales),
        "quats": _t(scene.quats), "logits": _t(scene.logits),
        "rgb": _t(scene.rgb), "feat": _t(scene.feat),
    }
    if requires_grad:
        for v in P.values():
            v.requires_grad_(True)
    return P


def _blocks(cam, rects, bs):
    """Pixel blocks (x0, y0, x1, y1), half-open, covering the rects."""
    if rects is None:
        rects = [(0, 0, cam.width, cam.height)]
    out = []
    for (x0, y0, w, h) in rects:
        for by in range(y0, y0 + h, bs):
            for bx in range(x0, x0 + w, bs):
                out.append((bx, by, min(bx + bs, x0 + w), min(by + bs, y0 + h)))
    return out


def _candidates(proj, blk, st, pad=1.0):
    """Visible Gaussians whose m2 <= cutoff2 ellipse box (plus `pad`) meets
    blk (half extents sqrt(cutoff2 Sigma'_xx), sqrt(cutoff2 Sigma'_yy))."""
    vis = proj["vis"]
    mu = proj["mu"].detach()
    cov = proj["cov2d"].detach()
    rx = torch.sqrt(st.cutoff2 * cov[:, 0]) + pad
    ry = torch.sqrt(st.cutoff2 * cov[:, 2]) + pad
    x0, y0, x1, y1 = blk
    hit = vis & (mu[:, 0] + rx >= x0) & (mu[:, 0] - rx <= x1 - 1) \
        & (mu[:, 1] + ry >= y0) & (mu[:, 1] - ry <= y1 - 1)
    return torch.nonzero(hit).flatten()


def _y_of(P, proj):
    return torch.cat([P["rgb"], proj["z"][:, None], P["feat"]], 1)   # [N, 4 + D]


def render(scene, cams, st: Settings = Settings(), rects=None, block=16,
           want_margin=True) -> list:
    """Forward render of every view.  Returns one dict per view with
    rgb [3,H,W], depth [H,W], feat [D,H,W] (D = the scene's feature
    dimension), T [H,W], n [H,W] (int64),
    margin {kind: [H,W]} (see ``composite``; inf where not evaluated) and the
    per-Gaussian projection (mu, conic, cov2d, opac, z, vis); pixels outside
    `rects` (per view list of (x0, y0, w, h)) are NaN."""
    P = _params(scene)
    outs = []
    with torch.no_grad():
        for vi, cam in enumerate(cams):
            proj = project_view(P, cam, torch.zeros(6, dtype=F64), st)
            y = _y_of(P, proj)
            C = y.shape[1]
            H, W = cam.height, cam.width
            Y = torch.full((C, H, W), math.nan, dtype=F64)
            T = torch.full((H, W), math.nan, dtype=F64)
            n = torch.full((H, W), -1, dtype=torch.int64)
            mg = {k: torch.full((H, W), math.inf, dtype=F64)
                  for k in ("m2", "alpha", "clamp", "T", "z")}
            for blk in _blocks(cam, None if rects is None else rects[vi], block):
                x0, y0, x1, y1 = blk
                yy, xx = torch.meshgrid(torch.arange(y0, y1, dtype=F64),
                                        torch.arange(x0, x1, dtype=F64), indexing="ij")
                px, py = xx.flatten(), yy.flatten()
                cand = _candidates(proj, blk, st)
                Yb, Tb, nb, mb = composite(px, py, proj["mu"][cand], proj["conic"][cand],
                                           proj["opac"][cand], proj["z"][cand], y[cand],
                                           cand, st, want_margin)
                h, w = y1 - y0, x1 - x0
                Y[:, y0:y1, x0:x1] = Yb.T.reshape(C, h, w)
                T[y0:y1, x0:x1] = Tb.reshape(h, w)
                n[y0:y1, x0:x1] = nb.reshape(h, w)
                if mb is not None:
                    for k in mg:
                        mg[k][y0:y1, x0:x1] = mb[k].reshape(h, w)
            outs.append({"rgb": Y[:3].numpy(), "depth": Y[3].numpy(), "feat": Y[4:].numpy(),
                         "T": T.numpy(), "n": n.numpy(),
                         "margin": {k: v.numpy() for k, v in mg.items()},
                         "vis": proj["vis"].numpy(),
                         "mu": proj["mu"].numpy(), "conic": proj["conic"].numpy(),
                         "opac": proj["opac"].numpy(), "z": proj["z"].numpy(),
                         "cov2d": proj["cov2d"].numpy()})
    return outs


def vjp(scene, cams, upstream, st: Settings = Settings(), upstream_T=None,
        rects=None, block=16) -> dict:
    """Vector-Jacobian product of the renderer.

    upstream: per view [4 + D, H, W] arrays dL/dY (RGB, depth, feature);
    upstream_T: optional per view [H, W] dL/dT.  Only pixels inside `rects`
    (per view; default: whole image) are evaluated, so the upstream gradient
    must vanish elsewhere.  Returns float64 numpy gradients: means [N,3],
    log_scales [N,3], quats [N,4], logits [N], rgb [N,3], feat [N,D],
    twist [V,6] (rho, phi)."""
    P = _params(scene, requires_grad=True)
    N = scene.n
    g_rgb = torch.zeros((N, 3), dtype=F64)
    D = scene.feat.shape[1]
    g_feat = torch.zeros((N, D), dtype=F64)
    twist = []
    for vi, cam in enumerate(cams):
        xi = torch.zeros(6, dtype=F64, requires_grad=True)
        proj = project_view(P, cam, xi, st)
        leaves = {k: proj[k].detach().clone().requires_grad_(True)
                  for k in ("mu", "conic", "opac", "z")}
        acc = {k: torch.zeros_like(v) for k, v in leaves.items()}
        up = _t(upstream[vi])
        upT = None if upstream_T is None else _t(upstream_T[vi])
        for blk in _blocks(cam, None if rects is None else rects[vi], block):
            x0, y0, x1, y1 = blk
            gb = up[:, y0:y1, x0:x1].reshape(4 + D, -1).T
            gT = None if upT is None else upT[y0:y1, x0:x1].reshape(-1)
            if not bool(gb.abs().sum() > 0) and (gT is None or not bool(gT.abs().sum() > 0)):
                continue
            cand = _candidates(proj, blk, st)
            if cand.numel() == 0:
                continue
            sub = {k: leaves[k].detach()[cand].clone().requires_grad_(True) for k in leaves}
            rgb_s = P["rgb"].detach()[cand].clone().requires_grad_(True)
            feat_s = P["feat"].detach()[cand].clone().requires_grad_(True)
            y = torch.cat([rgb_s, sub["z"][:, None], feat_s], 1)
            yy, xx = torch.meshgrid(torch.arange(y0, y1, dtype=F64),
                                    torch.arange(x0, x1, dtype=F64), indexing="ij")
            Yb, Tb, _, _ = composite(xx.flatten(), yy.flatten(), sub["mu"], sub["conic"],
                                     sub["opac"], sub["z"], y, cand, st)
            s = (Yb * gb).sum()
            if gT is not None:
                s = s + (Tb * gT).sum()
            grads = torch.autograd.grad(s, [sub["mu"], sub["conic"], sub["opac"], sub["z"],
                                            rgb_s, feat_s], allow_unused=True)
            for k, g in zip(("mu", "conic", "opac", "z"), grads[:4]):
                if g is not None:
                    acc[k].index_add_(0, cand, g)
            if grads[4] is not None:
                g_rgb.index_add_(0, cand, grads[4])
            if grads[5] is not None:
                g_feat.index_add_(0, cand, grads[5])
        outs = [proj[k] for k in ("mu", "conic", "opac", "z")]
        gouts = [acc[k] for k in ("mu", "conic", "opac", "z")]
        torch.autograd.backward(outs, gouts)
        twist.append(xi.grad.detach().clone() if xi.grad is not None else torch.zeros(6, dtype=F64))

    def g(k):
        return P[k].grad.numpy().copy() if P[k].grad is not None else np.zeros(P[k].shape)
    return {"means": g("means"), "log_scales": g("log_scales"), "quats": g("quats"),
            "logits": g("logits"), "rgb": g_rgb.numpy(), "feat": g_feat.numpy(),
            "twist": torch.stack(twist).numpy()}


# ---------------------------------------------------------------------------
# L1 loss of Eq. (1) without its D-SSIM term (the step downstream of render)
# ---------------------------------------------------------------------------
def l1_loss(outs, targets, loss_w) -> float:
    """Sum over views of  mean|RGB-RGB*| + w_d mean|D-D*| + w_f mean|F-F*|
    (each mean over that group's elements of the view); loss_w = (w_rgb,
    w_depth, w_feat)."""
    L = 0.0
    for o, t in zip(outs, targets):
        L += loss_w[0] * np.mean(np.abs(o["rgb"] - t.rgb))
        L += loss_w[1] * np.mean(np.abs(o["depth"] - t.depth))
        L += loss_w[2] * np.mean(np.abs(o["feat"] - t.feat))
    return float(L)


def l1_upstream(outs, targets, loss_w) -> list:
    """dL/dY of ``l1_loss``: w_group sign(Y - Y*) / n_group with sign(0) = 0,
    as per-view [4 + D, H, W] float64 arrays."""
    gs = []
    for o, t in zip(outs, targets):
        H, W = t.depth.shape
        D = t.feat.shape[0]
        g = np.empty((4 + D, H, W))
        g[:3] = loss_w[0] * np.sign(o["rgb"] - t.rgb) / (3 * H * W)
        g[3] = loss_w[1] * np.sign(o["depth"] - t.depth) / (H * W)
        g[4:] = loss_w[2] * np.sign(o["feat"] - t.feat) / (D * H * W)
        gs.append(g)
    return gs


def loss_and_grads(scene, cams, targets, loss_w, st: Settings = Settings()):
    """Forward, L1 loss, and its gradient (whole images)."""
    outs = render(scene, cams, st, want_margin=False)
    L = l1_loss(outs, targets, loss_w)
    g = l1_upstream(outs, targets, loss_w)
    return outs, L, vjp(scene, cams, g, st)


def settings_dict(st: Settings) -> dict:
    return asdict(st)
