"""Pure-Python (``math`` module) per-pixel brute force of the rasterizer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A second, deliberately different transcription of the same definition as
``raster_fp64`` (Sec. III-B.1, the 3DGS rasterizer; Eq. (1) for depth),
for tiny scenes (a few Gaussians, a few hundred pixels):

  * the rotation of a unit quaternion (w, v) is built as
    (w^2 - v.v) I + 2 v v^T + 2 w [v]_x  (not the expanded 3x3 table);
  * the world covariance is R S S R^T by explicit loops;
  * the pose perturbation Exp(xi) uses Rodrigues' formula and the SE(3)
    left Jacobian V (not a matrix exponential);
  * every pixel loops over every Gaussian, keeps the contributors and sorts
    them with ``sorted`` on (z, index).

It also returns a decision signature (culls, clamp sides, each pixel's ordered
contributor list and clamp flags) so finite-difference tests can drop the
parameters whose +-h evaluations change a discrete decision.
"""
from __future__ import annotations

import math


def _matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def _transpose(A):
    return [list(r) for r in zip(*A)]


def _rot_from_quat(q):
    w, x, y, z = q
    n = math.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    v = (x, y, z)
    vv = x * x + y * y + z * z
    skew = [[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]]
    return [[(w * w - vv) * (1.0 if i == j else 0.0) + 2.0 * v[i] * v[j] + 2.0 * w * skew[i][j]
             for j in range(3)] for i in range(3)]


def _so3_exp_and_V(phi):
    th2 = phi[0] ** 2 + phi[1] ** 2 + phi[2] ** 2
    K = [[0.0, -phi[2], phi[1]], [phi[2], 0.0, -phi[0]], [-phi[1], phi[0], 0.0]]
    K2 = _matmul(K, K)
    if th2 < 1e-12:
        a, b, c = 1.0 - th2 / 6.0, 0.5 - th2 / 24.0, 1.0 / 6.0 - th2 / 120.0
    else:
        th = math.sqrt(th2)
        a = math.sin(th) / th
        b = (1.0 - math.cos(th)) / th2
        c = (th - math.sin(th)) / (th2 * th)
    I = [[1.0 if i == j else 0.0 for j in range(3)] for i in range(3)]
    R = [[I[i][j] + a * K[i][j] + b * K2[i][j] for j in range(3)] for i in range(3)]
    V = [[I[i][j] + b * K[i][j] + c * K2[i][j] for j in range(3)] for i in range(3)]
    return R, V


def project_one(p, log_s, q, logit, cam, Rcw, tcw, st):
    """Returns None when culled, else a dict of screen quantities."""
    vals = list(p) + list(log_s) + list(q) + [logit]
    if not all(math.isfinite(v) for v in vals):
        return None
    if math.sqrt(sum(c * c for c in q)) == 0.0:
        return None
    xc = [sum(Rcw[i][k] * p[k] for k in range(3)) + tcw[i] for i in range(3)]
    z = xc[2]
    if not z > st.z_near:
        return None
    s = [math.exp(v) for v in log_s]
    R = _rot_from_quat(q)
    # Sigma = R S S R^T
    Sig = [[sum(R[i][k] * s[k] * s[k] * R[j][k] for k in range(3)) for j in range(3)]
           for i in range(3)]
    Sc = _matmul(_matmul(Rcw, Sig), _transpose(Rcw))
    fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy
    W, H = cam.width, cam.height
    X, Y = xc[0] / z, xc[1] / z
    limx = st.fov_clamp * max(cx + 0.5, W - 0.5 - cx) / fx
    limy = st.fov_clamp * max(cy + 0.5, H - 0.5 - cy) / fy
    Xc = min(max(X, -limx), limx)
    Yc = min(max(Y, -limy), limy)
    J = [[fx / z, 0.0, -fx * Xc / z], [0.0, fy / z, -fy * Yc / z]]
    S2 = _matmul(_matmul(J, Sc), _transpose(J))
    a = S2[0][0] + st.eps2d
    b = S2[0][1]
    c = S2[1][1] + st.eps2d
    det = a * c - b * b
    return {
        "mu": (fx * X + cx, fy * Y + cy),
        "conic": (c / det, -b / det, a / det),
        "opac": 1.0 / (1.0 + math.exp(-logit)),
        "z": z,
        "clamp": (abs(X) > limx, abs(Y) > limy),
    }


def render_view(scene, cam, st, xi=(0.0,) * 6):
    """Brute-force render of one view.

    scene: object with means, log_scales, quats, logits, rgb, feat (indexable
    rows).  Returns (Y [H][W][20], T [H][W], n [H][W], signature)."""
    Rphi, V = _so3_exp_and_V(xi[3:])
    rho = xi[:3]
    Rcw0 = [[float(cam.R_cw[i][j]) for j in range(3)] for i in range(3)]
    tcw0 = [float(cam.t_cw[i]) for i in range(3)]
    Rcw = _matmul(Rphi, Rcw0)
    tcw = [sum(Rphi[i][k] * tcw0[k] for k in range(3)) + sum(V[i][k] * rho[k] for k in range(3))
           for i in range(3)]
    N = len(scene.means)
    proj = []
    for i in range(N):
        pr = project_one([float(v) for v in scene.means[i]],
                         [float(v) for v in scene.log_scales[i]],
                         [float(v) for v in scene.quats[i]], float(scene.logits[i]),
                         cam, Rcw, tcw, st)
        if pr is not None and not (all(math.isfinite(float(v)) for v in scene.rgb[i])
                                   and all(math.isfinite(float(v)) for v in scene.feat[i])):
            pr = None
        proj.append(pr)
    sig = [None if pr is None else pr["clamp"] for pr in proj]
    H, W = cam.height, cam.width
    Yimg = [[None] * W for _ in range(H)]
    Timg = [[1.0] * W for _ in range(H)]
    nimg = [[0] * W for _ in range(H)]
    for j in range(H):
        for i in range(W):
            cands = []
            for g, pr in enumerate(proj):
                if pr is None:
                    continue
                dx = i - pr["mu"][0]
                dy = j - pr["mu"][1]
                qa, qb, qc = pr["conic"]
                m2 = qa * dx * dx + 2.0 * qb * dx * dy + qc * dy * dy
                if m2 > st.cutoff2:
                    continue
                ar = pr["opac"] * math.exp(-0.5 * m2)
                al = min(st.alpha_max, ar)
                if al < st.alpha_min:
                    continue
                cands.append((pr["z"], g, al, ar > st.alpha_max))
            cands.sort(key=lambda t: (t[0], t[1]))
            T = 1.0
            acc = [0.0] * 20
            used = []
            for (z, g, al, clamped) in cands:
                Tn = T * (1.0 - al)
                if Tn < st.T_eps:
                    break
                w = al * T
                y = [float(v) for v in scene.rgb[g]] + [proj[g]["z"]] + \
                    [float(v) for v in scene.feat[g]]
                for c in range(20):
                    acc[c] += w * y[c]
                T = Tn
                used.append((g, clamped))
            Yimg[j][i] = acc
            Timg[j][i] = T
            nimg[j][i] = len(used)
            sig.append(tuple(used))
    return Yimg, Timg, nimg, tuple(sig)


def loss_weighted(scene, cams, st, upstream, upstream_T=None, xis=None):
    """sum_v <upstream_v, Y_v> (+ <upstream_T_v, T_v>): a linear functional of
    the render whose gradient is the renderer's vector-Jacobian product.
    Returns (value, signature)."""
    total = 0.0
    sigs = []
    for vi, cam in enumerate(cams):
        xi = (0.0,) * 6 if xis is None else xis[vi]
        Y, T, n, sig = render_view(scene, cam, st, xi)
        g = upstream[vi]
        for j in range(cam.height):
            for i in range(cam.width):
                for c in range(20):
                    gc = float(g[c][j][i])
                    if gc != 0.0:
                        total += gc * Y[j][i][c]
                if upstream_T is not None:
                    total += float(upstream_T[vi][j][i]) * T[j][i]
        sigs.append(sig)
    return total, tuple(sigs)
