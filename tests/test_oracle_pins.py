"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test names the part of the definition it pins (see the oracle's module
docstring, O1-O13) and the kind of pin: closed form, invariant, brute force,
library routine, or finite differences.  The paper prints no per-pixel value,
so no test compares against a number taken from it.
"""
import copy
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.stats import multivariate_normal

import scenes
from oracle import brute
from oracle import raster_fp64 as R

ST = R.Settings()


def one_view(W, H, f, R_cw=None, t_cw=None, cx=None, cy=None):
    return scenes.Camera(W, H, f, f, (W - 1) / 2.0 if cx is None else cx,
                         (H - 1) / 2.0 if cy is None else cy,
                         np.eye(3, dtype=np.float32) if R_cw is None else R_cw,
                         np.zeros(3, np.float32) if t_cw is None else t_cw)


def make_scene(means, log_scales, quats, logits, rgb, feat):
    f = lambda a: np.asarray(a, dtype=np.float64)
    return scenes.Scene(f(means), f(log_scales), f(quats), f(logits), f(rgb), f(feat))


def posed_camera(seed, W=20, H=16, f=30.0):
    """A camera with a generic rotation and translation, and Gaussians
    placed in its frustum (world coordinates)."""
    rng = np.random.default_rng(seed)
    Rc = Rotation.from_rotvec(rng.normal(size=3) * 0.7).as_matrix()
    t = rng.normal(size=3)
    return one_view(W, H, f, Rc.astype(np.float64), t.astype(np.float64))


def scene_in_view(seed, cam, n, z=(1.2, 2.5), ls=(-2.2, 0.3), logit=(0.3, 1.0)):
    rng = np.random.default_rng(100 + seed)
    zz = rng.uniform(*z, size=n)
    u = rng.uniform(-1, cam.width, size=n)
    v = rng.uniform(-1, cam.height, size=n)
    xc = np.stack([(u - cam.cx) * zz / cam.fx, (v - cam.cy) * zz / cam.fy, zz], 1)
    Rcw = np.asarray(cam.R_cw, np.float64)
    means = (xc - np.asarray(cam.t_cw, np.float64)) @ Rcw     # R^T (xc - t)
    q = rng.normal(size=(n, 4))
    q *= rng.uniform(0.5, 2.0, size=(n, 1))                  # not normalised
    feat = rng.normal(size=(n, 16))
    return make_scene(means, rng.normal(ls[0], ls[1], size=(n, 3)), q,
                      rng.normal(logit[0], logit[1], size=n), rng.uniform(0, 1, (n, 3)), feat)


# --------------------------------------------------------------------------
# Projection (O1-O8)
# --------------------------------------------------------------------------
def test_isotropic_on_axis_closed_form():
    """Closed form: an isotropic Gaussian on the optical axis projects to the
    principal point with Sigma' = ((f s / z)^2 + eps) I and Q its inverse."""
    for (f, ls, z, W, H) in [(100.0, -3.0, 2.0, 128, 96), (577.0, -2.5, 3.7, 640, 480)]:
        cam = one_view(W, H, f)
        q = [[0.3, -0.5, 0.7, 0.2]]                # irrelevant for isotropic s
        sc = make_scene([[0, 0, z]], [[ls] * 3], q, [0.4], [[0.2, 0.5, 0.9]], [[0.1] * 16])
        o = R.render(sc, [cam], ST, rects=[[(0, 0, 1, 1)]])[0]
        s2 = (f * math.exp(ls) / z) ** 2 + ST.eps2d
        assert np.allclose(o["mu"][0], [cam.cx, cam.cy], rtol=0, atol=1e-12)
        assert np.allclose(o["cov2d"][0], [s2, 0.0, s2], rtol=1e-12, atol=1e-12)
        assert np.allclose(o["conic"][0], [1 / s2, 0.0, 1 / s2], rtol=1e-12)
        assert math.isclose(o["opac"][0], 1 / (1 + math.exp(-0.4)), rel_tol=1e-14)
        assert math.isclose(o["z"][0], z, rel_tol=1e-14)


def test_anisotropic_projection_vs_linearisation():
    """Library routine + numerical Jacobian: Sigma' - eps I equals
    J_num R_cw Sigma R_cw^T J_num^T, with Sigma built from scipy's quaternion
    rotation and J_num the central-difference Jacobian of the pinhole map;
    mu' equals the pinhole map of the mean.  Covers O1-O8 (unclamped)."""
    cam = posed_camera(3, W=64, H=48, f=55.0)
    sc = scene_in_view(3, cam, 25, ls=(-2.0, 0.6))
    o = R.render(sc, [cam], ST, rects=[[(0, 0, 1, 1)]])[0]
    Rcw = np.asarray(cam.R_cw, np.float64)
    t = np.asarray(cam.t_cw, np.float64)

    def pin(x):
        xc = Rcw @ x + t
        return np.array([cam.fx * xc[0] / xc[2] + cam.cx, cam.fy * xc[1] / xc[2] + cam.cy])

    for i in range(sc.n):
        w, x, y, z = sc.quats[i]
        Rq = Rotation.from_quat([x, y, z, w]).as_matrix()       # scipy: (x, y, z, w)
        S = np.diag(np.exp(sc.log_scales[i]) ** 2)
        Sig = Rq @ S @ Rq.T
        h = 1e-6
        Jw = np.stack([(pin(sc.means[i] + h * e) - pin(sc.means[i] - h * e)) / (2 * h)
                       for e in np.eye(3)], 1)                    # d mu / d p_world
        cov = Jw @ Sig @ Jw.T + ST.eps2d * np.eye(2)
        a, b, c = o["cov2d"][i]
        assert np.allclose([[a, b], [b, c]], cov, rtol=1e-7, atol=1e-9), i
        assert np.allclose(o["mu"][i], pin(sc.means[i]), rtol=1e-12, atol=1e-9)
        Q = np.array([[o["conic"][i][0], o["conic"][i][1]], [o["conic"][i][1], o["conic"][i][2]]])
        assert np.allclose(Q @ cov, np.eye(2), atol=1e-7)
        assert math.isclose(o["z"][i], (Rcw @ sc.means[i] + t)[2], rel_tol=1e-13)


def test_jacobian_clamp_side():
    """Closed form of O6 when the clamp is active: for a Gaussian far to the
    side (x/z beyond the limit), Sigma'_xx - eps = (fx s/z)^2 (1 + L^2) for an
    isotropic Gaussian (J row (fx/z, 0, -fx L/z))."""
    W, H, f = 40, 30, 50.0
    cam = one_view(W, H, f)
    L = ST.fov_clamp * max(cam.cx + 0.5, W - 0.5 - cam.cx) / f
    z, ls = 2.0, -2.0
    x = 3.0 * L * z                                            # well beyond the limit
    sc = make_scene([[x, 0, z]], [[ls] * 3], [[1, 0, 0, 0]], [0.0], [[1, 1, 1]], [[0] * 16])
    o = R.render(sc, [cam], ST, rects=[[(0, 0, 1, 1)]])[0]
    s = math.exp(ls)
    assert math.isclose(o["cov2d"][0][0] - ST.eps2d, (f * s / z) ** 2 * (1 + L * L), rel_tol=1e-12)
    assert math.isclose(o["cov2d"][0][2] - ST.eps2d, (f * s / z) ** 2, rel_tol=1e-12)


def test_quaternion_sign_and_scale_invariance():
    """Invariant: q -> -q and q -> 3.7 q leave every output unchanged."""
    cam = posed_camera(5)
    sc = scene_in_view(5, cam, 10)
    base = R.render(sc, [cam], ST)[0]
    for k in (-1.0, 3.7):
        sc2 = copy.copy(sc)
        sc2.quats = sc.quats * k
        o = R.render(sc2, [cam], ST)[0]
        for key in ("rgb", "depth", "feat", "T"):
            assert np.allclose(o[key], base[key], rtol=1e-12, atol=1e-13)


def test_culling_rules():
    """Special cases: zero quaternion, non-finite input and z <= z_near cull
    the Gaussian (no contribution)."""
    cam = one_view(9, 9, 10.0)
    base = dict(means=[[0, 0, 2.0]], log_scales=[[-1.0] * 3], quats=[[1, 0, 0, 0]],
                logits=[2.0], rgb=[[1, 1, 1]], feat=[[1] + [0] * 15])
    for k, v in [("quats", [[0, 0, 0, 0]]), ("logits", [math.nan]),
                 ("means", [[0, 0, 0.2]]), ("feat", [[math.inf] + [0] * 15])]:
        d = dict(base)
        d[k] = v
        o = R.render(make_scene(**d), [cam], ST)[0]
        assert np.all(o["T"] == 1.0) and np.all(o["rgb"] == 0.0) and np.all(o["n"] == 0), k
    o = R.render(make_scene(**base), [cam], ST)[0]
    assert o["n"][4, 4] == 1


# --------------------------------------------------------------------------
# Compositing (O9-O12)
# --------------------------------------------------------------------------
def _iso(z, ls, logit, rgb, feat, xy=(0.0, 0.0)):
    return dict(means=[xy[0] * z, xy[1] * z, z], ls=[ls] * 3, logit=logit, rgb=rgb, feat=feat)


def test_single_gaussian_closed_form():
    """Closed form of one isotropic on-axis Gaussian: inside the cut,
    Y = alpha [c, z, f] and T = 1 - alpha with alpha = min(0.99, o G),
    G = exp(-|u - c|^2 / (2 sigma^2)), sigma^2 = (f s/z)^2 + eps; outside,
    Y = 0 and T = 1."""
    W, H, f, z, ls, logit = 33, 25, 40.0, 2.0, -2.3, 0.7
    cam = one_view(W, H, f)
    c = [0.3, 0.6, 0.9]
    fe = list(np.linspace(-1, 1, 16))
    sc = make_scene([[0, 0, z]], [[ls] * 3], [[0.2, 0.4, 0.1, 0.9]], [logit], [c], [fe])
    o = R.render(sc, [cam], ST)[0]
    s2 = (f * math.exp(ls) / z) ** 2 + ST.eps2d
    op = 1 / (1 + math.exp(-logit))
    jj, ii = np.mgrid[0:H, 0:W]
    m2 = ((ii - cam.cx) ** 2 + (jj - cam.cy) ** 2) / s2
    al = np.minimum(0.99, op * np.exp(-0.5 * m2))
    inside = (m2 <= 9) & (al >= 1 / 255)
    a = np.where(inside, al, 0.0)
    assert inside.sum() > 20 and (~inside).sum() > 20
    assert np.allclose(o["T"], 1 - a, rtol=1e-13, atol=1e-15)
    for k in range(3):
        assert np.allclose(o["rgb"][k], a * c[k], rtol=1e-13, atol=1e-15)
    assert np.allclose(o["depth"], a * z, rtol=1e-13, atol=1e-15)
    for k in range(16):
        assert np.allclose(o["feat"][k], a * fe[k], rtol=1e-13, atol=1e-15)
    assert np.array_equal(o["n"], inside.astype(int))


def test_two_gaussians_closed_form():
    """Closed form: z1 < z2 at one pixel, Y = a1 y1 + (1 - a1) a2 y2 and
    T = (1 - a1)(1 - a2), whatever the input order."""
    W, H, f = 15, 11, 20.0
    cam = one_view(W, H, f)
    g1 = ([0.0, 0.0, 1.5], -2.0, 0.5, [1, 0, 0.5], [0.5] * 16)     # on the axis:
    g2 = ([0.0, 0.0, 2.5], -1.8, 1.2, [0, 1, 0.25], [-0.25] * 16)  # isotropic Sigma'
    for order in ([g2, g1], [g1, g2]):
        sc = make_scene([g[0] for g in order], [[g[1]] * 3 for g in order],
                        [[1, 0, 0, 0]] * 2, [g[2] for g in order],
                        [g[3] for g in order], [g[4] for g in order])
        o = R.render(sc, [cam], ST)[0]
        i, j = 8, 6
        vals = []
        for g in (g1, g2):
            z = g[0][2]
            mu = (f * g[0][0] / z + cam.cx, f * g[0][1] / z + cam.cy)
            s2 = (f * math.exp(g[1]) / z) ** 2 + ST.eps2d
            m2 = ((i - mu[0]) ** 2 + (j - mu[1]) ** 2) / s2
            assert m2 < 9
            vals.append(min(0.99, math.exp(-0.5 * m2) / (1 + math.exp(-g[2]))))
        a1, a2 = vals
        y1 = np.array(g1[3] + [g1[0][2]] + g1[4])
        y2 = np.array(g2[3] + [g2[0][2]] + g2[4])
        Y = a1 * y1 + (1 - a1) * a2 * y2
        got = np.concatenate([o["rgb"][:, j, i], [o["depth"][j, i]], o["feat"][:, j, i]])
        assert np.allclose(got, Y, rtol=1e-13)
        assert math.isclose(o["T"][j, i], (1 - a1) * (1 - a2), rel_tol=1e-13)


def test_termination_thirteen_layers():
    """Closed form of the early stop: 20 identical Gaussians on the axis with
    o = 0.5 give alpha = 0.5 at the centre pixel; 0.5^13 >= 1e-4 > 0.5^14, so
    exactly 13 contribute, T = 2^-13 and RGB = (1 - 2^-13) c.  A large logit
    clamps alpha to 0.99."""
    cam = one_view(9, 9, 30.0)                      # centre pixel (4, 4)
    n = 20
    zs = [1.0 + 0.1 * k for k in range(n)]
    c = [0.25, 0.5, 0.75]
    sc = make_scene([[0, 0, z] for z in zs], [[-2.5] * 3] * n, [[1, 0, 0, 0]] * n,
                    [0.0] * n, [c] * n, [[1.0] + [0.0] * 15] * n)
    o = R.render(sc, [cam], ST)[0]
    assert o["n"][4, 4] == 13
    assert o["T"][4, 4] == 2.0 ** -13
    assert np.allclose(o["rgb"][:, 4, 4], (1 - 2.0 ** -13) * np.array(c), rtol=1e-15)
    assert math.isclose(o["depth"][4, 4], sum(0.5 ** (k + 1) * zs[k] for k in range(13)),
                        rel_tol=1e-14)
    sc2 = make_scene([[0, 0, 1.0]], [[-2.5] * 3], [[1, 0, 0, 0]], [30.0], [c], [[0] * 16])
    o2 = R.render(sc2, [cam], ST)[0]
    assert math.isclose(o2["T"][4, 4], 0.01, rel_tol=1e-14)


def test_blend_weights_sum_to_one_minus_T():
    """Invariant (telescoping): sum_i w_i + T = 1 per pixel.  With c = 1 the
    RGB channels are 1 - T, with f = e1 the first feature is 1 - T and the
    others 0; with every Gaussian at camera depth z0, D = z0 (1 - T)."""
    wl = scenes.make_workload(1, n=600, res_scale=0.5)
    sc = wl.scene
    sc1 = copy.copy(sc)
    sc1.rgb = np.ones_like(sc.rgb)
    sc1.feat = np.zeros_like(sc.feat)
    sc1.feat[:, 0] = 1.0
    o = R.render(sc1, wl.cams, ST)[0]
    assert (o["n"] > 3).mean() > 0.3                     # the invariant is exercised
    for k in range(3):
        assert np.allclose(o["rgb"][k], 1 - o["T"], atol=1e-13)
    assert np.allclose(o["feat"][0], 1 - o["T"], atol=1e-13)
    assert np.all(o["feat"][1:] == 0)
    z0 = 2.0
    sc2 = copy.copy(sc1)
    sc2.means = sc.means / sc.means[:, 2:3] * z0           # identity pose: camera z = z0
    o2 = R.render(sc2, wl.cams, ST)[0]
    assert np.allclose(o2["depth"], z0 * (1 - o2["T"]), atol=1e-12)


def test_linearity_in_colour_and_feature():
    """Invariant: render(a f1 + b f2) = a render(f1) + b render(f2), and the
    same for colours (weights do not depend on c, f)."""
    wl = scenes.make_workload(1, n=300, res_scale=0.5)
    rng = np.random.default_rng(0)
    s1, s2 = copy.copy(wl.scene), copy.copy(wl.scene)
    s1.feat, s2.feat = rng.normal(size=s1.feat.shape), rng.normal(size=s1.feat.shape)
    s1.rgb, s2.rgb = rng.uniform(size=s1.rgb.shape), rng.uniform(size=s1.rgb.shape)
    s3 = copy.copy(wl.scene)
    s3.feat = 0.3 * s1.feat - 1.7 * s2.feat
    s3.rgb = 0.3 * s1.rgb - 1.7 * s2.rgb
    o1, o2, o3 = (R.render(s, wl.cams, ST, want_margin=False)[0] for s in (s1, s2, s3))
    for k in ("rgb", "feat"):
        assert np.allclose(o3[k], 0.3 * o1[k] - 1.7 * o2[k], atol=1e-12)


def test_textbook_sum_of_gaussians_at_low_opacity():
    """Special case reducing to a textbook formula: with the cuts removed and
    all opacities ~1e-3, T ~ 1 and Y equals sum_i o_i y_i N(u; mu'_i,
    Sigma'_i) 2 pi sqrt(det Sigma'_i) (scipy's normal pdf) within the bound
    (sum alpha)^2 max|y| of the first-order expansion."""
    cam = posed_camera(9, W=24, H=18, f=30.0)
    sc = scene_in_view(9, cam, 15, logit=(-6.9, 0.01))
    st = R.Settings(alpha_min=0.0, cutoff2=1e30)
    o = R.render(sc, [cam], st, want_margin=False)[0]
    Y = np.zeros((20, cam.height, cam.width))
    jj, ii = np.mgrid[0:cam.height, 0:cam.width]
    pts = np.stack([ii.ravel(), jj.ravel()], 1).astype(float)
    asum = np.zeros(pts.shape[0])
    for g in range(sc.n):
        a, b, c = o["cov2d"][g]
        cov = np.array([[a, b], [b, c]])
        G = multivariate_normal(mean=o["mu"][g], cov=cov).pdf(pts) * 2 * math.pi * math.sqrt(np.linalg.det(cov))
        al = o["opac"][g] * G
        asum += al
        y = np.concatenate([sc.rgb[g], [o["z"][g]], sc.feat[g]])
        Y += (al[:, None] * y[None, :]).T.reshape(20, cam.height, cam.width)
    got = np.concatenate([o["rgb"], o["depth"][None], o["feat"]], 0)
    ymax = max(np.abs(sc.rgb).max(), np.abs(o["z"]).max(), np.abs(sc.feat).max())
    bound = (asum ** 2).reshape(cam.height, cam.width) * ymax + 1e-15
    assert asum.max() > 1e-4
    assert np.all(np.abs(got - Y) <= bound[None])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_vectorised_matches_brute_force(seed):
    """Brute force (independent pure-Python transcription, every pixel x
    every Gaussian, sorted()) equals the vectorised oracle: RGB, depth,
    feature, T and the contributor counts, on tiny scenes at posed cameras,
    for several block sizes of the vectorised evaluation."""
    cam = posed_camera(seed, W=19, H=13, f=22.0)
    sc = scene_in_view(seed, cam, 10 + 4 * seed, ls=(-1.8, 0.5))
    Yb, Tb, nb, _ = brute.render_view(sc, cam, ST)
    Yb = np.array(Yb).transpose(2, 0, 1)
    for block in (4, 16):
        o = R.render(sc, [cam], ST, block=block)[0]
        got = np.concatenate([o["rgb"], o["depth"][None], o["feat"]], 0)
        assert np.allclose(got, Yb, rtol=1e-12, atol=1e-13)
        assert np.allclose(o["T"], np.array(Tb), rtol=1e-12, atol=1e-14)
        assert np.array_equal(o["n"], np.array(nb))
    assert np.array(nb).max() >= 3


# --------------------------------------------------------------------------
# Gradients (O13)
# --------------------------------------------------------------------------
def _richardson(vals, h):
    """Central differences with steps h and h/2 (values at +h, -h, +h/2,
    -h/2), combined by Richardson extrapolation (error O(h^4))."""
    d1 = (vals[0] - vals[1]) / (2 * h)
    d2 = (vals[2] - vals[3]) / h
    return (4 * d2 - d1) / 3


def _fd_check(sc, cams, up, upT, h=1e-4, tol=2e-6, params=None):
    G = R.vjp(sc, cams, up, ST, upstream_T=upT)
    f = lambda s, xis=None: brute.loss_weighted(s, cams, ST, up, upT, xis)
    _, sig0 = f(sc)
    checked = excluded = 0
    for key in params or ("means", "log_scales", "quats", "logits", "rgb", "feat"):
        arr = np.asarray(getattr(sc, key), np.float64)
        for idx in np.ndindex(arr.shape):
            vals = []
            same = True
            for s in (2, -2, 1, -1):
                a2 = arr.copy()
                a2[idx] += s * h / 2
                s2 = copy.copy(sc)
                setattr(s2, key, a2)
                v, sg = f(s2)
                vals.append(v)
                same &= sg == sig0
            if not same:
                excluded += 1
                continue
            fd = _richardson(vals, h)
            ad = G[key].reshape(arr.shape)[idx]
            assert abs(fd - ad) <= tol * max(1.0, abs(ad)), (key, idx, fd, ad)
            checked += 1
    for vi in range(len(cams)):
        for k in range(6):
            vals = []
            same = True
            for s in (2, -2, 1, -1):
                xis = [(0.0,) * 6 for _ in cams]
                xi = [0.0] * 6
                xi[k] = s * h / 2
                xis[vi] = tuple(xi)
                v, sg = f(sc, xis)
                vals.append(v)
                same &= sg == sig0
            if not same:
                excluded += 1
                continue
            fd = _richardson(vals, h)
            ad = G["twist"][vi][k]
            assert abs(fd - ad) <= tol * max(1.0, abs(ad)), ("twist", vi, k, fd, ad)
            checked += 1
    return checked, excluded


@pytest.mark.parametrize("seed", [0, 1])
def test_autodiff_vs_central_fd_of_brute_force(seed):
    """Finite differences (h = 1e-4, FP64, on the independent brute force)
    against the oracle's autodiff gradient for every parameter and the pose
    twist, with an upstream gradient on Y and on T; parameters whose +-h
    evaluations change a discrete decision are dropped (and counted)."""
    cam = posed_camera(10 + seed, W=14, H=11, f=18.0)
    sc = scene_in_view(10 + seed, cam, 5, ls=(-1.7, 0.4))
    up = scenes.random_upstream(seed, [cam])
    upT = [np.random.default_rng(seed).normal(size=(cam.height, cam.width))]
    checked, excluded = _fd_check(sc, [cam], up, upT)
    assert checked >= 0.9 * (5 * 30 + 6)
    assert excluded <= 0.1 * (5 * 30 + 6)


def test_autodiff_vs_fd_two_views_and_clamp():
    """FD pin with two views (twist per view, parameter gradients summed over
    views) and one Gaussian whose Jacobian clamp is active, one whose alpha is
    clamped at 0.99."""
    cam1 = posed_camera(21, W=12, H=10, f=16.0)
    cam2 = posed_camera(22, W=10, H=9, f=14.0)
    sc = scene_in_view(21, cam1, 4, ls=(-1.6, 0.3))
    sc.logits[0] = 6.0                                    # alpha clamped near its centre
    up = scenes.random_upstream(5, [cam1, cam2])
    checked, excluded = _fd_check(sc, [cam1, cam2], up, None)
    assert checked >= 100


def test_gradient_invariants():
    """Invariants of the exact gradient: <dL/dq_i, q_i> = 0 (q is used only
    through q/|q|) and dL/drho = R_cw sum_i dL/dp_i (moving every Gaussian by
    d in the world equals moving the camera by R_cw d)."""
    wl = scenes.make_workload(2, n=3000, res_scale=0.1)
    sc = wl.scene
    cam = wl.cams[0]
    up = scenes.random_upstream(1, wl.cams)
    G = R.vjp(sc, wl.cams, up, ST)
    dots = np.einsum("ij,ij->i", G["quats"], np.asarray(sc.quats, np.float64))
    assert np.abs(dots).max() <= 1e-9 * max(1.0, np.abs(G["quats"]).max())
    assert np.abs(G["quats"]).max() > 0
    lhs = G["twist"][0][:3]
    rhs = np.asarray(cam.R_cw, np.float64) @ G["means"].sum(0)
    assert np.allclose(lhs, rhs, rtol=1e-7, atol=1e-9 * np.abs(rhs).max())


def test_opacity_derivative_closed_form():
    """Closed form: for one unclamped Gaussian, dY_c/dlambda at a pixel is
    G y_c o (1 - o)."""
    cam = one_view(11, 9, 20.0)
    z, ls, logit = 2.0, -2.0, -0.3
    y = [0.3, 0.7, 0.1]
    sc = make_scene([[0.01, -0.02, z]], [[ls] * 3], [[1, 0, 0, 0]], [logit], [y], [[0.5] * 16])
    i, j = 6, 5
    up = [np.zeros((20, 9, 11))]
    up[0][1, j, i] = 1.0
    G = R.vjp(sc, [cam], up, ST)
    o = R.render(sc, [cam], ST)[0]
    op = o["opac"][0]
    dx, dy = i - o["mu"][0][0], j - o["mu"][0][1]
    qa, qb, qc = o["conic"][0]
    Gv = math.exp(-0.5 * (qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy))
    assert math.isclose(G["logits"][0], Gv * y[1] * op * (1 - op), rel_tol=1e-12)


def test_l1_loss_gradient_vs_fd():
    """The L1 upstream (Eq. (1) without D-SSIM, each term a mean over its
    elements, sign(0) = 0) composed with the renderer, against central FD of
    the loss computed on the brute-force render."""
    wl = scenes.tiny_scene(4, 5, 12, 10)
    wl.loss_w = (1.0, 0.1, 1.0)
    outs, L, G = R.loss_and_grads(wl.scene, wl.cams, wl.targets, wl.loss_w)

    def loss(sc):
        Y, T, n, sig = brute.render_view(sc, wl.cams[0], ST)
        Y = np.array(Y).transpose(2, 0, 1)
        t = wl.targets[0]
        return (wl.loss_w[0] * np.abs(Y[:3] - t.rgb).mean() + wl.loss_w[1] * np.abs(Y[3] - t.depth).mean()
                + wl.loss_w[2] * np.abs(Y[4:] - t.feat).mean()), sig
    L0, sig0 = loss(wl.scene)
    assert math.isclose(L, L0, rel_tol=1e-12)
    h = 1e-6
    n_ok = 0
    for key in ("means", "logits", "feat"):
        arr = np.asarray(getattr(wl.scene, key), np.float64)
        for idx in list(np.ndindex(arr.shape))[:12]:
            vs = []
            same = True
            for s in (1, -1):
                a2 = arr.copy()
                a2[idx] += s * h
                s2 = copy.copy(wl.scene)
                setattr(s2, key, a2)
                v, sg = loss(s2)
                vs.append(v)
                same &= sg == sig0
            if not same:
                continue
            fd = (vs[0] - vs[1]) / (2 * h)
            assert abs(fd - G[key].reshape(arr.shape)[idx]) <= 1e-6 * max(1e-3, abs(fd)), (key, idx)
            n_ok += 1
    assert n_ok >= 20


def test_margin_flags_threshold_pixels():
    """The decision margin is tiny exactly where a pixel sits on a cut:
    placing a Gaussian so that a pixel is at m2 = 9 (to 1e-9) makes that
    pixel's margin < 1e-6, while a generic pixel's margin is larger."""
    z, ls = 2.0, -1.5
    s2 = (20.0 * math.exp(ls) / z) ** 2 + ST.eps2d
    r = 3.0 * math.sqrt(s2)                   # pixel (10 + r, 10) sits on the cut
    shift = 10 + r - round(10 + r)
    cam = one_view(21, 21, 20.0, cx=10.0 - shift, cy=10.0)   # on-axis: isotropic Sigma'
    sc = make_scene([[0, 0, z]], [[ls] * 3], [[1, 0, 0, 0]], [3.0], [[1, 1, 1]], [[0] * 16])
    o = R.render(sc, [cam], ST)[0]
    px = int(round(10 + r))
    assert o["margin"]["m2"][10, px] < 1e-6
    assert o["margin"]["m2"][10, 10] > 1e-3
    assert o["margin"]["m2"][10, px - 2] > 1e-3


def test_margin_flags_depth_near_ties():
    """Two contributors of a pixel 1e-12 apart in depth give a depth-order
    margin ~1e-12 there; 0.5 apart they give ~0.3."""
    cam = one_view(9, 9, 10.0)
    for dz, lo, hi in [(1e-12, 0.0, 1e-11), (0.5, 0.1, 1.0)]:
        sc = make_scene([[0, 0, 2.0], [0, 0, 2.0 + dz]], [[-1.0] * 3] * 2, [[1, 0, 0, 0]] * 2,
                        [0.0, 0.0], [[1, 0, 0], [0, 1, 0]], [[0] * 16] * 2)
        o = R.render(sc, [cam], ST)[0]
        assert o["n"][4, 4] == 2
        assert lo <= o["margin"]["z"][4, 4] <= hi


def _with_feat(sc, feat):
    return scenes.Scene(sc.means, sc.log_scales, sc.quats, sc.logits, sc.rgb, np.ascontiguousarray(feat, np.float32),
                        "f32")


def test_feature_dimension_is_a_set_of_independent_groups():
    # The feature channels do not enter the blend weights: a 32-d render is
    # the two 16-d renders of its halves side by side, and its gradient is
    # the sum over the halves (the second half carrying no colour or depth
    # upstream).  An 8-d render is a 16-d render with the last 8 channels 0.
    wl = scenes.tiny_scene(3, 24, 20, 16)
    cams, sc = wl.cams, wl.scene
    rng = np.random.Generator(np.random.PCG64(77))
    f32 = rng.normal(size=(sc.n, 32)).astype(np.float32)
    full = R.render(_with_feat(sc, f32), cams, want_margin=False)[0]
    a = R.render(_with_feat(sc, f32[:, :16]), cams, want_margin=False)[0]
    b = R.render(_with_feat(sc, f32[:, 16:]), cams, want_margin=False)[0]
    for k in ("rgb", "depth", "T"):
        assert np.array_equal(full[k], a[k]) and np.array_equal(full[k], b[k])
    assert np.array_equal(full["feat"], np.concatenate([a["feat"], b["feat"]], 0))
    up = rng.normal(size=(36, 16, 20))
    g = R.vjp(_with_feat(sc, f32), cams, [up])
    ua = up[:20].copy()
    ub = np.concatenate([np.zeros((4, 16, 20)), up[20:]], 0)
    ga = R.vjp(_with_feat(sc, f32[:, :16]), cams, [ua])
    gb = R.vjp(_with_feat(sc, f32[:, 16:]), cams, [ub])
    for k in ("means", "log_scales", "quats", "logits", "twist"):
        assert np.allclose(g[k], ga[k] + gb[k], rtol=1e-12, atol=1e-14), k
    assert np.allclose(g["rgb"], ga["rgb"], rtol=1e-12, atol=1e-15)
    assert np.allclose(g["feat"], np.concatenate([ga["feat"], gb["feat"]], 1), rtol=1e-12, atol=1e-15)
    f8 = f32[:, :8]
    r8 = R.render(_with_feat(sc, f8), cams, want_margin=False)[0]
    r16 = R.render(_with_feat(sc, np.concatenate([f8, np.zeros((sc.n, 8), np.float32)], 1)), cams,
                   want_margin=False)[0]
    assert np.array_equal(r8["feat"], r16["feat"][:8]) and not r16["feat"][8:].any()
