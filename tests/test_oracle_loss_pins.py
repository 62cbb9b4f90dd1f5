"""Pins of the FP64 loss oracle (D-SSIM + L1 terms of Eq. (1)), CPU only.

Each test fixes part of ``oracle.loss_fp64`` against something other than
itself: a library routine (the window and the zero-padded local mean against
scipy), closed forms (constant images, where every local statistic is a
known multiple of the window mass inside the image), an invariant
(SSIM(X, X) = 1, so the D-SSIM gradient vanishes there), a pure-Python brute
force, and central finite differences of the loss.
"""
import numpy as np
import pytest
import torch
from scipy import ndimage
from scipy.signal import windows as sw

from oracle import loss_fp64 as LF
from oracle import raster_fp64 as R
from scenes import Targets


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_window_matches_scipy_gaussian():
    g = sw.gaussian(11, std=1.5)
    w2 = np.outer(g, g) / np.outer(g, g).sum()
    assert np.allclose(LF.gaussian_window(), w2, rtol=0, atol=1e-16)
    assert abs(LF.gaussian_window().sum() - 1.0) < 1e-15


def test_local_mean_is_zero_padded_gaussian_filter():
    # a non-square image with structure along one axis only: a transposed
    # window or image, or a different border rule, changes the result
    img = _rng(1).uniform(size=(2, 13, 23))
    img[1] = np.linspace(0, 1, 23)[None, :] ** 2
    win = torch.as_tensor(LF.gaussian_window())
    ours = LF._local_mean(torch.as_tensor(img), win).numpy()
    for c in range(2):
        ref = ndimage.gaussian_filter(img[c], sigma=1.5, truncate=5 / 1.5, mode="constant", cval=0.0)
        assert np.allclose(ours[c], ref, rtol=0, atol=1e-14)


def _mass_1d(n):
    """Window mass inside [0, n) for each position: sum of the normalised
    1-D weights of the taps that land in range."""
    g = sw.gaussian(11, std=1.5)
    g = g / g.sum()
    return np.array([sum(g[k + 5] for k in range(-5, 6) if 0 <= i + k < n) for i in range(n)])


@pytest.mark.parametrize("a,b", [(0.7, 0.7), (0.8, 0.3), (0.05, 0.9)])
def test_ssim_constant_images_closed_form(a, b):
    # X = a and Y = b everywhere: with window mass s inside the image,
    # mu_x = a s, E[X^2] = a^2 s, so var_x = a^2 s (1 - s), cov = a b s (1 - s)
    H, W = 9, 14
    s = np.outer(_mass_1d(H), _mass_1d(W))
    num = (2 * a * b * s * s + LF.SSIM_C1) * (2 * a * b * s * (1 - s) + LF.SSIM_C2)
    den = ((a * a + b * b) * s * s + LF.SSIM_C1) * ((a * a + b * b) * s * (1 - s) + LF.SSIM_C2)
    X = torch.full((1, H, W), a, dtype=torch.float64)
    Y = torch.full((1, H, W), b, dtype=torch.float64)
    S = LF.ssim_map(X, Y)[0].numpy()
    assert np.allclose(S, num / den, rtol=1e-12, atol=0)
    # interior pixels (window fully inside): the textbook luminance term
    Xb = torch.full((1, 12, 12), a, dtype=torch.float64)
    Yb = torch.full((1, 12, 12), b, dtype=torch.float64)
    Sb = LF.ssim_map(Xb, Yb)[0].numpy()
    assert np.allclose(Sb[5:7, 5:7], (2 * a * b + LF.SSIM_C1) / (a * a + b * b + LF.SSIM_C1), rtol=1e-12)


def test_ssim_of_an_image_with_itself_is_one():
    X = torch.as_tensor(_rng(2).uniform(size=(3, 17, 11)))
    assert np.allclose(LF.ssim_map(X, X).numpy(), 1.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed,shape", [(3, (2, 7, 9)), (4, (1, 3, 2)), (5, (1, 12, 4))])
def test_ssim_vectorised_matches_brute_force(seed, shape):
    rng = _rng(seed)
    X = rng.uniform(size=shape)
    Y = np.clip(X + rng.normal(0, 0.2, size=shape), 0, 1)
    ours = LF.ssim_map(torch.as_tensor(X), torch.as_tensor(Y)).numpy()
    assert np.allclose(ours, LF.ssim_brute(X, Y), rtol=0, atol=1e-13)


def _tiny_views(seed, sizes):
    rng = _rng(seed)
    outs, tgts = [], []
    for (W, H) in sizes:
        t = Targets(rng.uniform(size=(3, H, W)), rng.uniform(1, 3, size=(H, W)), rng.normal(size=(16, H, W)))
        o = {"rgb": np.clip(t.rgb + rng.normal(0, 0.15, size=t.rgb.shape), 0, 1),
             "depth": t.depth + rng.normal(0, 0.3, size=t.depth.shape),
             "feat": t.feat + rng.normal(0, 0.3, size=t.feat.shape)}
        outs.append(o)
        tgts.append(t)
    return outs, tgts


def test_loss_gradient_vs_central_fd():
    outs, tgts = _tiny_views(6, [(9, 7), (5, 12)])
    w = (1.0, 0.5, 0.8)
    L, terms, ups = LF.loss_and_upstream(outs, tgts, w, lam=0.3)
    assert abs(L - sum(w[0] * (0.7 * t[0] + 0.3 * t[1]) + w[1] * t[2] + w[2] * t[3] for t in terms)) < 1e-14
    rng = _rng(7)
    h = 1e-6
    for v in range(2):
        for k, lo, n in (("rgb", 0, 3), ("depth", 3, 1), ("feat", 4, 16)):
            for _ in range(6):
                H, W = outs[v]["depth"].shape
                c, i, j = rng.integers(n), rng.integers(H), rng.integers(W)
                base = outs[v][k]
                idx = (c, i, j) if base.ndim == 3 else (i, j)
                tv = getattr(tgts[v], k)[idx]
                if abs(base[idx] - tv) < 1e-3:       # away from the |x| kink
                    continue
                vals = []
                for sgn in (1, -1):
                    o2 = [dict(o) for o in outs]
                    o2[v] = dict(o2[v])
                    o2[v][k] = base.copy()
                    o2[v][k][idx] += sgn * h
                    vals.append(LF.loss_and_upstream(o2, tgts, w, lam=0.3)[0])
                fd = (vals[0] - vals[1]) / (2 * h)
                ad = ups[v][lo + (c if base.ndim == 3 else 0), i, j]
                assert abs(fd - ad) <= 1e-7 * max(1.0, abs(ad)) + 1e-9, (v, k, idx, fd, ad)


def test_dssim_gradient_vanishes_at_the_target():
    outs, tgts = _tiny_views(8, [(11, 6)])
    outs[0]["rgb"] = tgts[0].rgb.copy()
    L, terms, ups = LF.loss_and_upstream(outs, tgts, (1.0, 0.0, 0.0), lam=1.0)
    assert abs(terms[0][1]) < 1e-13 and abs(L) < 1e-13
    assert np.abs(ups[0][:3]).max() < 1e-12


def test_lambda_zero_is_the_l1_loss():
    outs, tgts = _tiny_views(9, [(6, 5), (8, 8)])
    w = (1.0, 0.7, 1.3)
    L, terms, ups = LF.loss_and_upstream(outs, tgts, w, lam=0.0)
    assert abs(L - R.l1_loss(outs, tgts, w)) < 1e-13
    for a, b in zip(ups, R.l1_upstream(outs, tgts, w)):
        assert np.allclose(a, b, rtol=0, atol=1e-15)
