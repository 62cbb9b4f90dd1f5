"""Plain FP64 definition of the mapping loss with its D-SSIM term.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product never
imports this file.

Definition followed (Sec. III-B.3, Eq. (1): the total loss is the photometric
loss plus weighted depth and feature terms; the photometric loss combines an
L1 term and a D-SSIM term between the rendered and the observed image; the
depth term is an L1 loss).  The paper gives neither the weighting of the two
photometric terms nor the SSIM window; the readings (marked [reading]) are the
3D Gaussian Splatting conventions the paper builds on:

  L_rgb   = (1 - lam) mean|I - I*| + lam (1 - SSIM(I, I*))   [reading: lam = 0.2]
  SSIM    = mean over the 3 colour channels and every pixel of the SSIM map
            S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
            where mu, s^2, s_xy are local means, variances and the covariance
            under an 11 x 11 Gaussian window, sigma = 1.5, weights summing to 1
            [reading]; windows that reach past the border see zeros there
            (zero padding, no renormalisation) and the map has one value per
            pixel [reading]; C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1) [reading]
  L_depth = mean|D - D*|,  L_feat = mean|F - F*|  (the decoder of Eq. (2)
            is not on the path: the 16-d target map is compared directly)
  L_total = w_rgb L_rgb + w_depth L_depth + w_feat L_feat per view; the views
            of a batch sum their losses.

The gradient with respect to the rendered images is taken by torch.autograd
(the subgradient of |x| at 0 is 0).  The local statistics are written as
their definitions, E[XY] - E[X]E[Y], with the window applied by a plain 2-D
correlation.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as Fn

F64 = torch.float64

SSIM_RADIUS = 5          # 11 x 11 window [reading]
SSIM_SIGMA = 1.5         # [reading]
SSIM_C1 = 0.01 ** 2      # [reading]
SSIM_C2 = 0.03 ** 2      # [reading]
SSIM_LAMBDA = 0.2        # weight of D-SSIM inside L_rgb [reading]


def gaussian_window(radius: int = SSIM_RADIUS, sigma: float = SSIM_SIGMA) -> np.ndarray:
    """2-D window: outer product of the sampled 1-D Gaussian, normalised so
    that its 2r+1 by 2r+1 weights sum to 1."""
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _local_mean(img: torch.Tensor, win: torch.Tensor) -> torch.Tensor:
    """Window-weighted local mean of every channel of img [C, H, W], zero
    padding, same size."""
    C = img.shape[0]
    r = win.shape[0] // 2
    k = win.expand(C, 1, *win.shape)
    return Fn.conv2d(img[None], k, padding=r, groups=C)[0]


def ssim_map(X: torch.Tensor, Y: torch.Tensor, radius: int = SSIM_RADIUS, sigma: float = SSIM_SIGMA,
             C1: float = SSIM_C1, C2: float = SSIM_C2) -> torch.Tensor:
    """Per-channel, per-pixel SSIM of X against Y ([C, H, W] float64)."""
    win = torch.as_tensor(gaussian_window(radius, sigma), dtype=F64)
    mx, my = _local_mean(X, win), _local_mean(Y, win)
    vx = _local_mean(X * X, win) - mx * mx
    vy = _local_mean(Y * Y, win) - my * my
    cxy = _local_mean(X * Y, win) - mx * my
    return (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))


def view_terms(out: dict, tgt, lam: float):
    """The four per-view terms as torch scalars: mean|I - I*|, 1 - SSIM
    (None when lam = 0: not evaluated), mean|D - D*|, mean|F - F*|.  `out`
    holds torch tensors (rgb [3,H,W], depth [H,W], feat [D,H,W]); `tgt` has
    numpy arrays of the same shapes."""
    trgb = torch.as_tensor(np.asarray(tgt.rgb, np.float64))
    l1 = (out["rgb"] - trgb).abs().mean()
    ds = (1.0 - ssim_map(out["rgb"], trgb).mean()) if lam != 0.0 else None
    ld = (out["depth"] - torch.as_tensor(np.asarray(tgt.depth, np.float64))).abs().mean()
    lf = (out["feat"] - torch.as_tensor(np.asarray(tgt.feat, np.float64))).abs().mean()
    return l1, ds, ld, lf


def loss_and_upstream(outs, targets, loss_w, lam: float = SSIM_LAMBDA):
    """L_total summed over views, its per-view terms, and dL/dY per view as
    [4 + D, H, W] float64 arrays (RGB 3, depth 1, feature D).  `outs` are the
    rendered images (numpy, any float dtype), `targets` the observed ones."""
    L = torch.zeros((), dtype=F64)
    leaves, terms = [], []
    for o, t in zip(outs, targets):
        v = {k: torch.tensor(np.asarray(o[k], np.float64), requires_grad=True) for k in ("rgb", "depth", "feat")}
        l1, ds, ld, lf = view_terms(v, t, lam)
        lrgb = (1.0 - lam) * l1 + (lam * ds if ds is not None else 0.0)
        L = L + loss_w[0] * lrgb + loss_w[1] * ld + loss_w[2] * lf
        leaves.append(v)
        terms.append([float(x.detach()) if x is not None else 0.0 for x in (l1, ds, ld, lf)])
    grads = torch.autograd.grad(L, [x for v in leaves for x in (v["rgb"], v["depth"], v["feat"])],
                                allow_unused=True) if leaves else []
    ups = []
    for i, v in enumerate(leaves):
        gr, gd, gf = (g if g is not None else torch.zeros_like(x)
                      for g, x in zip(grads[3 * i:3 * i + 3], (v["rgb"], v["depth"], v["feat"])))
        ups.append(torch.cat([gr, gd[None], gf], 0).numpy())
    return float(L.detach()), terms, ups


def ssim_brute(X: np.ndarray, Y: np.ndarray, radius: int = SSIM_RADIUS, sigma: float = SSIM_SIGMA,
               C1: float = SSIM_C1, C2: float = SSIM_C2) -> np.ndarray:
    """SSIM map by explicit loops over pixels and window taps (math module
    only), for tiny images: a second route to ``ssim_map``."""
    C, H, W = X.shape
    w1 = [math.exp(-(k * k) / (2.0 * sigma * sigma)) for k in range(-radius, radius + 1)]
    s = sum(w1)
    w1 = [v / s for v in w1]
    out = np.zeros((C, H, W))
    for c in range(C):
        for i in range(H):
            for j in range(W):
                m = [0.0] * 5
                for a in range(-radius, radius + 1):
                    for b in range(-radius, radius + 1):
                        ii, jj = i + a, j + b
                        if 0 <= ii < H and 0 <= jj < W:
                            wt = w1[a + radius] * w1[b + radius]
                            x, y = float(X[c, ii, jj]), float(Y[c, ii, jj])
                            m[0] += wt * x
                            m[1] += wt * y
                            m[2] += wt * x * x
                            m[3] += wt * y * y
                            m[4] += wt * x * y
                vx, vy, cxy = m[2] - m[0] ** 2, m[3] - m[1] ** 2, m[4] - m[0] * m[1]
                out[c, i, j] = ((2 * m[0] * m[1] + C1) * (2 * cxy + C2)) / \
                    ((m[0] ** 2 + m[1] ** 2 + C1) * (vx + vy + C2))
    return out
