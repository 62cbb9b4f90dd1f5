"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
(``paper_2511_16144_amd``) and the FP64 oracle on the same seeded inputs, and
compare them per channel group.

Metrics (per group: RGB, depth, feature, T; per gradient group):
    rel_L2  = ||X - R||_2 / ||R||_2
    rel_max = max|X - R| / max|R|
over the pixels (Gaussians) that are not ambiguous.  A pixel is ambiguous when
one of its discrete decisions sits closer to its threshold than FP32 can
resolve (the oracle reports each decision's relative margin); a Gaussian is
ambiguous when its cut-off box covers an ambiguous pixel.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import scenes

# relative margins under which FP32 and FP64 may legitimately take different
# branches (see the oracle's composite(): m2 cut, alpha cut, alpha clamp,
# termination, depth order).  The GPU's depth sort key keeps 28 mantissa bits
# of the FP64 depth, so contributors closer than 2^-28 (3.7e-9) relative keep
# index order there: the depth margin is 1e-8.
AMBIG = {"m2": 2e-5, "alpha": 2e-5, "clamp": 2e-5, "T": 5e-5, "z": 1e-8}

TOL_F32 = 1e-4     # FP32 path vs FP64 oracle on the same inputs
TOL_BF16 = 1e-2    # BF16-stored appearance vs the oracle on unrounded inputs


def mask_upstream(ups, ambs):
    """Zero the upstream gradient at ambiguous pixels (per view), so the
    gradient comparison can include every Gaussian: a pixel with zero upstream
    contributes nothing to any gradient, whichever branch it took."""
    out = []
    for u, a in zip(ups, ambs):
        u = np.array(u, np.float32, copy=True)
        u[:, a] = 0.0
        out.append(u)
    return out


def ambiguous(margin: dict) -> np.ndarray:
    m = np.zeros_like(margin["m2"], dtype=bool)
    for k, thr in AMBIG.items():
        m |= margin[k] < thr
    return m


def gpu_params(scene, device="cuda"):
    import paper_2511_16144_amd as P
    dt = torch.bfloat16 if scene.dtype == "bf16" else torch.float32
    return P.params_from_arrays(scene.means, scene.log_scales, scene.quats, scene.logits,
                                scene.rgb, scene.feat, device=device, appearance_dtype=dt)


def to_np(outs):
    return [{k: v.detach().float().cpu().numpy() if v.dtype != torch.int32 else v.cpu().numpy()
             for k, v in o.items()} for o in outs]


def rel_err(x, r, mask=None):
    x = np.asarray(x, np.float64)
    r = np.asarray(r, np.float64)
    if mask is not None:
        x = x[..., mask] if x.ndim > mask.ndim else x[mask]
        r = r[..., mask] if r.ndim > mask.ndim else r[mask]
    d = x - r
    nr = np.linalg.norm(r.ravel())
    mr = np.abs(r).max() if r.size else 0.0
    l2 = np.linalg.norm(d.ravel()) / nr if nr > 0 else np.linalg.norm(d.ravel())
    mx = np.abs(d).max() / mr if (r.size and mr > 0) else (np.abs(d).max() if d.size else 0.0)
    return float(l2), float(mx)


def forward_errors(gpu_out, ref_out, amb):
    keep = ~amb
    res = {}
    for k in ("rgb", "depth", "feat", "T"):
        res[k] = rel_err(gpu_out[k], ref_out[k], keep)
    return res


def gaussian_ambiguity(ref_out, amb, n):
    """Gaussians whose 3-sigma box (one pixel margin) covers an ambiguous
    pixel of this view."""
    bad = np.zeros(n, bool)
    ys, xs = np.nonzero(amb)
    if len(xs) == 0:
        return bad
    mu, cov, vis = ref_out["mu"], ref_out["cov2d"], ref_out["vis"]
    rx = 3.0 * np.sqrt(np.maximum(cov[:, 0], 0)) + 1.0
    ry = 3.0 * np.sqrt(np.maximum(cov[:, 2], 0)) + 1.0
    idx = np.nonzero(vis)[0]
    for g in idx:
        hit = (np.abs(xs - mu[g, 0]) <= rx[g]) & (np.abs(ys - mu[g, 1]) <= ry[g])
        if hit.any():
            bad[g] = True
    return bad


def grad_errors(gpu_g, ref_g, bad):
    keep = ~bad
    out = {}
    for k in ("means", "log_scales", "quats", "logits", "rgb", "feat"):
        gk = np.asarray(gpu_g[k], np.float64)
        gk = gk.T if gk.ndim == 2 else gk           # device SoA [k, N] -> [N, k]
        rk = np.asarray(ref_g[k], np.float64)
        out[k] = rel_err(gk[keep], rk[keep])
    out["twist"] = rel_err(gpu_g["twist"], ref_g["twist"])
    return out


def grads_np(g):
    return {k: v.detach().float().cpu().numpy() for k, v in g.items()}


def upstream_tensors(ups, device="cuda"):
    out = []
    for u in ups:
        t = torch.as_tensor(np.asarray(u, np.float32)).to(device)
        out.append({"rgb": t[:3].contiguous(), "depth": t[3].contiguous(), "feat": t[4:].contiguous()})
    return out


def fmt(res):
    return ", ".join(f"{k}: L2 {v[0]:.2e} max {v[1]:.2e}" for k, v in res.items())


def separate_targets(ref_outs, targets, delta=1e-4):
    """Targets moved at least `delta` away from the oracle's rendered values
    wherever they come closer (the kink of the L1 terms), so that every
    residual has the same sign in the FP32 render and the FP64 one outside
    ambiguous pixels.  Built from the oracle's images only."""
    from scenes import Targets
    out = []
    for o, t in zip(ref_outs, targets):
        d = {}
        for k in ("rgb", "depth", "feat"):
            r = np.asarray(o[k], np.float64)
            v = np.asarray(getattr(t, k), np.float64).copy()
            close = np.abs(v - r) < delta
            v[close] = r[close] + np.where(v[close] >= r[close], 2 * delta, -2 * delta)
            d[k] = v.astype(np.float32)
        out.append(Targets(d["rgb"], d["depth"], d["feat"]))
    return out


def dilate(mask, r):
    """Pixels within r (Chebyshev distance) of a set pixel: the reach of a
    (2r+1)-wide window."""
    from scipy import ndimage
    if not mask.any():
        return mask.copy()
    return ndimage.binary_dilation(mask, structure=np.ones((2 * r + 1, 2 * r + 1), bool))


def separate_decoder_targets(Z_fn, G, delta=2e-3, bf16=True, chunk=1 << 16):
    """Decoder targets moved at least `delta` away from the oracle's decoded
    values Z (Z_fn(s, e) returns the oracle's Z for pixels [s, e) as
    [C, e - s] float64), then rounded to BF16 when `bf16`, so that every
    sign(Z - F_gt) is the same in the matrix-core product and in FP64.
    Built from the oracle's values only."""
    C = G.shape[0]
    Gf = G.reshape(C, -1).astype(np.float32, copy=True)
    n = Gf.shape[1]
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        Z = Z_fn(s, e)
        g = Gf[:, s:e].astype(np.float64)
        if bf16:
            g = round_bf16_np(g)
        close = np.abs(g - Z) < delta
        sgn = np.where(g[close] >= Z[close], 1.0, -1.0)
        v = Z[close] + 3 * delta * sgn
        g[close] = round_bf16_np(v) if bf16 else v.astype(np.float32)
        Gf[:, s:e] = g
    return Gf.reshape(G.shape)


def round_bf16_np(x):
    """FP64/FP32 values rounded to BF16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32)
    r = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return r.view(np.float32).astype(np.float64)
