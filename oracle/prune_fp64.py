"""Plain FP64 definition of language-guided Gaussian pruning.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product never
imports this file.

Definition followed (Sec. III-C, Eq. (4)): each Gaussian G_i is checked
against its K nearest neighbours in 3-D; a neighbour G_j is redundant when it
is closer than tau_dist and the cosine similarity of the two language
features exceeds tau_sim; the pruned set is the union of the redundant
Gaussians and those that fail the usual geometric criteria.  The paper
publishes neither K nor the thresholds, and does not say which member of a
mutually redundant pair survives; the readings (marked [reading]):

  neighbours   the K nearest other Gaussians by Euclidean distance of the
               means, ties by index [reading: K = 16]
  redundant j  some i has j among its K nearest, |p_i - p_j| < tau_dist,
               cos(f_i, f_j) > tau_sim (0 when either feature is zero), and
               i dominates j: opacity logit_i > logit_j, or equal logits and
               i < j, so that one Gaussian of a redundant pair survives
               [reading]
  geometric    opacity sigmoid(logit) < min_opacity, or the largest scale
               exp(max log_scale) > max_scale, or a non-finite mean, logit or
               log-scale [reading: 3DGS-style opacity / size pruning]

Distances and similarities are evaluated in FP64 (squared distance
dx^2 + dy^2 + dz^2 against tau_dist^2).  Candidate neighbours come from
scipy's k-d tree queried beyond the distance threshold (a superset); the
order and the tests are then applied to exact FP64 values here.  The
thresholds of the geometric test are compared in logit / log space:
logit < log(min_opacity / (1 - min_opacity)), max log_scale > log(max_scale).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

DEFAULTS = {"k": 16, "tau_dist": 0.02, "tau_sim": 0.9, "min_opacity": 0.005, "max_scale": 0.3}


def geometric(means, logits, log_scales, min_opacity, max_scale):
    """Boolean [N]: fails the geometric criteria (or is not finite)."""
    finite = np.isfinite(means).all(1) & np.isfinite(logits) & np.isfinite(log_scales).all(1)
    lthr = math.log(min_opacity / (1.0 - min_opacity))
    sthr = math.log(max_scale)
    with np.errstate(invalid="ignore"):
        g = (logits.astype(np.float64) < lthr) | (log_scales.astype(np.float64).max(1) > sthr)
    return ~finite | g


def prune(means, feat, logits, log_scales, k=16, tau_dist=0.02, tau_sim=0.9, min_opacity=0.005,
          max_scale=0.3, extra=48, want_margins=False, rows=1 << 16):
    """means [N,3], feat [N,D], logits [N], log_scales [N,3] (any float
    dtype).  Returns (semantic [N] bool, geometric [N] bool) and, with
    want_margins, per Gaussian i the smallest relative margin of any decision
    it takes (distance vs tau_dist, the K-th / (K+1)-th distance order,
    similarity vs tau_sim).  Rows are processed `rows` Gaussians at a time."""
    P = np.asarray(means, np.float64)
    Fe = np.asarray(feat, np.float64)
    lam = np.asarray(logits, np.float64)
    N = P.shape[0]
    geo = geometric(np.asarray(means), np.asarray(logits), np.asarray(log_scales), min_opacity, max_scale)
    sem = np.zeros(N, bool)
    margin = np.full(N, np.inf)
    part = np.isfinite(P).all(1)          # Gaussians with a finite mean take part in the neighbour search
    idx = np.nonzero(part)[0]
    if len(idx) < 2:
        return (sem, geo, margin) if want_margins else (sem, geo)
    tree = cKDTree(P[idx])
    tau2 = tau_dist * tau_dist
    norm = np.sqrt((Fe * Fe).sum(1))
    for r0 in range(0, len(idx), rows):
        ii = idx[r0:r0 + rows]
        q = min(len(idx), k + 1 + extra)
        while True:   # enough candidates to hold every neighbour within the threshold
            dist, nb = tree.query(P[ii], k=q, distance_upper_bound=tau_dist * 1.001)
            if q == len(idx) or not np.isfinite(dist[:, -1]).any():
                break
            q = min(len(idx), 2 * q)
        ok = np.isfinite(dist)
        js = np.where(ok, idx[np.minimum(nb, len(idx) - 1)], -1)
        ok &= js != ii[:, None]                                   # not itself
        d = P[np.maximum(js, 0)] - P[ii][:, None, :]
        d2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
        if want_margins:
            dm = np.where(ok, np.abs(d2 - tau2) / tau2, np.inf).min(1)
            margin[ii] = np.minimum(margin[ii], dm)
        ok &= d2 < tau2
        # order each row by (squared distance, index); invalid entries last
        key_d = np.where(ok, d2, np.inf)
        key_j = np.where(ok, js, np.iinfo(np.int64).max)
        order = np.lexsort((key_j, key_d), axis=1)
        key_d = np.take_along_axis(key_d, order, 1)
        js = np.take_along_axis(np.where(ok, js, -1), order, 1)
        if want_margins and dist.shape[1] > k:
            # an exact tie (equal squared distances, e.g. duplicate means) is
            # the same on both sides and broken by index; only a near tie is a
            # decision that rounding could flip
            with np.errstate(invalid="ignore"):
                gap = (key_d[:, k] - key_d[:, k - 1]) / tau2
            margin[ii] = np.minimum(margin[ii], np.where(np.isfinite(gap) & (gap > 0), gap, np.inf))
        js = js[:, :k]
        valid = js >= 0
        jj = np.maximum(js, 0)
        den = norm[ii][:, None] * norm[jj]
        dot = np.einsum("rkd,rd->rk", Fe[jj], Fe[ii])
        sim = np.where(den > 0, dot / np.where(den > 0, den, 1.0), 0.0)
        if want_margins:
            sm = np.where(valid, np.abs(sim - tau_sim), np.inf).min(1)
            margin[ii] = np.minimum(margin[ii], sm)
        li, lj = lam[ii][:, None], lam[jj]
        dom = (li > lj) | ((li == lj) & (ii[:, None] < jj))
        hit = valid & (sim > tau_sim) & dom
        sem[jj[hit]] = True
    return (sem, geo, margin) if want_margins else (sem, geo)


def prune_brute(means, feat, logits, log_scales, k=16, tau_dist=0.02, tau_sim=0.9, min_opacity=0.005,
                max_scale=0.3):
    """The same definition by a full distance matrix (small N): a second
    route to ``prune`` for the tests."""
    P = np.asarray(means, np.float64)
    Fe = np.asarray(feat, np.float64)
    lam = np.asarray(logits, np.float64)
    N = P.shape[0]
    geo = geometric(np.asarray(means), np.asarray(logits), np.asarray(log_scales), min_opacity, max_scale)
    sem = np.zeros(N, bool)
    part = np.isfinite(P).all(1)
    for i in range(N):
        if not part[i]:
            continue
        best = []
        for j in range(N):
            if j == i or not part[j]:
                continue
            d2 = sum((P[j, a] - P[i, a]) ** 2 for a in range(3))
            best.append((d2, j))
        best.sort()
        for d2, j in best[:k]:
            if not d2 < tau_dist * tau_dist:
                continue
            ni, nj = math.sqrt(float(Fe[i] @ Fe[i])), math.sqrt(float(Fe[j] @ Fe[j]))
            sim = float(Fe[i] @ Fe[j]) / (ni * nj) if ni * nj > 0 else 0.0
            dom = lam[i] > lam[j] or (lam[i] == lam[j] and i < j)
            if sim > tau_sim and dom:
                sem[j] = True
    return sem, geo
