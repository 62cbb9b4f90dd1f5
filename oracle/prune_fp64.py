"""Plain FP64 definition of language-guided Gaussian pruning.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product never
imports this file.

Definition followed (Sec. III-D, Eq. (4)): each Gaussian G_i is checked
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
          max_scale=0.3, extra=48, want_margins=False):
    """means [N,3], feat [N,D], logits [N], log_scales [N,3] (any float
    dtype).  Returns (semantic [N] bool, geometric [N] bool) and, with
    want_margins, per Gaussian i the smallest relative margin of any decision
    it takes (distance vs tau_dist, the K-th / (K+1)-th distance order,
    similarity vs tau_sim)."""
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
    q = min(len(idx), k + 1 + extra)
    dist, nb = tree.query(P[idx], k=q, distance_upper_bound=tau_dist * 1.001)
    nb = np.where(np.isfinite(dist), nb, len(idx))
    if q == k + 1 + extra and np.isfinite(dist[:, -1]).any():
        raise RuntimeError("neighbour query saturated: raise `extra`")
    tau2 = tau_dist * tau_dist
    norm = np.sqrt((Fe * Fe).sum(1))
    for r, i in enumerate(idx):
        cand = nb[r][nb[r] < len(idx)]
        js = idx[cand]
        js = js[js != i]
        if len(js) == 0:
            continue
        d = P[js] - P[i]
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        if want_margins:
            margin[i] = min(margin[i], np.min(np.abs(d2 - tau2)) / tau2)
        keep = d2 < tau2
        js, d2 = js[keep], d2[keep]
        order = np.lexsort((js, d2))
        js, d2 = js[order], d2[order]
        if want_margins and len(d2) > k:
            margin[i] = min(margin[i], (d2[k] - d2[k - 1]) / tau2)
        js = js[:k]
        den = norm[i] * norm[js]
        sim = np.where(den > 0, (Fe[js] @ Fe[i]) / np.where(den > 0, den, 1.0), 0.0)
        if want_margins:
            margin[i] = min(margin[i], np.min(np.abs(sim - tau_sim)))
        dom = (lam[i] > lam[js]) | ((lam[i] == lam[js]) & (i < js))
        sem[js[(sim > tau_sim) & dom]] = True
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
