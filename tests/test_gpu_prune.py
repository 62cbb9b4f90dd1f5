"""GPU parity of language-guided pruning (lgs_prune, through the C ABI)
against the FP64 pruning oracle: the mask is compared bit for bit (integer
work).  Both sides take every distance and similarity decision in FP64;
decisions closer to their threshold than 1e-9 (relative) could still round
differently, so the neighbours of a Gaussian with such a decision are left
out of the comparison (their number is printed; it is 0 for these inputs).

Cases: the hand-built configurations of the oracle's pins (a redundant
pair, both thresholds, the K-nearest limit, zero features, the geometric
criteria, non-finite Gaussians); seeded clustered scenes with duplicate
means and equal opacities for K = 1, 4, 16, 32 and FP32 / BF16 features;
the batched workload's 500k room-surface Gaussians with object-coherent
features; no Gaussian; one Gaussian; a mean out of the grid's range.
"""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import prune_fp64 as PR
from parity import gpu_params

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_16144_amd as P
    c = P.Context(0)
    yield c
    c.close()


def f32(x):
    return float(np.float32(x))


def make(P, F, lam, ls, bf16=False):
    n = len(P)
    sc = scenes.Scene(np.asarray(P, np.float32), np.asarray(ls, np.float32),
                      np.tile(np.float32([1, 0, 0, 0]), (n, 1)), np.asarray(lam, np.float32),
                      np.zeros((n, 3), np.float32),
                      scenes.round_bf16(np.asarray(F, np.float32)) if bf16 else np.asarray(F, np.float32),
                      "bf16" if bf16 else "f32")
    return sc


def run_both(ctx, sc, k=16, tau_dist=0.02, tau_sim=0.9, min_opacity=0.005, max_scale=0.3):
    prm = dict(k=k, tau_dist=f32(tau_dist), tau_sim=f32(tau_sim), min_opacity=f32(min_opacity),
               max_scale=f32(max_scale))
    mask, counts = ctx.prune(gpu_params(sc), **prm)
    torch.cuda.synchronize()
    m = mask.cpu().numpy()
    sem, geo, margin = PR.prune(sc.means, sc.feat, sc.logits, sc.log_scales, want_margins=True, **prm)
    return m, counts, sem, geo, margin


def check(label, sc, m, counts, sem, geo, margin, tau_dist=0.02):
    amb = np.nonzero(margin < 1e-9)[0]
    keep = np.ones(sc.n, bool)
    if len(amb):
        P = sc.means.astype(np.float64)
        for i in amb:
            keep &= ~(((P - P[i]) ** 2).sum(1) < (1.5 * tau_dist) ** 2)
    exp = sem.astype(np.uint8) | (geo.astype(np.uint8) << 1)
    bad = np.nonzero((m != exp) & keep)[0]
    say(f"  {label}: n={sc.n} redundant {int(sem.sum())} geometric {int(geo.sum())} "
        f"ambiguous {len(amb)}; gpu counts {counts}; mismatches {len(bad)}")
    assert len(bad) == 0, (label, bad[:10], m[bad[:10]], exp[bad[:10]])
    if len(amb) == 0:
        assert counts == (int(sem.sum()), int(geo.sum()), int((sem | geo).sum()))


def test_hand_built_configurations(ctx):
    f = np.arange(1, 17, dtype=np.float64)
    f /= np.linalg.norm(f)
    # redundant pair (the less opaque one is marked), a far point
    sc = make([[0, 0, 0], [0.005, 0, 0], [1, 1, 1]], [f, f, f], [0.2, 1.5, 0.0], np.full((3, 3), -4.0))
    m, c, sem, geo, mg = run_both(ctx, sc)
    assert m.tolist() == [1, 0, 0]
    check("pair", sc, m, c, sem, geo, mg)
    # the K-nearest limit: a dominant centre and 20 satellites
    rng = np.random.Generator(np.random.PCG64(1))
    P, F = [[0.5, 0.5, 0.5]], [np.eye(16)[0]]
    for s in range(20):
        u = rng.normal(size=3)
        P.append(np.array([0.5, 0.5, 0.5]) + u / np.linalg.norm(u) * (0.004 + 0.0007 * s))
        g = np.zeros(16)
        g[0] = 0.93
        g[1 + (s % 15)] = math.sqrt(1 - 0.93 ** 2) * (1 if s < 15 else -1)
        F.append(g)
    sc = make(P, F, [5.0] + [0.0] * 20, np.full((21, 3), -4.0))
    m, c, sem, geo, mg = run_both(ctx, sc)
    assert m[1:17].all() and not m[17:].any() and m[0] == 0
    check("K limit", sc, m, c, sem, geo, mg)
    # zero features, geometric thresholds, non-finite Gaussians
    lo = math.log(0.005 / 0.995)
    sc = make([[0, 0, 0], [0.001, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0], [np.nan, 0, 0], [4, 0, 0]],
              [np.zeros(16), np.zeros(16), f, f, f, f, f],
              [1.0, 0.0, lo - 1e-3, lo + 1e-3, 0.0, 0.0, np.inf],
              [[-4] * 3, [-4] * 3, [-4] * 3, [-4] * 3, [-4, math.log(0.3) + 1e-3, -4], [-4] * 3, [-4] * 3])
    m, c, sem, geo, mg = run_both(ctx, sc)
    assert m.tolist() == [0, 0, 2, 0, 2, 2, 2]
    check("zero features + geometric", sc, m, c, sem, geo, mg)


@pytest.mark.parametrize("k,bf16", [(1, False), (4, True), (16, False), (32, True)])
def test_clustered_scene(ctx, k, bf16):
    rng = np.random.Generator(np.random.PCG64(10 + k))
    N = 20000
    centres = rng.uniform(-1, 1, size=(150, 3))
    which = rng.integers(150, size=N)
    P = centres[which] + rng.normal(0, 0.04, size=(N, 3))
    P[:200] = P[200:400]                              # duplicate means
    P[400:460] = P[460] + rng.normal(0, 0.002, size=(60, 3))   # one dense knot: the K limit binds
    base = rng.normal(size=(150, 16))
    F = base[which] + 0.3 * rng.normal(size=(N, 16))
    lam = rng.normal(size=N)
    lam[1000:1200] = lam[1200:1400]                   # equal opacities
    ls = rng.normal(-3, 0.8, size=(N, 3))
    sc = make(P, F, lam, ls, bf16)
    m, c, sem, geo, mg = run_both(ctx, sc, k=k)
    check(f"clustered k={k} bf16={bf16}", sc, m, c, sem, geo, mg)
    assert sem.sum() > 100


def test_batched_workload_scene(ctx):
    sc = scenes.prune_scene(0)
    say(f"[case] 500k room-surface Gaussians, object-coherent features")
    m, c, sem, geo, mg = run_both(ctx, sc)
    check("500k", sc, m, c, sem, geo, mg)
    assert 0.05 * sc.n < sem.sum() < 0.9 * sc.n


def test_degenerate_inputs(ctx):
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    f = np.ones((1, 16))
    sc = make([[0, 0, 0]], f, [0.0], [[-4, -4, -4]])
    m, c, sem, geo, mg = run_both(ctx, sc)
    assert m.tolist() == [0] and c == (0, 0, 0)
    # no Gaussian: nothing to do, counts zero
    g = B.lgs_gaussians(0, None, None, None, None, None, None, B.LGS_F32)
    p = B.lib().lgs_default_prune_params()
    cnt = (B.C.c_int64 * 3)(7, 7, 7)
    assert B.lib().lgs_prune(ctx._h, B.C.byref(g), B.C.byref(p), None, cnt, None) == B.LGS_OK
    assert tuple(cnt) == (0, 0, 0)
    # parameters out of range
    sc2 = make([[0, 0, 0], [0.001, 0, 0]], np.ones((2, 16)), [0.0, 0.0], np.full((2, 3), -4.0))
    for bad in (dict(k=0), dict(k=33), dict(tau_dist=0.0), dict(min_opacity=1.0)):
        with pytest.raises(B.LgsError) as e:
            ctx.prune(gpu_params(sc2), **bad)
        assert e.value.status == B.LGS_ERR_INVALID_ARG
    # a mean beyond 2^20 cells of tau_dist
    sc3 = make([[0, 0, 0], [1e5, 0, 0]], np.ones((2, 16)), [0.0, 0.0], np.full((2, 3), -4.0))
    with pytest.raises(B.LgsError) as e:
        ctx.prune(gpu_params(sc3))
    assert e.value.status == B.LGS_ERR_UNSUPPORTED
