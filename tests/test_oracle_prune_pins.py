"""Pins of the FP64 pruning oracle (Eq. (4) plus geometric criteria), CPU
only: hand-built configurations whose outcome follows from the definition
(a redundant pair and which member survives, the distance and similarity
thresholds, the K-nearest limit, zero features, ties by index), the
geometric thresholds, and the k-d-tree route against the brute-force
distance matrix on random clustered scenes."""
import math

import numpy as np
import pytest

from oracle import prune_fp64 as PR


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _scene(P, F, lam=None, ls=None):
    N = len(P)
    lam = np.zeros(N) if lam is None else np.asarray(lam, np.float64)
    ls = np.full((N, 3), -4.0) if ls is None else np.asarray(ls, np.float64)
    return np.asarray(P, np.float64), np.asarray(F, np.float64), lam, ls


def test_redundant_pair_keeps_the_more_opaque_one():
    f = _unit(np.arange(1, 17))
    P, F, lam, ls = _scene([[0, 0, 0], [0.005, 0, 0], [1, 1, 1]], [f, f, f], lam=[0.2, 1.5, 0.0])
    sem, geo = PR.prune(P, F, lam, ls)
    assert sem.tolist() == [True, False, False] and not geo.any()
    # equal opacities: the lower index survives
    sem, _ = PR.prune(P, F, np.zeros(3), ls)
    assert sem.tolist() == [False, True, False]


@pytest.mark.parametrize("dist,sim_angle,expect", [(0.019, 0.3, True), (0.021, 0.3, False),
                                                   (0.01, math.acos(0.89), False), (0.01, math.acos(0.91), True)])
def test_distance_and_similarity_thresholds(dist, sim_angle, expect):
    a = np.zeros(16)
    a[0] = 1.0
    b = np.zeros(16)
    b[0], b[1] = math.cos(sim_angle), math.sin(sim_angle)
    P, F, lam, ls = _scene([[0, 0, 0], [dist, 0, 0]], [a, b], lam=[1.0, 0.0])
    sem, _ = PR.prune(P, F, lam, ls)
    assert sem.tolist() == [False, expect]


def test_only_the_k_nearest_neighbours_are_checked():
    # a dominant centre and 20 satellites at increasing distances, each 0.93
    # similar to the centre and at most 0.865 to every other satellite:
    # exactly the K = 16 nearest satellites are redundant
    rng = np.random.Generator(np.random.PCG64(1))
    c = np.zeros(16)
    c[0] = 1.0
    P, F = [[0, 0, 0]], [c]
    for s in range(20):
        u = _unit(rng.normal(size=3))
        P.append(u * (0.004 + 0.0007 * s))
        f = np.zeros(16)
        f[0] = 0.93
        f[1 + (s % 15)] = math.sqrt(1 - 0.93 ** 2) * (1 if s < 15 else -1)
        F.append(f)
    lam = [5.0] + [0.0] * 20
    P, F, lam, ls = _scene(P, F, lam=lam)
    sem, _ = PR.prune(P, F, lam, ls, k=16)
    assert sem[1:17].all() and not sem[17:].any() and not sem[0]


def test_zero_features_are_never_similar():
    P, F, lam, ls = _scene([[0, 0, 0], [0.001, 0, 0]], [np.zeros(16), np.zeros(16)], lam=[1.0, 0.0])
    sem, _ = PR.prune(P, F, lam, ls)
    assert not sem.any()


def test_geometric_criteria():
    lo = math.log(0.005 / 0.995)
    P, F, lam, ls = _scene([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0], [np.nan, 0, 0]],
                           [np.ones(16)] * 5, lam=[lo - 1e-6, lo + 1e-6, 0.0, 0.0, 0.0],
                           ls=[[-4, -4, -4], [-4, -4, -4], [-4, math.log(0.3) + 1e-6, -4],
                               [-4, math.log(0.3) - 1e-6, -4], [-4, -4, -4]])
    _, geo = PR.prune(P, F, lam, ls)
    assert geo.tolist() == [True, False, True, False, True]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kdtree_route_equals_brute_force(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    N = 250
    centres = rng.uniform(0, 0.1, size=(6, 3))
    P = centres[rng.integers(6, size=N)] + rng.normal(0, 0.01, size=(N, 3))
    P[:5] = P[5:10]                       # exact duplicates: ties broken by index
    base = rng.normal(size=(6, 16))
    F = base[rng.integers(6, size=N)] + 0.25 * rng.normal(size=(N, 16))
    lam = rng.normal(size=N)
    lam[20:30] = lam[30:40]               # equal opacities
    ls = rng.normal(-3, 0.5, size=(N, 3))
    for k in (4, 16):
        a = PR.prune(P, F, lam, ls, k=k)
        b = PR.prune_brute(P, F, lam, ls, k=k)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert a[0].sum() > 5
