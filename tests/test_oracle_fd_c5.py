"""The oracle's gradient of the differentiation workload's loss against
central finite differences, on every parameter (CPU).

The workload: 2M Gaussians, 1296x968, f = 1170, BF16 colours and features,
loss L1(RGB) + 0.1 L1(depth) + L1(feature) (Sec. III-B.3, Eq. (1)).  Its
finite-difference check takes 64 Gaussians drawn with seed 5 among those
visible in its view, rendered alone at its camera and resolution with its
targets, and compares the oracle's autodiff gradient with central
differences (h = 1e-4, FP64) for all 64 x 30 parameters and the 6 pose-twist
components (Sec. III-B.2: pose refinement by the same loss).  The central
quotients at h and 2h are Richardson-extrapolated ((4 D(h) - D(2h)) / 3,
truncation error O(h^4)): at h alone the O(h^2) term reaches ~2e-5 relative
for the smallest footprints (a few pixels across at this focal length), above
the 1e-5 bound.  The quotients are taken over the pixels whose decisions and
residual signs do not change between the base and the four perturbed
evaluations, and compared with the autodiff gradient minus the autodiff share
of the remaining pixels (fd_helpers).  Spread over worker processes; a few
minutes of CPU time."""
import multiprocessing as mp
import os
import time

import numpy as np
import pytest

from fd_helpers import fd_worker_init, fd_worker_task

N_SUB = 64


def test_oracle_autodiff_vs_fd_all_parameters_c5_subset():
    workers = max(1, min(8, os.cpu_count() or 1))
    tasks = [("twist", j) for j in range(6)]
    tasks += [("gaussians", list(range(i, N_SUB, 16))) for i in range(16)]
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers, initializer=fd_worker_init) as pool:
        parts = pool.map(fd_worker_task, tasks, chunksize=1)
    res = [r for p, _ in parts for r in p]
    excluded = sum(e for _, e in parts)
    worst = 0.0
    names = set()
    for name, fd, ad, n_unstable in res:
        names.add(name)
        rel = abs(fd - ad) / max(abs(ad), 1e-12)
        worst = max(worst, rel if abs(fd - ad) > 1e-12 else 0.0)
        assert rel <= 1e-5 or abs(fd - ad) <= 1e-12, (name, fd, ad, n_unstable)
    total = N_SUB * 30 + 6
    print(f"\n  FD vs autodiff: {len(res)} of {total} scalars checked, {excluded} excluded "
          f"(a +-h evaluation changed a per-Gaussian decision), worst relative difference {worst:.2e}, "
          f"{time.time() - t0:.0f} s with {workers} processes", flush=True)
    assert all(f"twist[{j}]" in names for j in range(6))
    assert len(res) + excluded == total
    assert len(res) >= 0.95 * total
