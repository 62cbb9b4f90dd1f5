"""Differentiation at scale (the 2M-Gaussian, 1296x968, BF16 configuration):
64 Gaussians drawn with seed 5 among those visible in its view, rendered
alone at its camera and resolution with its targets and loss weights
(1, 0.1, 1).  The GPU gradient of the L1 step (lgs_forward +
lgs_backward_l1) against the oracle's autodiff gradient, for all 64 x 30
parameters and the 6 twist components (1e-4).  The oracle's autodiff
gradient of the same sub-scene is checked against central finite
differences on every one of those scalars by the CPU test
test_oracle_fd_c5.py."""
import numpy as np
import pytest
import torch

import scenes
from fd_helpers import base_gradient, subscene_64
from parity import TOL_F32, fmt, gpu_params, grad_errors, grads_np

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_c5_subset_gpu_vs_autodiff():
    import paper_2511_16144_amd as P
    wl = scenes.make_workload(5)
    sub, idx = subscene_64(wl)
    cam = wl.cams[0]
    say(f"[case] C5 64-Gaussian subset at {cam.width}x{cam.height}, BF16 appearance, loss {wl.loss_w}")
    ctx = P.Context(0)
    prm = gpu_params(sub)
    tg = [{"rgb": torch.as_tensor(t.rgb).cuda(), "depth": torch.as_tensor(t.depth).cuda(),
           "feat": torch.as_tensor(t.feat).cuda()} for t in wl.targets]
    outs, st = ctx.forward(prm, [cam], P.Settings(tile=16))
    g = grads_np(ctx.backward_l1(st, prm, outs, tg, wl.loss_w))
    torch.cuda.synchronize()
    st.release()
    ctx.close()
    _, AD = base_gradient(sub, cam, wl.targets[0], wl.loss_w)
    err = grad_errors(g, AD, np.zeros(sub.n, bool))
    say("  GPU vs autodiff (all 64 x 30 parameters and the twist):", fmt(err))
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)
