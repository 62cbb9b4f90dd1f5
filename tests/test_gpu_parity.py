"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every test prints the case it is about to run (flushed) before the GPU work,
so a failing run names its case.
"""
import sys

import numpy as np
import pytest
import torch

import scenes
from oracle import brute
from oracle import raster_fp64 as R
from parity import (TOL_F32, ambiguous, forward_errors, fmt, gpu_params,
                    grad_errors, grads_np, mask_upstream, rel_err, to_np, upstream_tensors)

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_16144_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = P.Context(0)
    yield c
    c.close()


def run_fwd(ctx, wl, tile=16, chunk=4, want_n=True, order=0):
    import paper_2511_16144_amd as P
    prm = gpu_params(wl.scene)
    st = P.Settings(tile=tile, chunk=chunk, order=order)
    outs, state = ctx.forward(prm, wl.cams, st, want_n=want_n)
    torch.cuda.synchronize()
    return prm, to_np(outs), state


@pytest.fixture(scope="module")
def c1():
    wl = scenes.make_workload(1)
    ref = R.render(wl.scene, wl.cams, R.Settings())
    return wl, ref


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_c1_forward_parity(ctx, c1, tile):
    wl, ref = c1
    say(f"[case] C1 forward tile={tile} n={wl.scene.n} {wl.cams[0].width}x{wl.cams[0].height}")
    prm, out, state = run_fwd(ctx, wl, tile=tile)
    state.release()
    amb = ambiguous(ref[0]["margin"])
    err = forward_errors(out[0], ref[0], amb)
    say(f"  ambiguous pixels {amb.sum()} / {amb.size}; {fmt(err)}")
    assert amb.mean() < 0.01
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)
    nn = out[0]["n"]
    assert np.array_equal(nn[~amb], ref[0]["n"][~amb])


def test_c1_tile_invariance_bitwise(ctx, c1):
    wl, _ = c1
    say("[case] C1 tile invariance 8/16/32, chunk 1/2/4, order 0/1/2")
    res = []
    for tile, chunk, order in [(8, 1, 0), (16, 4, 0), (32, 2, 0), (16, 1, 0), (32, 4, 1), (32, 4, 2), (8, 2, 2)]:
        _, out, state = run_fwd(ctx, wl, tile=tile, chunk=chunk, order=order)
        state.release()
        res.append(out[0])
    for o in res[1:]:
        for k in ("rgb", "depth", "feat", "T", "n"):
            assert np.array_equal(o[k], res[0][k]), k


def test_c1_backward_parity(ctx, c1):
    wl, ref = c1
    say("[case] C1 backward, seeded upstream on every pixel")
    amb = ambiguous(ref[0]["margin"])
    ups = mask_upstream(scenes.random_upstream(1, wl.cams), [amb])
    prm, out, state = run_fwd(ctx, wl)
    g = grads_np(ctx.backward(state, prm, upstream_tensors(ups)))
    torch.cuda.synchronize()
    state.release()
    gr = R.vjp(wl.scene, wl.cams, ups, R.Settings())
    err = grad_errors(g, gr, np.zeros(wl.scene.n, bool))
    say(f"  upstream zeroed at {amb.sum()} ambiguous pixels; every Gaussian compared; {fmt(err)}")
    for k, (l2, mx) in err.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (k, l2, mx)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_scenes_vs_brute_force(ctx, seed):
    wl = scenes.tiny_scene(seed, 12 + 6 * seed, 37, 29)
    say(f"[case] tiny seed={seed} n={wl.scene.n} 37x29")
    Yb, Tb, nb, _ = brute.render_view(wl.scene, wl.cams[0], R.Settings())
    Yb = np.array(Yb).transpose(2, 0, 1)
    for tile in (8, 16, 32):
        _, out, state = run_fwd(ctx, wl, tile=tile)
        state.release()
        got = np.concatenate([out[0]["rgb"], out[0]["depth"][None], out[0]["feat"]], 0)
        assert np.allclose(got, Yb, rtol=1e-4, atol=1e-5)
        assert np.allclose(out[0]["T"], np.array(Tb), rtol=1e-4, atol=1e-6)
        assert np.array_equal(out[0]["n"], np.array(nb))


def test_empty_scene_and_ragged_sizes(ctx):
    say("[case] n=0, 1x1, 13x7 images")
    import paper_2511_16144_amd as P
    for (W, H) in [(1, 1), (13, 7), (8, 8), (17, 9)]:
        wl = scenes.tiny_scene(5, 0, W, H)
        prm = gpu_params(wl.scene)
        outs, state = ctx.forward(prm, wl.cams, P.Settings(), want_n=True)
        torch.cuda.synchronize()
        o = to_np(outs)[0]
        assert np.all(o["T"] == 1.0) and np.all(o["rgb"] == 0.0) and np.all(o["n"] == 0)
        g = ctx.backward(state, prm, upstream_tensors(scenes.random_upstream(0, wl.cams)))
        torch.cuda.synchronize()
        assert g["twist"].abs().sum().item() == 0.0
        state.release()


def test_backward_repeated_on_one_state(ctx, c1):
    """Three backwards on one forward state (upstreams A, B, A): the third
    equals the first bitwise.  The slot mask of the backward's partial
    records is cleared by the reduction that reads it, so a stale mark left
    by one backward would show up in the next."""
    wl, _ = c1
    say("[case] C1 backward x3 on one state")
    ua = upstream_tensors(scenes.random_upstream(3, wl.cams))
    ub = upstream_tensors(scenes.random_upstream(4, wl.cams))
    prm, out, state = run_fwd(ctx, wl)
    ga = grads_np(ctx.backward(state, prm, ua))
    gb = grads_np(ctx.backward(state, prm, ub))
    ga2 = grads_np(ctx.backward(state, prm, ua))
    torch.cuda.synchronize()
    state.release()
    assert any(not np.array_equal(ga[k], gb[k]) for k in ga)
    for k in ga:
        assert np.array_equal(ga[k], ga2[k]), k


def test_backward_run_to_run_bitwise(ctx, c1):
    wl, _ = c1
    say("[case] C1 backward determinism (two runs)")
    ups = upstream_tensors(scenes.random_upstream(3, wl.cams))
    res = []
    for _ in range(2):
        prm, out, state = run_fwd(ctx, wl)
        g = grads_np(ctx.backward(state, prm, ups))
        torch.cuda.synchronize()
        state.release()
        res.append(g)
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_bf16_after_other_kernels(ctx, seed):
    """BF16-appearance forward on sparse scenes (most 8x8 blocks see fewer
    than 8 contributing entries, so the first batch a wave composites on the
    matrix cores is partial), run right after a batched forward + backward
    has left arbitrary data in LDS: every output finite and equal to the
    brute-force render of the BF16-rounded scene."""
    import paper_2511_16144_amd as P
    big = scenes.make_workload(4, n=60000, res_scale=0.25)
    say(f"[case] tiny BF16 seed={seed} after a batched step ({big.scene.n} Gaussians)")
    prm = gpu_params(big.scene)
    outs, st = ctx.forward(prm, big.cams, P.Settings(tile=16))
    ctx.backward(st, prm, upstream_tensors(scenes.random_upstream(7, big.cams)))
    torch.cuda.synchronize()
    st.release()
    wl = scenes.tiny_scene(seed, 10 + 5 * seed, 61, 45)
    sc = wl.scene
    s16 = scenes.Scene(sc.means, sc.log_scales, sc.quats, sc.logits, scenes.round_bf16(sc.rgb),
                       scenes.round_bf16(sc.feat), "bf16")
    wl16 = scenes.Workload(wl.name, s16, wl.cams, wl.targets)
    Yb, Tb, nb, _ = brute.render_view(s16, wl.cams[0], R.Settings())
    Yb = np.array(Yb).transpose(2, 0, 1)
    for tile in (8, 16):
        _, out, state = run_fwd(ctx, wl16, tile=tile)
        state.release()
        got = np.concatenate([out[0]["rgb"], out[0]["depth"][None], out[0]["feat"]], 0)
        assert np.isfinite(got).all()
        assert np.allclose(got, Yb, rtol=1e-4, atol=1e-5)
        assert np.allclose(out[0]["T"], np.array(Tb), rtol=1e-4, atol=1e-6)
        assert np.array_equal(out[0]["n"], np.array(nb))
