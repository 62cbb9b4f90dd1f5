"""GPU parity of the feature-distillation loss through the 1x1-conv decoder
(lgs_decoder_l1, through the C ABI) against the FP64 decoder oracle.

Inputs: ``scenes.decoder_inputs`` (seeded).  The targets are first moved at
least 2e-3 away from the oracle's decoded values and rounded to their
storage type (``parity.separate_decoder_targets``, from the oracle's values
only), so that every sign(Z - F_gt) is a decision both sides take the same
way; then every element of dL/dF, dL/dW and dL/db and the loss are compared
(1e-4 relative per group, rel_L2 and rel_max).  Sizes: 1x1, ragged (not a
multiple of the 32-pixel chunk, nor of 4), a multiple of the chunk, the
640x480 keyframe and the 1296x968 frame; BF16 and FP32 targets; C = 256
and 512.  The multi-view entry point (lgs_decoder_l1_views) against the
oracle's per-view results summed, with views of mixed ragged sizes (a
work-group's chunk run then crosses view boundaries), 16 views (the
maximum) and 8 equal views, and against the single-view entry point.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import scenes
from oracle import decoder_fp64 as DF
from parity import TOL_F32, fmt, rel_err, separate_decoder_targets

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2511_16144_amd as P
    c = P.Context(0)
    yield c
    c.close()


def prepared(seed, W, H, Cd, bf16):
    F, Wm, b, G = scenes.decoder_inputs(seed, W, H, Cd)
    Ff = F.reshape(16, -1).astype(np.float64)

    def z_fn(s, e):
        return Wm.astype(np.float64) @ Ff[:, s:e] + b.astype(np.float64)[:, None]
    G = separate_decoder_targets(z_fn, G, bf16=bf16)
    return F, Wm, b, G


def run_gpu(ctx, F, Wm, b, G, bf16, w_feat):
    dt = torch.bfloat16 if bf16 else torch.float32
    t = [torch.as_tensor(x).cuda() for x in (F, Wm, b)]
    g = torch.as_tensor(G).to(dt).cuda()
    loss, gf, gw, gb = ctx.decoder_l1(t[0], t[1], t[2], g, w_feat)
    torch.cuda.synchronize()
    return float(loss.item()), gf.cpu().numpy(), gw.cpu().numpy(), gb.cpu().numpy()


def check(label, gpu, ref, tol=TOL_F32):
    res = {"dF": rel_err(gpu[1], ref[1]), "dW": rel_err(gpu[2], ref[2]), "db": rel_err(gpu[3], ref[3])}
    say(f"  {label}: loss gpu {gpu[0]:.7g} oracle {ref[0]:.7g};", fmt(res))
    assert abs(gpu[0] - ref[0]) <= 1e-5 * abs(ref[0]), (label, gpu[0], ref[0])
    for k, (l2, mx) in res.items():
        assert l2 <= tol and mx <= tol, (label, k, l2, mx)


CASES = [
    ("1x1 C256 bf16", 1, 1, 256, True),
    ("7x5 C256 f32", 7, 5, 256, False),
    ("33x17 C512 bf16 ragged", 33, 17, 512, True),
    ("64x48 C512 bf16", 64, 48, 512, True),
    ("61x37 C512 f32 ragged", 61, 37, 512, False),
    ("640x480 C512 bf16", 640, 480, 512, True),
]


@pytest.mark.parametrize("label,W,H,Cd,bf16", CASES, ids=[c[0] for c in CASES])
def test_decoder_vs_oracle(ctx, label, W, H, Cd, bf16):
    say(f"[case] decoder {label}")
    F, Wm, b, G = prepared(W * 7 + H, W, H, Cd, bf16)
    gpu = run_gpu(ctx, F, Wm, b, G, bf16, 0.8)
    ref = DF.decoder_l1(F, Wm, b, G, w_feat=0.8)
    check(label, gpu, ref)


def test_decoder_full_frame_1296x968(ctx):
    say("[case] decoder 1296x968 C512 bf16")
    F, Wm, b, G = prepared(5, 1296, 968, 512, True)
    gpu = run_gpu(ctx, F, Wm, b, G, True, 1.0)
    ref = DF.decoder_l1(F, Wm, b, G, w_feat=1.0, chunk=1 << 17)
    check("1296x968", gpu, ref)


def test_decoder_deterministic_and_rejects_bad_arguments(ctx):
    from paper_2511_16144_amd import binding as B
    F, Wm, b, G = prepared(9, 50, 30, 256, True)
    a1 = run_gpu(ctx, F, Wm, b, G, True, 1.0)
    a2 = run_gpu(ctx, F, Wm, b, G, True, 1.0)
    assert a1[0] == a2[0]
    for x, y in zip(a1[1:], a2[1:]):
        assert np.array_equal(x, y)
    t = [torch.as_tensor(x).cuda() for x in (F, Wm, b)]
    g = torch.as_tensor(G).to(torch.bfloat16).cuda()
    out = [torch.empty(1, device="cuda"), torch.empty_like(t[0]), torch.empty_like(t[1]), torch.empty_like(t[2])]
    lib, h = B.lib(), ctx._h
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(), g.data_ptr(), B.LGS_BF16, C.c_float(1.0),
            out[1].data_ptr(), out[2].data_ptr(), out[3].data_ptr(), out[0].data_ptr(), s]
    assert lib.lgs_decoder_l1(h, 50, 30, 256, *args) == B.LGS_OK
    assert lib.lgs_decoder_l1(h, 50, 30, 128, *args) == B.LGS_ERR_UNSUPPORTED
    assert lib.lgs_decoder_l1(h, 0, 30, 256, *args) == B.LGS_ERR_INVALID_ARG
    bad = list(args)
    bad[6] = None
    assert lib.lgs_decoder_l1(h, 50, 30, 256, *bad) == B.LGS_ERR_INVALID_ARG
    bad = list(args)
    bad[5] = C.c_float(float("nan"))
    assert lib.lgs_decoder_l1(h, 50, 30, 256, *bad) == B.LGS_ERR_INVALID_ARG
    torch.cuda.synchronize()


VIEW_CASES = [
    ("3 views ragged C256 f32", [(7, 5), (33, 17), (1, 1)], 256, False),
    ("4 views ragged C512 bf16", [(61, 37), (64, 48), (1, 3), (33, 17)], 512, True),
    ("16 views C512 bf16", [(32 + 5 * v, 16 + 3 * v) for v in range(16)], 512, True),
    ("8 views 320x240 C512 bf16", [(320, 240)] * 8, 512, True),
]


@pytest.mark.parametrize("label,sizes,Cd,bf16", VIEW_CASES, ids=[c[0] for c in VIEW_CASES])
def test_decoder_views_vs_oracle(ctx, label, sizes, Cd, bf16):
    """lgs_decoder_l1_views: the views' Eq. (2) terms (each normalised by its
    own C H W) summed, dL/dF per view; against the oracle's per-view results
    summed in FP64, and against the single-view entry point called per view
    (up to FP32 summation order)."""
    say(f"[case] decoder views {label}")
    dt = torch.bfloat16 if bf16 else torch.float32
    _, Wm, b, _ = scenes.decoder_inputs(1, 1, 1, Cd)
    Fs, Gs, refs = [], [], []
    for v, (W, H) in enumerate(sizes):
        F, _, _, G = scenes.decoder_inputs(100 + v, W, H, Cd)
        Ff = F.reshape(16, -1).astype(np.float64)

        def z_fn(s, e, Ff=Ff):
            return Wm.astype(np.float64) @ Ff[:, s:e] + b.astype(np.float64)[:, None]
        G = separate_decoder_targets(z_fn, G, bf16=bf16)
        Fs.append(F)
        Gs.append(G)
        refs.append(DF.decoder_l1(F, Wm, b, G, w_feat=0.7))
    ref = (sum(r[0] for r in refs), None, sum(r[2] for r in refs), sum(r[3] for r in refs))
    tw, tb = torch.as_tensor(Wm).cuda(), torch.as_tensor(b).cuda()
    tf = [torch.as_tensor(F).cuda() for F in Fs]
    tg = [torch.as_tensor(G).to(dt).cuda() for G in Gs]
    loss, gfs, gw, gb = ctx.decoder_l1_views(tf, tw, tb, tg, 0.7)
    torch.cuda.synchronize()
    gpu = (float(loss.item()), None, gw.cpu().numpy(), gb.cpu().numpy())
    res = {"dW": rel_err(gpu[2], ref[2]), "db": rel_err(gpu[3], ref[3])}
    for v, r in enumerate(refs):
        res[f"dF{v}"] = rel_err(gfs[v].cpu().numpy(), r[1])
    say(f"  {label}: loss gpu {gpu[0]:.7g} oracle {ref[0]:.7g};", fmt(res))
    assert abs(gpu[0] - ref[0]) <= 1e-5 * abs(ref[0]), (label, gpu[0], ref[0])
    for k, (l2, mx) in res.items():
        assert l2 <= TOL_F32 and mx <= TOL_F32, (label, k, l2, mx)
    # the same sums from the single-view entry point
    one = [ctx.decoder_l1(f, tw, tb, g, 0.7) for f, g in zip(tf, tg)]
    torch.cuda.synchronize()
    s_loss = sum(float(o[0].item()) for o in one)
    s_gw = sum(o[2].double() for o in one).cpu().numpy()
    s_gb = sum(o[3].double() for o in one).cpu().numpy()
    assert abs(gpu[0] - s_loss) <= 1e-5 * abs(s_loss)
    for x, y in ((gpu[2], s_gw), (gpu[3], s_gb)):
        l2, mx = rel_err(x, y)
        assert l2 <= TOL_F32 and mx <= TOL_F32, (label, l2, mx)
    for v, o in enumerate(one):
        l2, mx = rel_err(gfs[v].cpu().numpy(), o[1].cpu().numpy())
        assert l2 <= TOL_F32 and mx <= TOL_F32, (label, v, l2, mx)


def test_decoder_views_rejects_bad_arguments(ctx):
    from paper_2511_16144_amd import binding as B
    F, Wm, b, G = prepared(9, 50, 30, 256, True)
    t = [torch.as_tensor(x).cuda() for x in (F, Wm, b)]
    g = torch.as_tensor(G).to(torch.bfloat16).cuda()
    gf, gw, gb, loss = torch.empty_like(t[0]), torch.empty_like(t[1]), torch.empty_like(t[2]), \
        torch.empty(1, device="cuda")
    lib, h = B.lib(), ctx._h
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    nv = 17
    ws, hs = (C.c_int32 * nv)(*([50] * nv)), (C.c_int32 * nv)(*([30] * nv))
    fp = (C.c_void_p * nv)(*([t[0].data_ptr()] * nv))
    tp = (C.c_void_p * nv)(*([g.data_ptr()] * nv))
    gp = (C.c_void_p * nv)(*([gf.data_ptr()] * nv))

    def call(n, ws=ws, fp=fp):
        return lib.lgs_decoder_l1_views(h, n, ws, hs, 256, fp, t[1].data_ptr(), t[2].data_ptr(), tp, B.LGS_BF16,
                                        C.c_float(1.0), gp, gw.data_ptr(), gb.data_ptr(), loss.data_ptr(), s)
    assert call(1) == B.LGS_OK
    assert call(0) == B.LGS_ERR_INVALID_ARG
    assert call(17) == B.LGS_ERR_UNSUPPORTED
    bad_w = (C.c_int32 * nv)(*([50] * nv))
    bad_w[1] = 0
    assert call(2, ws=bad_w) == B.LGS_ERR_INVALID_ARG
    bad_f = (C.c_void_p * nv)(*([t[0].data_ptr()] * nv))
    bad_f[1] = None
    assert call(2, fp=bad_f) == B.LGS_ERR_INVALID_ARG
    torch.cuda.synchronize()
