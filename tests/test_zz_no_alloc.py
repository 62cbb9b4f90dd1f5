"""The decoder-loss entry point that allocates nothing (lgs_decoder_l1_noalloc,
for callers that cannot allocate device memory) against lgs_decoder_l1, both
called through the C ABI.

They run the same kernels with the same launch; only where the work-groups'
partial sums live differs (a fixed device array instead of a context
buffer), so every output must be bitwise equal.  Two calls in a row on the
no-allocation entry point, the second with a smaller input (fewer pixels,
fewer channels, FP32 instead of BF16 targets), check that what the first call
left in the shared array does not leak into the second.  Every output buffer
is filled with NaN before each call, so an element a call fails to write is
caught too."""
import ctypes as C

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu

CASES = [(640, 480, 512, True, 1.0), (61, 37, 256, False, 0.5)]   # the second is smaller


def say(*a):
    print(*a, flush=True)


def inputs(seed, W, H, Cd, bf16):
    F, Wm, b, G = scenes.decoder_inputs(seed, W, H, Cd)
    dt = torch.bfloat16 if bf16 else torch.float32
    return [torch.as_tensor(x).cuda() for x in (F, Wm, b)] + [torch.as_tensor(G).to(dt).cuda()]


def call(fn, ctx, W, H, Cd, bf16, w_feat, x):
    from paper_2511_16144_amd import binding as B
    F, Wm, b, G = x
    out = [torch.full((1,), np.nan, device="cuda"), torch.full_like(F, np.nan), torch.full_like(Wm, np.nan),
           torch.full_like(b, np.nan)]
    st = fn(ctx._h, W, H, Cd, C.c_void_p(F.data_ptr()), C.c_void_p(Wm.data_ptr()), C.c_void_p(b.data_ptr()),
            C.c_void_p(G.data_ptr()), B.LGS_BF16 if bf16 else B.LGS_F32, C.c_float(w_feat),
            *[C.c_void_p(t.data_ptr()) for t in out[1:]], C.c_void_p(out[0].data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, B.lib().lgs_last_error(ctx._h).decode()
    return out


def test_noalloc_decoder_equals_allocating_entry_point_twice():
    import paper_2511_16144_amd as P
    lib = P.lib()
    ctx = P.Context(0)
    try:
        xs = [inputs(300 + i, *c[:4]) for i, c in enumerate(CASES)]
        ref = []
        for c, x in zip(CASES, xs):
            say(f"[case] lgs_decoder_l1 {c[0]}x{c[1]} C{c[2]} {'bf16' if c[3] else 'f32'} targets")
            ref.append([t.cpu().numpy() for t in call(lib.lgs_decoder_l1, ctx, *c, x)])
        torch.cuda.synchronize()
        # two no-allocation calls back to back, the second smaller
        got = []
        for c, x in zip(CASES, xs):
            say(f"[case] lgs_decoder_l1_noalloc {c[0]}x{c[1]} C{c[2]} {'bf16' if c[3] else 'f32'} targets")
            got.append(call(lib.lgs_decoder_l1_noalloc, ctx, *c, x))
        torch.cuda.synchronize()
        for c, r, g in zip(CASES, ref, got):
            g = [t.cpu().numpy() for t in g]
            for name, a, b in zip(("loss", "dF", "dW", "db"), g, r):
                assert np.all(np.isfinite(a)), (c, name)
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (c, name)
            say(f"  {c[0]}x{c[1]} C{c[2]}: loss {float(g[0][0]):.7g}, every output bitwise equal")
    finally:
        ctx.close()


def test_noalloc_decoder_rejects_bad_arguments():
    import paper_2511_16144_amd as P
    from paper_2511_16144_amd import binding as B
    lib = P.lib()
    ctx = P.Context(0)
    try:
        x = inputs(310, 8, 8, 256, False)
        for W, H, Cd, want in ((0, 8, 256, B.LGS_ERR_INVALID_ARG), (8, 8, 128, B.LGS_ERR_UNSUPPORTED)):
            F, Wm, b, G = x
            st = lib.lgs_decoder_l1_noalloc(ctx._h, W, H, Cd, C.c_void_p(F.data_ptr()), C.c_void_p(Wm.data_ptr()),
                                            C.c_void_p(b.data_ptr()), C.c_void_p(G.data_ptr()), B.LGS_F32,
                                            C.c_float(1.0), C.c_void_p(F.data_ptr()), C.c_void_p(Wm.data_ptr()),
                                            C.c_void_p(b.data_ptr()), None, None)
            assert st == want, lib.lgs_last_error(ctx._h).decode()
    finally:
        ctx.close()
