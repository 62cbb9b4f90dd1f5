"""Pins of the FP64 decoder-loss oracle (Eq. (2) through a 1x1-conv decoder),
CPU only: the identity decoder reduces to the plain feature L1 term (and to
the rasterizer oracle's feature upstream), a single pixel checked by explicit
loops, central finite differences, and invariance to the pixel chunking."""
import numpy as np
import pytest

from oracle import decoder_fp64 as DF
from oracle import raster_fp64 as R
from scenes import Targets


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_identity_decoder_is_the_feature_l1_term():
    rng = _rng(1)
    H, W = 5, 7
    F = rng.normal(size=(16, H, W))
    Fgt = rng.normal(size=(16, H, W))
    L, dF, dW, db = DF.decoder_l1(F, np.eye(16), np.zeros(16), Fgt, w_feat=0.7)
    assert np.allclose(DF.decode(F, np.eye(16), np.full(16, 0.25)), F + 0.25, rtol=0, atol=1e-15)
    assert abs(L - 0.7 * np.mean(np.abs(F - Fgt))) < 1e-14
    t = Targets(np.zeros((3, H, W)), np.zeros((H, W)), Fgt)
    o = {"rgb": np.zeros((3, H, W)), "depth": np.zeros((H, W)), "feat": F}
    up = R.l1_upstream([o], [t], (0.0, 0.0, 0.7))[0]
    assert np.allclose(dF, up[4:], rtol=0, atol=1e-16)


def test_single_pixel_by_explicit_loops():
    rng = _rng(2)
    C, d = 32, 16
    f = rng.normal(size=d)
    Wm = rng.normal(size=(C, d)) * 0.3
    b = rng.normal(size=C) * 0.1
    g = rng.normal(size=C)
    wf = 1.3
    z = [sum(Wm[c][k] * f[k] for k in range(d)) + b[c] for c in range(C)]
    s = [(1.0 if z[c] > g[c] else -1.0) for c in range(C)]
    L_ref = wf / C * sum(abs(z[c] - g[c]) for c in range(C))
    dF_ref = [wf / C * sum(Wm[c][k] * s[c] for c in range(C)) for k in range(d)]
    dW_ref = [[wf / C * s[c] * f[k] for k in range(d)] for c in range(C)]
    L, dF, dW, db = DF.decoder_l1(f.reshape(d, 1, 1), Wm, b, np.array(g).reshape(C, 1, 1), w_feat=wf)
    assert abs(L - L_ref) < 1e-13
    assert np.allclose(dF[:, 0, 0], dF_ref, rtol=0, atol=1e-15)
    assert np.allclose(dW, dW_ref, rtol=0, atol=1e-15)
    assert np.allclose(db, [wf / C * x for x in s], rtol=0, atol=1e-15)


def test_gradients_vs_central_fd():
    rng = _rng(3)
    C, H, W = 32, 3, 5
    F = rng.normal(size=(16, H, W))
    Wm = rng.normal(size=(C, 16)) * 0.3
    b = rng.normal(size=C) * 0.1
    Z = DF.decode(F, Wm, b)
    Fgt = Z + np.where(rng.uniform(size=Z.shape) < 0.5, -1, 1) * rng.uniform(0.05, 0.5, size=Z.shape)
    L, dF, dW, db = DF.decoder_l1(F, Wm, b, Fgt, w_feat=0.9)
    h = 1e-6

    def loss(F_, W_, b_):
        return DF.decoder_l1(F_, W_, b_, Fgt, w_feat=0.9)[0]
    for arr, grad, idxs in ((F, dF, [(0, 0, 0), (7, 2, 4), (15, 1, 2)]), (Wm, dW, [(0, 0), (31, 15), (9, 3)]),
                            (b, db, [(0,), (17,), (31,)])):
        for idx in idxs:
            ap, am = arr.copy(), arr.copy()
            ap[idx] += h
            am[idx] -= h
            args_p = [ap if arr is x else x for x in (F, Wm, b)]
            args_m = [am if arr is x else x for x in (F, Wm, b)]
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            assert abs(fd - grad[idx]) < 1e-9, (idx, fd, grad[idx])


@pytest.mark.parametrize("chunk", [1, 7, 64])
def test_pixel_chunking_does_not_change_the_result(chunk):
    rng = _rng(4)
    F = rng.normal(size=(16, 6, 11))
    Wm = rng.normal(size=(64, 16))
    b = rng.normal(size=64)
    Fgt = rng.normal(size=(64, 6, 11))
    a = DF.decoder_l1(F, Wm, b, Fgt, chunk=chunk)
    c = DF.decoder_l1(F, Wm, b, Fgt, chunk=1 << 20)
    assert abs(a[0] - c[0]) < 1e-13
    for x, y in zip(a[1:], c[1:]):
        assert np.allclose(x, y, rtol=0, atol=1e-15)
