"""ctypes binding of ``liblego_raster.so`` (the C ABI of include/lego_raster.h).

Argument marshalling only: every stage of the render and its gradient runs in
the library's HIP kernels.  torch provides device memory and the stream.
There is no CPU fallback: importing this module without the built library
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblego_raster.so")

LGS_OK, LGS_ERR_INVALID_ARG, LGS_ERR_HIP, LGS_ERR_CAPACITY, LGS_ERR_UNSUPPORTED, LGS_ERR_STATE = range(6)
LGS_F32, LGS_BF16 = 0, 1
# bits of lgs_settings.profile: stage events, compositing work counts
PROFILE_EVENTS, PROFILE_COUNTS = 1, 2


class lgs_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R_cw", C.c_float * 9), ("t_cw", C.c_float * 3)]


class lgs_settings(C.Structure):
    _fields_ = [("z_near", C.c_float), ("eps2d", C.c_float), ("fov_clamp", C.c_float),
                ("alpha_max", C.c_float), ("alpha_min", C.c_float), ("T_eps", C.c_float),
                ("cutoff2", C.c_float), ("tile", C.c_int32), ("chunk", C.c_int32), ("order", C.c_int32),
                ("profile", C.c_int32)]


class lgs_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity_logits", C.c_void_p), ("rgb", C.c_void_p),
                ("feat", C.c_void_p), ("appearance_dtype", C.c_int32), ("feat_dim", C.c_int32)]


class lgs_images(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("feat", C.c_void_p),
                ("final_T", C.c_void_p), ("n_contrib", C.c_void_p)]


class lgs_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("rgb", C.c_void_p), ("feat", C.c_void_p),
                ("twist", C.c_void_p)]


class lgs_prune_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("tau_dist", C.c_float), ("tau_sim", C.c_float), ("min_opacity", C.c_float),
                ("max_scale", C.c_float)]


class lgs_counts(C.Structure):
    _fields_ = [("n_visible", C.c_int64), ("n_pairs", C.c_int64), ("n_slots", C.c_int64),
                ("n_tiles", C.c_int64), ("n_items", C.c_int64), ("fwd_evals", C.c_int64),
                ("fwd_contrib", C.c_int64), ("bwd_evals", C.c_int64), ("bwd_contrib", C.c_int64),
                ("fwd_entries", C.c_int64), ("bwd_entries", C.c_int64), ("bwd_written", C.c_int64)]


EXPORTS = ["lgs_status_string", "lgs_last_error", "lgs_default_settings", "lgs_context_create",
           "lgs_context_destroy", "lgs_forward", "lgs_backward", "lgs_backward_l1", "lgs_loss", "lgs_decoder_l1",
           "lgs_decoder_l1_views", "lgs_decoder_l1_noalloc",
           "lgs_default_prune_params", "lgs_prune",
           "lgs_state_counts",
           "lgs_state_stage_ms",
           "lgs_state_release", "lgs_graph_create", "lgs_graph_launch", "lgs_graph_status",
           "lgs_graph_counts", "lgs_graph_stage_ms", "lgs_graph_destroy", "lgs_autotune"]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or paper_2511_16144_amd/build_lib.py)")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.lgs_status_string.restype = C.c_char_p
    lib.lgs_status_string.argtypes = [C.c_int]
    lib.lgs_last_error.restype = C.c_char_p
    lib.lgs_last_error.argtypes = [P]
    lib.lgs_default_settings.restype = lgs_settings
    lib.lgs_default_settings.argtypes = []
    lib.lgs_context_create.restype = C.c_int
    lib.lgs_context_create.argtypes = [C.c_int, C.POINTER(P)]
    lib.lgs_context_destroy.restype = None
    lib.lgs_context_destroy.argtypes = [P]
    lib.lgs_forward.restype = C.c_int
    lib.lgs_forward.argtypes = [P, C.POINTER(lgs_settings), C.POINTER(lgs_gaussians), C.c_int32,
                                C.POINTER(lgs_camera), C.POINTER(lgs_images), C.POINTER(P), P]
    lib.lgs_backward.restype = C.c_int
    lib.lgs_backward.argtypes = [P, P, C.POINTER(lgs_gaussians), C.POINTER(lgs_images),
                                 C.POINTER(lgs_grads), P]
    lib.lgs_backward_l1.restype = C.c_int
    lib.lgs_backward_l1.argtypes = [P, P, C.POINTER(lgs_gaussians), C.POINTER(lgs_images), C.POINTER(lgs_images),
                                    C.POINTER(C.c_float), C.POINTER(lgs_grads), P]
    lib.lgs_loss.restype = C.c_int
    lib.lgs_loss.argtypes = [P, C.c_int32, C.POINTER(lgs_camera), C.c_int32, C.POINTER(lgs_images),
                             C.POINTER(lgs_images),
                             C.POINTER(C.c_float), C.c_float, C.POINTER(lgs_images), P, P]
    lib.lgs_decoder_l1.restype = C.c_int
    lib.lgs_decoder_l1.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, C.c_int32, C.c_float,
                                   P, P, P, P, P]
    lib.lgs_decoder_l1_views.restype = C.c_int
    lib.lgs_decoder_l1_views.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                         C.POINTER(P), P, P, C.POINTER(P), C.c_int32, C.c_float, C.POINTER(P),
                                         P, P, P, P]
    lib.lgs_decoder_l1_noalloc.restype = C.c_int
    lib.lgs_decoder_l1_noalloc.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P, P, C.c_int32,
                                           C.c_float, P, P, P, P, P]
    lib.lgs_default_prune_params.restype = lgs_prune_params
    lib.lgs_default_prune_params.argtypes = []
    lib.lgs_prune.restype = C.c_int
    lib.lgs_prune.argtypes = [P, C.POINTER(lgs_gaussians), C.POINTER(lgs_prune_params), P,
                              C.POINTER(C.c_int64), P]
    lib.lgs_state_counts.restype = C.c_int
    lib.lgs_state_counts.argtypes = [P, C.POINTER(lgs_counts)]
    lib.lgs_state_stage_ms.restype = C.c_int
    lib.lgs_state_stage_ms.argtypes = [P, C.POINTER(C.c_float)]
    lib.lgs_state_release.restype = C.c_int
    lib.lgs_state_release.argtypes = [P, P]
    lib.lgs_graph_create.restype = C.c_int
    lib.lgs_graph_create.argtypes = [P, C.POINTER(lgs_settings), C.POINTER(lgs_gaussians), C.c_int32,
                                     C.POINTER(lgs_camera), C.POINTER(lgs_images), C.POINTER(C.c_float),
                                     C.c_float, C.POINTER(lgs_images), C.POINTER(lgs_grads), C.c_int64, P,
                                     C.POINTER(P)]
    lib.lgs_graph_launch.restype = C.c_int
    lib.lgs_graph_launch.argtypes = [P, P]
    lib.lgs_graph_status.restype = C.c_int
    lib.lgs_graph_status.argtypes = [P]
    lib.lgs_graph_counts.restype = C.c_int
    lib.lgs_graph_counts.argtypes = [P, C.POINTER(lgs_counts)]
    lib.lgs_graph_stage_ms.restype = C.c_int
    lib.lgs_graph_stage_ms.argtypes = [P, C.POINTER(C.c_float)]
    lib.lgs_graph_destroy.restype = None
    lib.lgs_graph_destroy.argtypes = [P]
    lib.lgs_autotune.restype = C.c_int
    lib.lgs_autotune.argtypes = [P, C.POINTER(lgs_settings), C.POINTER(lgs_gaussians), C.c_int32,
                                 C.POINTER(lgs_camera), C.POINTER(lgs_images), C.POINTER(C.c_float),
                                 C.POINTER(lgs_images), C.POINTER(lgs_grads), C.c_int64, P, C.c_char_p,
                                 C.POINTER(lgs_settings)]
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class LgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().lgs_status_string(status).decode()}: {msg}")
        self.status = status


@dataclass
class Settings:
    z_near: float = 0.2
    eps2d: float = 0.3
    fov_clamp: float = 1.3
    alpha_max: float = 0.99
    alpha_min: float = 1.0 / 255.0
    T_eps: float = 1e-4
    cutoff2: float = 9.0
    tile: int = 16
    chunk: int = 4
    order: int = 0
    profile: int = 0

    def to_c(self) -> lgs_settings:
        return lgs_settings(self.z_near, self.eps2d, self.fov_clamp, self.alpha_max, self.alpha_min,
                            self.T_eps, self.cutoff2, self.tile, self.chunk, self.order, self.profile)

    @staticmethod
    def from_c(s: lgs_settings) -> "Settings":
        return Settings(s.z_near, s.eps2d, s.fov_clamp, s.alpha_max, s.alpha_min, s.T_eps, s.cutoff2,
                        s.tile, s.chunk, s.order, s.profile)


def camera_c(cam) -> lgs_camera:
    """Any object with width, height, fx, fy, cx, cy, R_cw (3x3), t_cw (3)."""
    R = [float(x) for row in cam.R_cw for x in row]
    t = [float(x) for x in cam.t_cw]
    return lgs_camera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                      float(cam.cy), (C.c_float * 9)(*R), (C.c_float * 3)(*t))


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_param(t, rows, n, name, dtypes=(torch.float32,)):
    if t.dtype not in dtypes or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != ((rows, n) if rows else (n,)):
        raise ValueError(f"{name}: expected contiguous CUDA tensor of shape {(rows, n) if rows else (n,)} "
                         f"and dtype in {dtypes}, got {tuple(t.shape)} {t.dtype}")


def gaussians_c(means, log_scales, quats, logits, rgb, feat) -> lgs_gaussians:
    n = logits.shape[0]
    _check_param(means, 3, n, "means")
    _check_param(log_scales, 3, n, "log_scales")
    _check_param(quats, 4, n, "quats")
    _check_param(logits, 0, n, "logits")
    _check_param(rgb, 3, n, "rgb", (torch.float32, torch.bfloat16))
    D = feat.shape[0] if feat.dim() == 2 else -1
    _check_param(feat, D, n, "feat", (torch.float32, torch.bfloat16))
    if rgb.dtype != feat.dtype:
        raise ValueError("rgb and feat must share a dtype")
    dt = LGS_BF16 if rgb.dtype == torch.bfloat16 else LGS_F32
    return lgs_gaussians(n, _ptr(means), _ptr(log_scales), _ptr(quats), _ptr(logits), _ptr(rgb),
                         _ptr(feat), dt, D)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Context:
    """One library context (device workspace) on a HIP device."""

    def __init__(self, device: int = 0):
        self.device = device
        self._h = C.c_void_p()
        st = lib().lgs_context_create(device, C.byref(self._h))
        if st != LGS_OK:
            raise LgsError(st, "lgs_context_create failed")

    def close(self):
        if self._h:
            lib().lgs_context_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        raise LgsError(st, lib().lgs_last_error(self._h).decode())

    # -- eager forward / backward ------------------------------------------
    def forward(self, params, cams, settings: Settings | None = None, want_n: bool = False,
                stream=None, out=None):
        """params: dict of CUDA tensors means [3,N], log_scales [3,N], quats [4,N],
        logits [N], rgb [3,N], feat [D,N].  Returns (list of per-view dicts
        rgb [3,H,W], depth [H,W], feat [D,H,W], T [H,W] (and n [H,W] int32),
        state)."""
        settings = settings or Settings()
        g = gaussians_c(params["means"], params["log_scales"], params["quats"], params["logits"],
                        params["rgb"], params["feat"])
        dev = params["means"].device
        V = len(cams)
        outs, imgs = [], (lgs_images * V)()
        cams_c = (lgs_camera * V)(*[camera_c(c) for c in cams])
        for v, c in enumerate(cams):
            H, W = int(c.height), int(c.width)
            if out is not None:        # caller-provided output buffers (reused across steps)
                o = out[v]
            else:
                o = {"rgb": torch.empty((3, H, W), device=dev), "depth": torch.empty((H, W), device=dev),
                     "feat": torch.empty((g.feat_dim, H, W), device=dev), "T": torch.empty((H, W), device=dev)}
                if want_n:
                    o["n"] = torch.empty((H, W), device=dev, dtype=torch.int32)
            imgs[v] = lgs_images(_ptr(o["rgb"]), _ptr(o["depth"]), _ptr(o["feat"]), _ptr(o["T"]),
                                 _ptr(o.get("n")))
            outs.append(o)
        state = C.c_void_p()
        sc = settings.to_c()
        st = lib().lgs_forward(self._h, C.byref(sc), C.byref(g), V, cams_c, imgs, C.byref(state),
                               _stream(stream))
        if st != LGS_OK:
            self._raise(st)
        return outs, State(self, state, V, [(int(c.height), int(c.width)) for c in cams], g.feat_dim)

    def backward_l1(self, state, params, outs, targets, loss_w, stream=None, grads=None) -> dict:
        return backward_l1(self, state, params, outs, targets, loss_w, stream, grads)

    def loss(self, cams, outs, targets, loss_w, ssim_lambda: float = 0.2, stream=None, grad=None,
             want_terms: bool = True):
        """Mapping loss of Eq. (1) with its D-SSIM term and dL/dY (lgs_loss).
        outs / targets: per-view dicts rgb [3,H,W], depth [H,W], feat [D,H,W]
        (FP32 CUDA).  Returns (per-view gradient dicts, terms [V, 4] or None:
        mean|I-I*|, 1 - SSIM, mean|D-D*|, mean|F-F*|)."""
        V = len(cams)
        shapes = [(int(c.height), int(c.width)) for c in cams]
        dev = outs[0]["rgb"].device
        D = outs[0]["feat"].shape[0]
        if grad is None:
            grad = [{"rgb": torch.empty((3, H, W), device=dev), "depth": torch.empty((H, W), device=dev),
                     "feat": torch.empty((D, H, W), device=dev)} for (H, W) in shapes]
        terms = torch.empty((V, 4), device=dev) if want_terms else None
        cams_c = (lgs_camera * V)(*[camera_c(c) for c in cams])
        lw = (C.c_float * 3)(*[float(x) for x in loss_w])
        st = lib().lgs_loss(self._h, V, cams_c, D, _images_c(outs, shapes, False, D),
                            _images_c(targets, shapes, False, D), lw, float(ssim_lambda),
                            _images_c(grad, shapes, False, D), _ptr(terms), _stream(stream))
        if st != LGS_OK:
            self._raise(st)
        return grad, terms

    def decoder_l1(self, feat, weight, bias, target, w_feat: float = 1.0, stream=None, out=None,
                   noalloc: bool = False):
        """Feature-distillation loss of Eq. (2) through the 1x1-conv decoder
        (lgs_decoder_l1, or lgs_decoder_l1_noalloc with noalloc=True: no
        device allocation in the library; pass `out` to allocate nothing
        here either).  feat [16,H,W] FP32, weight [C,16], bias [C] FP32,
        target [C,H,W] BF16 or FP32 (CUDA, contiguous).  Returns (loss [1],
        grad_feat, grad_weight, grad_bias)."""
        d, H, W = feat.shape
        Cd = weight.shape[0]
        for t, shp, dts, name in ((feat, (16, H, W), (torch.float32,), "feat"),
                                  (weight, (Cd, 16), (torch.float32,), "weight"),
                                  (bias, (Cd,), (torch.float32,), "bias"),
                                  (target, (Cd, H, W), (torch.float32, torch.bfloat16), "target")):
            if tuple(t.shape) != shp or t.dtype not in dts or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name}: expected contiguous CUDA tensor of shape {shp}, dtype in {dts}")
        dev = feat.device
        if out is None:
            out = (torch.empty(1, device=dev), torch.empty_like(feat), torch.empty_like(weight),
                   torch.empty_like(bias))
        loss, gf, gw, gb = out
        dt = LGS_BF16 if target.dtype == torch.bfloat16 else LGS_F32
        fn = lib().lgs_decoder_l1_noalloc if noalloc else lib().lgs_decoder_l1
        st = fn(self._h, W, H, Cd, _ptr(feat), _ptr(weight), _ptr(bias), _ptr(target), dt,
                float(w_feat), _ptr(gf), _ptr(gw), _ptr(gb), _ptr(loss), _stream(stream))
        if st != LGS_OK:
            self._raise(st)
        return loss, gf, gw, gb

    def decoder_l1_views(self, feats, weight, bias, targets, w_feat: float = 1.0, stream=None, out=None):
        """The decoder loss summed over views in one launch
        (lgs_decoder_l1_views): feats / targets lists of per-view tensors as
        for decoder_l1 (sizes may differ between views, the targets share one
        dtype).  Returns (loss [1], [grad_feat per view], grad_weight,
        grad_bias)."""
        nv = len(feats)
        if nv != len(targets) or nv < 1:
            raise ValueError("feats and targets: one tensor per view, at least one view")
        Cd = weight.shape[0]
        for t, shp, name in ((weight, (Cd, 16), "weight"), (bias, (Cd,), "bias")):
            if tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name}: expected contiguous FP32 CUDA tensor of shape {shp}")
        tdt = targets[0].dtype
        for v, (f, tg) in enumerate(zip(feats, targets)):
            if (f.dim() != 3 or f.shape[0] != 16 or f.dtype != torch.float32 or not f.is_cuda
                    or not f.is_contiguous()):
                raise ValueError(f"feats[{v}]: expected contiguous FP32 CUDA tensor [16, H, W]")
            if (tuple(tg.shape) != (Cd,) + tuple(f.shape[1:]) or tg.dtype != tdt
                    or tdt not in (torch.float32, torch.bfloat16) or not tg.is_cuda or not tg.is_contiguous()):
                raise ValueError(f"targets[{v}]: expected contiguous CUDA tensor [{Cd}, H, W], "
                                 "BF16 or FP32 like targets[0]")
        dev = weight.device
        if out is None:
            out = (torch.empty(1, device=dev), [torch.empty_like(f) for f in feats], torch.empty_like(weight),
                   torch.empty_like(bias))
        loss, gfs, gw, gb = out
        ws = (C.c_int32 * nv)(*[int(f.shape[2]) for f in feats])
        hs = (C.c_int32 * nv)(*[int(f.shape[1]) for f in feats])
        fp = (C.c_void_p * nv)(*[_ptr(f) for f in feats])
        tp = (C.c_void_p * nv)(*[_ptr(t) for t in targets])
        gp = (C.c_void_p * nv)(*[_ptr(g) for g in gfs])
        dt = LGS_BF16 if tdt == torch.bfloat16 else LGS_F32
        st = lib().lgs_decoder_l1_views(self._h, nv, ws, hs, Cd, fp, _ptr(weight), _ptr(bias), tp, dt,
                                        float(w_feat), gp, _ptr(gw), _ptr(gb), _ptr(loss), _stream(stream))
        if st != LGS_OK:
            self._raise(st)
        return loss, gfs, gw, gb

    def prune(self, params, k=None, tau_dist=None, tau_sim=None, min_opacity=None, max_scale=None,
              stream=None, mask=None):
        """Language-guided + geometric pruning (lgs_prune).  params: the
        Gaussian tensors (as for forward).  Returns (mask [N] uint8: bit 0
        redundant, bit 1 geometric; counts (redundant, geometric, pruned))."""
        g = gaussians_c(params["means"], params["log_scales"], params["quats"], params["logits"],
                        params["rgb"], params["feat"])
        p = lib().lgs_default_prune_params()
        for name, v in (("k", k), ("tau_dist", tau_dist), ("tau_sim", tau_sim), ("min_opacity", min_opacity),
                        ("max_scale", max_scale)):
            if v is not None:
                setattr(p, name, v)
        if mask is None:
            mask = torch.empty(g.n, dtype=torch.uint8, device=params["means"].device)
        cnt = (C.c_int64 * 3)()
        st = lib().lgs_prune(self._h, C.byref(g), C.byref(p), _ptr(mask), cnt, _stream(stream))
        if st != LGS_OK:
            self._raise(st)
        return mask, tuple(cnt)

    def backward(self, state: "State", params, grad_outs, stream=None) -> dict:
        """grad_outs: per view dict rgb [3,H,W], depth [H,W], feat [D,H,W],
        optional T [H,W] (FP32 CUDA).  Returns FP32 gradients shaped like the
        parameters plus twist [V, 6]."""
        g = gaussians_c(params["means"], params["log_scales"], params["quats"], params["logits"],
                        params["rgb"], params["feat"])
        n = g.n
        dev = params["means"].device
        V = state.n_views
        ups = (lgs_images * V)()
        keep = []
        for v, go in enumerate(grad_outs):
            H, W = state.shapes[v]
            t = {k: go[k].contiguous().float() for k in ("rgb", "depth", "feat")}
            if go.get("T") is not None:
                t["T"] = go["T"].contiguous().float()
            for k, shp in (("rgb", (3, H, W)), ("depth", (H, W)), ("feat", (state.feat_dim, H, W))):
                if tuple(t[k].shape) != shp or not t[k].is_cuda:
                    raise ValueError(f"grad_outs[{v}][{k}] must be a CUDA tensor of shape {shp}")
            keep.append(t)
            ups[v] = lgs_images(_ptr(t["rgb"]), _ptr(t["depth"]), _ptr(t["feat"]), _ptr(t.get("T")), None)
        out = {"means": torch.empty((3, n), device=dev), "log_scales": torch.empty((3, n), device=dev),
               "quats": torch.empty((4, n), device=dev), "logits": torch.empty((n,), device=dev),
               "rgb": torch.empty((3, n), device=dev), "feat": torch.empty((g.feat_dim, n), device=dev),
               "twist": torch.empty((V, 6), device=dev)}
        gr = lgs_grads(_ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                       _ptr(out["logits"]), _ptr(out["rgb"]), _ptr(out["feat"]), _ptr(out["twist"]))
        st = lib().lgs_backward(self._h, state.handle, C.byref(g), ups, C.byref(gr), _stream(stream))
        if st != LGS_OK:
            self._raise(st)
        return out


def _images_c(ims, shapes, with_T, feat_dim=None):
    V = len(ims)
    arr = (lgs_images * V)()
    for v, im in enumerate(ims):
        H, W = shapes[v]
        D = im["feat"].shape[0] if feat_dim is None else feat_dim
        for k, shp in (("rgb", (3, H, W)), ("depth", (H, W)), ("feat", (D, H, W))):
            t = im[k]
            if tuple(t.shape) != shp or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"image {v} {k}: expected contiguous FP32 CUDA tensor of shape {shp}")
        arr[v] = lgs_images(_ptr(im["rgb"]), _ptr(im["depth"]), _ptr(im["feat"]),
                            _ptr(im.get("T")) if with_T else None, None)
    return arr


def _grad_buffers(n, V, dev, feat_dim=16):
    out = {"means": torch.empty((3, n), device=dev), "log_scales": torch.empty((3, n), device=dev),
           "quats": torch.empty((4, n), device=dev), "logits": torch.empty((n,), device=dev),
           "rgb": torch.empty((3, n), device=dev), "feat": torch.empty((feat_dim, n), device=dev),
           "twist": torch.empty((V, 6), device=dev)}
    gr = lgs_grads(_ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]), _ptr(out["logits"]),
                   _ptr(out["rgb"]), _ptr(out["feat"]), _ptr(out["twist"]))
    return out, gr


def backward_l1(context: "Context", state: "State", params, outs, targets, loss_w, stream=None,
                grads=None) -> dict:
    """Backward of the L1 mapping loss (Eq. (1) without D-SSIM) of the
    forward that produced `state`: outs are that forward's images, targets
    per-view dicts (rgb, depth, feat) of FP32 CUDA tensors."""
    g = gaussians_c(params["means"], params["log_scales"], params["quats"], params["logits"],
                    params["rgb"], params["feat"])
    if grads is None:
        grads = _grad_buffers(g.n, state.n_views, params["means"].device, g.feat_dim)
    out, gr = grads
    o = _images_c(outs, state.shapes, True, state.feat_dim)
    t = _images_c(targets, state.shapes, False, state.feat_dim)
    lw = (C.c_float * 3)(*[float(x) for x in loss_w])
    st = lib().lgs_backward_l1(context._h, state.handle, C.byref(g), o, t, lw, C.byref(gr), _stream(stream))
    if st != LGS_OK:
        context._raise(st)
    return out


class State:
    def __init__(self, ctx: Context, handle, n_views, shapes, feat_dim=16):
        self.ctx, self.handle, self.n_views, self.shapes = ctx, handle, n_views, shapes
        self.feat_dim = feat_dim

    def counts(self) -> dict:
        c = lgs_counts()
        lib().lgs_state_counts(self.handle, C.byref(c))
        return {k: getattr(c, k) for k, _ in lgs_counts._fields_}

    def stage_ms(self) -> list:
        buf = (C.c_float * 5)()
        st = lib().lgs_state_stage_ms(self.handle, buf)
        if st != LGS_OK:
            raise LgsError(st, lib().lgs_last_error(self.ctx._h).decode())
        return list(buf)

    def release(self):
        if self.handle:
            lib().lgs_state_release(self.ctx._h, self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class RasterFn(torch.autograd.Function):
    """Differentiable render of every view: returns per view (rgb, depth,
    feat, T), flattened.  The pose twist input is a [V, 6] zero leaf whose
    gradient is dL/d(rho, phi) of the left perturbation Exp(xi) T_cw.

    ``storage`` is the dtype the colours and features are handed to the
    library in (torch.float32 or torch.bfloat16).  With BF16 storage and FP32
    ``rgb`` / ``feat`` tensors (master copies), the forward passes their
    round-to-nearest-even BF16 copies and the backward returns the library's
    FP32 gradient with respect to the stored values as the masters' gradient,
    so that ``.grad`` stays FP32.  (Tensors that are BF16 already are passed as
    they are; autograd then casts their gradient to BF16.)"""

    @staticmethod
    def forward(ctx, context, cams, settings, storage, means, log_scales, quats, logits, rgb, feat, twist):
        if storage == torch.bfloat16:
            rgb_s, feat_s = rgb.to(torch.bfloat16).contiguous(), feat.to(torch.bfloat16).contiguous()
        elif storage == torch.float32:
            rgb_s, feat_s = rgb, feat
        else:
            raise ValueError(f"storage must be torch.float32 or torch.bfloat16, got {storage}")
        params = {"means": means, "log_scales": log_scales, "quats": quats, "logits": logits,
                  "rgb": rgb_s, "feat": feat_s}
        outs, state = context.forward(params, cams, settings)
        ctx.state = state
        ctx.context = context
        ctx.save_for_backward(means, log_scales, quats, logits, rgb_s, feat_s)
        flat = []
        for o in outs:
            flat += [o["rgb"], o["depth"], o["feat"], o["T"]]
        return tuple(flat)

    @staticmethod
    def backward(ctx, *grads):
        means, log_scales, quats, logits, rgb_s, feat_s = ctx.saved_tensors
        params = {"means": means, "log_scales": log_scales, "quats": quats, "logits": logits,
                  "rgb": rgb_s, "feat": feat_s}
        state = ctx.state
        gos = []
        for v in range(state.n_views):
            H, W = state.shapes[v]
            gr, gd, gf, gt = grads[4 * v: 4 * v + 4]
            dev = means.device
            gos.append({"rgb": gr if gr is not None else torch.zeros((3, H, W), device=dev),
                        "depth": gd if gd is not None else torch.zeros((H, W), device=dev),
                        "feat": gf if gf is not None else torch.zeros((state.feat_dim, H, W), device=dev),
                        "T": gt})
        g = ctx.context.backward(state, params, gos)
        state.release()
        return (None, None, None, None, g["means"], g["log_scales"], g["quats"], g["logits"],
                g["rgb"], g["feat"], g["twist"])


def render(context: Context, params: dict, cams, settings: Settings | None = None, twist=None,
           storage=None):
    """Autograd-enabled render; returns a list of per-view dicts (rgb, depth,
    feat, T).  ``storage``: dtype of the colours and features handed to the
    library (default: the dtype of params["rgb"]); see RasterFn."""
    V = len(cams)
    if twist is None:
        twist = torch.zeros((V, 6), device=params["means"].device, requires_grad=True)
    storage = params["rgb"].dtype if storage is None else storage
    flat = RasterFn.apply(context, cams, settings or Settings(), storage, params["means"], params["log_scales"],
                          params["quats"], params["logits"], params["rgb"], params["feat"], twist)
    return [{"rgb": flat[4 * v], "depth": flat[4 * v + 1], "feat": flat[4 * v + 2], "T": flat[4 * v + 3]}
            for v in range(V)]
