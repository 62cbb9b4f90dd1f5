"""Seeded synthetic inputs shaped like the paper's indoor RGB-D workloads.

This module only draws random inputs: Gaussian parameters, pinhole cameras and
loss targets.  It holds none of the rendering arithmetic, so both the FP64
oracle (``oracle/``) and the HIP path (``paper_2511_16144_amd``) may use it
without sharing any of the method.

The paper evaluates on Replica, TUM-RGBD and ScanNet (Sec. IV-A.1).  Those
datasets are not available here; these scenes stand in for them with the
Gaussian counts of the paper's maps (Table "pruning ablation": 0.6-1.8 M
Gaussians) and the usual RGB-D frame sizes.

Conventions (the paper states none of these; they are readings):
  * Gaussian parameters are stored structure-of-arrays in the C ABI; here they
    are row-major [N, k] numpy arrays (transposed when uploaded).
  * quaternions are (w, x, y, z), not necessarily normalised;
  * cameras are world->camera (R_cw, t_cw) in OpenCV axes (x right, y down,
    z forward); poses are drawn camera->world and inverted;
  * every float handed to either side is a float32 value, so the oracle sees
    exactly the numbers the GPU sees.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "Camera", "Scene", "Targets", "Workload", "make_workload", "round_bf16",
    "bf16_bits", "CONFIG_NAMES", "tiny_scene", "random_upstream",
]


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R_cw: np.ndarray  # [3, 3] float32, world -> camera rotation
    t_cw: np.ndarray  # [3] float32, world -> camera translation

    def as_tuple(self):
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                self.R_cw, self.t_cw)


@dataclass
class Scene:
    means: np.ndarray       # [N, 3] float32
    log_scales: np.ndarray  # [N, 3] float32
    quats: np.ndarray       # [N, 4] float32, (w, x, y, z)
    logits: np.ndarray      # [N] float32, opacity logit
    rgb: np.ndarray         # [N, 3] float32 (bf16-exact values when dtype == "bf16")
    feat: np.ndarray        # [N, 16] float32 (idem)
    dtype: str = "f32"      # storage of rgb / feat: "f32" or "bf16"
    rgb_unrounded: np.ndarray | None = None   # FP32 values before BF16 rounding
    feat_unrounded: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        sub = lambda a: None if a is None else np.ascontiguousarray(a[idx])
        return Scene(sub(self.means), sub(self.log_scales), sub(self.quats),
                     sub(self.logits), sub(self.rgb), sub(self.feat), self.dtype,
                     sub(self.rgb_unrounded), sub(self.feat_unrounded))

    def unrounded(self) -> "Scene":
        """The same scene with FP32 appearance (before BF16 rounding)."""
        if self.rgb_unrounded is None:
            return self
        return Scene(self.means, self.log_scales, self.quats, self.logits,
                     self.rgb_unrounded, self.feat_unrounded, "f32")


@dataclass
class Targets:
    rgb: np.ndarray    # [3, H, W] float32
    depth: np.ndarray  # [H, W] float32
    feat: np.ndarray   # [16, H, W] float32


@dataclass
class Workload:
    name: str
    scene: Scene
    cams: list
    targets: list
    loss_w: tuple = (1.0, 1.0, 1.0)   # weights of the RGB, depth, feature L1 terms
    meta: dict = field(default_factory=dict)

    @property
    def pixels(self) -> int:
        return sum(c.width * c.height for c in self.cams)


CONFIG_NAMES = {
    1: "C1 plain FP32 single view: 2k Gaussians, 128x96",
    2: "C2 plain FP32 single view: 300k Gaussians, 640x480",
    3: "C3 precision: 1M Gaussians, 1200x680, BF16 color/feature",
    4: "C4 batched: 500k Gaussians, 8 views (4x640x480 + 4x320x240), BF16",
    5: "C5 differentiation: 2M Gaussians, 1296x968, BF16",
}


# --------------------------------------------------------------------------
# BF16 storage helpers (input preparation: round-to-nearest-even of FP32)
# --------------------------------------------------------------------------
def bf16_bits(x: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns (uint16), round to nearest even."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16
    return u.astype(np.uint16)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """FP32 values rounded to BF16 and widened back to FP32."""
    b = bf16_bits(x).astype(np.uint32) << 16
    return b.view(np.float32).reshape(np.shape(x))


# --------------------------------------------------------------------------
# Gaussian parameter draws (draw order: means, log-scales, quats, logits,
# RGB, features; then cameras; then targets)
# --------------------------------------------------------------------------
def _draw_attributes(rng, n, feat_dim=16):
    log_scales = rng.normal(-3.0, 0.5, size=(n, 3)).astype(np.float32)
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    quats = quats.astype(np.float32)
    logits = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3)).astype(np.float32)
    feat = rng.normal(0.0, 1.0, size=(n, feat_dim))
    feat /= np.linalg.norm(feat, axis=1, keepdims=True)
    feat = feat.astype(np.float32)
    return log_scales, quats, logits, rgb, feat


def _room_surface_points(rng, n, jitter=0.02):
    """Uniform on the 6 inner faces of the box [-3,3]x[-3,3]x[0,3] (z up),
    area-weighted, plus isotropic N(0, jitter) noise."""
    # faces: floor, ceiling (6x6), walls x=+-3, y=+-3 (6x3)
    areas = np.array([36.0, 36.0, 18.0, 18.0, 18.0, 18.0])
    face = rng.choice(6, size=n, p=areas / areas.sum())
    a = rng.uniform(0.0, 1.0, size=n)
    b = rng.uniform(0.0, 1.0, size=n)
    p = np.empty((n, 3))
    u6 = -3.0 + 6.0 * a
    v6 = -3.0 + 6.0 * b
    v3 = 3.0 * b
    m = face == 0; p[m] = np.stack([u6[m], v6[m], np.zeros(m.sum())], 1)
    m = face == 1; p[m] = np.stack([u6[m], v6[m], np.full(m.sum(), 3.0)], 1)
    m = face == 2; p[m] = np.stack([np.full(m.sum(), -3.0), u6[m], v3[m]], 1)
    m = face == 3; p[m] = np.stack([np.full(m.sum(), 3.0), u6[m], v3[m]], 1)
    m = face == 4; p[m] = np.stack([u6[m], np.full(m.sum(), -3.0), v3[m]], 1)
    m = face == 5; p[m] = np.stack([u6[m], np.full(m.sum(), 3.0), v3[m]], 1)
    p += rng.normal(0.0, jitter, size=(n, 3))
    return p.astype(np.float32)


def _yaw_camera(center, yaw, W, H, f, cx, cy) -> Camera:
    """Camera at `center` looking horizontally along yaw (z up world),
    zero pitch and roll; returns the world->camera pose."""
    zc = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    xc = np.cross(zc, np.array([0.0, 0.0, 1.0]))
    yc = np.cross(zc, xc)
    R_wc = np.stack([xc, yc, zc], axis=1)           # columns = camera axes
    R_cw = R_wc.T
    t_cw = -R_cw @ np.asarray(center, dtype=np.float64)
    return Camera(int(W), int(H), float(np.float32(f)), float(np.float32(f)),
                  float(np.float32(cx)), float(np.float32(cy)),
                  R_cw.astype(np.float32), t_cw.astype(np.float32))


def _draw_targets(rng, cam: Camera, depth_range, feat_dim=16) -> Targets:
    H, W = cam.height, cam.width
    rgb = rng.uniform(0.0, 1.0, size=(3, H, W)).astype(np.float32)
    depth = rng.uniform(depth_range[0], depth_range[1], size=(H, W)).astype(np.float32)
    f = rng.normal(0.0, 1.0, size=(feat_dim, H, W))
    f /= np.linalg.norm(f, axis=0, keepdims=True)
    return Targets(rgb, depth, f.astype(np.float32))


def make_workload(k: int, n: int | None = None, res_scale: float = 1.0,
                  with_targets: bool = True, feat_dim: int = 16) -> Workload:
    """Config k in 1..5 with its default sizes, or smaller ones for parity
    tests (`n` Gaussians, image sides times `res_scale`).  Seed = k.
    `feat_dim` sets the language-feature dimension (16 in every config; the
    feature-dimension sweep varies it)."""
    rng = np.random.Generator(np.random.PCG64(k))

    def sz(w, h):
        return max(1, int(round(w * res_scale))), max(1, int(round(h * res_scale)))

    if k == 1:
        n = 2000 if n is None else n
        W, H = sz(128, 96)
        f = 100.0 * res_scale
        cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
        z = np.cbrt(rng.uniform(1.0, 125.0, size=n))
        u = rng.uniform(-0.5, W - 0.5, size=n)
        v = rng.uniform(-0.5, H - 0.5, size=n)
        means = np.stack([(u - cx) * z / f, (v - cy) * z / f, z], 1).astype(np.float32)
        attrs = _draw_attributes(rng, n, feat_dim)
        cams = [Camera(W, H, float(np.float32(f)), float(np.float32(f)),
                       float(np.float32(cx)), float(np.float32(cy)),
                       np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
        drange, dtype, loss_w = (1.0, 5.0), "f32", (1.0, 1.0, 1.0)
    elif k in (2, 3, 5):
        n_def, (W0, H0), f0, dtype, loss_w = {
            2: (300_000, (640, 480), 577.0, "f32", (1.0, 1.0, 1.0)),
            3: (1_000_000, (1200, 680), 600.0, "bf16", (1.0, 1.0, 1.0)),
            5: (2_000_000, (1296, 968), 1170.0, "bf16", (1.0, 0.1, 1.0)),
        }[k]
        n = n_def if n is None else n
        W, H = sz(W0, H0)
        f = f0 * res_scale
        means = _room_surface_points(rng, n)
        attrs = _draw_attributes(rng, n, feat_dim)
        center = rng.uniform([-2.5, -2.5, 0.5], [2.5, 2.5, 2.5])
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        cams = [_yaw_camera(center, yaw, W, H, f, (W - 1) / 2.0, (H - 1) / 2.0)]
        drange = (0.5, 6.0)
    elif k == 4:
        n = 500_000 if n is None else n
        means = _room_surface_points(rng, n)
        attrs = _draw_attributes(rng, n, feat_dim)
        cams = []
        for v in range(8):
            ang = 2.0 * math.pi * v / 8.0
            center = (2.0 * math.cos(ang), 2.0 * math.sin(ang), 1.5)
            if v % 2 == 0:
                W, H = sz(640, 480); f = 577.0 * res_scale
            else:
                W, H = sz(320, 240); f = 288.5 * res_scale
            cams.append(_yaw_camera(center, ang + math.pi, W, H, f,
                                    (W - 1) / 2.0, (H - 1) / 2.0))
        drange, dtype, loss_w = (0.5, 6.0), "bf16", (1.0, 1.0, 1.0)
    else:
        raise ValueError(f"unknown config {k}")

    log_scales, quats, logits, rgb, feat = attrs
    scene = Scene(means, log_scales, quats, logits, rgb, feat, "f32")
    if dtype == "bf16":
        scene = Scene(means, log_scales, quats, logits, round_bf16(rgb),
                      round_bf16(feat), "bf16", rgb, feat)
    targets = [_draw_targets(rng, c, drange, feat_dim) for c in cams] if with_targets else []
    return Workload(CONFIG_NAMES[k] if (n is None or res_scale == 1.0) else
                    f"C{k} reduced: {n} Gaussians, x{res_scale:g} resolution",
                    scene, cams, targets, loss_w,
                    {"config": k, "n": n, "res_scale": res_scale, "dtype": dtype})


def tiny_scene(seed: int, n: int, W: int, H: int, f: float = 40.0,
               z_range=(1.0, 3.0), log_scale=(-2.0, 0.4)) -> Workload:
    """A few Gaussians in front of an identity camera (brute-force sizes)."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    z = rng.uniform(*z_range, size=n)
    u = rng.uniform(-1.0, W, size=n)
    v = rng.uniform(-1.0, H, size=n)
    means = np.stack([(u - cx) * z / f, (v - cy) * z / f, z], 1).astype(np.float32)
    log_scales = rng.normal(log_scale[0], log_scale[1], size=(n, 3)).astype(np.float32)
    q = rng.normal(size=(n, 4)); q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.5, 1.0, size=n).astype(np.float32)
    rgb = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    feat = rng.normal(size=(n, 16)); feat /= np.linalg.norm(feat, axis=1, keepdims=True)
    scene = Scene(means, log_scales, q.astype(np.float32), logits, rgb,
                  feat.astype(np.float32), "f32")
    cam = Camera(W, H, float(np.float32(f)), float(np.float32(f)), cx, cy,
                 np.eye(3, dtype=np.float32), np.zeros(3, np.float32))
    tg = _draw_targets(rng, cam, (1.0, 3.0))
    return Workload(f"tiny seed={seed} n={n} {W}x{H}", scene, [cam], [tg])


def random_upstream(seed: int, cams, windows=None, feat_dim: int = 16) -> list:
    """Seeded upstream gradients dL/dY per view: [4 + feat_dim, H, W] float32
    (RGB 3, depth 1, feature feat_dim).  With `windows` (list per view of
    (x0, y0, w, h) rectangles) the gradient is zero outside them."""
    rng = np.random.Generator(np.random.PCG64(7000 + seed))
    out = []
    for vi, c in enumerate(cams):
        g = rng.normal(0.0, 1.0, size=(4 + feat_dim, c.height, c.width)).astype(np.float32)
        if windows is not None:
            m = np.zeros((c.height, c.width), bool)
            for (x0, y0, w, h) in windows[vi]:
                m[y0:y0 + h, x0:x0 + w] = True
            g *= m[None]
        out.append(g)
    return out


def crop_windows(seed: int, cam: Camera, k: int = 4, size: int = 64) -> list:
    """`k` non-overlapping size x size windows at seeded positions."""
    rng = np.random.Generator(np.random.PCG64(9000 + seed))
    wins = []
    tries = 0
    while len(wins) < k and tries < 1000:
        tries += 1
        x0 = int(rng.integers(0, max(1, cam.width - size + 1)))
        y0 = int(rng.integers(0, max(1, cam.height - size + 1)))
        ok = all(x0 + size <= a or a + size <= x0 or y0 + size <= b or b + size <= y0
                 for (a, b, _, _) in wins)
        if ok:
            wins.append((x0, y0, min(size, cam.width), min(size, cam.height)))
    return wins


def loss_images(seed: int, sizes, noise: float = 0.1, independent: bool = False):
    """Rendered-like images and targets for the loss alone, per view (W, H):
    targets drawn like the workloads' (RGB U[0,1], depth U[0.5, 6], unit
    16-d features); images = target + N(0, noise) noise (RGB clipped to
    [0, 1]; depth and features with 0.3), or independent draws.  About 1 in
    500 elements of each image equals its target exactly (sign(0) cases).
    Returns (list of dicts rgb/depth/feat float32, list of Targets)."""
    rng = np.random.Generator(np.random.PCG64(11000 + seed))
    outs, tgts = [], []
    for (W, H) in sizes:
        t = _draw_targets(rng, Camera(W, H, 1.0, 1.0, 0.0, 0.0, np.eye(3, dtype=np.float32),
                                      np.zeros(3, np.float32)), (0.5, 6.0))
        if independent:
            o = {"rgb": rng.uniform(0.0, 1.0, size=t.rgb.shape),
                 "depth": rng.uniform(0.5, 6.0, size=t.depth.shape),
                 "feat": rng.normal(0.0, 1.0, size=t.feat.shape)}
        else:
            o = {"rgb": np.clip(t.rgb + rng.normal(0.0, noise, size=t.rgb.shape), 0.0, 1.0),
                 "depth": t.depth + rng.normal(0.0, 0.3, size=t.depth.shape),
                 "feat": t.feat + rng.normal(0.0, 0.3, size=t.feat.shape)}
        for k in o:
            o[k] = o[k].astype(np.float32)
            eq = rng.uniform(size=o[k].shape) < 0.002
            o[k][eq] = getattr(t, k)[eq]
        outs.append(o)
        tgts.append(t)
    return outs, tgts


def decoder_inputs(seed: int, W: int, H: int, C: int = 512):
    """Inputs of the feature-decoder loss: a rendered-like 16-channel feature
    map F [16, H, W] (N(0, 0.25) per channel), decoder weights W [C, 16]
    (N(0, 1/16)), bias [C] (N(0, 0.05)) and extractor-like targets F_gt
    [C, H, W] (N(0, 0.25)), all float32."""
    rng = np.random.Generator(np.random.PCG64(12000 + seed))
    F = rng.normal(0.0, 0.25, size=(16, H, W)).astype(np.float32)
    Wm = rng.normal(0.0, 0.25, size=(C, 16)).astype(np.float32)
    b = rng.normal(0.0, 0.05, size=C).astype(np.float32)
    G = rng.normal(0.0, 0.25, size=(C, H, W)).astype(np.float32)
    return F, Wm, b, G


def prune_scene(seed: int, n: int = 500_000, objects: int = 64, spread: float = 0.08) -> Scene:
    """The batched workload's room-surface Gaussians with language features
    that follow objects: the room is split among `objects` random centres
    (each point belongs to its nearest centre), each object has a random unit
    feature, and a point's feature is that vector plus N(0, spread) noise per
    component, normalised (neighbours on one object then have cosine
    similarity near 1 / (1 + 16 spread^2)).  Appearance stored in BF16."""
    wl = make_workload(4, n=n, with_targets=False)
    sc = wl.scene
    rng = np.random.Generator(np.random.PCG64(13000 + seed))
    centres = rng.uniform([-3.0, -3.0, 0.0], [3.0, 3.0, 3.0], size=(objects, 3))
    obj = np.empty(n, np.int64)
    for s0 in range(0, n, 65536):
        d = ((sc.means[s0:s0 + 65536, None, :].astype(np.float64) - centres[None]) ** 2).sum(-1)
        obj[s0:s0 + 65536] = d.argmin(1)
    base = rng.normal(size=(objects, 16))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    f = base[obj] + rng.normal(0.0, spread, size=(n, 16))
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    f = f.astype(np.float32)
    return Scene(sc.means, sc.log_scales, sc.quats, sc.logits, sc.rgb, round_bf16(f), "bf16", sc.rgb_unrounded, f)
