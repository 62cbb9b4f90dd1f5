"""Device-side helpers of the GPU tests: a captured whole-step graph bound
to test-owned buffers, driven through the C ABI."""
import ctypes as C

import numpy as np
import torch

from parity import gpu_params


class GraphRun:
    """Owns the device buffers bound into one graph."""

    def __init__(self, ctx, wl, settings, capacity=0, dev="cuda", ssim_lambda=0.0):
        from paper_2511_16144_amd import binding as B
        self.B, self.ctx, self.wl = B, ctx, wl
        self.ssim_lambda = ssim_lambda
        self.params = gpu_params(wl.scene, dev)
        V = len(wl.cams)
        D = wl.scene.feat.shape[1]
        self.outs, self.tg = [], []
        self.imgs, self.tgts = (B.lgs_images * V)(), (B.lgs_images * V)()
        for v, c in enumerate(wl.cams):
            H, W = c.height, c.width
            o = {"rgb": torch.full((3, H, W), np.nan, device=dev), "depth": torch.full((H, W), np.nan, device=dev),
                 "feat": torch.full((D, H, W), np.nan, device=dev), "T": torch.full((H, W), np.nan, device=dev)}
            self.outs.append(o)
            self.imgs[v] = B.lgs_images(o["rgb"].data_ptr(), o["depth"].data_ptr(), o["feat"].data_ptr(),
                                        o["T"].data_ptr(), None)
            t = wl.targets[v]
            tt = {"rgb": torch.as_tensor(t.rgb).to(dev), "depth": torch.as_tensor(t.depth).to(dev),
                  "feat": torch.as_tensor(t.feat).to(dev)}
            self.tg.append(tt)
            self.tgts[v] = B.lgs_images(tt["rgb"].data_ptr(), tt["depth"].data_ptr(), tt["feat"].data_ptr(),
                                        None, None)
        n = wl.scene.n
        self.grads = {"means": torch.full((3, n), np.nan, device=dev),
                      "log_scales": torch.full((3, n), np.nan, device=dev),
                      "quats": torch.full((4, n), np.nan, device=dev), "logits": torch.full((n,), np.nan, device=dev),
                      "rgb": torch.full((3, n), np.nan, device=dev), "feat": torch.full((D, n), np.nan, device=dev),
                      "twist": torch.full((V, 6), np.nan, device=dev)}
        self.gr = B.lgs_grads(*[self.grads[k].data_ptr() for k in
                                ("means", "log_scales", "quats", "logits", "rgb", "feat", "twist")])
        p = self.params
        self.g = B.gaussians_c(p["means"], p["log_scales"], p["quats"], p["logits"], p["rgb"], p["feat"])
        self.cams = (B.lgs_camera * V)(*[B.camera_c(c) for c in wl.cams])
        self.lw = (C.c_float * 3)(*wl.loss_w)
        self.st = settings.to_c()
        self.h = C.c_void_p()
        rc = B.lib().lgs_graph_create(ctx._h, C.byref(self.st), C.byref(self.g), V, self.cams, self.tgts, self.lw,
                                      C.c_float(self.ssim_lambda),
                                      self.imgs, C.byref(self.gr), capacity, self.stream(), C.byref(self.h))
        self.rc = rc

    def stream(self):
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def launch(self):
        assert self.B.lib().lgs_graph_launch(self.h, self.stream()) == 0

    def status(self):
        return self.B.lib().lgs_graph_status(self.h)

    def counts(self):
        c = self.B.lgs_counts()
        assert self.B.lib().lgs_graph_counts(self.h, C.byref(c)) == 0
        return {k: getattr(c, k) for k, _ in self.B.lgs_counts._fields_}

    def snapshot(self):
        torch.cuda.synchronize()
        return ([{k: v.cpu().numpy().copy() for k, v in o.items()} for o in self.outs],
                {k: v.cpu().numpy().copy() for k, v in self.grads.items()})

    def destroy(self):
        if self.h:
            self.B.lib().lgs_graph_destroy(self.h)
            self.h = None
