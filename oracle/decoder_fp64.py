"""Plain FP64 definition of the feature-distillation loss through the decoder.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product never
imports this file.

Definition followed (Sec. III-B.3, Eq. (2): the rendered feature map passes
through a lightweight convolutional decoder that lifts it to the dimension of
the frozen extractor's features, and the loss is the L1 distance to those
features).  The paper gives neither the decoder's shape nor the extractor's
dimension; the readings (marked [reading]):

  D(F)(p) = W F(p) + b        a 1x1 convolution: one affine map R^16 -> R^C
                              per pixel, no activation [reading]
  C = 512                     dimension of F_gt [reading]; any multiple of 32
  L_feat = mean over C x H x W of |D(F) - F_gt|, times w_feat; sign(0) = 0
  F_gt at the render resolution (the lift is in channels, not in space),
  stored in BF16 [reading]; W [C, 16], b [C] and F [16, H, W] in FP32.

Gradients with respect to F, W and b by torch.autograd, pixel chunk by pixel
chunk (the loss is a sum over pixels, so the parameter gradients add up
across chunks).
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def decode(F: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """D(F) = W F + b per pixel: F [16, H, W] -> [C, H, W] (float64)."""
    d, H, Wd = F.shape
    Z = np.asarray(W, np.float64) @ np.asarray(F, np.float64).reshape(d, -1) + np.asarray(b, np.float64)[:, None]
    return Z.reshape(-1, H, Wd)


def decoder_l1(F: np.ndarray, W: np.ndarray, b: np.ndarray, Fgt: np.ndarray, w_feat: float = 1.0,
               chunk: int = 1 << 16):
    """Loss w_feat mean|W F + b - F_gt| and its gradients (dF [16, H, W],
    dW [C, 16], db [C]), float64.  F_gt is taken as given (already rounded
    to its storage type)."""
    d, H, Wd = F.shape
    C = W.shape[0]
    n = H * Wd
    Ff = np.asarray(F, np.float64).reshape(d, n)
    G = np.asarray(Fgt).reshape(C, n)          # converted to float64 chunk by chunk
    Wt = torch.tensor(np.asarray(W, np.float64), requires_grad=True)
    bt = torch.tensor(np.asarray(b, np.float64), requires_grad=True)
    scale = w_feat / (C * n)
    L = 0.0
    dF = np.empty((d, n))
    dW = np.zeros((C, d))
    db = np.zeros(C)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        Fc = torch.tensor(Ff[:, s:e], requires_grad=True)
        Z = Wt @ Fc + bt[:, None]
        Lc = scale * (Z - torch.as_tensor(np.asarray(G[:, s:e], np.float64))).abs().sum()
        gF, gW, gb = torch.autograd.grad(Lc, [Fc, Wt, bt])
        L += float(Lc.detach())
        dF[:, s:e] = gF.numpy()
        dW += gW.numpy()
        db += gb.numpy()
    return L, dF.reshape(d, H, Wd), dW, db
