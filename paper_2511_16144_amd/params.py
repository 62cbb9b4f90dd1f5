"""Marshalling of host arrays into the device layout the C ABI takes."""
from __future__ import annotations

import numpy as np
import torch


def params_from_arrays(means, log_scales, quats, logits, rgb, feat, device="cuda",
                       appearance_dtype=torch.float32) -> dict:
    """Row-major [N, k] host arrays -> structure-of-arrays [k, N] device
    tensors (means, log_scales, quats, logits FP32; rgb, feat in
    `appearance_dtype`, FP32 or BF16)."""
    def soa(a, dt=torch.float32):
        t = torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float32).T))
        return t.to(device=device, dtype=dt).contiguous()
    return {
        "means": soa(means), "log_scales": soa(log_scales), "quats": soa(quats),
        "logits": torch.as_tensor(np.asarray(logits, dtype=np.float32)).to(device).contiguous(),
        "rgb": soa(rgb, appearance_dtype), "feat": soa(feat, appearance_dtype),
    }

