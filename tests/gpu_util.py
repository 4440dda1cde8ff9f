"""Helpers for the GPU parity tests (HIP path vs the FP64 oracle)."""

import numpy as np


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device (run them with -m gpu on an MI355X)")
    import paper_1002_3675_amd._native as nat
    nat.lib()  # raises when the library is not built
    return torch


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype=None):
    import torch
    dtype = dtype or torch.float32
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def to_np(t):
    return t.detach().cpu().double().numpy()
