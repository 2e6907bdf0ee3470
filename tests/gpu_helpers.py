"""Helpers shared by the GPU parity tests (packing and error measures)."""
from __future__ import annotations

import numpy as np

# Relative error bars: FP64 kernels vs the FP64 oracle, FP32 kernels (FP32 inputs upcast
# exactly for the oracle) vs the oracle.
TOL64 = 1e-12
TOL32 = 1e-5


def dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda").reshape(-1)


def host(t):
    return t.detach().double().cpu().numpy()


def pack(arrs):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrs])


def unpack(vec, shapes):
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(vec[o:o + k].reshape(s))
        o += k
    return out


def rel(a, b, scale=None):
    """||a - b|| / ||scale|| (scale defaults to b)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    s = b if scale is None else np.asarray(scale, dtype=np.float64).ravel()
    d = np.linalg.norm(s)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def roundtrip32(x):
    """The float32 value of x, upcast exactly (the oracle sees the GPU's inputs)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)
