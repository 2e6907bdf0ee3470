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


# Floor of the element-wise bar, as a fraction of the RMS of the scale: an element whose own
# scale is tiny (cancellation in |Op||x| itself) is held to tol * FLOOR * rms(scale) instead.
FLOOR = 1e-2


def assert_close(got, exp, tol, scale=None, elementwise=None, msg=None, tol_inf=None):
    """Parity of `got` against `exp` at relative level `tol`, three ways:
      norm-wise     ||d||_2 / ||s||_2 < tol
      max-norm      ||d||_inf / ||s||_inf < tol
      element-wise  |d_i| <= tol * (s_i + FLOOR * rms(s)) for every i
    with d = got - exp and s = |scale| (a per-element forward-error scale such as |Op||x|)
    or |exp| when no scale is given.  The element-wise bar is applied when a scale is given
    (a per-element bound of the rounding error) unless elementwise=False, and for scale-less
    comparisons only when elementwise=True.  A seam or border of a few elements with an
    error far above rounding fails the max-norm or element-wise bar even when the 2-norm over
    millions of elements does not see it.  tol_inf (default tol) is the max-norm bar; solution-
    level comparisons of iterative FP32 pipelines set it apart from the norm-wise bar.
    Returns (norm-wise, max-norm) ratios."""
    a = np.asarray(got, dtype=np.float64).ravel()
    b = np.asarray(exp, dtype=np.float64).ravel()
    if scale is None:
        s = np.abs(b)
    else:
        sc = np.asarray(scale, dtype=np.float64)
        s = np.abs(sc.ravel() if sc.size == b.size else np.broadcast_to(sc, np.shape(exp)).ravel())
    d = np.abs(a - b)
    tag = "" if msg is None else f" [{msg}]"
    assert np.all(np.isfinite(a)), f"non-finite output{tag}"
    n2 = float(np.linalg.norm(s))
    r2 = float(np.linalg.norm(d)) / (n2 if n2 > 0 else 1.0)
    assert r2 < tol, f"norm-wise {r2:.3e} >= {tol:.1e}{tag}"
    ninf = float(s.max()) if s.size else 0.0
    rinf = float(d.max() if d.size else 0.0) / (ninf if ninf > 0 else 1.0)
    ti = tol if tol_inf is None else tol_inf
    assert rinf < ti, f"max-norm {rinf:.3e} >= {ti:.1e}{tag}"
    if elementwise is None:
        elementwise = scale is not None
    if elementwise and s.size:
        rms = n2 / np.sqrt(s.size)
        bound = tol * (s + FLOOR * rms)
        bad = d > bound
        if bad.any():
            i = int(np.argmax(d / bound))
            raise AssertionError(f"element-wise: {int(bad.sum())} of {s.size} elements above the bar, worst index "
                                 f"{i}: |d| = {d[i]:.3e}, scale = {s[i]:.3e}, rms scale = {rms:.3e}{tag}")
    return r2, rinf
