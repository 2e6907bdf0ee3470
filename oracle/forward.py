"""Forward operators H = blockdiag(H^1, ..., H^{n_t}) (Sec. 2.1), FP64.

Radon (parallel beam).  The paper builds H^t with a fan-beam toolbox and names
no projector model; the reading used here is the pixel-driven linear ("hat")
model with unit pixels and unit detector bins:

    pixel centre      X_p = x - (nx-1)/2,  Y_p = y - (ny-1)/2
    ray coordinate    tau_p(theta) = X_p cos(theta) + Y_p sin(theta)
    bin centre        d_j = j - (n_d-1)/2
    matrix entry      a_{(theta,j),p} = max(0, 1 - |tau_p(theta) - d_j|)

so (H^t u)_{theta,j} = sum_p a_{(theta,j),p} u_p and H^T uses the same entries.
Bins outside [0, n_d) are not measured (their weights are dropped).

Blur.  A 9x9 Gaussian (sigma = 2), normalised to unit sum, zero boundary,
output the size of the input; it is symmetric, so H^T is the same sum.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------- Radon


def hat_weights(ny: int, nx: int, theta: float, n_bins: int):
    """Candidate bins and weights a_{(theta,j),p} for every pixel p of one frame.

    Returns (j, a) of shape [4, ny*nx]: for each pixel the four bins around its ray
    coordinate with weight max(0, 1 - |tau - d_j|) (zero outside the hat's support
    and for bins outside [0, n_bins)).
    """
    y, x = np.mgrid[0:ny, 0:nx]
    X = (x - (nx - 1) / 2.0).ravel()
    Y = (y - (ny - 1) / 2.0).ravel()
    tau = X * np.cos(theta) + Y * np.sin(theta)
    pos = tau + (n_bins - 1) / 2.0            # tau in bin-index units (d_j = j - (n_d-1)/2)
    base = np.floor(pos).astype(np.int64)
    js, ws = [], []
    for off in (-1, 0, 1, 2):
        j = base + off
        a = np.maximum(0.0, 1.0 - np.abs(pos - j))
        a = np.where((j >= 0) & (j < n_bins), a, 0.0)
        js.append(np.clip(j, 0, n_bins - 1))
        ws.append(a)
    return np.stack(js), np.stack(ws)


def radon_project_angle(frame: np.ndarray, theta: float, n_bins: int) -> np.ndarray:
    """(H u)_{theta, :} for one frame and one angle."""
    ny, nx = frame.shape
    j, a = hat_weights(ny, nx, theta, n_bins)
    u = frame.ravel().astype(np.float64)
    return np.bincount(j.ravel(), weights=(a * u[None, :]).ravel(), minlength=n_bins)


def radon_fwd(u: np.ndarray, angles: np.ndarray, n_bins: int) -> np.ndarray:
    """b = H u for a stack u [n_t, ny, nx] with angles [n_t, n_theta] -> [n_t, n_theta, n_bins]."""
    n_t = u.shape[0]
    out = np.zeros((n_t, angles.shape[1], n_bins))
    for t in range(n_t):
        for k in range(angles.shape[1]):
            out[t, k] = radon_project_angle(u[t], float(angles[t, k]), n_bins)
    return out


def radon_adj(b: np.ndarray, angles: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """u = H^T b: every pixel gathers a_{(theta,j),p} b_{theta,j} over angles and bins."""
    n_t, n_theta, n_bins = b.shape
    out = np.zeros((n_t, ny * nx))
    for t in range(n_t):
        for k in range(n_theta):
            j, a = hat_weights(ny, nx, float(angles[t, k]), n_bins)
            out[t] += (a * b[t, k][j]).sum(axis=0)
    return out.reshape(n_t, ny, nx)


# ---------------------------------------------------------------------------- blur


def gaussian_kernel(ksize: int = 9, sigma: float = 2.0) -> np.ndarray:
    """K(i,j) = exp(-(i^2+j^2)/(2 sigma^2)) / sum, i,j in [-(ksize//2), ksize//2]."""
    r = ksize // 2
    i = np.arange(-r, r + 1, dtype=np.float64)
    K = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * sigma * sigma))
    return K / K.sum()


def blur(u: np.ndarray, ksize: int = 9, sigma: float = 2.0) -> np.ndarray:
    """(H u)(y,x) = sum_{i,j} K(i,j) u(y-i, x-j), u = 0 outside, per frame of u [n_t, ny, nx]."""
    K = gaussian_kernel(ksize, sigma)
    r = ksize // 2
    n_t, ny, nx = u.shape
    pad = np.zeros((n_t, ny + 2 * r, nx + 2 * r))
    pad[:, r:r + ny, r:r + nx] = u
    out = np.zeros((n_t, ny, nx))
    for i in range(-r, r + 1):
        for j in range(-r, r + 1):
            # u(y-i, x-j) lives at pad index (y-i+r, x-j+r)
            out += K[i + r, j + r] * pad[:, r - i:r - i + ny, r - j:r - j + nx]
    return out


def blur_adj(y: np.ndarray, ksize: int = 9, sigma: float = 2.0) -> np.ndarray:
    """H^T y = sum_{i,j} K(i,j) y(p+(i,j)); equal to ``blur`` because K(i,j) = K(-i,-j)."""
    K = gaussian_kernel(ksize, sigma)
    r = ksize // 2
    n_t, ny, nx = y.shape
    pad = np.zeros((n_t, ny + 2 * r, nx + 2 * r))
    pad[:, r:r + ny, r:r + nx] = y
    out = np.zeros((n_t, ny, nx))
    for i in range(-r, r + 1):
        for j in range(-r, r + 1):
            out += K[i + r, j + r] * pad[:, r + i:r + i + ny, r + j:r + j + nx]
    return out
