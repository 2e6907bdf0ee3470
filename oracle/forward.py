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

Fan beam (flat detector): see fan_rays and fan_matrix (Joseph's method).

Blur.  A 9x9 Gaussian (sigma = 2), normalised to unit sum, zero boundary,
output the size of the input; it is symmetric, so H^T is the same sum.
"""
from __future__ import annotations

import math

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


# ---------------------------------------------------------------------------- fan beam


def fan_rays(theta: float, n_bins: int, dso: float, dsd: float, du: float):
    """Source position and (unnormalised) directions of the rays of one angle.

    Fan beam with a flat detector (Sec. 5 builds its operators on such a geometry and names
    no projector model).  Reading, in the pixel frame of the parallel model: detector axis
    a = (cos theta, sin theta), central ray e = (-sin theta, cos theta), point source at
    S = -dso e, flat detector at distance dsd from the source with bins of width du centred at
    u_j = (j - (n_d-1)/2) du; ray j runs from S along d_j = dsd e + u_j a.  (The trig values
    come from the C library, math.cos / math.sin, like the library's table.)"""
    c, s = math.cos(theta), math.sin(theta)
    uj = (np.arange(n_bins) - (n_bins - 1) / 2.0) * du
    dx = -dsd * s + uj * c
    dy = dsd * c + uj * s
    return (dso * s, -dso * c), dx, dy


def fan_matrix(ny: int, nx: int, theta: float, n_bins: int, dso: float, dsd: float, du: float):
    """Rows of H for one angle by Joseph's method (ray-driven linear interpolation): a ray
    with |d_y| >= |d_x| is sampled on every pixel row at its crossing X_c(Y) = S_x + (Y - S_y)
    d_x / d_y, each sample being the linear interpolation between the two pixels around X_c
    (pixels outside the frame count as 0) and weighted by the path length per row |d| / |d_y|;
    other rays likewise on the columns.  Returns a dense [n_bins, ny*nx] matrix."""
    (sx, sy), dxs, dys = fan_rays(theta, n_bins, dso, dsd, du)
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    A = np.zeros((n_bins, ny * nx))
    for j in range(n_bins):
        dx, dy = dxs[j], dys[j]
        step = np.hypot(dx, dy)
        if abs(dy) >= abs(dx):
            for y in range(ny):
                xc = sx + ((y - cy) - sy) * dx / dy + cx
                x0 = math.floor(xc)
                f = xc - x0
                for x, w in ((x0, 1.0 - f), (x0 + 1, f)):
                    if 0 <= x < nx:
                        A[j, y * nx + x] += w * step / abs(dy)
        else:
            for x in range(nx):
                yc = sy + ((x - cx) - sx) * dy / dx + cy
                y0 = math.floor(yc)
                f = yc - y0
                for y, w in ((y0, 1.0 - f), (y0 + 1, f)):
                    if 0 <= y < ny:
                        A[j, y * nx + x] += w * step / abs(dx)
    return A


def fan_fwd(u: np.ndarray, angles: np.ndarray, n_bins: int, dso: float, dsd: float, du: float) -> np.ndarray:
    """b = H u (fan beam) for u [n_t, ny, nx], angles [n_t, n_theta] -> [n_t, n_theta, n_bins]."""
    n_t, ny, nx = u.shape
    out = np.zeros((n_t, angles.shape[1], n_bins))
    for t in range(n_t):
        for k in range(angles.shape[1]):
            out[t, k] = fan_matrix(ny, nx, float(angles[t, k]), n_bins, dso, dsd, du) @ u[t].ravel()
    return out


def fan_adj(b: np.ndarray, angles: np.ndarray, ny: int, nx: int, dso: float, dsd: float, du: float) -> np.ndarray:
    """u = H^T b (fan beam)."""
    n_t, n_theta, n_bins = b.shape
    out = np.zeros((n_t, ny * nx))
    for t in range(n_t):
        for k in range(n_theta):
            out[t] += fan_matrix(ny, nx, float(angles[t, k]), n_bins, dso, dsd, du).T @ b[t, k]
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
