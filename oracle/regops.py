"""Regularisation operators of the image subproblem, FP64.

Psi (Sec. 4.1, eq. L).  L_d in R^{(n_d-1) x n_d} is the first-difference matrix
(rows e_{i+1} - e_i, no boundary rows).  The paper calls it "rescaled" without a
scale; the reading here is unscaled +-1 (the regularisation parameter absorbs any
scale).  Per frame, with the x-fastest ordering p = y*nx + x used throughout,
L = [I_ny (x) L_nx ; L_ny (x) I_nx] (differences along x, then along y), and
Psi = blockdiag(L, ..., L).  Edge weights multiply the outputs row by row.

Motion matrices (Sec. 3).  M(s) maps u(t+1) to an approximation of u(t) by
pulling samples at r + s(r):
  * rounding and clipping (eq. m_matrix): the sample is taken at the pixel
    nearest to r + s(r) (round half to even), clipped into the image;
  * bilinear warping: the four neighbours of r' = r + s(r) with bilinear
    weights; here the sample coordinates are clipped to [0, n-1] (the clipping
    of the rounding variant carried over to the bilinear one).
M-bar(s) has block rows [.. I, -M(s(t)) ..] and M-bar'(s') block rows
[.. -M(s'(t+1)), I ..].  The library's flow operator is L(v) = -M-bar (and
-M-bar' for the reverse direction), so that its rows read
W(v)u(t+1) - u(t) ~ u_t + v . grad u; the sign does not change any norm.

Temporal difference (Sec. 5, the spatio-temporal regularisers of the method family: the
mode-3 product U x_3 L_t with L_t the first-difference matrix in time): for every frame pair,
(L_t u)_t = u(t+1) - u(t), stored [n_pairs, ny, nx] like a flow residual (it is the flow
operator with a zero flow).

Flow arrays are [n_pairs, 2, ny, nx] with component 0 = x, 1 = y.  The reverse
flow s'(t+1) is stored at pair index t (the earlier frame of the pair).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------- Psi


def diff_matrix(n: int) -> sp.csr_matrix:
    """L_d in R^{(n-1) x n}: (L_d x)_i = x_{i+1} - x_i."""
    if n < 2:
        return sp.csr_matrix((0, n))
    return sp.diags([-np.ones(n - 1), np.ones(n - 1)], [0, 1], shape=(n - 1, n), format="csr")


def psi_frame(ny: int, nx: int) -> sp.csr_matrix:
    """L = [I_ny (x) L_nx ; L_ny (x) I_nx] for one frame (eq. L, x-fastest ordering)."""
    Dx = sp.kron(sp.identity(ny), diff_matrix(nx))
    Dy = sp.kron(diff_matrix(ny), sp.identity(nx))
    return sp.vstack([Dx, Dy]).tocsr()


def grad_fwd(u: np.ndarray, wx=None, wy=None):
    """(gx, gy) = w (.) Psi u; gx [n_t, ny, nx-1], gy [n_t, ny-1, nx]."""
    n_t, ny, nx = u.shape
    L = psi_frame(ny, nx)
    nxr = ny * (nx - 1)
    gx = np.empty((n_t, ny, nx - 1))
    gy = np.empty((n_t, ny - 1, nx))
    for t in range(n_t):
        g = L @ u[t].ravel()
        gx[t] = g[:nxr].reshape(ny, nx - 1)
        gy[t] = g[nxr:].reshape(ny - 1, nx)
    if wx is not None:
        gx = gx * wx
    if wy is not None:
        gy = gy * wy
    return gx, gy


def grad_adj(gx: np.ndarray, gy: np.ndarray, wx=None, wy=None) -> np.ndarray:
    """u = Psi^T (w (.) g)."""
    n_t, ny, _ = gx.shape
    nx = gy.shape[2]
    if wx is not None:
        gx = gx * wx
    if wy is not None:
        gy = gy * wy
    L = psi_frame(ny, nx)
    out = np.empty((n_t, ny, nx))
    for t in range(n_t):
        out[t] = (L.T @ np.concatenate([gx[t].ravel(), gy[t].ravel()])).reshape(ny, nx)
    return out


# ----------------------------------------------------------------------- motion matrices


def motion_matrix(v2: np.ndarray, interp: str = "bilinear") -> sp.csr_matrix:
    """M(s) for one pair: v2 [2, ny, nx] -> sparse (ny*nx) x (ny*nx).

    Row i = y*nx + x is the target pixel r = (x, y); its entries sample the source
    image at r + s(r)."""
    _, ny, nx = v2.shape
    y, x = np.mgrid[0:ny, 0:nx]
    rows = (y * nx + x).ravel()
    if interp == "round":
        xs = np.clip(np.rint(x + v2[0]), 0, nx - 1).astype(np.int64).ravel()
        ys = np.clip(np.rint(y + v2[1]), 0, ny - 1).astype(np.int64).ravel()
        return sp.csr_matrix((np.ones(rows.size), (rows, ys * nx + xs)), shape=(ny * nx, ny * nx))
    xq = np.clip(x + v2[0], 0.0, nx - 1.0).ravel()
    yq = np.clip(y + v2[1], 0.0, ny - 1.0).ravel()
    x0 = np.floor(xq).astype(np.int64)
    y0 = np.floor(yq).astype(np.int64)
    fx = xq - x0
    fy = yq - y0
    x1 = np.minimum(x0 + 1, nx - 1)
    y1 = np.minimum(y0 + 1, ny - 1)
    r = np.concatenate([rows] * 4)
    c = np.concatenate([y0 * nx + x0, y0 * nx + x1, y1 * nx + x0, y1 * nx + x1])
    w = np.concatenate([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy])
    return sp.csr_matrix((w, (r, c)), shape=(ny * nx, ny * nx))  # duplicates are summed


def mbar(v: np.ndarray, n_t: int, interp: str = "bilinear") -> sp.csr_matrix:
    """M-bar(s): block rows t = 0..n_t-2 equal to [.., I (col t), -M(s(t)) (col t+1), ..]."""
    n_pairs, _, ny, nx = v.shape
    ns = ny * nx
    blocks = [[None] * n_t for _ in range(n_pairs)]
    for t in range(n_pairs):
        blocks[t][t] = sp.identity(ns, format="csr")
        blocks[t][t + 1] = -motion_matrix(v[t], interp)
    for t in range(n_pairs):
        for j in range(n_t):
            if blocks[t][j] is None:
                blocks[t][j] = sp.csr_matrix((ns, ns))
    return sp.bmat(blocks, format="csr")


def mbar_rev(vr: np.ndarray, n_t: int, interp: str = "bilinear") -> sp.csr_matrix:
    """M-bar'(s'): block rows [.., -M(s'(t+1)) (col t), I (col t+1), ..]; s'(t+1) = vr[t]."""
    n_pairs, _, ny, nx = vr.shape
    ns = ny * nx
    blocks = [[None] * n_t for _ in range(n_pairs)]
    for t in range(n_pairs):
        blocks[t][t] = -motion_matrix(vr[t], interp)
        blocks[t][t + 1] = sp.identity(ns, format="csr")
    for t in range(n_pairs):
        for j in range(n_t):
            if blocks[t][j] is None:
                blocks[t][j] = sp.csr_matrix((ns, ns))
    return sp.bmat(blocks, format="csr")


def flow_matrix(v: np.ndarray, n_t: int, direction: int = 1, interp: str = "bilinear") -> sp.csr_matrix:
    """L(v) = -M-bar(v) (direction +1) or -M-bar'(v) (direction -1) over the whole stack."""
    return -(mbar(v, n_t, interp) if direction > 0 else mbar_rev(v, n_t, interp))


def flow_fwd(u: np.ndarray, v: np.ndarray, direction: int = 1, interp: str = "bilinear") -> np.ndarray:
    """r [n_pairs, ny, nx]: forward r_t = W(v_t)u_{t+1} - u_t, reverse r_t = W(v_t)u_t - u_{t+1}."""
    n_t, ny, nx = u.shape
    return (flow_matrix(v, n_t, direction, interp) @ u.ravel()).reshape(n_t - 1, ny, nx)


def flow_adj(r: np.ndarray, v: np.ndarray, n_t: int, direction: int = 1, interp: str = "bilinear") -> np.ndarray:
    """u = L(v)^T r, shape [n_t, ny, nx]."""
    _, ny, nx = r.shape
    return (flow_matrix(v, n_t, direction, interp).T @ r.ravel()).reshape(n_t, ny, nx)


# ------------------------------------------------------------------- derivative in v


def warp_dv(src: np.ndarray, v2: np.ndarray):
    """Partial derivatives of the bilinear sample (W(v)src)(r) with respect to v_x(r), v_y(r).

    With x' = x + v_x in (0, nx-1), x0 = floor(x'), fx = x' - x0 (same in y):
      d/dv_x = (1-fy)(src[y0,x1]-src[y0,x0]) + fy(src[y1,x1]-src[y1,x0])
      d/dv_y = (1-fx)(src[y1,x0]-src[y0,x0]) + fx(src[y1,x1]-src[y0,x1])
    and 0 along an axis whose coordinate is clipped (outside [0, n-1]).  At an
    integer coordinate the cell [x0, x0+1] is used (one-sided derivative)."""
    ny, nx = src.shape
    y, x = np.mgrid[0:ny, 0:nx]
    xr = x + v2[0]
    yr = y + v2[1]
    xq = np.clip(xr, 0.0, nx - 1.0)
    yq = np.clip(yr, 0.0, ny - 1.0)
    x0 = np.floor(xq).astype(np.int64)
    y0 = np.floor(yq).astype(np.int64)
    fx = xq - x0
    fy = yq - y0
    x1 = np.minimum(x0 + 1, nx - 1)
    y1 = np.minimum(y0 + 1, ny - 1)
    s00, s01 = src[y0, x0], src[y0, x1]
    s10, s11 = src[y1, x0], src[y1, x1]
    dx = (1 - fy) * (s01 - s00) + fy * (s11 - s10)
    dy = (1 - fx) * (s10 - s00) + fx * (s11 - s01)
    dx = np.where((xr < 0.0) | (xr > nx - 1.0), 0.0, dx)
    dy = np.where((yr < 0.0) | (yr > ny - 1.0), 0.0, dy)
    return dx, dy


def flow_dv(u: np.ndarray, v: np.ndarray, w: np.ndarray, direction: int = 1, interp: str = "bilinear") -> np.ndarray:
    """g_v = (d r / d v)^T w, shape [n_pairs, 2, ny, nx] (zero for the rounding warp)."""
    n_pairs = v.shape[0]
    out = np.zeros_like(v, dtype=np.float64)
    if interp == "round":
        return out
    for t in range(n_pairs):
        src = u[t + 1] if direction > 0 else u[t]
        dx, dy = warp_dv(src, v[t])
        out[t, 0] = w[t] * dx
        out[t, 1] = w[t] * dy
    return out


# ----------------------------------------------------------------------------- L_t


def tdiff_fwd(u: np.ndarray) -> np.ndarray:
    """U x_3 L_t: r[t] = u[t+1] - u[t] for t < n_t - 1 ([n_t - 1, ny, nx])."""
    return u[1:] - u[:-1]


def tdiff_adj(r: np.ndarray) -> np.ndarray:
    """(U x_3 L_t)^T: u[t] = r[t-1] (t >= 1) - r[t] (t <= n_t - 2), [n_t, ny, nx]."""
    n_pairs = r.shape[0]
    u = np.zeros((n_pairs + 1,) + r.shape[1:])
    u[1:] += r
    u[:-1] -= r
    return u
