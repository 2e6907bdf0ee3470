"""Optical-flow subproblem, FP64.

Image derivatives (App. C).  The printed formulas are garbled (the same symbol is
used for the difference half-width and the averaging range, and the time
difference is written as central while the text calls it forward).  Reading,
with box radius dr (= Delta r) and half-sample-symmetric mirroring at borders
(index -1 -> 0, n -> n-1, "the image is flipped"):

  I_x(y,x) = 1/(2dr+1) sum_{j=-dr..dr} [u_t(y+j, x+dr) - u_t(y+j, x-dr)] / (2 dr)
  I_y(y,x) = 1/(2dr+1) sum_{j=-dr..dr} [u_t(y+dr, x+j) - u_t(y-dr, x+j)] / (2 dr)
  I_t(y,x) = 1/(2dr+1)^2 sum_{box} [u_{t+1} - u_t]

The spatial derivatives are taken on frame t (Upsilon(u(t)), Sec. 2.2); the flow
solver sees only the pair (u(t), u(t+1)) (Alg. 2), so the time difference is the
two-frame forward difference.

Flow update (eq. of_reg with p = q = 2, Horn-Schunck form).  Per pair, the energy
  E(s) = sum_p (I_x s_x + I_y s_y + I_t)^2 + gamma (||D s_x||^2 + ||D s_y||^2)
with D the first differences of regops (no boundary rows) is decreased by exact
2x2 block-Jacobi sweeps for grad E = 0:
  sbar(p)  = mean of s over the d_p in-image 4-neighbours of p
  s_new(p) = sbar - g (g . sbar + I_t) / (gamma d_p + |g|^2),   g = (I_x, I_y).
Horn-Schunck's alpha weights the smoothness term by alpha^2, so gamma = alpha^2.

Flow on rescaled frames (Sec. 4.2, cost reduction; Sec. 5 downsamples by 2 or 4 before
every flow computation and upscales the velocities).  The paper names no filters.
Reading, for a factor f: frames are reduced by f x f block means (a block at the right or
bottom edge averages its in-frame pixels only, so sizes become ceil(n / f)); the solver's
current flow is reduced the same way and divided by f as the warm start; the sweeps run on
the reduced pair; the result is sampled bilinearly at the reduced-grid position of every
pixel centre, ((x + 1/2) / f - 1/2, clamped to the grid), and multiplied by f.

Reverse flow (Remark on estimating the reverse optical flow): s'(r + s(r), t+1) =
-s(r, t), with r + s(r) rounded half-to-even to a pixel.  The paper is silent on
collisions and holes: all contributions to a pixel are averaged, pixels that
receive none get 0, targets outside the image are dropped.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .regops import diff_matrix

# ----------------------------------------------------------------------- derivatives


def of_derivs(u: np.ndarray, dr: int = 1) -> np.ndarray:
    """I [n_pairs, 3, ny, nx] = (I_x, I_y, I_t) for every pair (t, t+1) of u [n_t, ny, nx]."""
    n_t, ny, nx = u.shape
    out = np.empty((n_t - 1, 3, ny, nx))
    box = 2 * dr + 1
    for t in range(n_t - 1):
        a = np.pad(u[t], dr, mode="symmetric")
        b = np.pad(u[t + 1], dr, mode="symmetric")
        Ix = np.zeros((ny, nx))
        Iy = np.zeros((ny, nx))
        It = np.zeros((ny, nx))
        for j in range(-dr, dr + 1):
            # a[y+dr+j, x+dr+k] holds u_t(y+j, x+k)
            Ix += a[dr + j:dr + j + ny, 2 * dr:2 * dr + nx] - a[dr + j:dr + j + ny, 0:nx]
            Iy += a[2 * dr:2 * dr + ny, dr + j:dr + j + nx] - a[0:ny, dr + j:dr + j + nx]
            for k in range(-dr, dr + 1):
                It += b[dr + j:dr + j + ny, dr + k:dr + k + nx] - a[dr + j:dr + j + ny, dr + k:dr + k + nx]
        out[t, 0] = Ix / (box * 2 * dr)
        out[t, 1] = Iy / (box * 2 * dr)
        out[t, 2] = It / (box * box)
    return out


# ----------------------------------------------------------------------- HS sweeps


def neighbour_count(ny: int, nx: int) -> np.ndarray:
    """d_p: number of in-image 4-neighbours of each pixel."""
    d = np.full((ny, nx), 4.0)
    d[0, :] -= 1
    d[-1, :] -= 1
    d[:, 0] -= 1
    d[:, -1] -= 1
    return d


def neighbour_mean(s: np.ndarray) -> np.ndarray:
    """Mean of the in-image 4-neighbours of every pixel of s [ny, nx]."""
    acc = np.zeros_like(s)
    acc[1:, :] += s[:-1, :]
    acc[:-1, :] += s[1:, :]
    acc[:, 1:] += s[:, :-1]
    acc[:, :-1] += s[:, 1:]
    return acc / neighbour_count(*s.shape)


def hs_sweep(I: np.ndarray, s: np.ndarray, gamma: float) -> np.ndarray:
    """One block-Jacobi sweep for one pair: I [3, ny, nx], s [2, ny, nx] -> new s."""
    Ix, Iy, It = I
    d = neighbour_count(*Ix.shape)
    sx = neighbour_mean(s[0])
    sy = neighbour_mean(s[1])
    k = (Ix * sx + Iy * sy + It) / (gamma * d + Ix * Ix + Iy * Iy)
    return np.stack([sx - Ix * k, sy - Iy * k])


def hs_energy(I: np.ndarray, s: np.ndarray, gamma: float) -> float:
    Ix, Iy, It = I
    data = ((Ix * s[0] + Iy * s[1] + It) ** 2).sum()
    sm = 0.0
    for c in range(2):
        sm += (np.diff(s[c], axis=1) ** 2).sum() + (np.diff(s[c], axis=0) ** 2).sum()
    return float(data + gamma * sm)


def hs_direct(I: np.ndarray, gamma: float) -> np.ndarray:
    """Minimiser of E(s) for one pair: (Y^T Y + gamma blockdiag(D^T D, D^T D)) s = -Y^T I_t,
    Y = [diag(I_x) diag(I_y)] (the Upsilon of Sec. 2.2)."""
    Ix, Iy, It = I
    ny, nx = Ix.shape
    Dx = sp.kron(sp.identity(ny), diff_matrix(nx))
    Dy = sp.kron(diff_matrix(ny), sp.identity(nx))
    D = sp.vstack([Dx, Dy])
    Y = sp.hstack([sp.diags(Ix.ravel()), sp.diags(Iy.ravel())])
    R = sp.block_diag([D, D])
    A = (Y.T @ Y + gamma * (R.T @ R)).tocsc()
    rhs = -(Y.T @ It.ravel())
    s = spla.spsolve(A, rhs)
    return s.reshape(2, ny, nx)


def flow_update(u: np.ndarray, v: np.ndarray, alpha: float, n_sweeps: int, dr: int = 1) -> np.ndarray:
    """Warm-started Horn-Schunck update of v [n_pairs, 2, ny, nx] from the stack u."""
    gamma = alpha * alpha
    I = of_derivs(u, dr)
    out = np.array(v, dtype=np.float64, copy=True)
    for t in range(out.shape[0]):
        s = out[t]
        for _ in range(n_sweeps):
            s = hs_sweep(I[t], s, gamma)
        out[t] = s
    return out


# ------------------------------------------------------------------ rescaled flow


def box_down(u: np.ndarray, f: int) -> np.ndarray:
    """f x f block means of the last two axes; edge blocks average their in-frame pixels."""
    ny, nx = u.shape[-2:]
    nys, nxs = -(-ny // f), -(-nx // f)
    out = np.zeros(u.shape[:-2] + (nys, nxs))
    for by in range(nys):
        for bx in range(nxs):
            blk = u[..., by * f:min(by * f + f, ny), bx * f:min(bx * f + f, nx)]
            out[..., by, bx] = blk.sum(axis=(-2, -1)) / (blk.shape[-2] * blk.shape[-1])
    return out


def flow_up(vs: np.ndarray, f: int, ny: int, nx: int) -> np.ndarray:
    """f times the bilinear sample of vs [..., nys, nxs] at ((x + 1/2)/f - 1/2, (y + 1/2)/f - 1/2),
    positions clamped to the reduced grid -> [..., ny, nx]."""
    nys, nxs = vs.shape[-2:]
    Y = np.minimum(np.maximum((np.arange(ny) + 0.5) / f - 0.5, 0.0), nys - 1.0)
    X = np.minimum(np.maximum((np.arange(nx) + 0.5) / f - 0.5, 0.0), nxs - 1.0)
    y0 = np.minimum(np.floor(Y).astype(np.int64), nys - 1)
    x0 = np.minimum(np.floor(X).astype(np.int64), nxs - 1)
    y1 = np.minimum(y0 + 1, nys - 1)
    x1 = np.minimum(x0 + 1, nxs - 1)
    fy = (Y - y0)[:, None]          # per row
    fx = X - x0                     # per column
    a00 = vs[..., y0[:, None], x0[None, :]]
    a01 = vs[..., y0[:, None], x1[None, :]]
    a10 = vs[..., y1[:, None], x0[None, :]]
    a11 = vs[..., y1[:, None], x1[None, :]]
    return f * ((1 - fy) * ((1 - fx) * a00 + fx * a01) + fy * ((1 - fx) * a10 + fx * a11))


def flow_update_scaled(u: np.ndarray, v: np.ndarray, alpha: float, n_sweeps: int, dr: int = 1,
                       f: int = 1) -> np.ndarray:
    """flow_update on frames reduced by f (f = 1: flow_update itself)."""
    if f == 1:
        return flow_update(u, v, alpha, n_sweeps, dr)
    ny, nx = u.shape[-2:]
    vs = flow_update(box_down(u, f), box_down(v, f) / f, alpha, n_sweeps, dr)
    return flow_up(vs, f, ny, nx)


# ----------------------------------------------------------------------- reverse flow


def reverse_flow(v: np.ndarray) -> np.ndarray:
    """s'(t+1) at rint(r + s(r, t)) = -s(r, t), averaged over collisions, 0 at holes."""
    n_pairs, _, ny, nx = v.shape
    out = np.zeros_like(v, dtype=np.float64)
    y, x = np.mgrid[0:ny, 0:nx]
    for t in range(n_pairs):
        tx = np.rint(x + v[t, 0]).astype(np.int64)
        ty = np.rint(y + v[t, 1]).astype(np.int64)
        ok = (tx >= 0) & (tx < nx) & (ty >= 0) & (ty < ny)
        idx = (ty * nx + tx)[ok]
        cnt = np.bincount(idx, minlength=ny * nx)
        for c in range(2):
            acc = np.bincount(idx, weights=-v[t, c][ok], minlength=ny * nx)
            out[t, c] = np.where(cnt > 0, acc / np.maximum(cnt, 1), 0.0).reshape(ny, nx)
    return out
