"""Solve-OF (Alg. 2) with p = q = 2, FP64: the paper's own flow solver.

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check and the
benchmark's CPU baseline use it; the library never does.

For one pair (u(t), u(t+1)) the flow s = (s_x, s_y) minimises (eq.
subproblem_motion_estimation_redefined with p = q = 2)

    ||Y s + u_t||^2 + lambda ||L s||^2,   Y = [diag(I_x) diag(I_y)],  L = blockdiag(D, D),

with I_x, I_y, I_t the App. C derivatives (optflow.of_derivs), u_t = I_t and D the first
differences without boundary rows (regops.psi_frame, the same D as Psi).  Alg. 2 runs MMGKS
on (Y, L, b = -u_t); with p = q = 2 the majorant weights are identically 1, so MMGKS is the
generalized Krylov subspace method (GKS) on the fixed quadratic problem:

  1. V = ell Golub-Kahan steps on Y from b (mmgks.gkb);
  2. per iteration: Y V and L V; lambda by generalized cross-validation (eq.
     gcv_functional, Sec. 4.1.3); z from the projected problem (the stacked least-squares
     form of eq. minKryov2); s = V z;
  3. r = Y^T (Y V z - b) + lambda L^T L V z, r <- r - V (V^T r) twice, stop on breakdown
     (||r|| <= 1e-14 ||Y^T b||), else append r / ||r||;
  n_iter projected solves per call (Sec. 5 runs 20), the last one ends after s = V z.

Readings (the paper is silent or garbled):
  * ell: the image solver's 10 (the paper states no separate value for Solve-OF).
  * GCV as printed, with u_reg(lambda) = V z(lambda) the projected solution and
    H_reg^dagger(lambda) = V M^-1 (Y V)^T, M = (Y V)^T Y V + lambda (L V)^T L V:
        G(lambda) = ||Y V z - b||^2 / (m - trace(M^-1 (Y V)^T Y V))^2,  m = rows of Y;
    lambda is the minimiser over x = log10 lambda found by a grid search: 32 points evenly
    over c + [-12, 12], c = log10(||Y V||_F^2 / ||L V||_F^2), then 5 refinements, each with 8
    points evenly over [x* - h, x* + h] (h: the previous spacing) around the best point so
    far; points are visited in increasing x and a point replaces the best only when its G is
    smaller by more than a relative TIE (values closer than that are ties and the earlier
    point stays: G is nearly flat towards small lambda, and the choice must not depend on
    rounding); a G that is not finite (or an M that is not positive definite) never wins.
  * Y^T b = 0 (no temporal change, or none where the frame has a gradient) gives s = 0.
  * The reverse flow is not solved for: the Remark on the reverse optical flow forms it
    from s (optflow.reverse_flow).

The p = q = 1 variant (eq. of_reg_full with p = q = 1; the paper mentions it for flow problems
on their own) is MMGKS proper on ||Y s - b||_1 + lambda ||L s||_1 smoothed with eps
(phi_eps(x) = sqrt(x^2 + eps^2), majorized with the weights 1 / phi_eps as for the image
problem, eq. QuadraticMajorantQ): at iteration k the weights come from the current iterate s^(k) (s^(0) = 0),
W_d = diag((e^2 + eps^2)^(-1/2)) on the data rows (e = Y s^(k) - b) and
W_r = diag(((L s^(k))^2 + eps^2)^(-1/2)) on the rows of L; the projected problem, GCV and the
residual use Y -> W_d^(1/2) Y, b -> W_d^(1/2) b, L -> W_r^(1/2) L (so G is the printed functional
of the weighted problem); the rest as above.  Reading: eps = 1e-3, the image problem's value.
"""
from __future__ import annotations

import numpy as np

from . import mmgks, optflow, regops

GRID0 = 32          # points of the first grid
REFINE = 5          # refinement stages
GRID_R = 8          # points per refinement stage
SPAN = 12.0         # decades on either side of the centre
TIE = 1e-9          # relative improvement of G that a later point needs to win


def pair_ops(I: np.ndarray):
    """Y, Y^T, L and L^T of one pair, I [3, ny, nx]; s is [2 ny nx] (s_x then s_y)."""
    Ix, Iy = I[0].ravel(), I[1].ravel()
    ny, nx = I.shape[1:]
    n = ny * nx
    D = regops.psi_frame(ny, nx)

    def Y(s):
        return Ix * s[:n] + Iy * s[n:]

    def Yt(e):
        return np.concatenate([Ix * e, Iy * e])

    def L(s):
        return np.concatenate([D @ s[:n], D @ s[n:]])

    def Lt(g):
        k = g.size // 2
        return np.concatenate([D.T @ g[:k], D.T @ g[k:]])

    return Y, Yt, L, Lt


EPS_L1 = 1e-3


def l1_weights(I: np.ndarray, s: np.ndarray, eps: float = EPS_L1):
    """W_d and W_r (as vectors) of the p = q = 1 majorant at the iterate s [2 n]."""
    Y, _, L, _ = pair_ops(I)
    e = Y(s) + I[2].ravel()                  # Y s - b with b = -I_t
    g = L(s)
    return 1.0 / np.sqrt(e * e + eps * eps), 1.0 / np.sqrt(g * g + eps * eps)


def gcv_value(YV: np.ndarray, LV: np.ndarray, b: np.ndarray, lam: float):
    """G(lambda) of the projected solution and its z (inf when the problem is singular)."""
    m = b.size
    K = YV.shape[1]
    S = np.vstack([YV, np.sqrt(lam) * LV])
    if np.linalg.matrix_rank(S) < K:
        return np.inf, None
    z = np.linalg.lstsq(S, np.concatenate([b, np.zeros(LV.shape[0])]), rcond=None)[0]
    res = YV @ z - b
    M = YV.T @ YV + lam * (LV.T @ LV)
    t = np.trace(np.linalg.solve(M, YV.T @ YV))
    den = (m - t) ** 2
    g = float(res @ res) / den if den > 0 else np.inf
    return (g if np.isfinite(g) else np.inf), z


def gcv_lambda(YV: np.ndarray, LV: np.ndarray, b: np.ndarray) -> float:
    """The grid-search minimiser of G (readings above)."""
    c = np.log10(max((YV * YV).sum(), 1e-300) / max((LV * LV).sum(), 1e-300))
    best_g, best_x = np.inf, c
    xs = c - SPAN + 2.0 * SPAN * np.arange(GRID0) / (GRID0 - 1)
    h = 2.0 * SPAN / (GRID0 - 1)
    for stage in range(REFINE + 1):
        if stage > 0:
            xs = best_x - h + 2.0 * h * np.arange(GRID_R) / (GRID_R - 1)
            h = 2.0 * h / (GRID_R - 1)
        for x in xs:
            g = gcv_value(YV, LV, b, 10.0 ** x)[0]
            if g < best_g * (1.0 - TIE):
                best_g, best_x = g, x
    return 10.0 ** best_x


def solve_of_pair(I: np.ndarray, ell: int = 10, n_iter: int = 20, fixed_lambda: float = 0.0,
                  basis: list = None, p: int = 2, eps: float = EPS_L1, trace: list = None):
    """s [2, ny, nx] of one pair and the lambda of every iteration (`basis`, if given, receives
    the final V; `trace`, if given, the projected problem (Y V, L V, b) of every iteration, the
    arguments of gcv_value); p = 1: the p = q = 1 MM variant."""
    ny, nx = I.shape[1:]
    b = -I[2].ravel()
    Y, Yt, L, Lt = pair_ops(I)
    atb = np.linalg.norm(Yt(b))
    if atb == 0.0:                      # no temporal change, or none where the image varies
        return np.zeros((2, ny, nx)), []
    V = mmgks.gkb(Y, Yt, b, ell)[0]
    lams = []
    s = np.zeros(2 * ny * nx)
    for k in range(n_iter):
        if p == 1:
            wd, wr = l1_weights(I, s, eps)
        else:
            wd, wr = np.ones(b.size), None
        sd = np.sqrt(wd)
        YV = np.stack([sd * Y(V[:, j]) for j in range(V.shape[1])], axis=1)
        LV = np.stack([L(V[:, j]) for j in range(V.shape[1])], axis=1)
        if wr is not None:
            LV = np.sqrt(wr)[:, None] * LV
        bw = sd * b
        if trace is not None:
            trace.append((YV, LV, bw))
        lam = fixed_lambda if fixed_lambda > 0 else gcv_lambda(YV, LV, bw)
        lams.append(lam)
        z = gcv_value(YV, LV, bw, lam)[1]
        s = V @ z
        if k == n_iter - 1:
            break
        # r = Y^T W_d (Y s - b) + lambda L^T W_r L s  (W = I for p = 2)
        r = Yt(wd * (Y(s) - b)) + lam * Lt((wr if wr is not None else 1.0) * L(s))
        r = mmgks.reorth(V, r)
        nr = np.linalg.norm(r)
        if nr <= 1e-14 * atb:
            break
        V = np.concatenate([V, (r / nr)[:, None]], axis=1)
    if basis is not None:
        basis.append(V)
    return s.reshape(2, ny, nx), lams


def solve_of(u: np.ndarray, dr: int = 1, ell: int = 10, n_iter: int = 20, fixed_lambda: float = 0.0,
             f: int = 1, p: int = 2):
    """Flows [n_pairs, 2, ny, nx] of a sequence u [n_t, ny, nx] (each pair on its own), on
    frames reduced by f (optflow's block means and upscaling) when f > 1."""
    ny, nx = u.shape[1:]
    uw = optflow.box_down(u, f) if f > 1 else u
    I = optflow.of_derivs(uw, dr)
    out = np.stack([solve_of_pair(I[t], ell, n_iter, fixed_lambda, p=p)[0] for t in range(I.shape[0])])
    return optflow.flow_up(out, f, ny, nx) if f > 1 else out
