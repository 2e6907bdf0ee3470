"""MMGKS-OF (Alg. 1) in FP64, following the paper's steps in order.

Image subproblem (eq. rec_problem_s_fixed_joint): min ||H u - b||^2 + lambda ||Theta u||_1
with Theta = [Psi; M-bar(s); M-bar'(s')] (l1 on every row of Theta).

Regulariser variants (Sec. 5, table of methods, and the remark on its notation; `reg`):
  "psi"    M / M-OF:    Theta = [Psi], l1 on every row (the default above);
  "aniso"  D1 AnisoTV:  Theta = [Psi; L_t], l1 on every row (the vertical, horizontal and
                        temporal first differences of the tensor U);
  "iso"    D2 IsoTV:    Theta = [Psi; L_t]; the two spatial differences of a pixel (its
                        horizontal one unless it is in the last column, its vertical one
                        unless it is in the last row) form one group measured by its l2
                        norm, the temporal differences are l1;
  "gs"     D3 GS:       Theta = [Psi]; L_s U (every spatial difference of every frame) as a
                        matrix with one row per difference location and one column per
                        frame, measured by the l2,1 norm: each location's differences over
                        all frames of its sequence form one group;
each with the motion rows [M-bar(s); M-bar'(s')] appended for the -OF variant (use_flow).
A group g enters the smoothed objective as sqrt(||(Theta u)_g||^2 + eps^2) (an l1 row is a
group of one), and its MM weight is P^2 = 1 / sqrt(||(Theta u^(k))_g||^2 + eps^2) on every row
of the group: by concavity of sqrt in ||.||^2, the same quadratic tangent majorant as for the
l1 rows (eq. QuadraticMajorantQ) with these weights.

Per outer iteration k (Alg. 1):
  1. every tau iterations (k mod tau == 0) update the flow on u^(k) and the reverse
     flow from it (Sec. 4.1.4 strategies), which changes Theta;
  2. nu = Theta u^(k); P^2 = diag((nu^2 + eps^2)^(-1/2))  (so P = (.)^(-1/4));
  3. thin QR of H V and of P Theta V (eq. QR);
  4. lambda by the discrepancy principle (Sec. 4.1.3);
  5. z from the projected normal equations (eq. minKryov2);
  6. u^(k+1) = V z;
  7. r = H^T(H V z - b) + lambda Theta^T P^2 Theta V z (the residual of eq.
     normaleqQuadMajorant; Alg. 1 prints P where eqs. normaleqQuadMajorant and the
     residual have P^2 -- the squared weight is used);
  8. r <- r - V (V^T r), done twice (classical Gram-Schmidt with one
     re-orthogonalisation; Alg. 1 prints "r - V^T r");
  9. stop on breakdown (||r|| <= 1e-14 ||H^T b||), else append r/||r|| to V.
The last iteration stops after step 6.

Readings where the paper is silent: eps = 1e-3, eta = 1.01, u^(0) = 0 unless given,
zero initial flow.  The DP root is found by bisection in log10(lambda) over
[-12, 12] + log10(||R_H||_F^2 / ||R_Theta||_F^2) with 100 halvings; if the
discrepancy at the lower end already exceeds eta*delta the lower end is taken,
if it stays below at the upper end the upper end is taken.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import forward, optflow, regops


# ---------------------------------------------------------------------------- stack


@dataclass
class SeqGeom:
    n_t: int
    ny: int
    nx: int
    angles: Optional[np.ndarray] = None   # [n_t, n_theta] for Radon
    n_bins: Optional[int] = None
    ksize: int = 9
    sigma: float = 2.0

    @property
    def n(self) -> int:
        return self.n_t * self.ny * self.nx

    @property
    def m(self) -> int:
        if self.angles is None:
            return self.n
        return self.n_t * self.angles.shape[1] * self.n_bins


class StackOps:
    """H, Theta and the flow update over a batch of sequences stored one after another."""

    def __init__(self, seqs: List[SeqGeom], op: str, use_flow: bool = True, use_reverse: bool = True,
                 interp: str = "bilinear", flow_scale: int = 1, flow_solver: str = "hs", of_ell: int = 10,
                 of_iters: int = 20, fan: tuple = None, reg: str = "psi"):
        assert reg in ("psi", "aniso", "iso", "gs"), reg
        self.reg = reg
        self.tdiff = reg in ("aniso", "iso")   # Theta holds the temporal differences L_t
        self._groups = None
        self.seqs = seqs
        self.op = op
        self.use_flow = use_flow
        self.use_reverse = use_reverse
        self.interp = interp
        self.flow_scale = flow_scale  # flow computed on frames reduced by this factor
        self.fan = fan                # op "fan": (dso, dsd, du) of the flat-detector fan beam
        # "hs": warm-started Horn-Schunck sweeps; "gks": Solve-OF (Alg. 2, GKS with GCV)
        self.flow_solver = flow_solver
        self.of_ell = of_ell
        self.of_iters = of_iters
        self.n = sum(s.n for s in seqs)
        self.m = sum(s.m for s in seqs)
        self._mats = {}

    def _flow_mat(self, i, v, n_t, direction):
        # L(v) as a sparse matrix, rebuilt only when a different flow array is passed
        key = (i, direction)
        hit = self._mats.get(key)
        if hit is None or hit[0] is not v:
            hit = (v, regops.flow_matrix(v, n_t, direction, self.interp))
            self._mats[key] = hit
        return hit[1]

    # -- unpacking
    def split_u(self, u):
        out, o = [], 0
        for s in self.seqs:
            out.append(u[o:o + s.n].reshape(s.n_t, s.ny, s.nx))
            o += s.n
        return out

    def split_b(self, b):
        out, o = [], 0
        for s in self.seqs:
            shape = (s.n_t, s.ny, s.nx) if s.angles is None else (s.n_t, s.angles.shape[1], s.n_bins)
            out.append(b[o:o + s.m].reshape(shape))
            o += s.m
        return out

    # -- H
    def A(self, u):
        parts = []
        for s, us in zip(self.seqs, self.split_u(u)):
            if self.op == "radon":
                parts.append(forward.radon_fwd(us, s.angles, s.n_bins).ravel())
            elif self.op == "fan":
                parts.append(forward.fan_fwd(us, s.angles, s.n_bins, *self.fan).ravel())
            else:
                parts.append(forward.blur(us, s.ksize, s.sigma).ravel())
        return np.concatenate(parts)

    def At(self, b):
        parts = []
        for s, bs in zip(self.seqs, self.split_b(b)):
            if self.op == "radon":
                parts.append(forward.radon_adj(bs, s.angles, s.ny, s.nx).ravel())
            elif self.op == "fan":
                parts.append(forward.fan_adj(bs, s.angles, s.ny, s.nx, *self.fan).ravel())
            else:
                parts.append(forward.blur_adj(bs, s.ksize, s.sigma).ravel())
        return np.concatenate(parts)

    # -- flows
    def zero_flows(self):
        return [(np.zeros((s.n_t - 1, 2, s.ny, s.nx)), np.zeros((s.n_t - 1, 2, s.ny, s.nx))) for s in self.seqs]

    def update_flows(self, u, flows, alpha, n_sweeps, dr):
        from . import solve_of
        out = []
        for us, (v, _) in zip(self.split_u(u), flows):
            if self.flow_solver == "gks":
                vn = solve_of.solve_of(us, dr, self.of_ell, self.of_iters, 0.0, self.flow_scale)
            else:
                vn = optflow.flow_update_scaled(us, v, alpha, n_sweeps, dr, self.flow_scale)
            vr = optflow.reverse_flow(vn) if self.use_reverse else np.zeros_like(vn)
            out.append((vn, vr))
        return out

    # -- Theta
    def theta(self, u, flows):
        parts = []
        for i, (s, us, (v, vr)) in enumerate(zip(self.seqs, self.split_u(u), flows)):
            gx, gy = regops.grad_fwd(us)
            parts += [gx.ravel(), gy.ravel()]
            if self.tdiff:
                parts.append(regops.tdiff_fwd(us).ravel())
            if self.use_flow and s.n_t > 1:
                parts.append(self._flow_mat(i, v, s.n_t, 1) @ us.ravel())
                if self.use_reverse:
                    parts.append(self._flow_mat(i, vr, s.n_t, -1) @ us.ravel())
        return np.concatenate(parts)

    def thetaT(self, y, flows):
        parts, o = [], 0
        for i, (s, (v, vr)) in enumerate(zip(self.seqs, flows)):
            nt, ny, nx = s.n_t, s.ny, s.nx
            gx = y[o:o + nt * ny * (nx - 1)].reshape(nt, ny, nx - 1)
            o += gx.size
            gy = y[o:o + nt * (ny - 1) * nx].reshape(nt, ny - 1, nx)
            o += gy.size
            us = regops.grad_adj(gx, gy)
            if self.tdiff:
                npx = (nt - 1) * ny * nx
                us = us + regops.tdiff_adj(y[o:o + npx].reshape(nt - 1, ny, nx))
                o += npx
            if self.use_flow and nt > 1:
                npx = (nt - 1) * ny * nx
                rf = y[o:o + npx].reshape(nt - 1, ny, nx)
                o += npx
                us = us + (self._flow_mat(i, v, nt, 1).T @ rf.ravel()).reshape(nt, ny, nx)
                if self.use_reverse:
                    rr = y[o:o + npx].reshape(nt - 1, ny, nx)
                    o += npx
                    us = us + (self._flow_mat(i, vr, nt, -1).T @ rr.ravel()).reshape(nt, ny, nx)
            parts.append(us.ravel())
        return np.concatenate(parts)


    # -- groups of the regulariser and the MM weights
    def group_ids(self) -> np.ndarray:
        """The group of every row of Theta, in the row order of theta(): rows of one group
        share one smoothed l2 norm in the regulariser; an l1 row is a group of its own."""
        if self._groups is not None:
            return self._groups
        ids, nxt = [], 0

        def fresh(k):
            nonlocal nxt
            out = np.arange(nxt, nxt + k)
            nxt += k
            return out

        for s in self.seqs:
            nt, ny, nx = s.n_t, s.ny, s.nx
            t, y, x = np.meshgrid(np.arange(nt), np.arange(ny), np.arange(nx), indexing="ij")
            if self.reg == "iso":
                # one group per pixel: its horizontal and its vertical difference
                pix = fresh(nt * ny * nx).reshape(nt, ny, nx)
                ids += [pix[:, :, :-1].ravel(), pix[:, :-1, :].ravel()]
            elif self.reg == "gs":
                # one group per difference location, over all frames of the sequence
                locx = fresh(ny * (nx - 1)).reshape(ny, nx - 1)
                locy = fresh((ny - 1) * nx).reshape(ny - 1, nx)
                ids += [np.broadcast_to(locx, (nt, ny, nx - 1)).ravel(),
                        np.broadcast_to(locy, (nt, ny - 1, nx)).ravel()]
            else:
                ids += [fresh(nt * ny * (nx - 1)), fresh(nt * (ny - 1) * nx)]
            if self.tdiff:
                ids.append(fresh((nt - 1) * ny * nx))
            if self.use_flow and nt > 1:
                ids.append(fresh((nt - 1) * ny * nx))
                if self.use_reverse:
                    ids.append(fresh((nt - 1) * ny * nx))
        self._groups = np.concatenate(ids).astype(np.int64)
        return self._groups

    def group_sq_norms(self, nu: np.ndarray) -> np.ndarray:
        """||nu_g||^2 of every group."""
        ids = self.group_ids()
        return np.bincount(ids, weights=nu * nu, minlength=int(ids.max()) + 1)

    def weights(self, nu: np.ndarray, eps: float) -> np.ndarray:
        """Diagonal of P_eps^2 for the rows of Theta: 1 / sqrt(||nu_g||^2 + eps^2) of each
        row's group (for l1 rows the weights of mm_weights_sq)."""
        return 1.0 / np.sqrt(self.group_sq_norms(nu)[self.group_ids()] + eps * eps)

    def j_eps(self, Au_minus_b: np.ndarray, nu: np.ndarray, lam: float, eps: float) -> float:
        """||Hu - b||^2 + 2 lambda sum_g sqrt(||nu_g||^2 + eps^2) (j_eps with groups)."""
        return float(Au_minus_b @ Au_minus_b + 2.0 * lam * np.sqrt(self.group_sq_norms(nu) + eps * eps).sum())


# ------------------------------------------------------------------------ pieces


def mm_weights_sq(nu: np.ndarray, eps: float) -> np.ndarray:
    """Diagonal of P_eps^2 = diag(1/phi_eps(nu)), phi_eps(z) = sqrt(z^2 + eps^2) (Sec. 4.1.1)."""
    return 1.0 / np.sqrt(nu * nu + eps * eps)


def j_eps(Au_minus_b: np.ndarray, nu: np.ndarray, lam: float, eps: float) -> float:
    """||Hu - b||^2 + 2 lambda sum sqrt(nu^2 + eps^2): the smoothed objective whose quadratic
    tangent majorant is ||Hu-b||^2 + lambda ||P Theta u||^2 + c (eq. QuadraticMajorantQ)."""
    return float(Au_minus_b @ Au_minus_b + 2.0 * lam * np.sqrt(nu * nu + eps * eps).sum())


def reorth(V: np.ndarray, r: np.ndarray) -> np.ndarray:
    """r - V (V^T r), applied twice."""
    if V.shape[1] == 0:
        return r
    r = r - V @ (V.T @ r)
    r = r - V @ (V.T @ r)
    return r


def gkb(A, At, b: np.ndarray, ell: int):
    """ell Golub-Kahan steps from u_1 = b/||b|| (Sec. 4.1.1), both bases re-orthogonalised.

    Returns V [n, ell], U [m, ell+1] and the lower-bidiagonal B [ell+1, ell] with
    H V = U B."""
    beta = np.linalg.norm(b)
    U = [b / beta]
    v = At(U[0])
    alpha = np.linalg.norm(v)
    V = [v / alpha]
    B = np.zeros((ell + 1, ell))
    B[0, 0] = alpha
    for i in range(1, ell + 1):
        w = A(V[-1]) - alpha * U[-1]
        w = reorth(np.stack(U, axis=1), w)
        beta = np.linalg.norm(w)
        U.append(w / beta)
        B[i, i - 1] = beta
        if i == ell:
            break
        v = At(U[-1]) - beta * V[-1]
        v = reorth(np.stack(V, axis=1), v)
        alpha = np.linalg.norm(v)
        V.append(v / alpha)
        B[i, i] = alpha
    return np.stack(V, axis=1), np.stack(U, axis=1), B


def projected_solve(RA, QAtb, RT, lam):
    """z from (R_H^T R_H + lambda R_Theta^T R_Theta) z = R_H^T Q_H^T b (eq. minKryov2)."""
    M = RA.T @ RA + lam * (RT.T @ RT)
    return np.linalg.solve(M, RA.T @ QAtb)


def discrepancy(RA, QAtb, RT, lam, bnorm2):
    """||H V z_lambda - b|| from the projected quantities."""
    z = projected_solve(RA, QAtb, RT, lam)
    r = RA @ z - QAtb
    return float(np.sqrt(max(r @ r + (bnorm2 - QAtb @ QAtb), 0.0))), z


def dp_lambda(RA, QAtb, RT, bnorm2, target, steps: int = 100):
    """Discrepancy principle: lambda with ||H u_lambda - b|| = target (bisection in log10)."""
    s = np.log10((RA * RA).sum() / max((RT * RT).sum(), 1e-300))
    lo, hi = -12.0 + s, 12.0 + s
    if discrepancy(RA, QAtb, RT, 10.0 ** lo, bnorm2)[0] > target:
        return 10.0 ** lo, 2
    if discrepancy(RA, QAtb, RT, 10.0 ** hi, bnorm2)[0] < target:
        return 10.0 ** hi, 2
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if discrepancy(RA, QAtb, RT, 10.0 ** mid, bnorm2)[0] < target:
            lo = mid
        else:
            hi = mid
    return 10.0 ** (0.5 * (lo + hi)), 0


# ------------------------------------------------------------------------ solver


@dataclass
class SolveParams:
    ell: int = 10
    k_max: int = 20
    tau: int = 1
    eps: float = 1e-3
    eta: float = 1.01
    alpha: float = 0.1
    n_sweeps: int = 200
    delta_r: int = 1
    use_flow: bool = True
    use_reverse: bool = True
    fixed_lambda: Optional[float] = None   # bypasses the DP when set
    rre_target: float = 0.0


@dataclass
class SolveResult:
    u: np.ndarray
    flows: list
    lambdas: List[float] = field(default_factory=list)
    resid: List[float] = field(default_factory=list)    # ||H u^(k+1) - b||
    rre: List[float] = field(default_factory=list)
    jeps: List[float] = field(default_factory=list)     # J_eps(u^(k+1)) at lambda^(k), Theta^(k)
    dp_status: List[int] = field(default_factory=list)  # 0 root found, 2 clamped to an end
    status: int = 0
    iters: int = 0
    last_w2: Optional[np.ndarray] = None    # P^2 of the last iteration
    n_cols: int = 0                         # columns of V in the last projected solve


def rre(u, u_true) -> float:
    """||u - u_true|| / ||u_true|| over the whole stack (Sec. 5, quality measures)."""
    return float(np.linalg.norm(u - u_true) / np.linalg.norm(u_true))


def mmgks_of(ops: StackOps, b: np.ndarray, delta: float, p: SolveParams, u0=None, u_true=None,
             flows=None) -> SolveResult:
    n = ops.n
    u = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64).ravel()
    flows = ops.zero_flows() if flows is None else flows
    V, _, _ = gkb(ops.A, ops.At, b, p.ell)
    AV = np.stack([ops.A(V[:, j]) for j in range(V.shape[1])], axis=1)
    bnorm2 = float(b @ b)
    Atb_norm = np.linalg.norm(ops.At(b))
    res = SolveResult(u=u, flows=flows)
    for k in range(p.k_max):
        if ops.use_flow and k % p.tau == 0:
            flows = ops.update_flows(u, flows, p.alpha, p.n_sweeps, p.delta_r)
        nu = ops.theta(u, flows)
        w2 = ops.weights(nu, p.eps)
        TV = np.stack([ops.theta(V[:, j], flows) for j in range(V.shape[1])], axis=1)
        PTV = np.sqrt(w2)[:, None] * TV
        QA, RA = np.linalg.qr(AV)
        _, RT = np.linalg.qr(PTV)
        QAtb = QA.T @ b
        if p.fixed_lambda is not None:
            lam, st = p.fixed_lambda, 0
        else:
            lam, st = dp_lambda(RA, QAtb, RT, bnorm2, p.eta * delta)
        res.status = max(res.status, st)
        res.dp_status.append(st)
        z = projected_solve(RA, QAtb, RT, lam)
        u = V @ z
        Avz = AV @ z
        res.lambdas.append(lam)
        res.last_w2 = w2
        res.n_cols = V.shape[1]
        res.resid.append(float(np.linalg.norm(Avz - b)))
        res.jeps.append(ops.j_eps(Avz - b, TV @ z, lam, p.eps))
        if u_true is not None:
            res.rre.append(rre(u, u_true))
        res.iters = k + 1
        if u_true is not None and p.rre_target > 0 and res.rre[-1] <= p.rre_target:
            break
        if k == p.k_max - 1:
            break
        r = ops.At(Avz - b) + lam * ops.thetaT(w2 * (TV @ z), flows)
        r = reorth(V, r)
        nr = np.linalg.norm(r)
        if nr <= 1e-14 * Atb_norm:
            res.status = max(res.status, 3)
            break
        vnew = r / nr
        V = np.concatenate([V, vnew[:, None]], axis=1)
        AV = np.concatenate([AV, ops.A(vnew)[:, None]], axis=1)
    res.u = u
    res.flows = flows
    return res
