"""Pins of the oracle's regulariser variants (Sec. 5, table of methods: D1 AnisoTV, D2 IsoTV,
D3 GS, each with and without the motion rows), against their definitions written out here:

* Theta as the mode products of the tensor U (remark on the table's notation): L_h = I (x) I (x)
  D_nx (horizontal differences), L_v = I (x) D_ny (x) I, L_t = D_nt (x) I (x) I, as explicit
  Kronecker matrices on 7 x 8 x 3 frames (x fastest) -- Theta u and Theta^T y match;
* the regularisers R_1, R_2, R_3 summed by explicit loops over pixels, locations and frames
  equal the smoothed objective as eps -> 0;
* the group MM weights equal 1/sqrt(sum of the group's squares + eps^2) computed pixel by
  pixel (IsoTV) and location by location (GS); with one frame GS is the plain l1 weighting,
  and IsoTV of an image constant along y weights its horizontal differences as l1 does;
* the quadratic tangent majorant with these weights lies above the smoothed objective and
  touches it at u^(k) (eq. QuadraticMajorantQ for groups);
* at a fixed lambda and fixed Theta the MM iterates never increase the objective;
* with V spanning R^n the iterate solves the dense weighted normal equations.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mmgks
from synth import angles_shifted, bins_for, noisy

VARIANTS = ["aniso", "iso", "gs"]


def D(n):
    """First differences (x_{i+1} - x_i), (n-1) x n, written out."""
    M = np.zeros((n - 1, n))
    for i in range(n - 1):
        M[i, i], M[i, i + 1] = -1.0, 1.0
    return M


def theta_dense(reg, nt, ny, nx):
    I = np.eye
    Lh = np.kron(I(nt), np.kron(I(ny), D(nx)))
    Lv = np.kron(I(nt), np.kron(D(ny), I(nx)))
    Lt = np.kron(D(nt), np.kron(I(ny), I(nx)))
    rows = [Lh, Lv] + ([Lt] if reg in ("aniso", "iso") else [])
    return np.vstack(rows)


def _ops(reg, nt=3, ny=7, nx=8, use_flow=False, n_theta=4):
    ang = angles_shifted(nt, n_theta, math.radians(7.0))
    g = mmgks.SeqGeom(nt, ny, nx, ang, bins_for(max(ny, nx)))
    return mmgks.StackOps([g], "radon", use_flow=use_flow, reg=reg)


@pytest.mark.parametrize("reg", VARIANTS)
def test_theta_is_the_mode_products(reg):
    rng = np.random.default_rng(1)
    nt, ny, nx = 3, 7, 8
    ops = _ops(reg, nt, ny, nx)
    T = theta_dense(reg, nt, ny, nx)
    u = rng.standard_normal(ops.n)
    np.testing.assert_allclose(ops.theta(u, ops.zero_flows()), T @ u, atol=1e-13)
    y = rng.standard_normal(T.shape[0])
    np.testing.assert_allclose(ops.thetaT(y, ops.zero_flows()), T.T @ y, atol=1e-13)


def _regulariser_by_loops(reg, u):
    nt, ny, nx = u.shape
    total = 0.0
    if reg == "aniso":
        for t in range(nt):
            for y in range(ny):
                for x in range(nx):
                    if x + 1 < nx:
                        total += abs(u[t, y, x + 1] - u[t, y, x])
                    if y + 1 < ny:
                        total += abs(u[t, y + 1, x] - u[t, y, x])
    if reg == "iso":
        for t in range(nt):
            for y in range(ny):
                for x in range(nx):
                    gx = u[t, y, x + 1] - u[t, y, x] if x + 1 < nx else 0.0
                    gy = u[t, y + 1, x] - u[t, y, x] if y + 1 < ny else 0.0
                    total += math.sqrt(gx * gx + gy * gy)
    if reg in ("aniso", "iso"):
        for t in range(nt - 1):
            total += np.abs(u[t + 1] - u[t]).sum()
    if reg == "gs":
        for y in range(ny):
            for x in range(nx - 1):
                total += math.sqrt(sum((u[t, y, x + 1] - u[t, y, x]) ** 2 for t in range(nt)))
        for y in range(ny - 1):
            for x in range(nx):
                total += math.sqrt(sum((u[t, y + 1, x] - u[t, y, x]) ** 2 for t in range(nt)))
    return total


@pytest.mark.parametrize("reg", VARIANTS)
def test_smoothed_objective_tends_to_the_regulariser(reg):
    rng = np.random.default_rng(2)
    nt, ny, nx = 3, 5, 6
    ops = _ops(reg, nt, ny, nx)
    u = rng.standard_normal((nt, ny, nx))
    nu = ops.theta(u.ravel(), ops.zero_flows())
    r = np.zeros(3)
    # j_eps = ||r||^2 + 2 lambda sum_g sqrt(||nu_g||^2 + eps^2): with lambda = 1/2, r = 0
    val = ops.j_eps(r, nu, 0.5, 1e-9)
    assert abs(val - _regulariser_by_loops(reg, u)) <= 1e-7


def test_group_weights_pixel_by_pixel():
    rng = np.random.default_rng(3)
    nt, ny, nx, eps = 2, 5, 6, 0.3
    u = rng.standard_normal((nt, ny, nx))
    for reg in ("iso", "gs"):
        ops = _ops(reg, nt, ny, nx)
        nu = ops.theta(u.ravel(), ops.zero_flows())
        w = ops.weights(nu, eps)
        ngx, ngy = nt * ny * (nx - 1), nt * (ny - 1) * nx
        wx = w[:ngx].reshape(nt, ny, nx - 1)
        wy = w[ngx:ngx + ngy].reshape(nt, ny - 1, nx)
        for t in range(nt):
            for y in range(ny):
                for x in range(nx):
                    if reg == "iso":
                        gx = u[t, y, x + 1] - u[t, y, x] if x + 1 < nx else 0.0
                        gy = u[t, y + 1, x] - u[t, y, x] if y + 1 < ny else 0.0
                        e = 1.0 / math.sqrt(gx * gx + gy * gy + eps * eps)
                        if x + 1 < nx:
                            assert abs(wx[t, y, x] - e) <= 1e-14 * e
                        if y + 1 < ny:
                            assert abs(wy[t, y, x] - e) <= 1e-14 * e
                    else:
                        if x + 1 < nx:
                            s = sum((u[k, y, x + 1] - u[k, y, x]) ** 2 for k in range(nt))
                            e = 1.0 / math.sqrt(s + eps * eps)
                            assert abs(wx[t, y, x] - e) <= 1e-14 * e
                        if y + 1 < ny:
                            s = sum((u[k, y + 1, x] - u[k, y, x]) ** 2 for k in range(nt))
                            e = 1.0 / math.sqrt(s + eps * eps)
                            assert abs(wy[t, y, x] - e) <= 1e-14 * e
        if reg == "iso":   # the temporal rows are l1
            nu_t = nu[ngx + ngy:]
            np.testing.assert_array_equal(w[ngx + ngy:], mmgks.mm_weights_sq(nu_t, eps))


def test_special_cases_reduce_to_l1():
    rng = np.random.default_rng(4)
    eps = 0.1
    # GS over one frame: every group has one member
    ops_gs, ops_m = _ops("gs", 1, 5, 6), _ops("psi", 1, 5, 6)
    u = rng.standard_normal(ops_gs.n)
    nu = ops_gs.theta(u, ops_gs.zero_flows())
    np.testing.assert_array_equal(ops_gs.weights(nu, eps), mmgks.mm_weights_sq(nu, eps))
    np.testing.assert_array_equal(nu, ops_m.theta(u, ops_m.zero_flows()))
    # IsoTV of frames constant along y: the vertical differences vanish
    ops = _ops("iso", 2, 5, 6)
    u = np.broadcast_to(rng.standard_normal((2, 1, 6)), (2, 5, 6)).ravel()
    nu = ops.theta(u, ops.zero_flows())
    ngx = 2 * 5 * 5
    np.testing.assert_array_equal(ops.weights(nu, eps)[:ngx], mmgks.mm_weights_sq(nu[:ngx], eps))


def _problem(reg, use_flow, seed=0, n=8, nt=3):
    rng = np.random.default_rng(seed)
    u = np.zeros((nt, n, n))
    for t in range(nt):
        u[t, 2:5, 1 + t:4 + t] = 1.0
    ang = angles_shifted(nt, 4, math.radians(7.0))
    g = mmgks.SeqGeom(nt, n, n, ang, bins_for(n))
    ops = mmgks.StackOps([g], "radon", use_flow=use_flow, reg=reg)
    clean = ops.A(u.ravel())
    b = noisy(clean, rng.standard_normal(clean.shape), 0.02)
    return ops, u, b, float(np.linalg.norm(b - clean))


@pytest.mark.parametrize("reg", VARIANTS)
def test_group_majorant_above_objective_and_tangent(reg):
    rng = np.random.default_rng(5)
    ops, _, b, _ = _problem(reg, True, n=6, nt=2)
    flows = [(rng.uniform(-1, 1, f[0].shape), rng.uniform(-1, 1, f[1].shape)) for f in ops.zero_flows()]
    eps, lam = 0.05, 0.3
    uk = rng.standard_normal(ops.n)
    w2 = ops.weights(ops.theta(uk, flows), eps)
    Jk = ops.j_eps(ops.A(uk) - b, ops.theta(uk, flows), lam, eps)

    def Q(u):
        r = ops.A(u) - b
        t = ops.theta(u, flows)
        return r @ r + lam * (w2 * t * t).sum()
    c = Jk - Q(uk)
    for _ in range(30):
        u = uk + rng.standard_normal(ops.n) * rng.uniform(1e-3, 3)
        assert Q(u) + c >= ops.j_eps(ops.A(u) - b, ops.theta(u, flows), lam, eps) - 1e-10
    # tangent: the directional derivatives of Q + c and J agree at u_k
    d = rng.standard_normal(ops.n)
    h = 1e-6
    dq = (Q(uk + h * d) - Q(uk - h * d)) / (2 * h)
    dj = (ops.j_eps(ops.A(uk + h * d) - b, ops.theta(uk + h * d, flows), lam, eps) -
          ops.j_eps(ops.A(uk - h * d) - b, ops.theta(uk - h * d, flows), lam, eps)) / (2 * h)
    assert abs(dq - dj) <= 1e-6 * max(1.0, abs(dj))


@pytest.mark.parametrize("reg", VARIANTS)
@pytest.mark.parametrize("use_flow", [False, True])
def test_mm_objective_monotone_at_fixed_lambda(reg, use_flow):
    ops, _, b, delta = _problem(reg, use_flow)
    # tau beyond k_max: the only flow update is at u^(0) = 0, where it gives zero flows
    p = mmgks.SolveParams(ell=4, k_max=20, tau=1000, fixed_lambda=0.05, use_flow=use_flow, eps=1e-2)
    res = mmgks.mmgks_of(ops, b, delta, p)
    J0 = ops.j_eps(-b, ops.theta(np.zeros(ops.n), ops.zero_flows()), 0.05, 1e-2)
    seq = np.concatenate([[J0], res.jeps])
    assert (np.diff(seq) <= 1e-12 * seq[0]).all()
    assert seq[-1] < seq[0]


@pytest.mark.parametrize("reg", VARIANTS)
def test_full_subspace_equals_dense_normal_equations(reg):
    ops, u_true, b, delta = _problem(reg, True, n=6, nt=2)
    n = ops.n
    p = mmgks.SolveParams(ell=10, k_max=n - 10 + 1, tau=5, n_sweeps=20, alpha=0.3)
    res = mmgks.mmgks_of(ops, b, delta, p, u_true=u_true.ravel())
    assert res.n_cols == n
    lam, w2, flows = res.lambdas[-1], res.last_w2, res.flows
    A = np.stack([ops.A(np.eye(n)[:, j]) for j in range(n)], axis=1)
    T = np.stack([ops.theta(np.eye(n)[:, j], flows) for j in range(n)], axis=1)
    M = A.T @ A + lam * T.T @ (w2[:, None] * T)
    u = np.linalg.solve(M, A.T @ b)
    np.testing.assert_allclose(res.u, u, atol=1e-8 * np.abs(u).max())
