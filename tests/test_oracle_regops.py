"""Pins of the oracle's Psi, motion matrices and flow derivative.

Psi: agrees with numpy.diff; Psi^T Psi is the textbook 5-point graph Laplacian with
Neumann boundary (degree minus adjacency, built by explicit loops); constants map to 0,
ramps to constants; weighted adjoint identity.
Flow operator: exact zero residual for integer translations (bilinear and rounding),
v = 0 gives the temporal difference, rows of W(v) reproduce linear functions exactly
(bilinear interpolation is exact on affine data) so constants give a zero residual,
on a static bilinear image the residual is h v.grad f plus its exact second-order
remainder (the linearisation of Sec. 3), the rounding warp is the Kronecker-delta
permutation of eq. m_matrix for an interior integer shift, adjoint identity.
d/dv: central finite differences of the oracle's forward residual.
"""
import numpy as np
import pytest

from oracle import regops


def _rng(s=0):
    return np.random.default_rng(s)


def test_psi_matches_numpy_diff_and_weights():
    r = _rng(1)
    u = r.standard_normal((3, 7, 11))
    gx, gy = regops.grad_fwd(u)
    np.testing.assert_array_equal(gx, np.diff(u, axis=2))
    np.testing.assert_array_equal(gy, np.diff(u, axis=1))
    wx = r.random(gx.shape)
    wy = r.random(gy.shape)
    gxw, gyw = regops.grad_fwd(u, wx, wy)
    np.testing.assert_allclose(gxw, wx * np.diff(u, axis=2))
    a = r.standard_normal(gx.shape)
    b = r.standard_normal(gy.shape)
    lhs = (gxw * a).sum() + (gyw * b).sum()
    rhs = (u * regops.grad_adj(a, b, wx, wy)).sum()
    assert abs(lhs - rhs) < 1e-12


def test_psi_normal_is_neumann_laplacian():
    ny, nx = 5, 6
    L = regops.psi_frame(ny, nx).toarray()
    lap = np.zeros((ny * nx, ny * nx))
    for y in range(ny):
        for x in range(nx):
            p = y * nx + x
            for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                yy, xx = y + dy, x + dx
                if 0 <= yy < ny and 0 <= xx < nx:
                    lap[p, p] += 1
                    lap[p, yy * nx + xx] -= 1
    np.testing.assert_array_equal(L.T @ L, lap)


def test_psi_const_and_ramp():
    y, x = np.mgrid[0:6, 0:9]
    u = (2.5 * x - 1.25 * y + 3.0)[None]
    gx, gy = regops.grad_fwd(u)
    np.testing.assert_allclose(gx, 2.5)
    np.testing.assert_allclose(gy, -1.25)
    gx, gy = regops.grad_fwd(np.full((2, 4, 4), 7.0))
    assert np.abs(gx).max() == 0 and np.abs(gy).max() == 0


def _translating_square(n, n_t, vx, vy):
    u = np.zeros((n_t, n, n))
    for t in range(n_t):
        x0, y0 = 5 + vx * t, 6 + vy * t
        u[t, y0:y0 + 4, x0:x0 + 5] = 1.0 + 0.1 * np.arange(5)[None, :]
    return u


@pytest.mark.parametrize("interp", ["bilinear", "round"])
def test_flow_integer_translation_zero_residual(interp):
    n, n_t, vx, vy = 20, 4, 2, -1
    u = _translating_square(n, n_t, vx, vy)
    # pulling u(t+1) at r + s gives u(t) when s is the displacement t -> t+1
    v = np.zeros((n_t - 1, 2, n, n))
    v[:, 0], v[:, 1] = vx, vy
    r = regops.flow_fwd(u, v, 1, interp)
    assert np.abs(r).max() == 0.0
    # reverse pairing: sample u(t) at r - s to reach u(t+1)
    rr = regops.flow_fwd(u, -v, -1, interp)
    assert np.abs(rr).max() == 0.0


def test_flow_zero_velocity_is_time_difference():
    u = _rng(2).standard_normal((4, 6, 7))
    v = np.zeros((3, 2, 6, 7))
    np.testing.assert_array_equal(regops.flow_fwd(u, v, 1), u[1:] - u[:-1])
    np.testing.assert_array_equal(regops.flow_fwd(u, v, -1), u[:-1] - u[1:])


def test_bilinear_reproduces_affine_and_constants():
    n = 12
    r = _rng(3)
    v = r.uniform(-1.5, 1.5, size=(1, 2, n, n))
    y, x = np.mgrid[0:n, 0:n]
    f = 0.7 * x - 0.3 * y + 2.0
    u = np.stack([np.zeros((n, n)), f])
    res = regops.flow_fwd(u, v, 1)[0]
    xq = np.clip(x + v[0, 0], 0, n - 1)
    yq = np.clip(y + v[0, 1], 0, n - 1)
    np.testing.assert_allclose(res, 0.7 * xq - 0.3 * yq + 2.0, atol=1e-13)
    uc = np.full((3, n, n), 4.0)
    vv = r.uniform(-3, 3, size=(2, 2, n, n))
    assert np.abs(regops.flow_fwd(uc, vv, 1)).max() < 1e-13
    assert np.abs(regops.flow_fwd(uc, vv, -1)).max() < 1e-13


def test_flow_taylor_exact_on_bilinear_functions():
    # Bilinear interpolation is exact on f = a + b x + c y + d x y, so the warp residual
    # of a static image equals f(r + hv) - f(r) = h v.grad f(r) + h^2 d v_x v_y exactly:
    # the first-order (Upsilon s) term plus the known second-order remainder.
    n = 16
    y, x = np.mgrid[0:n, 0:n].astype(float)
    a, b, c, d = 0.3, 0.7, -0.4, 0.05
    f = a + b * x + c * y + d * x * y
    r = _rng(4)
    dir_ = r.uniform(-1, 1, size=(1, 2, n, n))
    inner = (slice(2, -2), slice(2, -2))
    for h in (0.8, 0.3, 0.05):
        res = regops.flow_fwd(np.stack([f, f]), h * dir_, 1)[0]
        vx, vy = h * dir_[0, 0], h * dir_[0, 1]
        first = vx * (b + d * y) + vy * (c + d * x)
        np.testing.assert_allclose(res[inner], (first + d * vx * vy)[inner], atol=1e-12)


def test_round_warp_is_permutation_for_interior_shift():
    n = 9
    v = np.zeros((2, n, n))
    v[0], v[1] = 1.0, -2.0
    M = regops.motion_matrix(v, "round").toarray()
    # Kronecker-delta form (eq. m_matrix): row r has a single 1 at r + s (clipped)
    E = np.zeros((n * n, n * n))
    for yy in range(n):
        for xx in range(n):
            E[yy * n + xx, min(max(yy - 2, 0), n - 1) * n + min(max(xx + 1, 0), n - 1)] = 1.0
    np.testing.assert_array_equal(M, E)
    rows_inner = [yy * n + xx for yy in range(2, n) for xx in range(0, n - 1)]
    sub = M[rows_inner]
    assert (sub.sum(axis=0) <= 1).all() and (sub.sum(axis=1) == 1).all()


@pytest.mark.parametrize("direction", [1, -1])
def test_flow_adjoint(direction):
    r = _rng(5)
    n_t, ny, nx = 4, 9, 8
    u = r.standard_normal((n_t, ny, nx))
    v = r.uniform(-2.5, 2.5, size=(n_t - 1, 2, ny, nx))
    w = r.standard_normal((n_t - 1, ny, nx))
    lhs = (regops.flow_fwd(u, v, direction) * w).sum()
    rhs = (u * regops.flow_adj(w, v, n_t, direction)).sum()
    assert abs(lhs - rhs) < 1e-12


@pytest.mark.parametrize("direction", [1, -1])
def test_flow_dv_central_differences(direction):
    from synth import nudge_off_kinks

    r = _rng(6)
    n_t, n = 3, 10
    u = r.standard_normal((n_t, n, n))
    v = nudge_off_kinks(r.uniform(-3, 3, size=(n_t - 1, 2, n, n)), 1e-3)
    w = r.standard_normal((n_t - 1, n, n))
    g = regops.flow_dv(u, v, w, direction)
    h = 1e-4
    fd = np.zeros_like(v)
    # every velocity entry only affects its own output pixel: perturb all at once per component
    for c in range(2):
        e = np.zeros_like(v)
        e[:, c] = h
        fp = regops.flow_fwd(u, v + e, direction)
        fm = regops.flow_fwd(u, v - e, direction)
        fd[:, c] = w * (fp - fm) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-9)
