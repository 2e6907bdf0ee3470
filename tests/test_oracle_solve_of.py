"""Pins of the oracle's Solve-OF (Alg. 2, p = q = 2: GKS with GCV).

* The GCV value of the projected solution equals the printed functional evaluated densely
  on matrices built entry by entry (so Y, L and the formula are all pinned), for the
  identity basis and for any orthonormal basis of the whole space.
* With a fixed lambda and a basis that grows to the whole space, the GKS flow is the
  minimiser of the p = q = 2 flow energy, i.e. the direct Horn-Schunck solve with
  gamma = lambda (itself pinned against the normal equations).
* Each new basis vector is the energy gradient at the current iterate, orthogonalised
  (dense matrices), and the iterate minimises the energy over the basis.
* The grid search finds the minimum of G over 24 decades that a dense brute-force scan
  finds.
* Scaling the frames by 4 leaves the flow unchanged and multiplies every lambda by 16
  (the data term scales by 16, the regulariser does not).
* No temporal change gives zero flow; a smooth pattern translating by half a pixel gets a
  flow along the shift of a size between 0.2 and 0.6 px in the interior.
"""
import numpy as np
import pytest

from oracle import mmgks, optflow, solve_of


def _dense_ops(I):
    """Y and L as dense matrices, entry by entry."""
    _, ny, nx = I.shape
    n = ny * nx
    Y = np.zeros((n, 2 * n))
    for p in range(n):
        Y[p, p] = I[0].ravel()[p]
        Y[p, n + p] = I[1].ravel()[p]
    rows = []
    for y in range(ny):
        for x in range(nx - 1):
            r = np.zeros(n)
            r[y * nx + x + 1], r[y * nx + x] = 1.0, -1.0
            rows.append(r)
    for y in range(ny - 1):
        for x in range(nx):
            r = np.zeros(n)
            r[(y + 1) * nx + x], r[y * nx + x] = 1.0, -1.0
            rows.append(r)
    D = np.array(rows)
    Z = np.zeros_like(D)
    L = np.block([[D, Z], [Z, D]])
    return Y, L


def _pair(seed, ny=3, nx=4):
    r = np.random.default_rng(seed)
    u = r.standard_normal((2, ny, nx))
    return optflow.of_derivs(u, 1)[0]


def _dense_gcv(Y, L, b, lam):
    M = Y.T @ Y + lam * L.T @ L
    x = np.linalg.solve(M, Y.T @ b)
    res = Y @ x - b
    hat = Y @ np.linalg.solve(M, Y.T)
    return float(res @ res) / (np.trace(np.eye(Y.shape[0]) - hat)) ** 2


@pytest.mark.parametrize("lam", [1e-3, 0.1, 7.0])
def test_gcv_value_equals_dense_functional(lam):
    I = _pair(1)
    Y, L = _dense_ops(I)
    b = -I[2].ravel()
    exp = _dense_gcv(Y, L, b, lam)
    N = Y.shape[1]
    got, _ = solve_of.gcv_value(Y, L, b, lam)                     # V = identity
    assert abs(got - exp) <= 1e-10 * exp
    Q = np.linalg.qr(np.random.default_rng(2).standard_normal((N, N)))[0]
    got, _ = solve_of.gcv_value(Y @ Q, L @ Q, b, lam)             # any orthonormal basis
    assert abs(got - exp) <= 1e-10 * exp
    # the oracle's operator closures are the dense matrices
    Yf, Ytf, Lf, Ltf = solve_of.pair_ops(I)
    s = np.random.default_rng(3).standard_normal(N)
    assert np.allclose(Yf(s), Y @ s, atol=1e-14) and np.allclose(Lf(s), L @ s, atol=1e-14)
    e, g = np.random.default_rng(4).standard_normal(Y.shape[0]), np.random.default_rng(5).standard_normal(L.shape[0])
    assert np.allclose(Ytf(e), Y.T @ e, atol=1e-14) and np.allclose(Ltf(g), L.T @ g, atol=1e-14)


@pytest.mark.parametrize("lam", [0.05, 2.0])
def test_full_space_gks_is_the_flow_energy_minimiser(lam):
    I = _pair(6)
    s, lams = solve_of.solve_of_pair(I, ell=6, n_iter=40, fixed_lambda=lam)
    exp = optflow.hs_direct(I, lam)
    assert np.linalg.norm(s - exp) <= 1e-9 * np.linalg.norm(exp)
    assert all(x == lam for x in lams)


@pytest.mark.parametrize("k", [1, 3])
def test_basis_grows_by_the_energy_gradient(k):
    """After k projected solves at a fixed lambda, the new basis vector is the part of the
    gradient of ||Y s - b||^2 + lambda ||L s||^2 at s_k (dense matrices) orthogonal to the
    basis; the basis stays orthonormal."""
    I = _pair(10, 4, 5)
    Y, L = _dense_ops(I)
    b = -I[2].ravel()
    lam = 0.3
    Vs, Vn = [], []
    s, _ = solve_of.solve_of_pair(I, ell=4, n_iter=k, fixed_lambda=lam, basis=Vs)
    solve_of.solve_of_pair(I, ell=4, n_iter=k + 1, fixed_lambda=lam, basis=Vn)
    V, W = Vs[0], Vn[0]
    assert W.shape[1] == V.shape[1] + 1 and np.allclose(W[:, :-1], V, atol=1e-15)
    grad = Y.T @ (Y @ s.ravel() - b) + lam * (L.T @ (L @ s.ravel()))
    g = grad - V @ (V.T @ grad)
    np.testing.assert_allclose(W[:, -1], g / np.linalg.norm(g), atol=1e-10)
    np.testing.assert_allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-12)
    # s_k minimises the energy over the span of V: its gradient is orthogonal to V
    assert np.abs(V.T @ grad).max() <= 1e-10 * np.abs(grad).max()


def test_grid_search_finds_the_dense_minimum():
    """On the projected problem the solver meets (8 Golub-Kahan columns of a noisy
    translating pattern; G has an interior minimum): the search's G is the minimum of a
    brute-force scan over the same 24 decades."""
    ny, nx = 6, 7
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    r = np.random.default_rng(0)
    pat = lambda sx: np.sin(0.6 * (x - sx)) + np.cos(0.5 * y)
    u = np.stack([pat(0.0) + 0.05 * r.standard_normal((ny, nx)), pat(0.4) + 0.05 * r.standard_normal((ny, nx))])
    I = optflow.of_derivs(u, 1)[0]
    Y, L = _dense_ops(I)
    b = -I[2].ravel()
    Yf, Ytf, _, _ = solve_of.pair_ops(I)
    V = mmgks.gkb(Yf, Ytf, b, 8)[0]
    YV, LV = Y @ V, L @ V
    lam = solve_of.gcv_lambda(YV, LV, b)
    g_found = _dense_gcv(YV, LV, b, lam)
    c = np.log10((YV * YV).sum() / (LV * LV).sum())
    xs = np.linspace(c - 12, c + 12, 24001)
    gs = np.array([_dense_gcv(YV, LV, b, 10.0 ** x) for x in xs])
    assert 0 < gs.argmin() < xs.size - 1
    assert g_found <= gs.min() * (1 + 1e-9)
    assert gs[0] > g_found and gs[-1] > g_found


def test_scaling_the_frames():
    r = np.random.default_rng(8)
    u = np.cumsum(np.cumsum(r.standard_normal((2, 10, 12)), axis=1), axis=2) * 0.1
    I1 = optflow.of_derivs(u, 1)[0]
    I4 = optflow.of_derivs(4.0 * u, 1)[0]
    s1, l1 = solve_of.solve_of_pair(I1, ell=5, n_iter=6)
    s4, l4 = solve_of.solve_of_pair(I4, ell=5, n_iter=6)
    assert np.linalg.norm(s4 - s1) <= 1e-9 * np.linalg.norm(s1)
    np.testing.assert_allclose(np.array(l4), 16.0 * np.array(l1), rtol=1e-9)


def test_no_change_and_translation():
    ny, nx = 24, 26
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    def pattern(sx):
        return np.sin(0.35 * (x - sx)) + np.cos(0.27 * y)
    u0 = np.stack([pattern(0.0), pattern(0.0)])
    assert not np.any(solve_of.solve_of(u0, n_iter=4))
    u = np.stack([pattern(0.0), pattern(0.5)])         # content moves +0.5 px in x
    s = solve_of.solve_of(u, ell=10, n_iter=20)[0]
    inner = (slice(4, -4), slice(4, -4))
    # 20 projected solves reach part of the way (GCV picks a small lambda; the basis is
    # the regulariser): the right direction and about half to all of the shift
    assert 0.2 < np.median(s[0][inner]) < 0.6
    assert abs(np.median(s[1][inner])) < 0.05


# ------------------------------------------------------------------ p = q = 1 variant


def _j_l1(I, s, lam, eps):
    Y, _, L, _ = solve_of.pair_ops(I)
    e = Y(s.ravel()) + I[2].ravel()
    g = L(s.ravel())
    return float(np.sqrt(e * e + eps * eps).sum() + lam * np.sqrt(g * g + eps * eps).sum())


def test_l1_with_huge_eps_is_the_quadratic_solver():
    """eps far above every residual makes both weights the same constant 1/eps: the weighted
    problem is the p = q = 2 one scaled, with the same GCV choice and the same flow."""
    I = optflow.of_derivs(np.stack([np.sin(0.5 * np.arange(11))[None, :] * np.ones((9, 1)),
                                    np.sin(0.5 * (np.arange(11) - 0.3))[None, :] * np.ones((9, 1))]) +
                          0.01 * np.random.default_rng(11).standard_normal((2, 9, 11)), 1)[0]
    s2, l2 = solve_of.solve_of_pair(I, ell=5, n_iter=6)
    s1, l1 = solve_of.solve_of_pair(I, ell=5, n_iter=6, p=1, eps=1e8)
    assert np.linalg.norm(s1 - s2) <= 1e-8 * np.linalg.norm(s2)
    np.testing.assert_allclose(l1, l2, rtol=1e-8)


@pytest.mark.parametrize("lam", [0.05, 0.5])
def test_l1_majorize_minimize_decreases_the_objective(lam):
    """At a fixed lambda every MM iterate lowers the smoothed l1 objective (the iterate of
    step k lies in the grown basis of step k + 1, and the quadratic majorant touches J there)."""
    I = _pair(12, 5, 6)
    eps = 1e-2
    prev = None
    for k in range(1, 12):
        s, _ = solve_of.solve_of_pair(I, ell=4, n_iter=k, fixed_lambda=lam, p=1, eps=eps)
        j = _j_l1(I, s, lam, eps)
        if prev is not None:
            assert j <= prev * (1 + 1e-12), k
        prev = j


def test_l1_converges_to_a_stationary_point():
    """With a basis that grows to the whole space and a fixed lambda, the iterates approach
    a zero of the gradient of the smoothed objective (dense matrices)."""
    I = _pair(13, 3, 4)
    Y, L = _dense_ops(I)
    b = -I[2].ravel()
    lam, eps = 0.2, 1e-1
    s, _ = solve_of.solve_of_pair(I, ell=4, n_iter=32, fixed_lambda=lam, p=1, eps=eps)
    x = s.ravel()
    e, g = Y @ x - b, L @ x
    grad = Y.T @ (e / np.sqrt(e * e + eps * eps)) + lam * L.T @ (g / np.sqrt(g * g + eps * eps))
    g0 = Y.T @ (-b / np.sqrt(b * b + eps * eps))
    assert np.linalg.norm(grad) <= 1e-3 * np.linalg.norm(g0)


def test_trace_holds_each_iterations_problem_and_a_worse_lambda_is_detected():
    """The per-iteration projected problems (the `trace` hook) reproduce the chosen lambdas,
    and moving a chosen lambda by two decades raises G by far more than the 1e-9 a GPU choice
    is allowed (so that validity check can fail)."""
    I = _pair(11, 6, 7)
    trace = []
    _, lams = solve_of.solve_of_pair(I, 3, 4, 0.0, trace=trace)
    assert len(trace) == len(lams) == 4
    for (YV, LV, bw), lam in zip(trace, lams):
        assert YV.shape[1] == LV.shape[1]
        assert solve_of.gcv_lambda(YV, LV, bw) == lam
        g0 = solve_of.gcv_value(YV, LV, bw, lam)[0]
        for f in (1e-2, 1e2):
            assert solve_of.gcv_value(YV, LV, bw, lam * f)[0] > (1.0 + 1e-9) * g0
