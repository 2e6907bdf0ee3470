"""GPU parity of the projected-problem steps of MMGKS (FP64 Krylov side) at every basis size.

* weighted Gram X^T diag(w2) X on the matrix cores vs numpy, K = 1..256 (all block-grid shapes,
  the 64-column tiles beyond 64 and a ragged last tile);
* projected solve + discrepancy principle vs the oracle's bisection on the same Grams, on the
  one-wave path (K <= 64) and the multi-wave path (up to 256);
* the Gram, inner products and column combinations on bases whose columns are only
  element-aligned (odd leading dimension, base one element past a 16-byte boundary).
"""
import numpy as np
import pytest

from oracle import mmgks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_2501_12497_amd import binding
    return binding


# 17, 20, 24, 33, 36, 39, 40, 52, 56: full blocks plus a tail of at most 8 columns (vector-ALU
# tail path); 31, 47, 63: tails of more than 8 (padded block)
@pytest.mark.parametrize("K", [1, 5, 16, 17, 20, 24, 31, 33, 36, 39, 40, 47, 48, 52, 56, 63, 64, 65, 97, 130, 210,
                               256])
@pytest.mark.parametrize("which", ["f64", "f32"])
def test_weighted_gram(B, K, which):
    import torch
    dt = torch.float64 if which == "f64" else torch.float32
    r = np.random.default_rng(K)
    n = (50000 if K <= 64 else 20000) + 37 * K
    X = r.standard_normal((K, n))
    nu = r.standard_normal(n) * np.logspace(-4, 0, n)
    if dt == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        nu = nu.astype(np.float32).astype(np.float64)
    G = B.weighted_gram(torch.as_tensor(X, dtype=dt, device="cuda"), torch.as_tensor(nu, dtype=dt, device="cuda"),
                        1e-3).cpu().numpy()
    w = mmgks.mm_weights_sq(nu, 1e-3)
    exp = X @ (w[:, None] * X.T)
    assert np.abs(G - exp).max() <= 1e-12 * np.abs(exp).max()
    G1 = B.weighted_gram(torch.as_tensor(X, dtype=dt, device="cuda")).cpu().numpy()
    assert np.abs(G1 - X @ X.T).max() <= 1e-12 * np.abs(X @ X.T).max()


@pytest.mark.parametrize("K", [3, 20, 39, 64, 65, 100, 131, 210, 256])
def test_projected_solve_matches_oracle_dp(B, K):
    import torch
    r = np.random.default_rng(100 + K)
    m, n = 3 * K + 50, 2 * K + 40
    RA = r.standard_normal((m, K))
    RT = r.standard_normal((n, K)) * r.uniform(0.1, 10, size=K)
    b = r.standard_normal(m) * 3 + RA @ r.standard_normal(K)
    QA, RAq = np.linalg.qr(RA)
    _, RTq = np.linalg.qr(RT)
    QAtb = QA.T @ b
    bb = float(b @ b)
    # a target between the two ends so that a root exists
    lo_d = mmgks.discrepancy(RAq, QAtb, RTq, 1e-8, bb)[0]
    hi_d = mmgks.discrepancy(RAq, QAtb, RTq, 1e8, bb)[0]
    target = 0.5 * (lo_d + hi_d)
    lam_or, st_or = mmgks.dp_lambda(RAq, QAtb, RTq, bb, target)
    z_or = mmgks.projected_solve(RAq, QAtb, RTq, lam_or)
    GA, GT, d = RA.T @ RA, RT.T @ RT, RA.T @ b
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    z, lam, D2, st = B.projected_solve(dev(GA), dev(GT), dev(d), bb, target * target)
    assert st == st_or == 0
    assert abs(lam - lam_or) <= 1e-9 * lam_or
    np.testing.assert_allclose(z.cpu().numpy(), z_or, rtol=1e-7, atol=1e-9 * np.abs(z_or).max())
    assert abs(np.sqrt(D2) - target) <= 1e-10 * target
    # clamped ends
    z, lam, D2, st = B.projected_solve(dev(GA), dev(GT), dev(d), bb, (0.1 * lo_d) ** 2)
    assert st == 2
    z, lam, D2, st = B.projected_solve(dev(GA), dev(GT), dev(d), bb, (10 * hi_d) ** 2)
    assert st == 2


def test_weighted_gram_is_symmetric_and_rejects_more_than_256_columns(B):
    import torch
    from paper_2501_12497_amd._lib import MMOFError
    r = np.random.default_rng(5)
    X = torch.as_tensor(r.standard_normal((150, 3001)), device="cuda")
    G = B.weighted_gram(X, torch.as_tensor(r.standard_normal(3001), device="cuda")).cpu().numpy()
    assert np.array_equal(G, G.T)
    with pytest.raises(MMOFError) as e:
        B.weighted_gram(torch.zeros((257, 10), dtype=torch.float64, device="cuda"))
    assert e.value.code == -2


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("K", [7, 39, 70])
def test_unaligned_bases(B, which, K):
    """The Gram, the inner products and the column combinations on a basis that starts one
    element past a 16-byte boundary and has an odd leading dimension: every column then starts
    at an address that is only element-aligned, which their vector loads must accept."""
    import torch
    dt = torch.float64 if which == "f64" else torch.float32
    r = np.random.default_rng(7 * K)
    n = 40001 + 2 * K
    X = r.standard_normal((K, n))
    nu = r.standard_normal(n) * np.logspace(-3, 0, n)
    if dt == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        nu = nu.astype(np.float32).astype(np.float64)
    buf = torch.zeros(K * n + 1, dtype=dt, device="cuda")
    buf[1:] = torch.as_tensor(X.ravel(), dtype=dt, device="cuda")
    Xd = buf[1:].view(K, n)
    assert Xd.data_ptr() % 16 != 0
    w = mmgks.mm_weights_sq(nu, 1e-3)
    G = B.weighted_gram(Xd, torch.as_tensor(nu, dtype=dt, device="cuda"), 1e-3).cpu().numpy()
    exp = X @ (w[:, None] * X.T)
    assert np.abs(G - exp).max() <= 1e-12 * np.abs(exp).max()
    y = r.standard_normal(n)
    d = B.block_dot(Xd, torch.as_tensor(y, device="cuda")).cpu().numpy()
    ed = X @ y
    assert np.abs(d - ed).max() <= 1e-12 * np.abs(X).sum(axis=1).max() * np.abs(y).max()
    z = r.standard_normal(K)
    u = B.block_combine(Xd, torch.as_tensor(z, device="cuda")).cpu().numpy()
    eu = z @ X
    assert np.abs(u - eu).max() <= 1e-12 * (np.abs(z) @ np.abs(X)).max()


@pytest.mark.parametrize("K", [1, 9, 39, 64, 100])
def test_reorth_auto_one_pass_when_enough(B, K):
    """A vector with a large part outside span(Q): the first pass keeps most of its norm, so
    the automatic mode stops after it -- its result is bit for bit the single pass
    x - Q (Q^T x) formed by the block inner product and column combination -- and that result is
    orthogonal to Q to working precision and equal to the exact projection (numpy, FP64)."""
    import torch
    r = np.random.default_rng(700 + K)
    n = 40000 + 13 * K
    Qh, _ = np.linalg.qr(r.standard_normal((n, K)))
    Q = torch.as_tensor(np.ascontiguousarray(Qh.T), device="cuda")
    x0 = r.standard_normal(n) + Qh @ r.standard_normal(K)
    x = torch.as_tensor(x0, device="cuda")
    h = B.block_dot(Q, x)
    one = B.block_combine(Q, h, -1.0, x, 1.0).cpu().numpy()
    sq = B.reorth(Q, x, "auto")
    got = x.cpu().numpy()
    np.testing.assert_array_equal(got, one)
    exp = x0 - Qh @ (Qh.T @ x0)
    assert np.abs(got - exp).max() <= 1e-13 * np.abs(x0).max()
    assert abs(sq - float(got @ got)) <= 1e-12 * sq
    assert np.abs(Qh.T @ got).max() <= 1e-13 * np.sqrt(sq)


@pytest.mark.parametrize("K", [1, 9, 39, 64, 100])
def test_reorth_auto_second_pass_when_needed(B, K):
    """A vector within 1e-9 of span(Q): one pass leaves the rounding of the cancelled part
    (about 1e-16 ||x||, i.e. 1e-7 of what remains) along Q, so Kahan's test asks for the
    second pass; afterwards Q^T x is at working precision relative to the remainder, as with
    two passes always (mmof_cgs2), and both agree with the exact projection."""
    import torch
    r = np.random.default_rng(800 + K)
    n = 40000 + 13 * K
    Qh, _ = np.linalg.qr(r.standard_normal((n, K)))
    Q = torch.as_tensor(np.ascontiguousarray(Qh.T), device="cuda")
    w = r.standard_normal(n)
    w -= Qh @ (Qh.T @ w)
    w -= Qh @ (Qh.T @ w)
    w /= np.linalg.norm(w)
    c = r.standard_normal(K)
    x0 = Qh @ c + 1e-9 * np.linalg.norm(c) * w
    for mode in ("auto", "twice"):
        x = torch.as_tensor(x0, device="cuda")
        sq = B.reorth(Q, x, mode)
        got = x.cpu().numpy()
        rem = 1e-9 * np.linalg.norm(c)
        assert abs(np.sqrt(sq) - rem) <= 1e-5 * rem, mode
        assert np.abs(got - 1e-9 * np.linalg.norm(c) * w).max() <= 1e-13 * np.abs(x0).max(), mode
        assert np.abs(Qh.T @ got).max() <= 1e-12 * np.sqrt(sq), mode


def test_reorth_rejects_bad_mode(B):
    import torch
    from paper_2501_12497_amd._lib import MMOFError
    Q = torch.eye(4, 16, dtype=torch.float64, device="cuda")
    x = torch.ones(16, dtype=torch.float64, device="cuda")
    with pytest.raises(MMOFError) as e:
        B.reorth(Q, x, 7)
    assert e.value.code == -1


def _implicit_basis(r, n, K, spread):
    """An orthonormal V (n x K) and a unit upper-triangular T with off-diagonal entries of size
    `spread`; the stored columns Vs = V T^-1, so that V = Vs T."""
    Q, _ = np.linalg.qr(r.standard_normal((n, K)))
    T = np.eye(K) + np.triu(r.standard_normal((K, K)) * spread, 1)
    Vs = Q @ np.linalg.inv(T)
    return Q, T, Vs


def _device_T(T):
    import torch
    K = T.shape[0]
    Tt = np.zeros((256, 256))
    Tt[:K, :K] = T.T          # row j of the buffer = column j of T
    return torch.as_tensor(Tt, device="cuda")


@pytest.mark.parametrize("K", [1, 10, 39, 100, 255])
def test_basis_extend_implicit_step(B, K):
    """A direction with most of its norm outside span(V): one pass over Vs gives g = V^T r,
    rho^2 = ||r||^2 - ||g||^2 and the new column of T, e_K - T g / rho; r is left as it is, and
    the new basis vector r / rho - V g / rho is a unit vector orthogonal to V (numpy, FP64)."""
    import torch
    r = np.random.default_rng(900 + K)
    n = 20000 + 7 * K
    Q, T, Vs = _implicit_basis(r, n, K, 1e-3)
    x0 = r.standard_normal(n) + Q @ r.standard_normal(K)
    x = torch.as_tensor(x0, device="cuda")
    Td = _device_T(T)
    rho2 = B.basis_extend(torch.as_tensor(np.ascontiguousarray(Vs.T), device="cuda"), x, Td)
    np.testing.assert_array_equal(x.cpu().numpy(), x0)
    g = Q.T @ x0
    exp2 = x0 @ x0 - g @ g
    assert abs(rho2 - exp2) <= 1e-12 * exp2
    col = Td.cpu().numpy()[K, :K + 1]
    exp_col = -(T @ g) / np.sqrt(exp2)
    assert np.abs(col[:K] - exp_col).max() <= 1e-12 * (np.abs(T) @ np.abs(g)).max() / np.sqrt(exp2) + 1e-15
    assert col[K] == 1.0
    vK = x0 / np.sqrt(rho2) + Vs @ col[:K]
    assert abs(np.linalg.norm(vK) - 1.0) <= 1e-12
    assert np.abs(Q.T @ vK).max() <= 1e-12
    np.testing.assert_array_equal(Td.cpu().numpy()[:K, :K], T.T)   # the earlier columns untouched


@pytest.mark.parametrize("K", [1, 10, 39, 100])
def test_basis_extend_explicit_pass_when_needed(B, K):
    """A direction within 1e-9 of span(V): the device test takes the explicit pass r <- r - V g
    first (r changes), then the implicit step on what is left; the new basis vector is still a
    unit vector orthogonal to V to working precision relative to it."""
    import torch
    r = np.random.default_rng(950 + K)
    n = 20000 + 7 * K
    Q, T, Vs = _implicit_basis(r, n, K, 1e-3)
    w = r.standard_normal(n)
    w -= Q @ (Q.T @ w)
    w -= Q @ (Q.T @ w)
    w /= np.linalg.norm(w)
    c = r.standard_normal(K)
    x0 = Q @ c + 1e-9 * np.linalg.norm(c) * w
    x = torch.as_tensor(x0, device="cuda")
    Td = _device_T(T)
    rho2 = B.basis_extend(torch.as_tensor(np.ascontiguousarray(Vs.T), device="cuda"), x, Td)
    x1 = x.cpu().numpy()
    assert np.linalg.norm(x1) <= 1e-6 * np.linalg.norm(x0)        # the explicit pass ran
    rem = 1e-9 * np.linalg.norm(c)
    assert abs(np.sqrt(rho2) - rem) <= 1e-5 * rem
    col = Td.cpu().numpy()[K, :K + 1]
    vK = x1 / np.sqrt(rho2) + Vs @ col[:K]
    assert abs(np.linalg.norm(vK) - 1.0) <= 1e-9
    assert np.abs(Q.T @ vK).max() <= 1e-12
    assert np.abs(vK - w).max() <= 1e-5 * np.abs(w).max()
