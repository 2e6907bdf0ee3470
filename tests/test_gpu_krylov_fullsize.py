"""The FP64 Krylov passes at the lengths of the 1024x1024x64 solve, through the C ABI.

Theta V of that solve has R = 266,207,232 rows (gx and gy of 64 frames of 1024 x 1024 and two
flow directions over 63 pairs) and V has n = 67,108,864 rows; with 39 columns, R*K and n*K
exceed 2^31, so these tests hold the 64-bit offsets and the large-grid paths of the kernels.
Columns are drawn on the device from a seeded generator; sampled results are compared with
host FP64 sums over the same values (numpy on the columns copied back):
  * weighted Gram of 39 FP32 columns (three 16-column blocks, the last one ragged);
  * inner products V^T y, column combinations V z at sampled rows (including the first and
    last rows), and CGS2 against an orthonormal basis with disjoint supports, FP64.
Bar: 1e-12 of the absolute sums (sum |a||b|), the FP64 rounding level of sums of this length.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

R_THETA = 64 * 1024 * 1023 * 2 + 2 * 63 * 1024 * 1024   # rows of Theta V at 1024 x 1024 x 64
N_PIX = 64 * 1024 * 1024
K = 39


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_2501_12497_amd import binding
    return binding


def test_weighted_gram_at_theta_length(B):
    import torch
    assert R_THETA == 266_207_232
    g = torch.Generator(device="cuda").manual_seed(7)
    print(f"wgram: {K} x {R_THETA} FP32", flush=True)
    X = torch.randn((K, R_THETA), generator=g, device="cuda", dtype=torch.float32)
    nu = torch.randn(R_THETA, generator=g, device="cuda", dtype=torch.float32)
    eps = 1e-3
    G = B.weighted_gram(X, nu, eps).cpu().numpy()
    assert np.array_equal(G, G.T)
    w = 1.0 / np.sqrt(nu.cpu().numpy().astype(np.float64) ** 2 + eps * eps)
    cols = {}
    for i, j in ((0, 0), (0, 38), (17, 33), (38, 38), (5, 20), (31, 32)):
        for c in (i, j):
            if c not in cols:
                cols[c] = X[c].cpu().numpy().astype(np.float64)
        a, b = cols[i], cols[j]
        exp = float(np.dot(a * w, b))
        scale = float(np.dot(np.abs(a) * w, np.abs(b)))
        assert abs(G[i, j] - exp) <= 1e-12 * scale, (i, j, G[i, j], exp, scale)
    del X, nu
    torch.cuda.empty_cache()


def test_block_dot_and_combine_at_basis_length(B):
    import torch
    g = torch.Generator(device="cuda").manual_seed(8)
    print(f"block dot / combine: {K} x {N_PIX} FP64", flush=True)
    V = torch.randn((K, N_PIX), generator=g, device="cuda", dtype=torch.float64)
    y = torch.randn(N_PIX, generator=g, device="cuda", dtype=torch.float64)
    z = torch.randn(K, generator=g, device="cuda", dtype=torch.float64)
    d = B.block_dot(V, y).cpu().numpy()
    yh = y.cpu().numpy()
    for j in (0, 19, 38):
        vj = V[j].cpu().numpy()
        exp = float(np.dot(vj, yh))
        assert abs(d[j] - exp) <= 1e-12 * float(np.dot(np.abs(vj), np.abs(yh))), j
    u = B.block_combine(V, z, 1.0, y, -0.5)   # V z - y / 2
    rows = np.concatenate([[0, 1, 2, 255, 256, N_PIX // 2, N_PIX - 2, N_PIX - 1],
                           np.random.default_rng(9).integers(0, N_PIX, 2000)])
    idx = torch.as_tensor(rows, device="cuda")
    Vs = V[:, idx].cpu().numpy()
    zh = z.cpu().numpy()
    exp = zh @ Vs - 0.5 * yh[rows]
    scale = np.abs(zh) @ np.abs(Vs) + 0.5 * np.abs(yh[rows])
    got = u[idx].cpu().numpy()
    assert np.all(np.abs(got - exp) <= 1e-13 * scale)
    del V, y, u
    torch.cuda.empty_cache()


def test_cgs2_at_basis_length(B):
    """Q: 39 orthonormal columns with disjoint supports (column j lives on rows
    [j*nb, (j+1)*nb)), so x - Q (Q^T x) is known block by block; the second pass removes only
    rounding.  Checked on every row of sampled blocks, and Q^T x ~ 0 afterwards."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(10)
    print(f"cgs2: {K} x {N_PIX} FP64", flush=True)
    nb = N_PIX // K
    Q = torch.zeros((K, N_PIX), dtype=torch.float64, device="cuda")
    for j in range(K):
        q = torch.randn(nb, generator=g, device="cuda", dtype=torch.float64)
        Q[j, j * nb:(j + 1) * nb] = q / torch.linalg.vector_norm(q)
    x = torch.randn(N_PIX, generator=g, device="cuda", dtype=torch.float64)
    x0 = x.cpu().numpy()
    sq = B.cgs2(Q, x)
    xh = x.cpu().numpy()
    for j in (0, 1, 20, 38):
        qj = Q[j, j * nb:(j + 1) * nb].cpu().numpy()
        blk = x0[j * nb:(j + 1) * nb]
        h = float(np.dot(qj, blk))
        exp = blk - qj * h
        assert np.all(np.abs(xh[j * nb:(j + 1) * nb] - exp) <= 1e-12 * (np.abs(blk) + np.abs(qj) * abs(h)) + 1e-15), j
    np.testing.assert_array_equal(xh[K * nb:], x0[K * nb:])   # rows no column touches
    assert abs(sq - float(np.dot(xh, xh))) <= 1e-12 * sq
    h2 = B.block_dot(Q, x).cpu().numpy()
    assert np.abs(h2).max() <= 1e-13 * np.sqrt(sq)
    del Q, x
    torch.cuda.empty_cache()


def test_block_dot_ragged_length_all_columns(B):
    """A length just past 2^26 (odd): the inner products then use their largest number of row
    chunks (8192) of 8194 rows with a short last chunk of odd length, and 21 columns take three
    column groups (8, 8, 5) on the one-dimensional grid; every column is checked, and the
    column combination at rows around the chunk seams and the end."""
    import torch
    n = N_PIX + 12345
    k = 21
    g = torch.Generator(device="cuda").manual_seed(11)
    print(f"block dot ragged: {k} x {n} FP64", flush=True)
    V = torch.randn((k, n), generator=g, device="cuda", dtype=torch.float64)
    y = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
    z = torch.randn(k, generator=g, device="cuda", dtype=torch.float64)
    d = B.block_dot(V, y).cpu().numpy()
    yh = y.cpu().numpy()
    for j in range(k):
        vj = V[j].cpu().numpy()
        exp = float(np.dot(vj, yh))
        assert abs(d[j] - exp) <= 1e-12 * float(np.dot(np.abs(vj), np.abs(yh))), j
    u = B.block_combine(V, z)
    chunk = 8194
    seams = [c * chunk + o for c in (1, 4095, 8190, 8191) for o in (-1, 0, 1)]
    rows = np.array(sorted(set(seams + [0, n // 2, n - 3, n - 2, n - 1])))
    idx = torch.as_tensor(rows, device="cuda")
    Vs = V[:, idx].cpu().numpy()
    zh = z.cpu().numpy()
    exp = zh @ Vs
    got = u[idx].cpu().numpy()
    assert np.all(np.abs(got - exp) <= 1e-13 * (np.abs(zh) @ np.abs(Vs)))
    del V, y, u
    torch.cuda.empty_cache()
