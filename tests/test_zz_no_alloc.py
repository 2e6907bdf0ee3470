"""The allocation-free weighted Gram (mmof_weighted_gram_noalloc) against mmof_weighted_gram,
through the C ABI: two calls in a row on one context, the second with a smaller input (the
fixed scratch array keeps the first call's partials), in FP32 and FP64, weighted and not.

Bar: the two entry points compute the same FP64 sums in another grouping of the partials, so
every entry agrees to 1e-12 of sum_r w_r |x_ri| |x_rj| (the FP64 rounding bound of the sum,
far above its actual size at these lengths)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _gram_pair(dt, n, K, weighted, seed):
    import torch
    from paper_2501_12497_amd import binding as B
    from paper_2501_12497_amd._lib import check
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn((K, n), generator=g, device="cuda", dtype=torch.float64).to(dt).contiguous()
    nu = torch.randn(n, generator=g, device="cuda", dtype=torch.float64).to(dt).contiguous() if weighted else None
    ctx = B.context()
    code = B._dtcode(dt)
    eps = 1e-3
    G_ref = torch.full((K, K), float("nan"), dtype=torch.float64, device="cuda")
    G_na = torch.full((K, K), float("nan"), dtype=torch.float64, device="cuda")
    ctx.bind()
    check(ctx.lib.mmof_weighted_gram(ctx.h, code, n, K, B._ptr(X), n, B._ptr(nu), eps, B._ptr(G_ref), K))
    check(ctx.lib.mmof_weighted_gram_noalloc(ctx.h, code, n, K, B._ptr(X), n, B._ptr(nu), eps, B._ptr(G_na), K))
    torch.cuda.synchronize()
    Xd = X.double()
    w = (1.0 / torch.sqrt(nu.double() ** 2 + eps * eps)) if weighted else torch.ones(n, dtype=torch.float64,
                                                                                      device="cuda")
    scale = (Xd.abs() * w).matmul(Xd.abs().t())     # sum_r w_r |x_ri| |x_rj|
    return G_ref.cpu().numpy(), G_na.cpu().numpy(), scale.cpu().numpy()


@pytest.mark.parametrize("which", ["f32", "f64"])
@pytest.mark.parametrize("weighted", [True, False])
def test_noalloc_gram_matches_the_allocating_entry_point(which, weighted):
    import torch
    dt = torch.float32 if which == "f32" else torch.float64
    # a long call (every one of the 256 scratch partials used, K in the fourth column block),
    # then a shorter one with fewer columns on the same scratch
    for n, K, seed in ((3_000_003, 57, 1), (40_001, 19, 2)):
        print(f"noalloc gram {which} weighted={weighted} n={n} K={K}", flush=True)
        G_ref, G_na, scale = _gram_pair(dt, n, K, weighted, seed)
        assert np.all(np.isfinite(G_na)), (n, K)
        assert np.array_equal(G_na, G_na.T), (n, K)
        d = np.abs(G_na - G_ref)
        assert np.all(d <= 1e-12 * scale), (n, K, float((d / scale).max()))


def test_noalloc_gram_refuses_sizes_beyond_its_limit():
    import torch
    from paper_2501_12497_amd import binding as B
    ctx = B.context()
    X = torch.zeros(65 * 8, dtype=torch.float64, device="cuda")
    G = torch.zeros(65 * 65, dtype=torch.float64, device="cuda")
    ctx.bind()
    rc = ctx.lib.mmof_weighted_gram_noalloc(ctx.h, 1, 8, 65, B._ptr(X), 8, None, 1e-3, B._ptr(G), 65)
    assert rc == -2
    assert "Krylov columns" in ctx.lib.mmof_last_error(None).decode() or "Gram sizes" in \
        ctx.lib.mmof_last_error(None).decode()
