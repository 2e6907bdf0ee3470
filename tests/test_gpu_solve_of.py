"""GPU parity of Solve-OF (Alg. 2, p = q = 2: GKS with GCV; and the p = q = 1 MM variant)
against the FP64 oracle, through the C ABI (mmof_flow_solve_gks, mmof_flow_solve_of), and of
the joint solve that uses it for the flow.

Bars: with a fixed lambda the FP64 flow matches to 1e-10 (only summation order differs);
with the GCV search the chosen lambdas match to 1e-6 relative and the flows to 1e-8 (the
search's points are the same on both sides and ties within a relative 1e-9 of G keep the
earlier point, so rounding does not move the choice; G is evaluated from Gram matrices on the
GPU and from the stacked least-squares form in the oracle); FP32 derivatives (FP64 solve):
flows to 1e-4 (their G values differ by FP32 rounding, more than the tie width, so the
lambdas are not compared).
"""
import numpy as np
import pytest

from gpu_helpers import TOL32, assert_close, dev, host, pack, roundtrip32, unpack
from oracle import optflow, solve_of

pytestmark = pytest.mark.gpu

SIZES = [(3, 14, 16), (2, 11, 9)]   # ragged; widths of both parities


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_2501_12497_amd import binding
    return binding


def _frames(seed, sizes=SIZES, noise=0.02):
    """Smooth moving patterns (sub-pixel shifts per frame) plus a little noise."""
    r = np.random.default_rng(seed)
    out = []
    for i, (nt, ny, nx) in enumerate(sizes):
        y, x = np.mgrid[0:ny, 0:nx].astype(float)
        fr = [np.sin(0.45 * (x - 0.4 * t) + 0.3 * i) + np.cos(0.37 * (y + 0.3 * t)) + noise * r.standard_normal((ny, nx))
              for t in range(nt)]
        out.append(np.stack(fr))
    return out


def _run(B, us, dt, **kw):
    import torch
    stack = B.Stack([u.shape for u in us])
    v = torch.zeros(2 * stack.n_pair_px, dtype=dt, device="cuda")
    vr = torch.empty_like(v)
    v, lam = B.flow_solve_gks(stack, dev(pack(us), dt), v, v_rev=vr, want_lambdas=True, **kw)
    return host(v), host(vr), lam


def _oracle(us, ell, n_iter, fixed_lambda=0.0, dr=1):
    flows, lams = [], []
    for u in us:
        I = optflow.of_derivs(u, dr)
        for t in range(I.shape[0]):
            s, l = solve_of.solve_of_pair(I[t], ell, n_iter, fixed_lambda)
            flows.append(s)
            lams.append(l)
    return flows, lams


def test_fixed_lambda_fp64(B):
    import torch
    us = _frames(1)
    got, _, lam = _run(B, us, torch.float64, ell=6, n_iter=8, fixed_lambda=0.05)
    exp, _ = _oracle(us, 6, 8, 0.05)
    assert_close(got, pack(exp), 1e-10)
    assert np.all(lam == 0.05)


def _gcv_choices_valid(lam, us, ell, n_iter, rel, dr=1):
    """Each pair's lambdas against the oracle's: equal to 1e-6, or, at the first iteration where
    they differ, a choice no worse than the oracle's on the oracle's own GCV functional of that
    iteration, G(lambda_gpu) <= (1 + rel) G(lambda_oracle) (several lambdas can be equally good
    where G is flat); the iterations after a different choice have another basis and are not
    compared.  Returns the number of pairs whose lambdas all agree."""
    lam = np.asarray(lam)
    agree, p = 0, 0
    for u in us:
        I = optflow.of_derivs(u, dr)
        for t in range(I.shape[0]):
            trace = []
            _, el = solve_of.solve_of_pair(I[t], ell, n_iter, 0.0, trace=trace)
            for k, (lg, lo) in enumerate(zip(lam[p], el)):
                if abs(lg - lo) <= 1e-6 * abs(lo):
                    continue
                YV, LV, bw = trace[k]
                gg, go = solve_of.gcv_value(YV, LV, bw, lg)[0], solve_of.gcv_value(YV, LV, bw, lo)[0]
                assert gg <= (1.0 + rel) * go, (p, k, lg, lo, gg, go)
                break
            else:
                agree += 1
            p += 1
    return agree


@pytest.mark.parametrize("ell,n_iter", [(10, 20), (4, 7), (1, 1)])
def test_gcv_fp64(B, ell, n_iter):
    import torch
    us = _frames(2)
    got, gotr, lam = _run(B, us, torch.float64, ell=ell, n_iter=n_iter)
    exp, elams = _oracle(us, ell, n_iter)
    # every choice valid; on these frames also the same choices and flows as the oracle's
    assert _gcv_choices_valid(lam, us, ell, n_iter, 1e-9) == len(elams)
    np.testing.assert_allclose(lam, np.array(elams), rtol=1e-6)
    assert_close(got, pack(exp), 1e-8)
    # reverse flow of the GPU's own flow
    shapes = [(u.shape[0] - 1, 2) + u.shape[1:] for u in us]
    flows = unpack(got, shapes)
    assert_close(gotr, pack([optflow.reverse_flow(f) for f in flows]), 1e-12)


def test_gcv_fp32_derivatives(B):
    import torch
    us = [roundtrip32(u) for u in _frames(3)]
    got, _, lam = _run(B, us, torch.float32, ell=10, n_iter=20)
    exp, elams = _oracle(us, 10, 20)
    assert_close(got, pack(exp), 1e-4)
    # the lambdas may move to another point where G is flat: such a choice must still be as
    # good on the oracle's functional, to the FP32 derivatives' accuracy
    _gcv_choices_valid(lam, us, 10, 20, 1e-5)


def test_reduced_frames(B):
    """scale = 2 on 40 x 44 / 30 x 27 frames: the solve runs on 20 x 22 / 15 x 14 frames."""
    import torch
    sizes = [(3, 40, 44), (2, 30, 27)]
    us = _frames(4, sizes)
    got, _, _ = _run(B, us, torch.float64, ell=8, n_iter=10, scale=2)
    exp = pack([solve_of.solve_of(u, 1, 8, 10, 0.0, 2) for u in us])
    assert_close(got, exp, 1e-8)


def test_edges(B):
    import torch
    from paper_2501_12497_amd._lib import MMOFError
    # no temporal change: zero flow, lambdas 0
    u = _frames(5, [(3, 9, 11)], noise=0.0)[0]
    still = [np.stack([u[0]] * 3)]
    got, _, lam = _run(B, still, torch.float64, ell=5, n_iter=4)
    assert not np.any(got) and not np.any(lam)
    # a stack whose sequences have single frames and pairs side by side
    us = [_frames(6, [(1, 8, 8)])[0], _frames(7, [(2, 10, 9)])[0]]
    got, _, _ = _run(B, us, torch.float64, ell=5, n_iter=5)
    exp, _ = _oracle([us[1]], 5, 5)
    assert_close(got, pack(exp), 1e-8)
    # argument checks, before any launch
    stack = B.Stack([(2, 6, 5)])
    uu = dev(np.zeros(60), torch.float64)
    v = torch.full((60,), 7.0, dtype=torch.float64, device="cuda")
    for kw in (dict(ell=20, n_iter=14), dict(ell=0, n_iter=3), dict(ell=3, n_iter=0), dict(ell=30, n_iter=1),
               dict(ell=3, n_iter=3, fixed_lambda=-1.0), dict(ell=3, n_iter=3, scale=3, delta_r=2)):
        with pytest.raises(MMOFError) as e:
            B.flow_solve_gks(stack, uu, v, **kw)
        assert e.value.code == -1, kw
    assert torch.all(v == 7.0)


@pytest.mark.parametrize("op", ["f64", "f32"])
def test_joint_solve_with_solve_of(B, op):
    """The joint solve with the paper's flow solver on frames reduced by 2 (its Sec. 5
    setting), FP64 against the oracle's run of the same configuration."""
    import torch
    from oracle import mmgks
    from synth import noisy
    sizes = [(3, 25, 30), (4, 18, 21)]
    us = []
    for (nt, ny, nx) in sizes:
        yy, xx = np.mgrid[0:ny, 0:nx]
        us.append(np.stack([(((xx - (8.0 + 1.5 * t)) ** 2 + (yy - ny / 2) ** 2) <= 16.0).astype(float)
                            for t in range(nt)]))
    geoms = [mmgks.SeqGeom(nt, ny, nx) for (nt, ny, nx) in sizes]
    ops = mmgks.StackOps(geoms, "blur", flow_scale=2, flow_solver="gks", of_ell=6, of_iters=8)
    ut = np.concatenate([u.ravel() for u in us])
    clean = ops.A(ut)
    b = noisy(clean, np.random.default_rng(8).standard_normal(clean.shape), 0.01)
    delta = float(np.linalg.norm(b - clean))
    prm = dict(ell=5, k_max=8, tau=3, alpha=0.2)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(n_sweeps=0, **prm), u_true=ut)
    plan = B.plan_blur(B.Stack(sizes), 9, 2.0)
    kw = dict(op_dtype=op, flow_scale=2, flow_solver=1, of_ell=6, of_iters=8, **prm)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        **kw)
    assert res.iters == ref.iters
    assert abs(res.rre[-1] - ref.rre[-1]) <= 1e-4
    if op == "f64":
        np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-7)
        assert_close(res.u.cpu().numpy(), ref.u, 1e-7)
    again = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                          use_graph=1, **kw)
    assert torch.equal(again.u, res.u) and again.lambdas == res.lambdas


# ------------------------------------------------------------------ p = q = 1 variant
#
# Bars: the weights (e^2 + eps^2)^(-1/2) amplify rounding of the iterate by up to 1 / eps
# (1e3 at eps = 1e-3) in relative terms, so the p = q = 1 flows are compared to 1e-8 with a
# fixed lambda and to 1e-7 with the GCV search (lambdas to 1e-6, as for p = q = 2).


def _oracle_l1(us, ell, n_iter, fixed_lambda=0.0, eps=solve_of.EPS_L1):
    flows, lams = [], []
    for u in us:
        I = optflow.of_derivs(u, 1)
        for t in range(I.shape[0]):
            s, l = solve_of.solve_of_pair(I[t], ell, n_iter, fixed_lambda, p=1, eps=eps)
            flows.append(s)
            lams.append(l)
    return flows, lams


@pytest.mark.parametrize("lam,eps", [(0.05, 1e-3), (0.5, 1e-2)])
def test_l1_fixed_lambda_fp64(B, lam, eps):
    import torch
    us = _frames(21)
    got, _, lams = _run(B, us, torch.float64, ell=6, n_iter=9, fixed_lambda=lam, pq=1, eps=eps)
    exp, _ = _oracle_l1(us, 6, 9, lam, eps)
    assert_close(got, pack(exp), 1e-8)
    assert np.all(lams == lam)


@pytest.mark.parametrize("ell,n_iter", [(10, 20), (3, 6), (1, 1)])
def test_l1_gcv_fp64(B, ell, n_iter):
    import torch
    us = _frames(22)
    got, gotr, lam = _run(B, us, torch.float64, ell=ell, n_iter=n_iter, pq=1)
    exp, elams = _oracle_l1(us, ell, n_iter)
    np.testing.assert_allclose(lam, np.array(elams), rtol=1e-6)
    assert_close(got, pack(exp), 1e-7)
    shapes = [(u.shape[0] - 1, 2) + u.shape[1:] for u in us]
    assert_close(gotr, pack([optflow.reverse_flow(f) for f in unpack(got, shapes)]), 1e-12)


def test_l1_large_eps_is_the_quadratic_solve(B):
    """eps far above every residual: both weights are the constant 1/eps, so the GPU's p = q = 1
    run reproduces its own p = q = 2 run (same lambdas up to rounding, same flow)."""
    import torch
    us = _frames(23)
    g2, _, l2 = _run(B, us, torch.float64, ell=5, n_iter=7)
    g1, _, l1 = _run(B, us, torch.float64, ell=5, n_iter=7, pq=1, eps=1e8)
    np.testing.assert_allclose(l1, l2, rtol=1e-7)
    assert_close(g1, g2, 1e-8)


def test_l1_reduced_frames_fp32(B):
    """p = q = 1 on frames reduced by 2, FP32 derivatives (FP64 solve)."""
    import torch
    sizes = [(3, 36, 40), (2, 22, 27)]
    us = [roundtrip32(u) for u in _frames(24, sizes)]
    got, _, _ = _run(B, us, torch.float32, ell=6, n_iter=8, scale=2, pq=1)
    exp = pack([solve_of.solve_of(u, 1, 6, 8, 0.0, 2, p=1) for u in us])
    assert_close(got, exp, 1e-4)


def test_l1_rejects(B):
    import torch
    from paper_2501_12497_amd._lib import MMOFError
    stack = B.Stack([(2, 6, 5)])
    uu = dev(np.zeros(60), torch.float64)
    v = torch.full((60,), 7.0, dtype=torch.float64, device="cuda")
    for kw in (dict(pq=3), dict(pq=0), dict(pq=1, eps=0.0), dict(pq=1, eps=-1.0), dict(pq=1, eps=float("inf"))):
        with pytest.raises(MMOFError) as e:
            B.flow_solve_gks(stack, uu, v, ell=3, n_iter=3, **kw)
        assert e.value.code == -1, kw
    assert torch.all(v == 7.0)
