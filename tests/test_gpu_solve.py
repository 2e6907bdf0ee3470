"""GPU parity of the full MMGKS-OF solve (Alg. 1) against the FP64 oracle, through the C ABI.

The oracle runs the same algorithm step by step (QR of the projected matrices, the
projected normal equations, bisection for the discrepancy principle); the GPU uses
Gram matrices, Cholesky and a safeguarded Newton root.  Bars: the FP64 GPU solve
reproduces the oracle's iterates to ~1e-8 and its RRE to 1e-4 (the solve bar); the
FP32-operator solve (FP64 Krylov) reproduces the RRE to 1e-4.
"""
import math

import numpy as np
from gpu_helpers import assert_close
import pytest

from oracle import mmgks
from synth import angles_shifted, bins_for, cfg_disk32, noisy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_2501_12497_amd import binding
    return binding


def _problem(n=20, n_t=3, n_theta=6, seed=0, level=0.02):
    y, x = np.mgrid[0:n, 0:n]
    u = np.stack([(((x - (7.0 + t)) ** 2 + (y - 10.0) ** 2) <= 12.0).astype(float) for t in range(n_t)])
    ang = angles_shifted(n_t, n_theta, math.radians(4.0))
    nb = bins_for(n)
    g = mmgks.SeqGeom(n_t, n, n, ang, nb)
    return u, ang, nb, g


def _run_both(B, u, ang, nb, g, b, delta, op="f64", **prm):
    import torch
    ops = mmgks.StackOps([g], "radon", use_flow=bool(prm.get("use_flow", True)),
                         interp={0: "bilinear", 1: "round"}[prm.get("interp", 0)])
    okeys = {k: v for k, v in prm.items() if k in mmgks.SolveParams.__dataclass_fields__}
    okeys["use_flow"] = bool(okeys.get("use_flow", True))
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**okeys), u_true=u.ravel())
    stack = B.Stack.single(g.n_t, g.ny, g.nx)
    plan = B.plan_radon(stack, [ang.shape[1]], [nb], ang.ravel())
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta,
                        u_true=torch.as_tensor(u.ravel(), device="cuda"), op_dtype=op, **prm)
    return ref, res


def test_solve_fixed_lambda_no_flow_fp64(B):
    u, ang, nb, g = _problem()
    ops = mmgks.StackOps([g], "radon", use_flow=False)
    clean = ops.A(u.ravel())
    b = noisy(clean, np.random.default_rng(1).standard_normal(clean.shape), 0.02)
    delta = float(np.linalg.norm(b - clean))
    ref, res = _run_both(B, u, ang, nb, g, b, delta, ell=6, k_max=12, use_flow=0, fixed_lambda=0.05)
    got = res.u.cpu().numpy()
    assert_close(got, ref.u, 1e-9)
    np.testing.assert_allclose(res.rre, ref.rre, rtol=1e-9)


@pytest.mark.parametrize("interp", [0, 1])
def test_solve_with_flow_and_dp_fp64(B, interp):
    u, ang, nb, g = _problem()
    ops = mmgks.StackOps([g], "radon")
    clean = ops.A(u.ravel())
    b = noisy(clean, np.random.default_rng(2).standard_normal(clean.shape), 0.02)
    delta = float(np.linalg.norm(b - clean))
    ref, res = _run_both(B, u, ang, nb, g, b, delta, ell=6, k_max=12, tau=3, n_sweeps=40, alpha=0.2,
                         interp=interp)
    assert res.iters == ref.iters
    assert res.dp_status == ref.dp_status
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-7)
    np.testing.assert_allclose(res.resid, ref.resid, rtol=1e-8)
    got = res.u.cpu().numpy()
    assert_close(got, ref.u, 1e-7)
    assert abs(res.rre[-1] - ref.rre[-1]) <= 1e-4
    v_or = ref.flows[0][0].ravel()
    assert np.linalg.norm(res.v.cpu().numpy() - v_or) <= 1e-6 * max(np.linalg.norm(v_or), 1e-30)


def _disk32_data():
    wl = cfg_disk32()
    s = wl.seqs[0]
    g = mmgks.SeqGeom(s.n_t, s.ny, s.nx, s.angles, s.n_bins)
    ops = mmgks.StackOps([g], "radon")
    clean = ops.A(s.u_true.ravel())
    b = noisy(clean, s.noise_g, wl.noise_level)
    return wl, s, g, b, float(np.linalg.norm(b - clean))


@pytest.mark.parametrize("op", ["f64", "f32"])
def test_solve_disk32_workload(B, op):
    """32x32x8 translating disk, 10 shifted angles, 1% noise, 20 alternations (tau = 1)."""
    wl, s, g, b, delta = _disk32_data()
    prm = dict(ell=10, k_max=20, tau=1, n_sweeps=200, alpha=0.1, eps=1e-3, eta=1.01, delta_r=1)
    ref, res = _run_both(B, s.u_true, s.angles, s.n_bins, g, b, delta, op=op, **prm)
    assert res.iters == ref.iters == 20
    assert abs(res.rre[-1] - ref.rre[-1]) <= 1e-4, (res.rre[-1], ref.rre[-1])
    if op == "f64":
        np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-6)
        got = res.u.cpu().numpy()
        assert_close(got, ref.u, 1e-6)


def test_solve_disk32_refined(B):
    """FP32 operators with the last outer iterations on FP64 operators (the FP64 phase takes
    over the FP32 phase's basis and flows and continues the iteration count)."""
    import torch
    wl, s, g, b, delta = _disk32_data()
    prm = dict(ell=10, k_max=20, tau=1, n_sweeps=200, alpha=0.1, eps=1e-3, eta=1.01, delta_r=1)
    ref, res = _run_both(B, s.u_true, s.angles, s.n_bins, g, b, delta, op="f32", refine_iters=5, **prm)
    assert res.iters == ref.iters == 20
    assert abs(res.rre[-1] - ref.rre[-1]) <= 1e-4, (res.rre[-1], ref.rre[-1])
    assert res.v.dtype == torch.float32 and res.n_cols == ref.n_cols
    # refinement over the whole solve is the FP64 solve
    stack = B.Stack.single(g.n_t, g.ny, g.nx)
    plan = B.plan_radon(stack, [s.angles.shape[1]], [s.n_bins], s.angles.ravel())
    bt = torch.as_tensor(b, device="cuda")
    ut = torch.as_tensor(s.u_true.ravel(), device="cuda")
    full = B.solve_joint(plan, bt, delta, u_true=ut, op_dtype="f32", refine_iters=20, **prm)
    f64 = B.solve_joint(plan, bt, delta, u_true=ut, op_dtype="f64", **prm)
    assert full.rre == f64.rre and full.lambdas == f64.lambdas
    assert torch.equal(full.u, f64.u)
    # a target reached during the FP32 phase ends the solve there
    tgt = res.rre[4]
    early = B.solve_joint(plan, bt, delta, u_true=ut, op_dtype="f32", refine_iters=5, rre_target=tgt, **prm)
    assert early.iters <= 15 and early.rre[-1] <= tgt and early.status == 0
    # the returned solution is the iterate whose RRE stopped the solve (formed after the stop)
    rre_u = float(torch.linalg.vector_norm(early.u - ut) / torch.linalg.vector_norm(ut))
    assert abs(rre_u - early.rre[-1]) <= 1e-9 * early.rre[-1], (rre_u, early.rre[-1])


@pytest.mark.parametrize("sizes", [[(3, 24, 30), (4, 18, 18)], [(3, 24, 32), (4, 18, 20)]], ids=["ragged", "vec4"])
def test_solve_blur_ragged_fp64(B, sizes):
    import torch
    r = np.random.default_rng(5)
    us = []
    for (nt, ny, nx) in sizes:
        yy, xx = np.mgrid[0:ny, 0:nx]
        us.append(np.stack([(((xx - (8.0 + t)) ** 2 + (yy - ny / 2) ** 2) <= 16.0).astype(float) for t in range(nt)]))
    geoms = [mmgks.SeqGeom(nt, ny, nx) for (nt, ny, nx) in sizes]
    ops = mmgks.StackOps(geoms, "blur")
    ut = np.concatenate([u.ravel() for u in us])
    clean = ops.A(ut)
    b = noisy(clean, r.standard_normal(clean.shape), 0.01)
    delta = float(np.linalg.norm(b - clean))
    prm = dict(ell=5, k_max=8, tau=4, n_sweeps=30, alpha=0.2)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    plan = B.plan_blur(B.Stack(sizes), 9, 2.0)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype="f64", **prm)
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-7)
    assert_close(res.u.cpu().numpy(), ref.u, 1e-7)


@pytest.mark.parametrize("op", ["f64", "f32"])
def test_solve_blur_flow_on_reduced_frames(B, op):
    """flow_scale = 2: every flow update runs on frames reduced by 2 (odd sides, so the
    border blocks are partial) and is upscaled; the oracle's StackOps does the same."""
    import torch
    sizes = [(3, 25, 30), (4, 18, 21)]
    us = []
    for (nt, ny, nx) in sizes:
        yy, xx = np.mgrid[0:ny, 0:nx]
        us.append(np.stack([(((xx - (8.0 + 1.5 * t)) ** 2 + (yy - ny / 2) ** 2) <= 16.0).astype(float)
                            for t in range(nt)]))
    geoms = [mmgks.SeqGeom(nt, ny, nx) for (nt, ny, nx) in sizes]
    ops = mmgks.StackOps(geoms, "blur", flow_scale=2)
    ut = np.concatenate([u.ravel() for u in us])
    clean = ops.A(ut)
    b = noisy(clean, np.random.default_rng(7).standard_normal(clean.shape), 0.01)
    delta = float(np.linalg.norm(b - clean))
    prm = dict(ell=5, k_max=8, tau=3, n_sweeps=30, alpha=0.2)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    plan = B.plan_blur(B.Stack(sizes), 9, 2.0)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype=op, flow_scale=2, **prm)
    assert res.iters == ref.iters
    assert abs(res.rre[-1] - ref.rre[-1]) <= 1e-4
    if op == "f64":
        np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-7)
        assert_close(res.u.cpu().numpy(), ref.u, 1e-7)
        v_or = np.concatenate([fl[0].ravel() for fl in ref.flows])
        assert np.linalg.norm(res.v.cpu().numpy() - v_or) <= 1e-6 * max(np.linalg.norm(v_or), 1e-30)
    # graph replay of the reduced-frame flow update gives the eager result bit for bit
    again = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                          op_dtype=op, flow_scale=2, use_graph=1, **prm)
    assert torch.equal(again.u, res.u) and again.lambdas == res.lambdas


def test_solve_rejects_bad_arguments(B):
    import torch
    from paper_2501_12497_amd._lib import MMOFError
    u, ang, nb, g = _problem()
    plan = B.plan_radon(B.Stack.single(g.n_t, g.ny, g.nx), [ang.shape[1]], [nb], ang.ravel())
    b = torch.zeros(plan.m, dtype=torch.float64, device="cuda")
    with pytest.raises(MMOFError) as e:
        B.solve_joint(plan, b, 0.1, ell=10, k_max=248)   # basis of 257 columns: above the capacity
    assert e.value.code == -2
    with pytest.raises(MMOFError) as e:
        B.solve_joint(plan, b, 0.1, eps=-1.0)
    assert e.value.code == -1
    with pytest.raises(MMOFError) as e:
        B.solve_joint(plan, b, 0.1, op_dtype="f32", refine_iters=-1)
    assert e.value.code == -1
    with pytest.raises(MMOFError) as e:
        B.solve_joint(plan, b, 0.1, flow_scale=65)
    assert e.value.code == -1
    with pytest.raises(MMOFError) as e:   # 20 x 20 frames reduced by 10 leave no room for delta_r = 2
        B.solve_joint(plan, b, 0.1, flow_scale=10, delta_r=2)
    assert e.value.code == -1
