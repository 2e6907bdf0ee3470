"""HIP-graph replay of the solve's fixed launch sequences, and the tile-shape autotuner.

* A solve with use_graph=1 runs the flow update and the residual's operator applications
  eagerly on first use, captures them on the second and replays them afterwards (also in
  later solves, from the context's cache).  Every replay must give exactly the eager
  result: solves are repeated with eager work in between and compared bit for bit.
* Every tile-shape candidate of the tunable kernels computes the same values; the
  autotuner's report names a candidate for every tunable kernel of the plan.
"""
import numpy as np
import pytest

from synth import noisy

pytestmark = pytest.mark.gpu

SIZES = [(3, 40, 70), (5, 33, 33), (2, 64, 20)]
# widths that are multiples of 4: the stencil kernels take their vector forms
SIZES4 = [(3, 40, 72), (5, 33, 36), (2, 64, 20)]


def _ragged_blur_problem(B, torch, dtype, sizes=SIZES):
    r = np.random.default_rng(31)
    us = []
    for (nt, ny, nx) in sizes:
        yy, xx = np.mgrid[0:ny, 0:nx]
        cx, cy = nx * 0.4, ny * 0.5
        us.append(np.stack([(((xx - (cx + 1.5 * t)) ** 2 / 60.0 + (yy - cy) ** 2 / 30.0) <= 1.0).astype(float)
                            for t in range(nt)]))
    ut = np.concatenate([u.ravel() for u in us])
    plan = B.plan_blur(B.Stack(sizes), 9, 2.0)
    clean = B.apply_A(plan, torch.as_tensor(ut, device="cuda")).cpu().numpy()
    b = noisy(clean, r.standard_normal(clean.shape), 0.01)
    return plan, torch.as_tensor(b, device="cuda"), float(np.linalg.norm(b - clean)), \
        torch.as_tensor(ut, device="cuda")


def _solve(B, plan, b, delta, ut, op, use_graph, **extra):
    prm = dict(ell=5, k_max=9, tau=2, n_sweeps=20, alpha=0.2, op_dtype=op, use_graph=use_graph)
    prm.update(extra)
    return B.solve_joint(plan, b, delta, u_true=ut, **prm)


@pytest.mark.parametrize("op", ["f64", "f32"])
@pytest.mark.parametrize("sizes", [SIZES, SIZES4], ids=["ragged", "vec4"])
def test_graph_replays_match_eager(op, sizes):
    import torch
    from paper_2501_12497_amd import binding as B
    plan, b, delta, ut = _ragged_blur_problem(B, torch, op, sizes)
    ref = _solve(B, plan, b, delta, ut, op, 0)
    for rep in range(3):
        got = _solve(B, plan, b, delta, ut, op, 1)
        assert torch.equal(got.u, ref.u), rep
        assert torch.equal(got.v, ref.v) and torch.equal(got.v_rev, ref.v_rev), rep
        assert got.rre == ref.rre and got.lambdas == ref.lambdas, rep
        assert got.counts == ref.counts, (got.counts, ref.counts)
        # eager work between replays
        mid = _solve(B, plan, b, delta, ut, op, 0, k_max=4)
        assert mid.iters == 4


def test_graph_radon_solve_matches_eager():
    import torch
    from paper_2501_12497_amd import binding as B
    from synth import angles_shifted, bins_for
    n, nt = 24, 4
    yy, xx = np.mgrid[0:n, 0:n]
    u = np.stack([(((xx - (8.0 + t)) ** 2 + (yy - 12.0) ** 2) <= 16.0).astype(float) for t in range(nt)])
    ang = angles_shifted(nt, 8, np.radians(3.0))
    nb = bins_for(n)
    plan = B.plan_radon(B.Stack.single(nt, n, n), [8], [nb], ang.ravel())
    ut = torch.as_tensor(u.ravel(), device="cuda")
    clean = B.apply_A(plan, ut).cpu().numpy()
    b = torch.as_tensor(noisy(clean, np.random.default_rng(4).standard_normal(clean.shape), 0.02), device="cuda")
    delta = float(np.linalg.norm(b.cpu().numpy() - clean))
    ref = _solve(B, plan, b, delta, ut, "f32", 0)
    for _ in range(2):
        got = _solve(B, plan, b, delta, ut, "f32", 1)
        assert torch.equal(got.u, ref.u) and got.rre == ref.rre


@pytest.mark.parametrize("sizes", [SIZES, SIZES4], ids=["ragged", "vec4"])
def test_every_tile_candidate_gives_the_same_solve(sizes):
    import torch
    from paper_2501_12497_amd import binding as B
    plan, b, delta, ut = _ragged_blur_problem(B, torch, "f64", sizes)
    ref = _solve(B, plan, b, delta, ut, "f64", 0)
    x = torch.as_tensor(np.random.default_rng(5).standard_normal(plan.n), device="cuda")
    ax0 = B.apply_A(plan, x)
    n_cand = {"blur": 5, "grad_fwd": 4, "grad_adj": 4, "flow_fwd": 4, "flow_adj": 4}
    for c in range(1, 5):
        for k, nc in n_cand.items():
            plan.set_tile(k, min(c, nc - 1), torch.float64)
        assert torch.equal(B.apply_A(plan, x), ax0), c
        got = _solve(B, plan, b, delta, ut, "f64", 0)
        assert torch.equal(got.u, ref.u) and got.rre == ref.rre, c
    for k in n_cand:
        plan.set_tile(k, 0, torch.float64)


@pytest.mark.parametrize("sizes", [SIZES, SIZES4], ids=["ragged", "vec4"])
def test_autotune_report_and_errors(sizes):
    import torch
    from paper_2501_12497_amd import binding as B
    from paper_2501_12497_amd._lib import MMOFError
    plan, b, delta, ut = _ragged_blur_problem(B, torch, "f32", sizes)
    rep = plan.autotune(torch.float32)
    names = [item.split("=")[0] for item in rep.split()]
    assert names == ["blur", "grad_fwd", "grad_adj", "flow_fwd", "flow_adj"], rep
    got = _solve(B, plan, b, delta, ut, "f32", 1)
    ref = _solve(B, plan, b, delta, ut, "f32", 0)
    assert torch.equal(got.u, ref.u)
    with pytest.raises(MMOFError) as e:
        plan.set_tile("blur", 99, torch.float32)
    assert e.value.code == -1
    with pytest.raises(MMOFError) as e:
        plan.set_tile("nonesuch", 0, torch.float32)
    assert e.value.code == -1
