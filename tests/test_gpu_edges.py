"""Edge cases of the solve and the boundary, against the oracle where a value is defined.

* a ragged batch holding a single-frame sequence (no frame pair, so no flow rows) beside
  a moving sequence;
* noise-free data (delta = 0): the discrepancy equation has no root above the lower end of
  the lambda bracket, which is taken with the clamped status;
* the largest basis of the one-wave projected solve (ell + k_max - 1 = 64), and the paper's
  iteration budget (210 columns: the multi-wave solve and the tiled Gram);
* stacks the library must refuse (no sequences, a frame side above 65535, a single
  pixel row) and flow operators on a stack without frame pairs.
"""
import math

import numpy as np
from gpu_helpers import assert_close
import pytest

from oracle import mmgks
from synth import angles_shifted, bins_for, noisy

pytestmark = pytest.mark.gpu


def _disk_seq(nt, n, x0, r2=10.0):
    yy, xx = np.mgrid[0:n, 0:n]
    return np.stack([(((xx - (x0 + t)) ** 2 + (yy - n / 2) ** 2) <= r2).astype(float) for t in range(nt)])


def _radon_problem(sizes, n_th, level, seed):
    us = [_disk_seq(nt, n, 0.3 * n) for (nt, n, *_) in sizes]
    angs = [angles_shifted(nt, n_th, math.radians(5.0)) for (nt, *_) in sizes]
    geoms = [mmgks.SeqGeom(nt, n, n, a, bins_for(n)) for (nt, n, *_), a in zip(sizes, angs)]
    ut = np.concatenate([u.ravel() for u in us])
    ops = mmgks.StackOps(geoms, "radon")
    clean = ops.A(ut)
    b = noisy(clean, np.random.default_rng(seed).standard_normal(clean.shape), level) if level > 0 else clean
    return ops, geoms, angs, ut, b, float(np.linalg.norm(b - clean))


def _gpu_plan(B, geoms, angs):
    stack = B.Stack([(g.n_t, g.ny, g.nx) for g in geoms])
    return B.plan_radon(stack, [a.shape[1] for a in angs], [g.n_bins for g in geoms],
                        np.concatenate([a.ravel() for a in angs]))


def test_ragged_batch_with_a_single_frame_sequence():
    import torch
    from paper_2501_12497_amd import binding as B
    sizes = [(1, 20), (4, 16)]
    ops, geoms, angs, ut, b, delta = _radon_problem(sizes, 6, 0.02, 1)
    prm = dict(ell=6, k_max=8, tau=3, n_sweeps=30, alpha=0.2)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    plan = _gpu_plan(B, geoms, angs)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype="f64", **prm)
    assert res.iters == ref.iters
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-7)
    assert_close(res.u.cpu().numpy(), ref.u, 1e-7)
    assert res.v.numel() == 2 * 3 * 16 * 16  # only the moving sequence has pairs


def test_noise_free_data_clamps_lambda():
    import torch
    from paper_2501_12497_amd import binding as B
    ops, geoms, angs, ut, b, delta = _radon_problem([(3, 16)], 6, 0.0, 2)
    assert delta == 0.0
    prm = dict(ell=5, k_max=6, tau=2, n_sweeps=20, alpha=0.2)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    plan = _gpu_plan(B, geoms, angs)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype="f64", **prm)
    assert res.status == 2 and all(s == 2 for s in res.dp_status)
    assert ref.dp_status == res.dp_status
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-9)
    assert np.all(np.isfinite(res.u.cpu().numpy()))
    assert_close(res.u.cpu().numpy(), ref.u, 1e-7)


def test_largest_krylov_basis():
    import torch
    from paper_2501_12497_amd import binding as B
    ops, geoms, angs, ut, b, delta = _radon_problem([(2, 14)], 8, 0.02, 3)
    prm = dict(ell=10, k_max=55, tau=20, n_sweeps=20, alpha=0.2)   # 64 columns in the last solve
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    plan = _gpu_plan(B, geoms, angs)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype="f64", **prm)
    assert res.n_cols == ref.n_cols == 64
    assert abs(res.rre[-1] - ref.rre[-1]) <= 1e-6
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-5)


def test_paper_iteration_budget_210_columns():
    """The paper's iteration budget (Sec. 5: ell = 10, up to 200 MM iterations, flow every 20):
    201 iterations, so the last projected problems have up to 210 columns -- the Gram tiles
    beyond 64 columns, the four-wave projected solve and the two-pass CGS2 all run.  Against the
    oracle's stored run (tests/golden/krylov210.json, written by make_krylov210.py from the
    oracle alone): the lambda of every iteration, the RRE trajectory and the final u."""
    import json
    import os
    import torch
    from paper_2501_12497_amd import binding as B
    from synth import cfg_krylov210, noisy
    G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "krylov210.json")))
    wl = cfg_krylov210()
    s = wl.seqs[0]
    g = mmgks.SeqGeom(s.n_t, s.ny, s.nx, s.angles, s.n_bins)
    clean = mmgks.StackOps([g], "radon").A(s.u_true.ravel())
    b = noisy(clean, s.noise_g, wl.noise_level)
    delta = float(np.linalg.norm(b - clean))
    plan = _gpu_plan(B, [g], [s.angles])
    prm = dict(G["params"])
    print("krylov210: solve ell 10, 201 iterations", flush=True)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta,
                        u_true=torch.as_tensor(s.u_true.ravel(), device="cuda"), op_dtype="f64", **prm)
    assert res.iters == G["iters"] == 201
    assert res.n_cols == G["n_cols"] == 210
    assert res.dp_status == G["dp_status"]
    np.testing.assert_allclose(res.lambdas, G["lambdas"], rtol=1e-6)
    np.testing.assert_allclose(res.rre, G["rre"], rtol=0, atol=1e-7)
    assert_close(res.u.cpu().numpy(), np.asarray(G["u"]), 1e-6)


def test_refused_stacks():
    """The geometry is checked before any launch, so the operands can be tiny placeholders."""
    import torch
    from paper_2501_12497_amd import _lib, binding as B
    from paper_2501_12497_amd._lib import MMOFError
    ctx = B.context()
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    p = x.data_ptr()
    for sizes in ([], [(2, 70000, 4)], [(2, 1, 8)], [(0, 4, 4)]):
        st = B.Stack(sizes)
        ctx.bind()
        rc = ctx.lib.mmof_apply_grad(ctx.h, st.ref, _lib.MMOF_F64, 0, None, None, p, p, p)
        assert rc == -2, (sizes, rc)
    single = B.Stack([(1, 4, 4)])
    rc = ctx.lib.mmof_apply_flow_op(ctx.h, single.ref, _lib.MMOF_F64, _lib.MMOF_FLOW_FWD, 1, 0, p, p, None, p)
    assert rc == -2, rc


@pytest.mark.parametrize("where,val", [("b", float("nan")), ("b", float("inf")), ("u0", float("nan"))])
def test_nonfinite_input_is_refused(where, val):
    """A NaN or an infinity in b or in the initial estimate is found on the device before
    the first iteration and returned as MMOF_ERR_NONFINITE (-6); u_inout is left as given."""
    import torch
    from paper_2501_12497_amd import binding as B
    from paper_2501_12497_amd._lib import MMOFError
    sizes = [(3, 16)]
    ops, geoms, angs, ut, b, delta = _radon_problem(sizes, 5, 0.02, 2)
    plan = _gpu_plan(B, geoms, angs)
    bt = torch.as_tensor(b, device="cuda").clone()
    u0 = torch.zeros(plan.n, dtype=torch.float64, device="cuda")
    (bt if where == "b" else u0)[7] = val
    with pytest.raises(MMOFError) as e:
        B.solve_joint(plan, bt, delta, u0=u0, ell=4, k_max=3, tau=2, n_sweeps=5, op_dtype="f64")
    assert e.value.code == -6
    assert "NaN or Inf" in str(e.value)
