"""The batched deblurring workload at its full size: 40 sequences of uneven sizes
(64^2..256^2, 8..32 frames, about 2.1e7 pixels), 9x9 Gaussian blur, in one packed stack.

* Sampled parity: H (blur), Psi and L(v) in FP32 on the whole stack in one launch each; the
  oracle recomputes the first and last frame (or pair) of every sequence in FP64 from the
  same FP32 inputs.
* A ragged subset of five sequences solved against the oracle's stored run (FP64 and FP32).
* The solve in its benchmark configuration (FP32 operators, FP64 Krylov, autotuned tiles)
  with the launch sequences replayed from HIP graphs gives bit for bit the eagerly launched
  solve, and its error decreases.  (The oracle's full solve at this size would take hours;
  the ragged blur solve is held to the oracle at a small size in test_gpu_solve.)
"""
import numpy as np
import pytest

from gpu_helpers import TOL32, assert_close
from oracle import forward, regops
from synth import cfg_blur_ragged, smooth_flow_coarse

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rag():
    import torch
    from paper_2501_12497_amd import binding as B
    wl = cfg_blur_ragged()
    sizes = [(s.n_t, s.ny, s.nx) for s in wl.seqs]
    stack = B.Stack(sizes)
    plan = B.plan_blur(stack, 9, 2.0)
    u32 = [s.u_true.astype(np.float32) for s in wl.seqs]
    u = torch.from_numpy(np.concatenate([x.ravel() for x in u32])).cuda()
    return dict(B=B, torch=torch, wl=wl, sizes=sizes, stack=stack, plan=plan, u32=u32, u=u)


def _split(vec, shapes):
    out, o = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        out.append(vec[o:o + k].reshape(sh))
        o += k
    return out


def test_blur_psi_flow_ragged40_sampled(rag):
    B, torch, sizes, u32 = rag["B"], rag["torch"], rag["sizes"], rag["u32"]
    assert rag["stack"].n > 2e7
    # H
    hb = _split(B.apply_A(rag["plan"], rag["u"]).cpu().numpy(), sizes)
    for i, (nt, ny, nx) in enumerate(sizes):
        for t in (0, nt - 1):
            ut = u32[i][t:t + 1].astype(np.float64)
            exp = forward.blur(ut)[0]
            sc = forward.blur(np.abs(ut))[0]
            assert_close(hb[i][t], exp, TOL32, sc, msg=(i, t))
    # Psi
    gx, gy = B.apply_grad(rag["stack"], rag["u"])
    gxs = _split(gx.cpu().numpy(), [(nt, ny, nx - 1) for nt, ny, nx in sizes])
    gys = _split(gy.cpu().numpy(), [(nt, ny - 1, nx) for nt, ny, nx in sizes])
    for i, (nt, ny, nx) in enumerate(sizes):
        ut = u32[i][[0, nt - 1]].astype(np.float64)
        ex, ey = regops.grad_fwd(ut)
        assert_close(gxs[i][[0, nt - 1]], ex, TOL32, np.abs(ut[:, :, 1:]) + np.abs(ut[:, :, :-1]), msg=i)
        assert_close(gys[i][[0, nt - 1]], ey, TOL32, np.abs(ut[:, 1:, :]) + np.abs(ut[:, :-1, :]), msg=i)
    # L(v), forward direction, with a smooth flow of up to 2 px per sequence
    from paper_2501_12497_amd import _lib
    vs = [smooth_flow_coarse(nt - 1, nx, seed=40 + i, coarse=8, vmax=2.0).astype(np.float32)
          for i, (nt, ny, nx) in enumerate(sizes)]
    v = torch.from_numpy(np.concatenate([x.ravel() for x in vs])).cuda()
    r = B.apply_flow_op(rag["stack"], _lib.MMOF_FLOW_FWD, 1, _lib.MMOF_INTERP_BILINEAR, rag["u"], v)
    rs = _split(r.cpu().numpy(), [(nt - 1, ny, nx) for nt, ny, nx in sizes])
    for i, (nt, ny, nx) in enumerate(sizes):
        for p in (0, nt - 2):
            ut = u32[i][p:p + 2].astype(np.float64)
            vp = vs[i][p:p + 1].astype(np.float64)
            exp = regops.flow_fwd(ut, vp, 1)[0]
            M = abs(regops.motion_matrix(vp[0]))
            sc = (M @ np.abs(ut[1]).ravel()).reshape(ny, nx) + np.abs(ut[0])
            assert_close(rs[i][p], exp, TOL32, sc, msg=(i, p))


def test_solve_ragged40_graph_matches_eager(rag):
    B, torch, wl = rag["B"], rag["torch"], rag["wl"]
    plan = rag["plan"]
    ut = torch.as_tensor(np.concatenate([s.u_true.ravel() for s in wl.seqs]), dtype=torch.float64, device="cuda")
    clean = B.apply_A(plan, ut)
    g = torch.as_tensor(np.concatenate([s.noise_g.ravel() for s in wl.seqs]), dtype=torch.float64, device="cuda")
    e = 0.01 * torch.linalg.vector_norm(clean) * g / torch.linalg.vector_norm(g)
    b = (clean + e).contiguous()
    delta = float(torch.linalg.vector_norm(e))
    plan.autotune(torch.float32)
    prm = dict(ell=10, k_max=6, tau=3, n_sweeps=40, alpha=0.1, eps=1e-3, eta=1.01, delta_r=1, op_dtype="f32")
    ref = B.solve_joint(plan, b, delta, u_true=ut, use_graph=0, **prm)
    for rep in range(2):
        got = B.solve_joint(plan, b, delta, u_true=ut, use_graph=1, **prm)
        assert torch.equal(got.u, ref.u), rep
        assert got.rre == ref.rre and got.lambdas == ref.lambdas, rep
    assert ref.iters == 6 and all(np.isfinite(ref.rre))
    assert ref.rre[-1] < ref.rre[0]


@pytest.mark.parametrize("op", ["f64", "f32"])
def test_ragged_subset_solve_against_oracle(op):
    """The five smallest sequences of the 40 (80^2 x 8 .. 115^2 x 12, 410,305 pixels) as one
    ragged batch, 13 iterations with one flow update on a nonzero image, against the oracle's
    stored run (tests/golden/ragged5.json, written by make_ragged5.py): FP64 operators give the
    oracle's lambda of every iteration and its RRE trajectory; FP32 operators its final RRE to
    1e-4 (the solve bar)."""
    import json
    import os
    import sys
    import torch
    from paper_2501_12497_amd import binding as B
    here = os.path.join(os.path.dirname(__file__), "golden")
    sys.path.insert(0, here)
    try:
        from make_ragged5 import subset
    finally:
        sys.path.remove(here)
    G = json.load(open(os.path.join(here, "ragged5.json")))
    wl, pick, seqs, ops, ut, b, delta = subset()
    assert pick == G["pick"]
    stack = B.Stack([(s.n_t, s.ny, s.nx) for s in seqs])
    plan = B.plan_blur(stack, 9, 2.0)
    print(f"ragged subset solve {op}", flush=True)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype=op, **G["params"])
    assert res.iters == G["iters"]
    if op == "f64":
        assert res.dp_status == G["dp_status"]
        np.testing.assert_allclose(res.lambdas, G["lambdas"], rtol=1e-6)
        np.testing.assert_allclose(res.rre, G["rre"], rtol=0, atol=1e-8)
    else:
        assert abs(res.rre[-1] - G["rre"][-1]) <= 1e-4, (res.rre[-1], G["rre"][-1])
