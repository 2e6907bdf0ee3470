"""GPU parity of the regulariser variants (Sec. 5, table of methods: D1 AnisoTV, D2 IsoTV,
D3 GS, each with and without the motion rows) against the FP64 oracle, through the C ABI:

* the temporal difference L_t and its adjoint on ragged stacks (a single-frame sequence among
  them), FP64 to 1e-12 and FP32 to 1e-5 of the per-element forward-error scale;
* the MM weights of every variant (groups over a pixel's two spatial differences, over a
  location's differences in all frames of its sequence) from the same Theta u;
* whole joint solves of every variant on a ragged batch of two moving sequences: FP64 against
  the oracle's lambda of every iteration and its u, FP32 operators to 1e-4 in RRE.
The oracle orders Theta's rows sequence by sequence, the library block by block over the
stack; the tests permute between the two."""
import math

import numpy as np
import pytest

from gpu_helpers import TOL32, TOL64, assert_close, dev, host, pack, roundtrip32
from oracle import mmgks, regops
from synth import angles_shifted, bins_for, noisy

pytestmark = pytest.mark.gpu

SIZES = [(3, 37, 75), (1, 20, 30), (4, 33, 33), (2, 9, 8)]


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_2501_12497_amd import binding
    return binding


@pytest.mark.parametrize("which", ["f64", "f32"])
def test_tdiff_forward_and_adjoint(B, which):
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    r = np.random.default_rng(40)
    us = [r.standard_normal(s) for s in SIZES]
    rs = [r.standard_normal((s[0] - 1, s[1], s[2])) for s in SIZES]
    if dt == torch.float32:
        us, rs = [roundtrip32(u) for u in us], [roundtrip32(x) for x in rs]
    stack = B.Stack(SIZES)
    got = host(B.apply_tdiff(stack, dev(pack(us), dt)))
    exp = pack([regops.tdiff_fwd(u) for u in us])
    sc = pack([np.abs(u[1:]) + np.abs(u[:-1]) for u in us])
    assert_close(got, exp, tol, sc)
    got = host(B.apply_tdiff(stack, dev(pack(rs), dt), transpose=True))
    exp = pack([regops.tdiff_adj(x) for x in rs])

    def abs_adj(x):   # |r(t-1)| + |r(t)|: the forward-error scale of the adjoint
        u = np.zeros((x.shape[0] + 1,) + x.shape[1:])
        u[1:] += np.abs(x)
        u[:-1] += np.abs(x)
        return u
    assert_close(got, exp, tol, pack([abs_adj(x) for x in rs]))


def _blocks(nt, ny, nx, reg, use_flow):
    """Row-block sizes of one sequence's Theta in the oracle's order."""
    npx = (nt - 1) * ny * nx
    b = [("gx", nt * ny * (nx - 1)), ("gy", nt * (ny - 1) * nx)]
    if reg in ("aniso", "iso"):
        b.append(("td", npx))
    if use_flow:
        b += [("f", npx), ("r", npx)]
    return b


def _to_stack_order(per_seq, sizes, reg, use_flow):
    """Oracle rows (sequence by sequence) -> library rows (block by block over the stack)."""
    parts = {}
    for vec, (nt, ny, nx) in zip(per_seq, sizes):
        o = 0
        for name, k in _blocks(nt, ny, nx, reg, use_flow):
            parts.setdefault(name, []).append(vec[o:o + k])
            o += k
    order = ["gx", "gy", "td", "f", "r"]
    return np.concatenate([np.concatenate(parts[k]) for k in order if k in parts])


@pytest.mark.parametrize("reg", ["psi", "aniso", "iso", "gs"])
@pytest.mark.parametrize("which", ["f64", "f32"])
def test_reg_weights_match_oracle(B, reg, which):
    import torch
    dt = torch.float64 if which == "f64" else torch.float32
    r = np.random.default_rng(41)
    eps = 0.05
    nus, ws = [], []
    for nt, ny, nx in SIZES:
        g = mmgks.SeqGeom(nt, ny, nx)
        ops = mmgks.StackOps([g], "blur", use_flow=nt > 1, reg=reg)
        nrow = sum(k for _, k in _blocks(nt, ny, nx, reg, nt > 1))
        nu = r.standard_normal(nrow) * r.choice([1e-3, 1.0], size=nrow)
        if dt == torch.float32:
            nu = roundtrip32(nu)
        nus.append(nu)
        ws.append(ops.weights(nu, eps))
    nu_s = _to_stack_order(nus, SIZES, reg, True)
    w_exp = _to_stack_order(ws, SIZES, reg, True)
    w = B.reg_weights(B.Stack(SIZES), reg, dev(nu_s, dt), eps).cpu().numpy()
    assert_close(w, w_exp, 1e-13, elementwise=True)


@pytest.mark.parametrize("eps", [1e-3, 0.05, 10.0])
def test_mm_weight_precision(B, eps):
    """The FP64 weight 1/sqrt(nu^2 + eps^2) of every weight path (hardware reciprocal square root
    and two Newton steps) against the correctly rounded division and square root of numpy, over
    |nu| from 1e-12 to 1e12: within 1e-15 relative (a few ulp), element by element."""
    import torch
    r = np.random.default_rng(43)
    nrow = sum(sum(k for _, k in _blocks(nt, ny, nx, "aniso", nt > 1)) for nt, ny, nx in SIZES)
    nu = r.choice([-1.0, 1.0], size=nrow) * 10.0 ** r.uniform(-12, 12, size=nrow)
    nu[:4] = [0.0, eps, -eps, 1e-300]
    w = B.reg_weights(B.Stack(SIZES), "aniso", dev(nu, torch.float64), eps).cpu().numpy()
    w_exp = 1.0 / np.sqrt(nu * nu + eps * eps)
    rel = np.abs(w - w_exp) / w_exp
    assert rel.max() <= 1e-15, (rel.max(), nu[np.argmax(rel)])


def _disk_seq(nt, n, x0, r2=10.0):
    yy, xx = np.mgrid[0:n, 0:n]
    return np.stack([(((xx - (x0 + t)) ** 2 + (yy - n / 2) ** 2) <= r2).astype(float) for t in range(nt)])


def _problem(sizes, reg, use_flow, seed=5):
    us = [_disk_seq(nt, n, 0.3 * n) for nt, n in sizes]
    angs = [angles_shifted(nt, 7, math.radians(5.0)) for nt, _ in sizes]
    geoms = [mmgks.SeqGeom(nt, n, n, a, bins_for(n)) for (nt, n), a in zip(sizes, angs)]
    ut = np.concatenate([u.ravel() for u in us])
    ops = mmgks.StackOps(geoms, "radon", use_flow=use_flow, reg=reg)
    clean = ops.A(ut)
    b = noisy(clean, np.random.default_rng(seed).standard_normal(clean.shape), 0.02)
    return ops, geoms, angs, ut, b, float(np.linalg.norm(b - clean))


@pytest.mark.parametrize("reg", ["aniso", "iso", "gs"])
@pytest.mark.parametrize("use_flow", [False, True])
def test_variant_solve_matches_oracle_fp64(B, reg, use_flow):
    import torch
    sizes = [(3, 16), (4, 14)]
    ops, geoms, angs, ut, b, delta = _problem(sizes, reg, use_flow)
    prm = dict(ell=6, k_max=9, tau=3, n_sweeps=30, alpha=0.2, use_flow=use_flow)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    stack = B.Stack([(g.n_t, g.ny, g.nx) for g in geoms])
    plan = B.plan_radon(stack, [a.shape[1] for a in angs], [g.n_bins for g in geoms],
                        np.concatenate([a.ravel() for a in angs]))
    print(f"variant solve {reg} flow={use_flow}", flush=True)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype="f64", reg=reg, **{k: v for k, v in prm.items() if k != "use_flow"},
                        use_flow=1 if use_flow else 0)
    assert res.iters == ref.iters and res.dp_status == ref.dp_status
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-7)
    np.testing.assert_allclose(res.rre, ref.rre, rtol=0, atol=1e-9)
    assert_close(res.u.cpu().numpy(), ref.u, 1e-7)


@pytest.mark.parametrize("reg", ["aniso", "iso", "gs"])
def test_variant_solve_fp32_operators(B, reg):
    import torch
    sizes = [(3, 16), (4, 14)]
    ops, geoms, angs, ut, b, delta = _problem(sizes, reg, True)
    prm = dict(ell=6, k_max=9, tau=3, n_sweeps=30, alpha=0.2)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    stack = B.Stack([(g.n_t, g.ny, g.nx) for g in geoms])
    plan = B.plan_radon(stack, [a.shape[1] for a in angs], [g.n_bins for g in geoms],
                        np.concatenate([a.ravel() for a in angs]))
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(ut, device="cuda"),
                        op_dtype="f32", reg=reg, **prm)
    assert res.iters == ref.iters
    assert abs(res.rre[-1] - ref.rre[-1]) <= 1e-4, (res.rre[-1], ref.rre[-1])
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-4)
