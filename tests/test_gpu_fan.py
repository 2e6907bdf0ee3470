"""GPU parity of the flat-detector fan-beam projector (Joseph's method) and of a joint solve
that uses it, against the FP64 oracle, through the C ABI.

Cases: a ragged stack (20 x 24 and 17 x 13 frames) under the three angle schedules of Sec. 5
plus angles at multiples of 45 degrees (rays exactly on the row / column diagonal: the
row-or-column choice must follow the oracle's bit for bit), FP64 (1e-12) and FP32 (1e-5 of
the projection of |u|); the adjoint identity on the GPU; a disk's projection at 256 x 256
against the oracle on sampled angles; argument checks; the joint solve on a fan-beam plan.
"""
import math

import numpy as np
import pytest

from gpu_helpers import TOL32, TOL64, assert_close, dev, host, pack, roundtrip32
from oracle import forward
from synth import angle_schedule

pytestmark = pytest.mark.gpu

SIZES = [(3, 20, 24), (2, 17, 13)]
GEO = dict(dso=40.0, dsd=70.0, du=1.3)
NB = [41, 33]


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_2501_12497_amd import binding
    return binding


def _angles(kind, sizes, n_views):
    if kind == "diag":
        return [np.tile(np.arange(n_views) * (math.pi / 4), (nt, 1)) for nt, _, _ in sizes]
    return [angle_schedule(kind, nt, n_views) for nt, _, _ in sizes]


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["fixed", "equal", "shifted", "diag"])
def test_fan_forward_and_adjoint(B, which, kind):
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    nv = 8 if kind == "diag" else 7
    angs = _angles(kind, SIZES, nv)
    r = np.random.default_rng(3)
    us = [r.standard_normal(s) for s in SIZES]
    if dt == torch.float32:
        us = [roundtrip32(u) for u in us]
    plan = B.plan_fan(B.Stack(SIZES), [nv] * 2, NB, np.concatenate([a.ravel() for a in angs]), **GEO)
    got = host(B.apply_A(plan, dev(pack(us), dt)))
    exp = pack([forward.fan_fwd(u, a, nb, **GEO) for u, a, nb in zip(us, angs, NB)])
    sc = pack([forward.fan_fwd(np.abs(u), a, nb, **GEO) for u, a, nb in zip(us, angs, NB)])
    assert_close(got, exp, tol, sc)
    bs = [r.standard_normal((nt, nv, nb)) for (nt, _, _), nb in zip(SIZES, NB)]
    if dt == torch.float32:
        bs = [roundtrip32(b) for b in bs]
    got = host(B.apply_At(plan, dev(pack(bs), dt)))
    exp = pack([forward.fan_adj(b, a, ny, nx, **GEO) for b, a, (_, ny, nx) in zip(bs, angs, SIZES)])
    sc = pack([forward.fan_adj(np.abs(b), a, ny, nx, **GEO) for b, a, (_, ny, nx) in zip(bs, angs, SIZES)])
    assert_close(got, exp, tol, sc)


def test_fan_adjoint_identity_fp64(B):
    import torch
    angs = _angles("shifted", SIZES, 9)
    plan = B.plan_fan(B.Stack(SIZES), [9, 9], NB, np.concatenate([a.ravel() for a in angs]), **GEO)
    g = torch.Generator(device="cuda").manual_seed(5)
    u = torch.randn(plan.n, dtype=torch.float64, device="cuda", generator=g)
    b = torch.randn(plan.m, dtype=torch.float64, device="cuda", generator=g)
    lhs = float(torch.dot(B.apply_A(plan, u), b))
    rhs = float(torch.dot(u, B.apply_At(plan, b)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_fan_disk_256_sampled(B):
    import torch
    n, nv, nb = 256, 12, 301
    geo = dict(dso=300.0, dsd=500.0, du=1.4)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    c = (n - 1) / 2.0
    disk = (((x - c - 20) ** 2 + (y - c + 10) ** 2) <= 80.0 ** 2).astype(float)
    ang = angle_schedule("shifted", 1, nv)
    plan = B.plan_fan(B.Stack.single(1, n, n), [nv], [nb], ang.ravel(), **geo)
    got = host(B.apply_A(plan, dev(disk.ravel(), torch.float32))).reshape(nv, nb)
    for k in (0, 5, 11):
        exp = forward.fan_fwd(disk[None], ang[:, k:k + 1], nb, **geo)[0, 0]
        assert_close(got[k], exp, TOL32, msg=k)


def test_fan_rejects_bad_geometry(B):
    from paper_2501_12497_amd._lib import MMOFError
    st = B.Stack.single(2, 20, 20)
    ang = np.zeros(4)
    for geo in (dict(dso=40.0, dsd=30.0, du=1.0), dict(dso=12.0, dsd=50.0, du=1.0), dict(dso=40.0, dsd=70.0, du=0.0)):
        with pytest.raises(MMOFError) as e:
            B.plan_fan(st, [2], [31], ang, **geo)
        assert e.value.code == -1, geo


def test_joint_solve_on_fan_beam(B):
    """MMGKS-OF with the fan-beam H (shifted schedule, 6 views per frame), FP64 against the
    oracle's run of the same configuration."""
    import torch
    from oracle import mmgks
    from synth import noisy
    n, nt, nv, nb = 20, 3, 6, 37
    geo = dict(dso=45.0, dsd=80.0, du=1.6)
    yy, xx = np.mgrid[0:n, 0:n]
    u = np.stack([(((xx - (7.0 + t)) ** 2 + (yy - 10.0) ** 2) <= 12.0).astype(float) for t in range(nt)])
    ang = angle_schedule("shifted", nt, nv)
    g = mmgks.SeqGeom(nt, n, n, ang, nb)
    ops = mmgks.StackOps([g], "fan", fan=(geo["dso"], geo["dsd"], geo["du"]))
    clean = ops.A(u.ravel())
    b = noisy(clean, np.random.default_rng(4).standard_normal(clean.shape), 0.02)
    delta = float(np.linalg.norm(b - clean))
    prm = dict(ell=6, k_max=10, tau=3, n_sweeps=40, alpha=0.2)
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=u.ravel())
    plan = B.plan_fan(B.Stack.single(nt, n, n), [nv], [nb], ang.ravel(), **geo)
    res = B.solve_joint(plan, torch.as_tensor(b, device="cuda"), delta, u_true=torch.as_tensor(u.ravel(), device="cuda"),
                        op_dtype="f64", **prm)
    assert res.iters == ref.iters
    np.testing.assert_allclose(res.lambdas, ref.lambdas, rtol=1e-7)
    assert_close(res.u.cpu().numpy(), ref.u, 1e-7)


@pytest.mark.parametrize("which", ["f64", "f32"])
def test_fan_source_close_to_the_frame(B, which):
    """A source 0.2 px beyond the bound the plan accepts and a fine detector: the transpose's
    FP32 candidate bounds would need a margin above half a bin, so it takes the FP64 bounds,
    and a tile's rays span more bins than are staged, so it reads the ray table directly."""
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    sizes = [(2, 24, 20)]
    geo = dict(dso=0.5 * math.hypot(24, 20) + 2.2, dsd=30.0, du=0.2)
    nv, nb = 6, 81
    angs = _angles("equal", sizes, nv)
    r = np.random.default_rng(17)
    bs = [r.standard_normal((2, nv, nb))]
    us = [r.standard_normal(sizes[0])]
    if dt == torch.float32:
        bs = [roundtrip32(b) for b in bs]
        us = [roundtrip32(u) for u in us]
    plan = B.plan_fan(B.Stack(sizes), [nv], [nb], angs[0].ravel(), **geo)
    got = host(B.apply_At(plan, dev(pack(bs), dt)))
    exp = forward.fan_adj(bs[0], angs[0], 24, 20, **geo).ravel()
    sc = forward.fan_adj(np.abs(bs[0]), angs[0], 24, 20, **geo).ravel()
    assert np.abs(exp).max() > 0
    assert_close(got, exp, tol, sc)
    got = host(B.apply_A(plan, dev(pack(us), dt)))
    exp = forward.fan_fwd(us[0], angs[0], nb, **geo).ravel()
    sc = forward.fan_fwd(np.abs(us[0]), angs[0], nb, **geo).ravel()
    assert_close(got, exp, tol, sc)
