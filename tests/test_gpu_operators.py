"""GPU parity of every operator kernel against the FP64 oracle, through the C ABI.

Stacks are ragged batches whose frames span several kernel tiles and end in partial
tiles.  FP64 kernels must match to 1e-12 (norm-wise relative); FP32 kernels get FP32
inputs (the oracle sees the same values upcast) and must match to 1e-5 relative to the
forward-error scale ||Op| |x|| (for cancellation-prone outputs) or to ||y||.
"""
import math

import numpy as np
import pytest

from gpu_helpers import TOL32, TOL64, assert_close, dev, host, pack, roundtrip32, unpack
from oracle import forward, optflow, regops
from synth import bins_for, nudge_off_kinks

pytestmark = pytest.mark.gpu

SIZES = [(3, 37, 75), (2, 20, 130), (4, 33, 33)]   # (n_t, ny, nx) per sequence
# every width a multiple of 4: the stencil kernels take their vector forms (4 pixels per
# lane); ragged heights and widths that end in partial tiles of every candidate, and a
# frame one vector wide
SIZES4 = [(3, 37, 76), (2, 21, 132), (4, 33, 36), (2, 9, 8), (2, 6, 4)]
LAYOUTS = {"ragged": SIZES, "vec4": SIZES4}


@pytest.fixture(scope="module")
def B():
    import torch  # noqa: F401
    from paper_2501_12497_amd import binding
    return binding


def _rand_stack(seed, sizes=SIZES):
    r = np.random.default_rng(seed)
    return [r.standard_normal(s) for s in sizes]


def _dtypes():
    import torch
    return [(torch.float64, TOL64), (torch.float32, TOL32)]


# --------------------------------------------------------------------------- Radon


def _angles(r, n_t, n_th):
    a = r.uniform(0, math.pi, size=(n_t, n_th))
    a[0, :4] = [0.0, math.pi / 2, math.pi / 4, 3 * math.pi / 4][: min(4, n_th)]
    return a


@pytest.mark.parametrize("cand", [0, 1, 2, 3])   # angle groups of 1, 2, 4, 8 per workgroup
@pytest.mark.parametrize("which", ["f64", "f32"])
def test_radon_forward_and_adjoint(B, which, cand):
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    r = np.random.default_rng(10)
    us = _rand_stack(11)
    n_th = [7, 5, 9]
    nbins = [bins_for(max(SIZES[0][1], SIZES[0][2])), 23, bins_for(33)]
    angs = [_angles(r, s[0], k) for s, k in zip(SIZES, n_th)]
    stack = B.Stack(SIZES)
    plan = B.plan_radon(stack, n_th, nbins, np.concatenate([a.ravel() for a in angs]))
    plan.set_tile("radon_fwd", cand, dt)
    if dt == torch.float32:
        us = [roundtrip32(u) for u in us]
    b = host(B.apply_A(plan, dev(pack(us), dt)))
    exp = [forward.radon_fwd(u, a, nb) for u, a, nb in zip(us, angs, nbins)]
    scale = pack([forward.radon_fwd(np.abs(u), a, nb) for u, a, nb in zip(us, angs, nbins)])
    assert_close(b, pack(exp), tol, scale)
    bs = [r.standard_normal(e.shape) for e in exp]
    if dt == torch.float32:
        bs = [roundtrip32(x) for x in bs]
    u = host(B.apply_At(plan, dev(pack(bs), dt)))
    expu = [forward.radon_adj(x, a, s[1], s[2]) for x, a, s in zip(bs, angs, SIZES)]
    scale = pack([forward.radon_adj(np.abs(x), a, s[1], s[2]) for x, a, s in zip(bs, angs, SIZES)])
    assert_close(u, pack(expu), tol, scale)


@pytest.mark.parametrize("cand", [0, 3])
@pytest.mark.parametrize("which", ["f64", "f32"])
def test_radon_forward_wide_frames(B, which, cand):
    """Non-square frames of several hundred pixels (two 300 x 700 frames and a 620 x 90 one),
    angles that include 0, 45, 90 and 135 degrees and a detector wider than the frames'
    diagonal, with one and with eight angles per workgroup, against the oracle element by
    element."""
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    r = np.random.default_rng(14)
    sizes = [(2, 300, 700), (1, 620, 90)]
    us = [r.uniform(0.0, 1.0, (nt, ny, nx)) for nt, ny, nx in sizes]
    base = np.array([0.0, 0.25, 0.5, 0.75]) * math.pi
    angs = [np.stack([np.concatenate([base, r.uniform(0, math.pi, 5)]) for _ in range(s[0])]) for s in sizes]
    nbins = [bins_for(700) + 40, bins_for(620)]
    plan = B.plan_radon(B.Stack(sizes), [9, 9], nbins, np.concatenate([a.ravel() for a in angs]))
    plan.set_tile("radon_fwd", cand, dt)
    if dt == torch.float32:
        us = [roundtrip32(u) for u in us]
    b = host(B.apply_A(plan, dev(pack(us), dt)))
    exp = pack([forward.radon_fwd(u, a, nb) for u, a, nb in zip(us, angs, nbins)])
    scale = pack([forward.radon_fwd(np.abs(u), a, nb) for u, a, nb in zip(us, angs, nbins)])
    assert_close(b, exp, tol, scale)


@pytest.mark.parametrize("which", ["f64", "f32"])
def test_radon_forward_frames_of_quarter_widths(B, which):
    """Frames whose sides are multiples of 4 but not of 32 (100 x 68 and 36 x 132, offsets then
    multiples of 4 too): the frame transpose takes its vector form on tiles the frame edges cut;
    steep and flat angles, against the oracle element by element."""
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    r = np.random.default_rng(15)
    sizes = [(3, 100, 68), (2, 36, 132)]
    us = [r.uniform(0.0, 1.0, (nt, ny, nx)) for nt, ny, nx in sizes]
    base = np.array([0.0, 0.25, 0.5, 0.75]) * math.pi
    angs = [np.stack([np.concatenate([base, r.uniform(0, math.pi, 3)]) for _ in range(s[0])]) for s in sizes]
    nbins = [bins_for(100), bins_for(132)]
    plan = B.plan_radon(B.Stack(sizes), [7, 7], nbins, np.concatenate([a.ravel() for a in angs]))
    if dt == torch.float32:
        us = [roundtrip32(u) for u in us]
    b = host(B.apply_A(plan, dev(pack(us), dt)))
    exp = pack([forward.radon_fwd(u, a, nb) for u, a, nb in zip(us, angs, nbins)])
    scale = pack([forward.radon_fwd(np.abs(u), a, nb) for u, a, nb in zip(us, angs, nbins)])
    assert_close(b, exp, tol, scale)


def test_radon_adjoint_identity_fp64(B):
    import torch
    r = np.random.default_rng(12)
    sizes = [(2, 64, 64), (1, 50, 70)]
    stack = B.Stack(sizes)
    plan = B.plan_radon(stack, [30, 11], [bins_for(64), 87], r.uniform(0, 2 * math.pi, 2 * 30 + 11))
    u = torch.randn(plan.n, dtype=torch.float64, device="cuda")
    b = torch.randn(plan.m, dtype=torch.float64, device="cuda")
    lhs = float((B.apply_A(plan, u) * b).sum())
    rhs = float((u * B.apply_At(plan, b)).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# --------------------------------------------------------------------------- blur


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("ksize,sigma", [(9, 2.0), (5, 1.0)])   # compiled-in 9-tap path and the general one
def test_blur(B, which, ksize, sigma):
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    us = _rand_stack(13)
    if dt == torch.float32:
        us = [roundtrip32(u) for u in us]
    plan = B.plan_blur(B.Stack(SIZES), ksize, sigma)
    y = host(B.apply_A(plan, dev(pack(us), dt)))
    exp = pack([forward.blur(u, ksize, sigma) for u in us])
    sc = pack([forward.blur(np.abs(u), ksize, sigma) for u in us])
    assert_close(y, exp, tol, sc)
    y2 = host(B.apply_At(plan, dev(pack(us), dt)))
    assert_close(y2, pack([forward.blur_adj(u, ksize, sigma) for u in us]), tol, sc)


# --------------------------------------------------------------------------- gradient


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("layout", ["ragged", "vec4"])
def test_grad_forward_and_adjoint(B, which, weighted, layout):
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    sizes = LAYOUTS[layout]
    nseq = len(sizes)
    r = np.random.default_rng(14)
    us = _rand_stack(15, sizes)
    gxs = [r.standard_normal((s[0], s[1], s[2] - 1)) for s in sizes]
    gys = [r.standard_normal((s[0], s[1] - 1, s[2])) for s in sizes]
    wxs = [r.random(g.shape) for g in gxs] if weighted else None
    wys = [r.random(g.shape) for g in gys] if weighted else None
    if dt == torch.float32:
        us, gxs, gys = [list(map(roundtrip32, a)) for a in (us, gxs, gys)]
        if weighted:
            wxs, wys = list(map(roundtrip32, wxs)), list(map(roundtrip32, wys))
    stack = B.Stack(sizes)
    wx = dev(pack(wxs), dt) if weighted else None
    wy = dev(pack(wys), dt) if weighted else None
    gx, gy = B.apply_grad(stack, dev(pack(us), dt), wx=wx, wy=wy)
    ex = [regops.grad_fwd(u, *((a, b) if weighted else ())) for u, a, b in
          zip(us, wxs or [None] * nseq, wys or [None] * nseq)]
    # per-element forward-error scales |w| (|u_right| + |u_left|)
    sx = pack([(wxs[i] if weighted else 1.0) * (np.abs(u[:, :, 1:]) + np.abs(u[:, :, :-1])) for i, u in enumerate(us)])
    sy = pack([(wys[i] if weighted else 1.0) * (np.abs(u[:, 1:, :]) + np.abs(u[:, :-1, :])) for i, u in enumerate(us)])
    assert_close(host(gx), pack([e[0] for e in ex]), tol, sx)
    assert_close(host(gy), pack([e[1] for e in ex]), tol, sy)
    u = host(B.apply_grad(stack, gx=dev(pack(gxs), dt), gy=dev(pack(gys), dt), wx=wx, wy=wy, transpose=True))
    exp = pack([regops.grad_adj(a, b, *((c, d) if weighted else ())) for a, b, c, d in
                zip(gxs, gys, wxs or [None] * nseq, wys or [None] * nseq)])
    scale = []
    for i, (a, b) in enumerate(zip(gxs, gys)):
        a = np.abs(a) * (wxs[i] if weighted else 1.0)
        b = np.abs(b) * (wys[i] if weighted else 1.0)
        sc = np.zeros(sizes[i])
        sc[:, :, 1:] += a
        sc[:, :, :-1] += a
        sc[:, 1:, :] += b
        sc[:, :-1, :] += b
        scale.append(sc)
    scale = pack(scale)
    assert_close(u, exp, tol, scale)


# --------------------------------------------------------------------------- flow operator


def _flows(seed, vmax, sizes=SIZES, nudge=False):
    r = np.random.default_rng(seed)
    vs = [r.uniform(-vmax, vmax, size=(s[0] - 1, 2, s[1], s[2])) for s in sizes]
    return [nudge_off_kinks(v) for v in vs] if nudge else vs


def _abs_warp(u, v, direction, interp, adjoint=False, r=None):
    """Forward-error scale |W| |src| + |sub| (or its adjoint counterpart)."""
    n_t = u.shape[0] if not adjoint else r.shape[0] + 1
    out = []
    for t in range(v.shape[0]):
        M = abs(regops.motion_matrix(v[t], interp))
        if not adjoint:
            src = u[t + 1] if direction > 0 else u[t]
            sub = u[t] if direction > 0 else u[t + 1]
            out.append((M @ np.abs(src).ravel()).reshape(src.shape) + np.abs(sub))
    if adjoint:
        acc = np.zeros((n_t,) + r.shape[1:])
        for t in range(r.shape[0]):
            M = abs(regops.motion_matrix(v[t], interp))
            back = (M.T @ np.abs(r[t]).ravel()).reshape(r.shape[1:])
            if direction > 0:
                acc[t + 1] += back
                acc[t] += np.abs(r[t])
            else:
                acc[t] += back
                acc[t + 1] += np.abs(r[t])
        return acc
    return np.stack(out)


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("interp", ["bilinear", "round"])
@pytest.mark.parametrize("vmax", [3.5, 11.0])   # LDS-staged adjoint (radius <= 8) and the wide-window path
@pytest.mark.parametrize("layout", ["ragged", "vec4"])
def test_flow_operator(B, which, direction, interp, vmax, layout):
    import torch
    from paper_2501_12497_amd import _lib
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    sizes = LAYOUTS[layout]
    us = _rand_stack(16, sizes)
    vs = _flows(17, vmax, sizes)
    rs = [np.random.default_rng(18 + i).standard_normal((s[0] - 1, s[1], s[2])) for i, s in enumerate(sizes)]
    if dt == torch.float32:
        us, vs, rs = [list(map(roundtrip32, a)) for a in (us, vs, rs)]
    stack = B.Stack(sizes)
    ip = _lib.MMOF_INTERP_BILINEAR if interp == "bilinear" else _lib.MMOF_INTERP_ROUND
    du, dv, dr = dev(pack(us), dt), dev(pack(vs), dt), dev(pack(rs), dt)
    y = host(B.apply_flow_op(stack, _lib.MMOF_FLOW_FWD, direction, ip, du, dv))
    exp = pack([regops.flow_fwd(u, v, direction, interp) for u, v in zip(us, vs)])
    scale = pack([_abs_warp(u, v, direction, interp) for u, v in zip(us, vs)])
    assert_close(y, exp, tol, scale)
    ya = B.apply_flow_op(stack, _lib.MMOF_FLOW_ADJ, direction, ip, None, dv, dr)
    exp = pack([regops.flow_adj(r, v, s[0], direction, interp) for r, v, s in zip(rs, vs, sizes)])
    scale = pack([_abs_warp(None, v, direction, interp, True, r) for r, v in zip(rs, vs)])
    assert_close(host(ya), exp, tol, scale)
    # the adjoint is a deterministic gather: bitwise reproducible
    ya2 = B.apply_flow_op(stack, _lib.MMOF_FLOW_ADJ, direction, ip, None, dv, dr)
    assert torch.equal(ya, ya2)


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("direction", [1, -1])
def test_flow_dv(B, which, direction):
    import torch
    from paper_2501_12497_amd import _lib
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    us = _rand_stack(19)
    vs = _flows(20, 3.0, nudge=True)
    ws = [np.random.default_rng(21 + i).standard_normal((s[0] - 1, s[1], s[2])) for i, s in enumerate(SIZES)]
    if dt == torch.float32:
        us, vs, ws = [list(map(roundtrip32, a)) for a in (us, vs, ws)]
    stack = B.Stack(SIZES)
    g = host(B.apply_flow_op(stack, _lib.MMOF_FLOW_DV, direction, _lib.MMOF_INTERP_BILINEAR,
                             dev(pack(us), dt), dev(pack(vs), dt), dev(pack(ws), dt)))
    exp = pack([regops.flow_dv(u, v, w, direction) for u, v, w in zip(us, vs, ws)])
    scale = pack([2 * np.abs(w)[:, None] * np.abs(u).max() * np.ones((1, 2, 1, 1)) for u, w in zip(us, ws)])
    assert_close(g, exp, tol, scale)


# --------------------------------------------------------------------------- optical flow pieces


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("dr,layout", [(1, "ragged"), (2, "ragged"), (1, "vec4"), (2, "vec4"), (3, "vec4"),
                                       (4, "vec4"), (5, "vec4")])
def test_of_derivs(B, which, dr, layout):
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    sizes = LAYOUTS[layout]
    if layout == "vec4":   # radius below every frame side
        sizes = [s for s in sizes if min(s[1], s[2]) > dr]
    us = _rand_stack(22, sizes)
    if dt == torch.float32:
        us = [roundtrip32(u) for u in us]
    I = host(B.of_derivs(B.Stack(sizes), dev(pack(us), dt), dr))
    exp = pack([optflow.of_derivs(u, dr) for u in us])
    scale = pack([optflow.of_derivs(np.abs(u), dr) * 0 + np.abs(u).max() for u in us])
    assert_close(I, exp, tol, scale)


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["ragged", "vec4"])
def test_flow_update_and_reverse(B, which, layout):
    import torch
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    sizes = LAYOUTS[layout]
    r = np.random.default_rng(23)
    us = [np.cumsum(np.cumsum(r.standard_normal(s), axis=1), axis=2) * 0.05 for s in sizes]   # smooth-ish images
    vs0 = _flows(24, 0.5, sizes)
    if dt == torch.float32:
        us, vs0 = [list(map(roundtrip32, a)) for a in (us, vs0)]
    stack = B.Stack(sizes)
    v = dev(pack(vs0), dt)
    vr = torch.empty_like(v)
    B.flow_update(stack, dev(pack(us), dt), v, alpha=0.3, n_sweeps=25, delta_r=1, v_rev=vr)
    exp = [optflow.flow_update(u, v0, 0.3, 25, 1) for u, v0 in zip(us, vs0)]
    got = host(v)
    assert_close(got, pack(exp), TOL64 if dt == torch.float64 else 1e-4)
    # reverse flow of the GPU's own flow (rounding decisions must see identical inputs)
    gshapes = [e.shape for e in exp]
    exp_r = pack([optflow.reverse_flow(x) for x in unpack(got, gshapes)])
    assert_close(host(vr), exp_r, tol)


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["ragged", "vec4"])
@pytest.mark.parametrize("scale", [2, 3])
def test_flow_update_scaled(B, which, layout, scale):
    """The flow computed on frames reduced by `scale` (block means, warm start v/scale, HS on
    the reduced frames, bilinear upscaling times scale) against the oracle; frame sides not
    divisible by the scale leave partial border blocks."""
    import torch
    dt = torch.float64 if which == "f64" else torch.float32
    sizes = LAYOUTS[layout]
    r = np.random.default_rng(27)
    us = [np.cumsum(np.cumsum(r.standard_normal(s), axis=1), axis=2) * 0.05 for s in sizes]
    vs0 = _flows(28, 1.0, sizes)
    if dt == torch.float32:
        us, vs0 = [list(map(roundtrip32, a)) for a in (us, vs0)]
    stack = B.Stack(sizes)
    v = dev(pack(vs0), dt)
    vr = torch.empty_like(v)
    B.flow_update_scaled(stack, dev(pack(us), dt), v, alpha=0.3, n_sweeps=25, delta_r=1, scale=scale, v_rev=vr)
    exp = [optflow.flow_update_scaled(u, v0, 0.3, 25, 1, scale) for u, v0 in zip(us, vs0)]
    got = host(v)
    assert_close(got, pack(exp), TOL64 if dt == torch.float64 else 1e-4)
    gshapes = [e.shape for e in exp]
    exp_r = pack([optflow.reverse_flow(x) for x in unpack(got, gshapes)])
    assert_close(host(vr), exp_r, TOL64 if dt == torch.float64 else TOL32)


@pytest.mark.parametrize("which", ["f64", "f32"])
@pytest.mark.parametrize("scale", [4, 8])
def test_flow_update_scaled_wide_blocks(B, which, scale):
    """Reduction factors 4 and 8 (block rows read as one vector of the block width) on frames
    whose sides leave partial border blocks, and reduced frames narrower than four columns
    (the upscaling's element-load path) next to wider ones, against the oracle."""
    import torch
    dt = torch.float64 if which == "f64" else torch.float32
    sizes = [(3, 37, 75), (2, 40, 130), (2, 64, 64), (2, 28, 20)]
    r = np.random.default_rng(29)
    us = [np.cumsum(np.cumsum(r.standard_normal(s), axis=1), axis=2) * 0.05 for s in sizes]
    vs0 = _flows(30, 1.0, sizes)
    if dt == torch.float32:
        us, vs0 = [list(map(roundtrip32, a)) for a in (us, vs0)]
    stack = B.Stack(sizes)
    v = dev(pack(vs0), dt)
    B.flow_update_scaled(stack, dev(pack(us), dt), v, alpha=0.3, n_sweeps=25, delta_r=1, scale=scale)
    exp = [optflow.flow_update_scaled(u, v0, 0.3, 25, 1, scale) for u, v0 in zip(us, vs0)]
    assert_close(host(v), pack(exp), TOL64 if dt == torch.float64 else 1e-4)


def test_flow_update_scaled_edges(B):
    """scale 1 is the plain update bit for bit; a scale that leaves a reduced side <= delta_r
    is rejected before any launch; frames that reduce to 2 x 2 still work."""
    import torch
    from paper_2501_12497_amd._lib import MMOFError
    sizes = [(3, 9, 8), (2, 4, 7)]
    r = np.random.default_rng(29)
    us = [r.standard_normal(sz) for sz in sizes]
    vs0 = [r.uniform(-1, 1, (sz[0] - 1, 2, sz[1], sz[2])) for sz in sizes]
    stack = B.Stack(sizes)
    u = dev(pack(us), torch.float64)
    a, b = dev(pack(vs0), torch.float64), dev(pack(vs0), torch.float64)
    B.flow_update(stack, u, a, alpha=0.2, n_sweeps=9, delta_r=1)
    B.flow_update_scaled(stack, u, b, alpha=0.2, n_sweeps=9, delta_r=1, scale=1)
    assert torch.equal(a, b)
    c = dev(pack(vs0), torch.float64)
    B.flow_update_scaled(stack, u, c, alpha=0.2, n_sweeps=9, delta_r=1, scale=3)   # (4,4,3,3) -> (3,3), (2,3)
    exp = pack([optflow.flow_update_scaled(x, v0, 0.2, 9, 1, 3) for x, v0 in zip(us, vs0)])
    assert_close(host(c), exp, TOL64, elementwise=True)
    # automatic factor: the smallest power of two that brings the sides below 50
    big = [(2, 100, 120), (2, 30, 44)]
    ub = dev(pack([r.standard_normal(sz) for sz in big]), torch.float64)
    vb = pack([r.uniform(-1, 1, (sz[0] - 1, 2, sz[1], sz[2])) for sz in big])
    got = {}
    for sc in (-1, 2, 4):
        got[sc] = dev(vb, torch.float64)
        B.flow_update_scaled(B.Stack(big), ub, got[sc], alpha=0.2, n_sweeps=5, delta_r=1, scale=sc)
    assert torch.equal(got[-1], got[4]) and not torch.equal(got[-1], got[2])
    before = c.clone()
    for sc, dr in ((4, 1), (2, 2), (65, 1), (-2, 1)):   # (2,4,7)/4 -> 1 x 2;  /2 -> 2 x 4 with dr 2
        with pytest.raises(MMOFError) as e:
            B.flow_update_scaled(stack, u, c, alpha=0.2, n_sweeps=9, delta_r=dr, scale=sc)
        assert e.value.code == -1
    assert torch.equal(c, before)


@pytest.mark.parametrize("n_sweeps", [0, 1, 8, 9, 40])
def test_flow_update_sweep_counts_small_frames(B, n_sweeps):
    """Sweep counts around the per-launch block of sweeps, on frames smaller than one tile
    and its halo (2x2, 5x3, 3x70 frames in one ragged stack), FP64 against the oracle."""
    import torch
    sizes = [(2, 2, 2), (3, 5, 3), (2, 3, 70)]
    r = np.random.default_rng(26)
    us = [r.standard_normal(sz) for sz in sizes]
    vs0 = [r.uniform(-1, 1, (sz[0] - 1, 2, sz[1], sz[2])) for sz in sizes]
    v = dev(pack(vs0), torch.float64)
    B.flow_update(B.Stack(sizes), dev(pack(us), torch.float64), v, alpha=0.2, n_sweeps=n_sweeps, delta_r=1)
    exp = pack([optflow.flow_update(u, v0, 0.2, n_sweeps, 1) for u, v0 in zip(us, vs0)])
    assert_close(host(v), exp, TOL64, elementwise=True)


@pytest.mark.parametrize("which", ["f64", "f32"])
def test_reverse_flow_with_outliers(B, which):
    """Mostly small displacements plus a few of 35 px, and in a 1200-px-wide frame some of
    1100 px (more than 64 block columns in the window): the block reach table must not drop
    any source.  FP64 sums in the oracle's order (raster order of the sources): equal."""
    import torch
    dt = torch.float64 if which == "f64" else torch.float32
    sizes = [(3, 40, 70), (2, 12, 1200)]
    r = np.random.default_rng(31)
    vs = []
    for (nt, ny, nx), big in zip(sizes, (35.0, 1100.0)):
        v = r.uniform(-2, 2, size=(nt - 1, 2, ny, nx))
        for _ in range(6):
            t, c, y, x = r.integers(nt - 1), r.integers(2), r.integers(ny), r.integers(nx)
            v[t, c, y, x] = big * (1 if r.random() < 0.5 else -1) + r.uniform(-0.4, 0.4)
        vs.append(roundtrip32(v) if dt == torch.float32 else v)
    got = host(B.reverse_flow(B.Stack(sizes), dev(pack(vs), dt)))
    exp = pack([optflow.reverse_flow(v) for v in vs])
    if dt == torch.float64:
        assert np.array_equal(got, exp)
    else:
        np.testing.assert_allclose(got, exp, rtol=1e-6, atol=1e-6)


def test_reverse_flow_exact_on_half_integers(B):
    import torch
    sizes = [(2, 9, 11)]
    r = np.random.default_rng(25)
    v = (np.round(r.uniform(-3, 3, size=(1, 2, 9, 11)) * 2) / 2)    # many exact .5 ties
    exp = optflow.reverse_flow(v).ravel()
    got = host(B.reverse_flow(B.Stack(sizes), dev(v, torch.float64)))
    assert np.array_equal(got, exp)
    # FP32: identical rounding decisions; the averages differ only by FP32 rounding
    got = host(B.reverse_flow(B.Stack(sizes), dev(v, torch.float32)))
    np.testing.assert_allclose(got, exp, rtol=1e-6, atol=0)


@pytest.mark.parametrize("which", ["f64", "f32"])
def test_mm_weights(B, which):
    import torch
    from oracle import mmgks
    dt, tol = (torch.float64, TOL64) if which == "f64" else (torch.float32, TOL32)
    nu = np.random.default_rng(26).standard_normal(10007) * np.logspace(-5, 1, 10007)
    if dt == torch.float32:
        nu = roundtrip32(nu)
    w = host(B.mm_weights(dev(nu, dt), 1e-3))
    assert_close(w, mmgks.mm_weights_sq(nu, 1e-3), tol)
