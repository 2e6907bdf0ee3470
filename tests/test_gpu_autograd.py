"""Autograd over H, Psi and L(v) at 256x256x16 (FP32 forward, FP64 checks).

Loss f(u, v) = <w1, H u> + <w2x, gx> + <w2y, gy> + <w3, L(v) u> with random weights.
Its gradient comes from the adjoint kernels through torch.autograd; it is compared with
  * the oracle's adjoints applied to the same weights (FP64 oracle, FP32 and FP64 GPU),
  * central finite differences of the GPU's own FP64 loss, h = 1e-4, along random
    directions (the flow is kept at least 1e-3 away from the bilinear kinks, so the
    loss is smooth within +-h).
"""
import numpy as np
from gpu_helpers import assert_close
import pytest

from oracle import forward, regops
from synth import cfg_autograd256

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2501_12497_amd import binding as B
    wl = cfg_autograd256()
    s = wl.seqs[0]
    v = wl.params["flow"]
    r = np.random.default_rng(wl.params["loss_seed"])
    n_t, n = s.n_t, s.ny
    w1 = r.standard_normal((n_t, s.angles.shape[1], s.n_bins))
    w2x = r.standard_normal((n_t, n, n - 1))
    w2y = r.standard_normal((n_t, n - 1, n))
    w3 = r.standard_normal((n_t - 1, n, n))
    stack = B.Stack.single(n_t, n, n)
    plan = B.plan_radon(stack, [s.angles.shape[1]], [s.n_bins], s.angles.ravel())
    return dict(B=B, s=s, v=v, w=(w1, w2x, w2y, w3), stack=stack, plan=plan)


def _loss(AG, u, v, S, ws):
    import torch
    w1, w2x, w2y, w3 = ws
    b = AG.forward_op(u, S["plan"])
    gx, gy = AG.gradient_op(u, S["stack"])
    r = AG.flow_op(u, v, S["stack"], 1)
    return (w1 * b).sum() + (w2x * gx).sum() + (w2y * gy).sum() + (w3 * r).sum()


def _oracle_grads(S, u, v, ws):
    s = S["s"]
    w1, w2x, w2y, w3 = ws
    gu = forward.radon_adj(w1, s.angles, s.ny, s.nx) + regops.grad_adj(w2x, w2y) + \
        regops.flow_adj(w3, v, s.n_t, 1)
    gv = regops.flow_dv(u, v, w3, 1)
    return gu, gv


@pytest.mark.parametrize("which", ["f32", "f64"])
def test_autograd_matches_oracle_adjoints(setup, which):
    import torch
    from paper_2501_12497_amd import autograd as AG
    S = setup
    dt = torch.float32 if which == "f32" else torch.float64
    u_np, v_np = S["s"].u_true, S["v"]
    if dt == torch.float32:
        u_np = u_np.astype(np.float32).astype(np.float64)
        v_np = v_np.astype(np.float32).astype(np.float64)
        ws = [w.astype(np.float32).astype(np.float64) for w in S["w"]]
    else:
        ws = S["w"]
    u = torch.tensor(u_np.ravel(), dtype=dt, device="cuda", requires_grad=True)
    v = torch.tensor(v_np.ravel(), dtype=dt, device="cuda", requires_grad=True)
    wt = [torch.tensor(w.ravel(), dtype=dt, device="cuda") for w in ws]
    f = _loss(AG, u, v, S, wt)
    f.backward()
    gu_or, gv_or = _oracle_grads(S, u_np, v_np, ws)
    tol = 1e-5 if dt == torch.float32 else 1e-12
    gu = u.grad.double().cpu().numpy()
    gv = v.grad.double().cpu().numpy()
    # forward-error scales: the adjoints with absolute weights applied to |weights|
    s = S["s"]
    w1, w2x, w2y, w3 = ws
    sg = np.zeros(u_np.shape)
    sg[:, :, 1:] += np.abs(w2x)
    sg[:, :, :-1] += np.abs(w2x)
    sg[:, 1:, :] += np.abs(w2y)
    sg[:, :-1, :] += np.abs(w2y)
    sf = np.zeros(u_np.shape)
    for t in range(s.n_t - 1):
        sf[t + 1] += (abs(regops.motion_matrix(v_np[t])).T @ np.abs(w3[t]).ravel()).reshape(s.ny, s.nx)
        sf[t] += np.abs(w3[t])
    scale_u = forward.radon_adj(np.abs(w1), s.angles, s.ny, s.nx) + sg + sf
    assert_close(gu, gu_or.ravel(), tol, scale_u)
    scale_v = 2 * np.abs(w3)[:, None] * np.abs(u_np).max() * np.ones((1, 2, 1, 1))
    assert_close(gv, gv_or.ravel(), tol, scale_v)
    # the value of the loss itself
    f_or = (w1 * forward.radon_fwd(u_np, s.angles, s.n_bins)).sum() + \
        sum((a * b).sum() for a, b in zip((w2x, w2y), regops.grad_fwd(u_np))) + \
        (w3 * regops.flow_fwd(u_np, v_np, 1)).sum()
    assert abs(float(f.detach()) - f_or) <= (1e-4 if dt == torch.float32 else 1e-11) * abs(f_or)


def test_autograd_central_differences_fp64(setup):
    import torch
    from paper_2501_12497_amd import autograd as AG
    S = setup
    u = torch.tensor(S["s"].u_true.ravel(), dtype=torch.float64, device="cuda", requires_grad=True)
    v = torch.tensor(S["v"].ravel(), dtype=torch.float64, device="cuda", requires_grad=True)
    wt = [torch.tensor(w.ravel(), dtype=torch.float64, device="cuda") for w in S["w"]]
    f = _loss(AG, u, v, S, wt)
    f.backward()
    r = np.random.default_rng(7)
    h = 1e-4
    for _ in range(3):
        du = torch.tensor(r.standard_normal(u.numel()), dtype=torch.float64, device="cuda")
        dv = torch.tensor(r.uniform(-1, 1, v.numel()), dtype=torch.float64, device="cuda")
        with torch.no_grad():
            fp = _loss(AG, u + h * du, v + h * dv, S, wt)
            fm = _loss(AG, u - h * du, v - h * dv, S, wt)
        fd = float((fp - fm) / (2 * h))
        an = float((u.grad * du).sum() + (v.grad * dv).sum())
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_gradcheck_small():
    """torch.autograd.gradcheck on a 2x9x11 stack (FP64, flow away from the kinks)."""
    import torch
    from paper_2501_12497_amd import _lib, autograd as AG, binding as B
    from synth import nudge_off_kinks
    r = np.random.default_rng(3)
    st = B.Stack.single(3, 9, 11)
    u = torch.tensor(r.standard_normal(st.n), dtype=torch.float64, device="cuda", requires_grad=True)
    v = torch.tensor(nudge_off_kinks(r.uniform(-2, 2, 2 * st.n_pair_px), 1e-2), dtype=torch.float64,
                     device="cuda", requires_grad=True)
    for direction in (1, -1):
        assert torch.autograd.gradcheck(lambda a, b: AG.flow_op(a, b, st, direction), (u, v), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(lambda a: AG.gradient_op(a, st), (u,), eps=1e-6, atol=1e-7)
