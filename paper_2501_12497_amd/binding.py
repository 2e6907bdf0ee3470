"""Thin Python binding of the C ABI: argument marshalling only.

Every function takes torch tensors that already live on the GPU (PyTorch provides
device memory and streams), checks shapes and dtypes, and calls the entry point of
the same name in libmmof.so on the current torch stream.  All arithmetic happens in
the HIP kernels.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import check

_DT = {torch.float32: _lib.MMOF_F32, torch.float64: _lib.MMOF_F64}
# largest Krylov basis of a solve and leading dimension of the projected matrices
KRYLOV_MAX = 256

# Library objects still alive at interpreter exit are released while the HIP runtime is
# still up (plans before contexts); later finalizers then do nothing.
_LIVE_PLANS = weakref.WeakSet()
_LIVE_CTX = weakref.WeakSet()
_SHUTDOWN = [False]


@atexit.register
def _release_all():
    for p in list(_LIVE_PLANS):
        p.close()
    for c in list(_LIVE_CTX):
        c.close()
    _SHUTDOWN[0] = True


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dt(*ts: torch.Tensor) -> int:
    dts = {t.dtype for t in ts if t is not None}
    if len(dts) != 1 or next(iter(dts)) not in _DT:
        raise TypeError(f"tensors must share one dtype, float32 or float64 (got {dts})")
    return _DT[next(iter(dts))]


def _dtcode(dtype) -> int:
    if isinstance(dtype, str):
        dtype = {"f32": torch.float32, "f64": torch.float64}[dtype]
    if dtype not in _DT:
        raise TypeError(f"dtype must be float32 or float64 (got {dtype})")
    return _DT[dtype]


def _need(t: torch.Tensor, numel: int, name: str):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


# ----------------------------------------------------------------------------- context


class Context:
    """A library context bound to the current torch stream of one device."""

    def __init__(self, device: Optional[int] = None):
        self.lib = _lib.load()
        self.device = torch.cuda.current_device() if device is None else device
        with torch.cuda.device(self.device):
            h = C.c_void_p()
            check(self.lib.mmof_create(C.byref(h), C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        self.h = h
        _LIVE_CTX.add(self)

    def bind(self):
        """Point the context at torch's current stream (call before every launch)."""
        check(self.lib.mmof_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))
        return self.h

    def close(self):
        if self.h and not _SHUTDOWN[0]:
            self.lib.mmof_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # timing of a named kernel with HIP events on the bound stream
    def profile_kernel(self, name: Optional[str]):
        check(self.lib.mmof_profile_kernel(self.h, None if not name else name.encode()))

    def kernel_timing(self) -> Tuple[int, float, float, float]:
        """(launches, total ms, algorithmic bytes, algorithmic flops) of the profiled kernel."""
        n = C.c_int64()
        ms, by, fl = C.c_double(), C.c_double(), C.c_double()
        check(self.lib.mmof_kernel_timing(self.h, C.byref(n), C.byref(ms), C.byref(by), C.byref(fl)))
        return int(n.value), float(ms.value), float(by.value), float(fl.value)


_CTX = {}


def context(device: Optional[int] = None) -> Context:
    d = torch.cuda.current_device() if device is None else device
    if d not in _CTX:
        _CTX[d] = Context(d)
    return _CTX[d]


# ----------------------------------------------------------------------------- stacks


@dataclass
class Stack:
    """Sizes of a packed batch of sequences: [(n_t, ny, nx), ...]."""
    sizes: List[Tuple[int, int, int]]
    _arrs: tuple = field(default=None, repr=False)
    _s: object = field(default=None, repr=False)

    def __post_init__(self):
        self.sizes = [tuple(int(v) for v in s) for s in self.sizes]
        nt = (C.c_int32 * len(self.sizes))(*[s[0] for s in self.sizes])
        ny = (C.c_int32 * len(self.sizes))(*[s[1] for s in self.sizes])
        nx = (C.c_int32 * len(self.sizes))(*[s[2] for s in self.sizes])
        self._arrs = (nt, ny, nx)
        self._s = _lib.mmof_stack(len(self.sizes), nt, ny, nx)

    @classmethod
    def single(cls, n_t: int, ny: int, nx: int) -> "Stack":
        return cls([(n_t, ny, nx)])

    @property
    def ref(self):
        return C.byref(self._s)

    @property
    def n(self) -> int:
        return sum(t * y * x for t, y, x in self.sizes)

    @property
    def n_pair_px(self) -> int:
        return sum((t - 1) * y * x for t, y, x in self.sizes)

    @property
    def n_gx(self) -> int:
        return sum(t * y * (x - 1) for t, y, x in self.sizes)

    @property
    def n_gy(self) -> int:
        return sum(t * (y - 1) * x for t, y, x in self.sizes)


# ----------------------------------------------------------------------------- plans


class Plan:
    def __init__(self, h, ctx: Context, stack: Stack, kind: str):
        self.h = h
        self.ctx = ctx
        self.stack = stack
        self.kind = kind
        n = C.c_int64()
        m = C.c_int64()
        check(ctx.lib.mmof_plan_sizes(h, C.byref(n), C.byref(m)))
        self.n, self.m = int(n.value), int(m.value)
        _LIVE_PLANS.add(self)

    def autotune(self, dtype=torch.float32) -> str:
        """Times the tile-shape candidates of this plan's stencil kernels; returns the report."""
        buf = C.create_string_buffer(1024)
        self.ctx.bind()
        check(self.ctx.lib.mmof_autotune(self.h, _dtcode(dtype), buf, 1024))
        return buf.value.decode()

    def set_tile(self, kernel: str, choice: int, dtype=torch.float32):
        """Forces tile candidate `choice` of a tunable kernel for this plan."""
        check(self.ctx.lib.mmof_set_tile(self.h, kernel.encode(), _dtcode(dtype), int(choice)))

    def close(self):
        if self.h and not _SHUTDOWN[0]:
            self.ctx.lib.mmof_plan_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_radon(stack: Stack, n_angles: Sequence[int], n_bins: Sequence[int], angles_rad: np.ndarray,
               ctx: Optional[Context] = None) -> Plan:
    """Parallel-beam projector plan; angles_rad holds sum_s n_t[s]*n_angles[s] radians."""
    ctx = ctx or context()
    na = (C.c_int32 * len(n_angles))(*[int(v) for v in n_angles])
    nb = (C.c_int32 * len(n_bins))(*[int(v) for v in n_bins])
    ang = np.ascontiguousarray(np.asarray(angles_rad, dtype=np.float64).ravel())
    want = sum(s[0] * a for s, a in zip(stack.sizes, n_angles))
    if ang.size != want:
        raise ValueError(f"angles_rad has {ang.size} entries, expected {want}")
    h = C.c_void_p()
    ctx.bind()
    check(ctx.lib.mmof_plan_radon(ctx.h, stack.ref, na, nb, ang.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)))
    return Plan(h, ctx, stack, "radon")


def plan_fan(stack: Stack, n_angles: Sequence[int], n_bins: Sequence[int], angles_rad: np.ndarray, dso: float,
             dsd: float, du: float, ctx: Optional[Context] = None) -> Plan:
    """Flat-detector fan-beam projector plan (Joseph's method); sizes and angles as plan_radon."""
    ctx = ctx or context()
    na = (C.c_int32 * len(n_angles))(*[int(v) for v in n_angles])
    nb = (C.c_int32 * len(n_bins))(*[int(v) for v in n_bins])
    ang = np.ascontiguousarray(np.asarray(angles_rad, dtype=np.float64).ravel())
    want = sum(s[0] * a for s, a in zip(stack.sizes, n_angles))
    if ang.size != want:
        raise ValueError(f"angles_rad has {ang.size} entries, expected {want}")
    h = C.c_void_p()
    ctx.bind()
    check(ctx.lib.mmof_plan_fan(ctx.h, stack.ref, na, nb, ang.ctypes.data_as(C.POINTER(C.c_double)), float(dso),
                                float(dsd), float(du), C.byref(h)))
    return Plan(h, ctx, stack, "fan")


def plan_blur(stack: Stack, ksize: int = 9, sigma: float = 2.0, ctx: Optional[Context] = None) -> Plan:
    ctx = ctx or context()
    h = C.c_void_p()
    ctx.bind()
    check(ctx.lib.mmof_plan_blur(ctx.h, stack.ref, int(ksize), float(sigma), C.byref(h)))
    return Plan(h, ctx, stack, "blur")


# ----------------------------------------------------------------------------- operators


def apply_A(plan: Plan, u: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    _need(u, plan.n, "u")
    out = torch.empty(plan.m, dtype=u.dtype, device=u.device) if out is None else out
    _need(out, plan.m, "out")
    plan.ctx.bind()
    check(plan.ctx.lib.mmof_apply_A(plan.h, _dt(u, out), _ptr(u), _ptr(out)))
    return out


def apply_At(plan: Plan, b: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    _need(b, plan.m, "b")
    out = torch.empty(plan.n, dtype=b.dtype, device=b.device) if out is None else out
    _need(out, plan.n, "out")
    plan.ctx.bind()
    check(plan.ctx.lib.mmof_apply_At(plan.h, _dt(b, out), _ptr(b), _ptr(out)))
    return out


def apply_grad(stack: Stack, u: Optional[torch.Tensor] = None, gx: Optional[torch.Tensor] = None,
               gy: Optional[torch.Tensor] = None, wx=None, wy=None, transpose: bool = False,
               ctx: Optional[Context] = None):
    """transpose=False: returns (gx, gy) = w (.) Psi u.  transpose=True: returns Psi^T (w (.) g)."""
    ctx = ctx or context()
    ref = u if not transpose else gx
    if transpose:
        _need(gx, stack.n_gx, "gx")
        _need(gy, stack.n_gy, "gy")
        u = torch.empty(stack.n, dtype=gx.dtype, device=gx.device) if u is None else u
    else:
        _need(u, stack.n, "u")
        gx = torch.empty(stack.n_gx, dtype=u.dtype, device=u.device) if gx is None else gx
        gy = torch.empty(stack.n_gy, dtype=u.dtype, device=u.device) if gy is None else gy
    _need(u, stack.n, "u")
    _need(gx, stack.n_gx, "gx")
    _need(gy, stack.n_gy, "gy")
    if wx is not None:
        _need(wx, stack.n_gx, "wx")
    if wy is not None:
        _need(wy, stack.n_gy, "wy")
    ctx.bind()
    check(ctx.lib.mmof_apply_grad(ctx.h, stack.ref, _dt(ref, u, gx, gy, wx, wy), int(bool(transpose)), _ptr(wx),
                                  _ptr(wy), _ptr(u), _ptr(gx), _ptr(gy)))
    return u if transpose else (gx, gy)


def apply_flow_op(stack: Stack, mode: int, direction: int, interp: int, u: Optional[torch.Tensor],
                  v: torch.Tensor, inp: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                  ctx: Optional[Context] = None) -> torch.Tensor:
    """mode FWD: L(v) u;  ADJ: L(v)^T inp;  DV: (d(L(v)u)/dv)^T inp."""
    ctx = ctx or context()
    P = stack.n_pair_px
    _need(v, 2 * P, "v")
    if mode == _lib.MMOF_FLOW_FWD:
        _need(u, stack.n, "u")
        n_out = P
    elif mode == _lib.MMOF_FLOW_ADJ:
        _need(inp, P, "inp")
        n_out = stack.n
    elif mode == _lib.MMOF_FLOW_DV:
        _need(u, stack.n, "u")
        _need(inp, P, "inp")
        n_out = 2 * P
    else:
        raise ValueError("bad mode")
    out = torch.empty(n_out, dtype=v.dtype, device=v.device) if out is None else out
    _need(out, n_out, "out")
    ctx.bind()
    check(ctx.lib.mmof_apply_flow_op(ctx.h, stack.ref, _dt(u, v, inp, out), int(mode), int(direction), int(interp),
                                     _ptr(u), _ptr(v), _ptr(inp), _ptr(out)))
    return out


def mm_weights(nu: torch.Tensor, eps: float, out: Optional[torch.Tensor] = None,
               ctx: Optional[Context] = None) -> torch.Tensor:
    ctx = ctx or context()
    out = torch.empty_like(nu) if out is None else out
    _need(nu, nu.numel(), "nu")
    _need(out, nu.numel(), "out")
    ctx.bind()
    check(ctx.lib.mmof_mm_weights(ctx.h, _dt(nu, out), nu.numel(), _ptr(nu), float(eps), _ptr(out)))
    return out


def of_derivs(stack: Stack, u: torch.Tensor, delta_r: int = 1, out: Optional[torch.Tensor] = None,
              ctx: Optional[Context] = None) -> torch.Tensor:
    ctx = ctx or context()
    _need(u, stack.n, "u")
    out = torch.empty(3 * stack.n_pair_px, dtype=u.dtype, device=u.device) if out is None else out
    _need(out, 3 * stack.n_pair_px, "out")
    ctx.bind()
    check(ctx.lib.mmof_of_derivs(ctx.h, stack.ref, _dt(u, out), _ptr(u), _ptr(out), int(delta_r)))
    return out


def flow_update(stack: Stack, u: torch.Tensor, v: torch.Tensor, alpha: float, n_sweeps: int, delta_r: int = 1,
                v_rev: Optional[torch.Tensor] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Horn-Schunck sweeps, in place on v; fills v_rev with the reverse flow when given."""
    return flow_update_scaled(stack, u, v, alpha, n_sweeps, delta_r, 1, v_rev, ctx)


def flow_update_scaled(stack: Stack, u: torch.Tensor, v: torch.Tensor, alpha: float, n_sweeps: int,
                       delta_r: int = 1, scale: int = 1, v_rev: Optional[torch.Tensor] = None,
                       ctx: Optional[Context] = None) -> torch.Tensor:
    """flow_update computed on frames reduced by `scale` and upscaled (in place on v)."""
    ctx = ctx or context()
    _need(u, stack.n, "u")
    _need(v, 2 * stack.n_pair_px, "v")
    if v_rev is not None:
        _need(v_rev, 2 * stack.n_pair_px, "v_rev")
    ctx.bind()
    check(ctx.lib.mmof_flow_update_scaled(ctx.h, stack.ref, _dt(u, v, v_rev), _ptr(u), _ptr(v), _ptr(v_rev),
                                          float(alpha), int(n_sweeps), int(delta_r), int(scale)))
    return v


def flow_solve_gks(stack: Stack, u: torch.Tensor, v: torch.Tensor, delta_r: int = 1, ell: int = 10,
                   n_iter: int = 20, fixed_lambda: float = 0.0, scale: int = 1,
                   v_rev: Optional[torch.Tensor] = None, want_lambdas: bool = False,
                   pq: int = 2, eps: float = 1e-3, ctx: Optional[Context] = None):
    """Solve-OF (lambda by GCV) into v: pq = 2 GKS on the quadratic flow problem, pq = 1 the
    smoothed-l1 MM variant; returns v, or (v, lambdas [pairs, n_iter]) when asked."""
    ctx = ctx or context()
    _need(u, stack.n, "u")
    _need(v, 2 * stack.n_pair_px, "v")
    if v_rev is not None:
        _need(v_rev, 2 * stack.n_pair_px, "v_rev")
    n_pairs = sum(t - 1 for t, _, _ in stack.sizes)
    lam = np.zeros((max(n_pairs, 1), max(int(n_iter), 1))) if want_lambdas else None
    ctx.bind()
    lp = None if lam is None else lam.ctypes.data_as(C.c_void_p)
    if pq == 2:
        check(ctx.lib.mmof_flow_solve_gks(ctx.h, stack.ref, _dt(u, v, v_rev), _ptr(u), _ptr(v), _ptr(v_rev),
                                          int(delta_r), int(ell), int(n_iter), float(fixed_lambda), int(scale), lp))
    else:
        check(ctx.lib.mmof_flow_solve_of(ctx.h, stack.ref, _dt(u, v, v_rev), _ptr(u), _ptr(v), _ptr(v_rev),
                                         int(delta_r), int(ell), int(n_iter), float(fixed_lambda), int(scale),
                                         int(pq), float(eps), lp))
    return (v, lam[:n_pairs]) if want_lambdas else v


def reverse_flow(stack: Stack, v: torch.Tensor, out: Optional[torch.Tensor] = None,
                 ctx: Optional[Context] = None) -> torch.Tensor:
    ctx = ctx or context()
    _need(v, 2 * stack.n_pair_px, "v")
    out = torch.empty_like(v) if out is None else out
    _need(out, 2 * stack.n_pair_px, "out")
    ctx.bind()
    check(ctx.lib.mmof_reverse_flow(ctx.h, stack.ref, _dt(v, out), _ptr(v), _ptr(out)))
    return out


# ----------------------------------------------------------------------------- projected steps


def weighted_gram(X: torch.Tensor, nu: Optional[torch.Tensor] = None, eps: float = 1e-3,
                  ctx: Optional[Context] = None) -> torch.Tensor:
    """G = X^T diag(1/sqrt(nu^2+eps^2)) X for X of shape [K, n] (K columns, each contiguous)."""
    ctx = ctx or context()
    K, n = X.shape
    _need(X, K * n, "X")
    if nu is not None:
        _need(nu, n, "nu")
    G = torch.empty((K, K), dtype=torch.float64, device=X.device)
    ctx.bind()
    check(ctx.lib.mmof_weighted_gram(ctx.h, _dt(X, nu), n, K, _ptr(X), n, _ptr(nu), float(eps), _ptr(G), K))
    return G


def apply_tdiff(stack: Stack, x: torch.Tensor, transpose: bool = False, out: Optional[torch.Tensor] = None,
                ctx: Optional[Context] = None) -> torch.Tensor:
    """L_t x (x: n pixels -> pair pixels) or L_t^T x (pair pixels -> n pixels)."""
    ctx = ctx or context()
    n_in, n_out = (stack.n_pair_px, stack.n) if transpose else (stack.n, stack.n_pair_px)
    _need(x, n_in, "x")
    out = torch.empty(n_out, dtype=x.dtype, device=x.device) if out is None else out
    _need(out, n_out, "out")
    ctx.bind()
    check(ctx.lib.mmof_apply_tdiff(ctx.h, stack.ref, _dt(x, out), 1 if transpose else 0, _ptr(x), _ptr(out)))
    return out


def reg_weights(stack: Stack, reg, nu: torch.Tensor, eps: float = 1e-3, ctx: Optional[Context] = None) -> torch.Tensor:
    """FP64 MM weights of the rows of Theta u (nu) for a regulariser ("psi", "aniso", "iso", "gs")."""
    ctx = ctx or context()
    code = _lib.REGS[reg] if isinstance(reg, str) else int(reg)
    _need(nu, nu.numel(), "nu")
    w2 = torch.empty(nu.numel(), dtype=torch.float64, device=nu.device)
    ctx.bind()
    check(ctx.lib.mmof_reg_weights(ctx.h, stack.ref, _dt(nu), code, nu.numel(), _ptr(nu), float(eps), _ptr(w2)))
    return w2


def block_dot(X: torch.Tensor, y: torch.Tensor, ctx: Optional[Context] = None) -> torch.Tensor:
    """out[j] = X_j^T y for X of shape [K, n] (float32 or float64) and an FP64 y of n entries."""
    ctx = ctx or context()
    K, n = X.shape
    _need(X, K * n, "X")
    _need(y, n, "y")
    if y.dtype != torch.float64:
        raise TypeError("y must be float64")
    out = torch.empty(K, dtype=torch.float64, device=X.device)
    ctx.bind()
    check(ctx.lib.mmof_block_dot(ctx.h, _dt(X), n, K, _ptr(X), n, _ptr(y), _ptr(out)))
    return out


def block_combine(X: torch.Tensor, z: torch.Tensor, alpha: float = 1.0, y: Optional[torch.Tensor] = None,
                  beta: float = 0.0, ctx: Optional[Context] = None) -> torch.Tensor:
    """alpha X^T z + beta y (X of shape [K, n], z FP64 of K entries, y FP64 of n entries or None)."""
    ctx = ctx or context()
    K, n = X.shape
    _need(X, K * n, "X")
    _need(z, K, "z")
    if z.dtype != torch.float64 or (y is not None and y.dtype != torch.float64):
        raise TypeError("z and y must be float64")
    if y is not None:
        _need(y, n, "y")
    out = torch.empty(n, dtype=torch.float64, device=X.device)
    ctx.bind()
    check(ctx.lib.mmof_block_combine(ctx.h, _dt(X), n, K, _ptr(X), n, _ptr(z), float(alpha), _ptr(y), float(beta),
                                     _ptr(out)))
    return out


def cgs2(Q: torch.Tensor, x: torch.Tensor, ctx: Optional[Context] = None) -> float:
    """x <- x - Q^T (Q x), twice, in place (Q FP64 of shape [K, n]); returns ||x||^2."""
    return reorth(Q, x, "twice", ctx)


def reorth(Q: torch.Tensor, x: torch.Tensor, mode="auto", ctx: Optional[Context] = None) -> float:
    """x <- x - Q^T (Q x) in place (Q FP64 of shape [K, n]), a second time always ("twice") or
    only when the first pass kept less than 1/sqrt(2) of ||x|| ("auto"); returns ||x||^2."""
    if isinstance(mode, str):
        mode = _lib.REORTHS[mode]
    ctx = ctx or context()
    K, n = Q.shape
    _need(Q, K * n, "Q")
    _need(x, n, "x")
    if Q.dtype != torch.float64 or x.dtype != torch.float64:
        raise TypeError("Q and x must be float64")
    sq = torch.empty(1, dtype=torch.float64, device=x.device)
    ctx.bind()
    check(ctx.lib.mmof_reorth(ctx.h, n, K, _ptr(Q), n, _ptr(x), _ptr(sq), int(mode)))
    return float(sq.item())


def basis_extend(Vs: torch.Tensor, r: torch.Tensor, T: torch.Tensor, ctx: Optional[Context] = None) -> float:
    """One step of the implicit basis V = Vs T: Vs FP64 [K, n] (row k = stored column k), T FP64
    [256, 256] with T[j, i] = T(i, j) (row j = the coefficients of v_j in Vs).  Writes row K of T
    (e_K - T g / rho, g = V^T r) and returns rho^2 = ||r||^2 - ||g||^2; r is replaced by r - V g
    when it keeps less than 1/sqrt(2) of its norm outside the basis."""
    ctx = ctx or context()
    K, n = Vs.shape
    _need(Vs, K * n, "Vs")
    _need(r, n, "r")
    _need(T, KRYLOV_MAX * KRYLOV_MAX, "T")
    if Vs.dtype != torch.float64 or r.dtype != torch.float64 or T.dtype != torch.float64:
        raise TypeError("Vs, r and T must be float64")
    sq = torch.empty(1, dtype=torch.float64, device=r.device)
    ctx.bind()
    check(ctx.lib.mmof_basis_extend(ctx.h, n, K, _ptr(Vs), n, _ptr(r), _ptr(T), _ptr(sq)))
    return float(sq.item())


def projected_solve(GA: torch.Tensor, GT: torch.Tensor, d: torch.Tensor, bnorm2: float, target: float,
                    prev_lambda: float = 0.0, fixed_lambda: float = 0.0, ctx: Optional[Context] = None):
    """(G_H + lambda G_T) z = d with lambda from the discrepancy principle; returns (z, lambda, D^2, status)."""
    ctx = ctx or context()
    K = d.numel()
    if not 1 <= K <= KRYLOV_MAX:
        raise ValueError(f"K must be in [1, {KRYLOV_MAX}] (got {K})")
    pad = lambda M: torch.nn.functional.pad(M.to(torch.float64), (0, KRYLOV_MAX - K, 0, KRYLOV_MAX - K)).contiguous()
    A64, T64 = pad(GA), pad(GT)
    sc = torch.tensor([bnorm2, target, prev_lambda], dtype=torch.float64, device=d.device)
    z = torch.empty(K, dtype=torch.float64, device=d.device)
    res = torch.empty(4, dtype=torch.float64, device=d.device)
    dd = d.to(torch.float64).contiguous()
    ctx.bind()
    check(ctx.lib.mmof_projected_solve(ctx.h, K, _ptr(A64), _ptr(T64), _ptr(dd), _ptr(sc), float(fixed_lambda),
                                       _ptr(z), _ptr(res)))
    r = res.cpu().tolist()
    return z, r[0], r[1], int(r[2])


# ----------------------------------------------------------------------------- solve


def solve_params(**kw) -> _lib.mmof_solve_params:
    p = _lib.mmof_solve_params()
    _lib.load().mmof_solve_defaults(C.byref(p))
    for k, val in kw.items():
        if k == "op_dtype" and isinstance(val, str):
            val = {"f32": _lib.MMOF_F32, "f64": _lib.MMOF_F64}[val]
        if k == "reg" and isinstance(val, str):
            val = _lib.REGS[val]
        if k == "reorth" and isinstance(val, str):
            val = _lib.REORTHS[val]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, val)
    return p


@dataclass
class SolveResult:
    u: torch.Tensor
    v: Optional[torch.Tensor]
    v_rev: Optional[torch.Tensor]
    status: int
    iters: int
    n_cols: int
    lambdas: List[float]
    resid: List[float]
    rre: List[float]
    dp_status: List[int]
    counts: dict


def solve_joint(plan: Plan, b: torch.Tensor, noise_norm: float, u0: Optional[torch.Tensor] = None,
                u_true: Optional[torch.Tensor] = None, **params) -> SolveResult:
    """MMGKS-OF solve; b, u0, u_true are FP64 GPU tensors; params as in mmof_solve_params."""
    p = solve_params(**params)
    # the library reads b and u_inout as FP64 device arrays of m and n values: every dtype
    # and device is checked before a pointer is handed over
    if b.dtype != torch.float64:
        raise TypeError(f"b must be float64 (got {b.dtype})")
    if u0 is not None:
        if u0.dtype != torch.float64:
            raise TypeError(f"u0 must be float64 (got {u0.dtype})")
        if u0.device != b.device:
            raise ValueError(f"u0 is on {u0.device}, b on {b.device}")
    if u_true is not None and u_true.dtype != torch.float64:
        raise TypeError(f"u_true must be float64 (got {u_true.dtype})")
    _need(b, plan.m, "b")
    u = torch.zeros(plan.n, dtype=torch.float64, device=b.device) if u0 is None else u0.clone()
    _need(u, plan.n, "u0")
    if u_true is not None:
        _need(u_true, plan.n, "u_true")
        if u_true.device != b.device:
            raise ValueError(f"u_true is on {u_true.device}, b on {b.device}")
        p.u_true = u_true.data_ptr()
    opdt = torch.float32 if p.op_dtype == _lib.MMOF_F32 else torch.float64
    P = plan.stack.n_pair_px
    v = torch.zeros(2 * P, dtype=opdt, device=b.device) if (p.use_flow and P) else None
    vr = torch.zeros(2 * P, dtype=opdt, device=b.device) if (p.use_flow and P) else None
    cap = max(1, int(p.k_max))
    lam = (C.c_double * cap)()
    res = (C.c_double * cap)()
    rre = (C.c_double * cap)()
    dps = (C.c_int32 * cap)()
    rep = _lib.mmof_report()
    rep.capacity = cap
    rep.lambda_, rep.resid, rep.rre, rep.dp_status = lam, res, rre, dps
    plan.ctx.bind()
    rc = check(plan.ctx.lib.mmof_solve_joint(plan.h, _ptr(b), float(noise_norm), C.byref(p), _ptr(u), _ptr(v),
                                            _ptr(vr), C.byref(rep)))
    k = rep.iters
    return SolveResult(u=u, v=v, v_rev=vr, status=rc, iters=k, n_cols=rep.n_cols, lambdas=list(lam[:k]),
                       resid=list(res[:k]), rre=list(rre[:k]) if u_true is not None else [],
                       dp_status=list(dps[:k]),
                       counts=dict(A=rep.n_A, At=rep.n_At, theta=rep.n_theta, thetaT=rep.n_thetaT,
                                   flow_updates=rep.n_flow_updates, L=rep.n_L,
                                   factorizations=rep.n_factorizations))
