"""Benchmark of the MMGKS-OF hot path on one MI355X.

Workload: 128x128 pixels x 16 frames, three ellipses translating with integer
velocities in [-2, 2] px/frame, 30 parallel-beam angles per frame rotated 6 deg per
frame, 181 detector bins, 2% Gaussian noise (synthetic, seeded).  One step is one
complete joint solve (MMGKS-OF, Alg. 1): Golub-Kahan start (ell = 10), 30 outer
MM iterations, Horn-Schunck flow update (200 sweeps) every 10 iterations, with FP32
operator applications and the FP64 generalized-Krylov projection, Gram matrices,
projected solve and discrepancy principle.  Inputs are resident on the GPU before
the timed region starts.

Printed JSON fields beyond the driver's contract:
  roofline         the dominant kernel's algorithmic bytes / its mean launch time
                   (HIP events on the library's stream over the timed region)
  time_to_solution FP32-operator vs FP64-operator solve to the same RRE target
  cpu_baseline     the FP64 oracle on the host cores, on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Published MI355X compute peaks (TFLOP/s) of the unit each profiled kernel computes on.
COMPUTE = {
    "wgram": ("mfma", 78.6),        # FP64 matrix cores (FP32 operands widened to FP64)
    "radon_fwd": ("alu", 157.3),    # FP32 vector ALU
    "radon_adj": ("alu", 157.3),
    "blur": ("alu", 157.3),
    "flow_fwd": ("alu", 157.3),
    "flow_adj": ("alu", 157.3),
    "grad_fwd": ("alu", 157.3),
    "grad_adj": ("alu", 157.3),
    "hs_multi": ("alu", 157.3),
    "of_derivs": ("alu", 157.3),
    "box_down": ("alu", 157.3),
    "fan_fwd": ("alu", 157.3),
    "fan_adj": ("alu", 157.3),
    "flow_up": ("alu", 157.3),
    "mdot": ("alu", 78.6),          # FP64 vector ALU
}
# The committed HBM-traffic summary of a kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE runs) and
# the source file it was measured on: traffic is reported only while that source is unchanged.
TRAFFIC = {
    "wgram": ("profiles/wgram_ellipse128_traffic.txt", "paper_2501_12497_amd/csrc/k_krylov.hip"),
}


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, or None."""
    import hashlib
    if kernel not in TRAFFIC:
        return None
    summ, src = (os.path.join(ROOT, x) for x in TRAFFIC[kernel])
    if not (os.path.exists(summ) and os.path.exists(src)):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    fields = {}
    for line in open(summ):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source sha256") != digest:
        return None
    try:
        return float(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


# FP32+FP64-refined solves: the last outer iterations run with FP64 operators
REFINE_ITERS = 10


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload():
    from synth import cfg_ellipse128
    return cfg_ellipse128()


def gpu_data(wl, B, torch):
    s = wl.seqs[0]
    stack = B.Stack.single(s.n_t, s.ny, s.nx)
    plan = B.plan_radon(stack, [s.angles.shape[1]], [s.n_bins], s.angles.ravel())
    u_true = torch.as_tensor(s.u_true.ravel(), dtype=torch.float64, device="cuda")
    clean = B.apply_A(plan, u_true)          # data synthesis on the GPU (FP64)
    g = torch.as_tensor(s.noise_g.ravel(), dtype=torch.float64, device="cuda")
    e = wl.noise_level * torch.linalg.vector_norm(clean) * g / torch.linalg.vector_norm(g)
    b = (clean + e).contiguous()
    delta = float(torch.linalg.vector_norm(e))
    return stack, plan, u_true, b, delta


def operators_large(B, torch, reps=5, before_ops=None):
    """Per-kernel rates of the operators on the 1024x1024x64 workload (FP32; 90 angles per
    frame shifted by the golden angle, 1449 bins; a smooth flow of up to 3 px): HIP-event
    mean over `reps` launches, algorithmic bytes and flops as the library counts them."""
    from paper_2501_12497_amd import _lib
    from synth import cfg_large1024, smooth_flow_coarse
    wl = cfg_large1024()
    s = wl.seqs[0]
    stack = B.Stack.single(s.n_t, s.ny, s.nx)
    plan = B.plan_radon(stack, [s.angles.shape[1]], [s.n_bins], s.angles.ravel())
    ctx = plan.ctx
    u = torch.as_tensor(s.u_true.ravel(), dtype=torch.float32, device="cuda")
    v = torch.as_tensor(smooth_flow_coarse(s.n_t - 1, s.nx, seed=11, coarse=16, vmax=3.0).ravel(),
                        dtype=torch.float32, device="cuda")
    b = B.apply_A(plan, u)
    gx, gy = B.apply_grad(stack, u)
    r = B.apply_flow_op(stack, _lib.MMOF_FLOW_FWD, 1, 0, u, v)
    w = torch.zeros_like(v)
    tuned = plan.autotune(torch.float32)
    log(f"large autotune: {tuned}")
    ops = {
        "radon_fwd": lambda: B.apply_A(plan, u, out=b),
        "radon_adj": lambda: B.apply_At(plan, b),
        "grad_fwd": lambda: B.apply_grad(stack, u),
        "grad_adj": lambda: B.apply_grad(stack, gx=gx, gy=gy, transpose=True),
        "flow_fwd": lambda: B.apply_flow_op(stack, _lib.MMOF_FLOW_FWD, 1, 0, u, v),
        "flow_adj": lambda: B.apply_flow_op(stack, _lib.MMOF_FLOW_ADJ, 1, 0, None, v, r),
        "of_derivs": lambda: B.of_derivs(stack, u, 1),
        "hs_multi": lambda: B.flow_update(stack, u, w, alpha=0.1, n_sweeps=8, delta_r=1),
        # frames and flow reduced by 4 (both block means) and the flow upscaled, no sweeps
        "box_down": lambda: B.flow_update_scaled(stack, u, w, alpha=0.1, n_sweeps=0, delta_r=1, scale=4),
        "flow_up": lambda: B.flow_update_scaled(stack, u, w, alpha=0.1, n_sweeps=0, delta_r=1, scale=4),
    }
    # the same frames through a flat-detector fan beam (source 1500 px from the centre,
    # detector 2500 px from the source, bins of 5/3 px: one pixel at the centre per bin)
    fplan = B.plan_fan(stack, [s.angles.shape[1]], [s.n_bins], s.angles.ravel(), 1500.0, 2500.0, 2500.0 / 1500.0)
    bf = B.apply_A(fplan, u)
    ops["fan_fwd"] = lambda: B.apply_A(fplan, u, out=bf)
    ops["fan_adj"] = lambda: B.apply_At(fplan, bf)
    if before_ops is not None:
        before_ops()
    table = {}
    for name, f in ops.items():
        f()
        torch.cuda.synchronize()
        ctx.profile_kernel(name)
        for _ in range(reps):
            f()
        n, ms, by, fl = ctx.kernel_timing()
        ctx.profile_kernel(None)
        if not n:
            continue
        sec = ms * 1e-3
        unit, peak = COMPUTE[name]
        ent = {"us": round(ms * 1e3 / n, 1), "GB/s": round(by / sec / 1e9, 1), "hbm_frac": round(by / sec / 1e9 / HBM_PEAK_GBS, 3),
               "TFLOP/s": round(fl / sec / 1e12, 2), "compute_frac": round(fl / sec / 1e12 / peak, 3)}
        if name == "hs_multi":
            ent["sweeps_per_launch"] = 8
        table[name] = ent
    # one whole flow update (derivatives, 200 warm-started sweeps, reverse flow) on the full
    # frames and on frames reduced by 2, 4 and the automatic factor: HIP-event time
    upd = {}
    vr = torch.empty_like(v)
    for sc in (1, 2, 4, _lib.MMOF_FLOW_SCALE_AUTO):
        f = lambda: B.flow_update_scaled(stack, u, w, alpha=0.1, n_sweeps=200, delta_r=1, scale=sc, v_rev=vr)
        f()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(3):
            f()
        ev1.record()
        torch.cuda.synchronize()
        upd["auto" if sc < 0 else str(sc)] = round(ev0.elapsed_time(ev1) / 3, 3)
    # Solve-OF (GKS with GCV: 10 Golub-Kahan steps, 20 projected solves, one workgroup per
    # pair) on the frames reduced by the automatic factor (32 x 32), with the reverse flow
    # and its p = q = 1 variant (smoothed-l1 weights, Gram matrices rebuilt per solve)
    for key, pq in (("solve_of_auto", 2), ("solve_of_l1_auto", 1)):
        f = lambda: B.flow_solve_gks(stack, u, w, delta_r=1, ell=10, n_iter=20, scale=_lib.MMOF_FLOW_SCALE_AUTO,
                                     v_rev=vr, pq=pq)
        f()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(3):
            f()
        ev1.record()
        torch.cuda.synchronize()
        upd[key] = round(ev0.elapsed_time(ev1) / 3, 3)
    del plan, fplan
    return {"workload": "large1024x1024x64: 12 moving/rotating ellipses, 90 golden-angle-shifted angles/frame, "
                        "1449 bins, smooth flow |v| <= 3 px", "dtype": "f32", "tiles": tuned, "kernels": table,
            "flow_update_ms": upd}


def large_solve(B, torch, k_ref=30, k_cap=40):
    """Time to solution on the 1024x1024x64 workload: the target is the RRE of the
    FP64-operator solve after k_ref iterations (x 1.01); FP64, FP32 and FP32 + FP64-refined
    solves run to it (at most k_cap iterations), timed by the wall clock of solve_joint with
    the inputs resident.  (k_cap bounds the Krylov basis: 49 columns of V, H V and Theta V
    in both precisions take about 200 GB of HBM.)"""
    from synth import cfg_large1024
    wl = cfg_large1024()
    stack, plan, u_true, b, delta = gpu_data(wl, B, torch)
    p = wl.params
    prm = dict(ell=p["ell"], k_max=k_ref, tau=p["tau"], n_sweeps=p["n_sweeps"], alpha=p["alpha"],
               eps=p["eps"], eta=p["eta"], delta_r=p["delta_r"])
    for dt in (torch.float32, torch.float64):
        log(f"large autotune {dt}: {plan.autotune(dt)}")
    out = {"workload": "large1024x1024x64", "n_pixels": plan.n, "n_data": plan.m, "params": dict(prm),
           "k_cap": k_cap}
    t0 = time.perf_counter()
    ref = B.solve_joint(plan, b, delta, u_true=u_true, op_dtype="f64", **prm)
    torch.cuda.synchronize()
    out["f64_reference"] = {"seconds": time.perf_counter() - t0, "iters": ref.iters, "rre": ref.rre[-1]}
    log(f"large f64 reference: {out['f64_reference']}")
    target = ref.rre[-1] * 1.01
    out["rre_target"] = target
    prm["k_max"] = k_cap
    for name, kw in (("f64", dict(op_dtype="f64")), ("f32", dict(op_dtype="f32")),
                     ("f32+refine", dict(op_dtype="f32", refine_iters=REFINE_ITERS))):
        # untimed one-iteration solve of the same configuration: the workspaces (tens of GB
        # at this size) are allocated outside the timed run
        B.solve_joint(plan, b, delta, u_true=u_true, rre_target=1.0, **dict(prm, **kw))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = B.solve_joint(plan, b, delta, u_true=u_true, rre_target=target, **dict(prm, **kw))
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "iters": r.iters, "rre": r.rre[-1],
                     "reached": bool(r.rre[-1] <= target)}
        log(f"large {name}: {out[name]}")
    free, total = torch.cuda.mem_get_info()
    out["hbm_used_gb"] = round((total - free) / 1e9, 1)
    # the FP64 Krylov kernels at this size: HIP-event time and algorithmic bytes of every
    # launch of one kernel over one FP32 solve of k_ref iterations (one solve per kernel)
    ctx = plan.ctx
    kry = {}
    prm["k_max"] = k_ref
    for kname in ("wgram", "mdot", "gemv_mdot", "gemv"):
        ctx.profile_kernel(kname)
        B.solve_joint(plan, b, delta, u_true=u_true, op_dtype="f32", **prm)
        torch.cuda.synchronize()
        nl, ms, by, fl = ctx.kernel_timing()
        ctx.profile_kernel(None)
        if nl:
            sec = ms * 1e-3
            kry[kname] = {"launches": nl, "avg_us": round(ms * 1e3 / nl, 1), "GB/s": round(by / sec / 1e9, 1),
                          "hbm_frac": round(by / sec / 1e9 / HBM_PEAK_GBS, 3), "TFLOP/s": round(fl / sec / 1e12, 2)}
    out["krylov_kernels"] = kry
    log(f"large krylov kernels: {kry}")
    return out


def ragged_blur(B, torch, reps=2):
    """The batched deblurring workload (40 sequences of 64^2..256^2 x 8..32 frames, 9x9
    Gaussian blur, 1% noise): FP32-operator solves with the launch sequences replayed from
    HIP graphs and the autotuned tiles, the same solves launched eagerly, and the FP64
    solve; wall time per solve (median of `reps` after a warm-up), inputs resident."""
    from synth import cfg_blur_ragged
    wl = cfg_blur_ragged()
    sizes = [(s.n_t, s.ny, s.nx) for s in wl.seqs]
    stack = B.Stack(sizes)
    plan = B.plan_blur(stack, wl.params["ksize"], wl.params["sigma"])
    u_true = torch.as_tensor(np.concatenate([s.u_true.ravel() for s in wl.seqs]), dtype=torch.float64,
                             device="cuda")
    clean = B.apply_A(plan, u_true)
    g = torch.as_tensor(np.concatenate([s.noise_g.ravel() for s in wl.seqs]), dtype=torch.float64, device="cuda")
    e = wl.noise_level * torch.linalg.vector_norm(clean) * g / torch.linalg.vector_norm(g)
    b = (clean + e).contiguous()
    delta = float(torch.linalg.vector_norm(e))
    tiles = {str(dt): plan.autotune(dt) for dt in (torch.float32, torch.float64)}
    log(f"ragged autotune: {tiles}")
    p = wl.params
    out = {"workload": f"blur_ragged40: {len(sizes)} sequences, {min(s[1] for s in sizes)}^2..{max(s[1] for s in sizes)}^2 "
                       f"x {min(s[0] for s in sizes)}..{max(s[0] for s in sizes)} frames, 9x9 Gaussian blur, 1% noise",
           "n_pixels": plan.n, "tiles": tiles}
    for name, op, graph in (("f32_graph", "f32", 1), ("f32_eager", "f32", 0), ("f64_graph", "f64", 1)):
        kw = dict(ell=p["ell"], k_max=p["k_max"], tau=p["tau"], n_sweeps=p["n_sweeps"], alpha=p["alpha"],
                  eps=p["eps"], eta=p["eta"], delta_r=p["delta_r"], op_dtype=op, use_graph=graph)
        r = B.solve_joint(plan, b, delta, u_true=u_true, **kw)   # warm-up (graphs captured)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = B.solve_joint(plan, b, delta, u_true=u_true, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        sec = float(np.median(ts))
        mv = r.counts["A"] + r.counts["At"] + r.counts["L"]
        out[name] = {"seconds": sec, "iters": r.iters, "rre": r.rre[-1], "matvecs": mv,
                     "matvecs_per_s": mv / sec}
        log(f"ragged {name}: {out[name]}")
    del plan
    return out


def autograd_step(B, torch, reps=10):
    """The differentiation workload (256x256x16, Radon with 30 angles, a smooth flow of up to
    3 px): one forward and backward pass of f(u, v) = <w1, H u> + <w2, Psi u> + <w3, L(v) u>
    through the library's autograd functions (backward = the adjoint kernels and dL/dv), FP32
    and FP64; wall time per pass, median of `reps` after a warm-up."""
    from paper_2501_12497_amd import autograd as AG
    from synth import cfg_autograd256
    wl = cfg_autograd256()
    s = wl.seqs[0]
    n_t, n = s.n_t, s.ny
    stack = B.Stack.single(n_t, n, n)
    plan = B.plan_radon(stack, [s.angles.shape[1]], [s.n_bins], s.angles.ravel())
    r = np.random.default_rng(wl.params["loss_seed"])
    ws = [r.standard_normal(sh) for sh in ((n_t, s.angles.shape[1], s.n_bins), (n_t, n, n - 1), (n_t, n - 1, n),
                                            (n_t - 1, n, n))]
    out = {"workload": "autograd256: 256x256x16, 30 angles/frame, 363 bins, smooth flow |v| <= 3 px; "
                       "loss <w1,Hu> + <w2,Psi u> + <w3,L(v)u>, gradients in u and v"}
    for dt in (torch.float32, torch.float64):
        wt = [torch.as_tensor(w.ravel(), dtype=dt, device="cuda") for w in ws]
        u0 = torch.as_tensor(s.u_true.ravel(), dtype=dt, device="cuda")
        v0 = torch.as_tensor(np.asarray(wl.params["flow"]).ravel(), dtype=dt, device="cuda")

        def step():
            u = u0.clone().requires_grad_(True)
            v = v0.clone().requires_grad_(True)
            b = AG.forward_op(u, plan)
            gx, gy = AG.gradient_op(u, stack)
            rr = AG.flow_op(u, v, stack, 1)
            f = (wt[0] * b).sum() + (wt[1] * gx).sum() + (wt[2] * gy).sum() + (wt[3] * rr).sum()
            f.backward()
            return u.grad, v.grad
        step()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out["f32" if dt == torch.float32 else "f64"] = {"ms_per_forward_backward": round(float(np.median(ts)) * 1e3, 3)}
    log(f"autograd: {out}")
    return out


def solve_params(wl, op, graph=True):
    p = wl.params
    return dict(ell=p["ell"], k_max=p["k_max"], tau=p["tau"], n_sweeps=p["n_sweeps"], alpha=p["alpha"],
                eps=p["eps"], eta=p["eta"], delta_r=p["delta_r"], op_dtype=op, use_graph=1 if graph else 0)


def cpu_baseline(wl, k_iters: int = 3):
    """The FP64 oracle's solve on the same workload, stopped after k_iters outer iterations
    (one flow update included); matvecs counted by wrapping the oracle's operators."""
    from oracle import mmgks
    from synth import noisy

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    s = wl.seqs[0]
    g = mmgks.SeqGeom(s.n_t, s.ny, s.nx, s.angles, s.n_bins)
    ops = mmgks.StackOps([g], "radon")
    clean = ops.A(s.u_true.ravel())
    b = noisy(clean, s.noise_g, wl.noise_level)
    delta = float(np.linalg.norm(b - clean))
    cnt = dict(A=0, At=0, L=0)
    fA, fAt, fT, fTT = ops.A, ops.At, ops.theta, ops.thetaT

    def A(x):
        cnt["A"] += 1
        return fA(x)

    def At(x):
        cnt["At"] += 1
        return fAt(x)

    def T(x, f):
        cnt["L"] += 2
        return fT(x, f)

    def TT(x, f):
        cnt["L"] += 2
        return fTT(x, f)

    ops.A, ops.At, ops.theta, ops.thetaT = A, At, T, TT
    p = wl.params
    prm = mmgks.SolveParams(ell=p["ell"], k_max=k_iters, tau=p["tau"], n_sweeps=p["n_sweeps"], alpha=p["alpha"],
                            eps=p["eps"], eta=p["eta"], delta_r=p["delta_r"])
    t0 = time.perf_counter()
    mmgks.mmgks_of(ops, b, delta, prm, u_true=s.u_true.ravel())
    dt = time.perf_counter() - t0
    n = cnt["A"] + cnt["At"] + cnt["L"]
    return {"value": n / dt, "unit": "matvecs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 oracle MMGKS-OF on the same 128x128x16 data, {k_iters} outer iterations "
                      f"(1 flow update of {p['n_sweeps']} sweeps), {n} A/At/L(v) applications in {dt:.1f} s; "
                      f"sparse products single-threaded, dense QR/solves on {threads} BLAS threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--profile-kernel", default="wgram")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the operator table at 1024x1024x64")
    ap.add_argument("--no-autotune", action="store_true", help="use the default tile shapes")
    ap.add_argument("--no-ragged", action="store_true", help="skip the batched-deblurring (40 sequences) solves")
    ap.add_argument("--no-autograd", action="store_true", help="skip the autograd forward/backward timing")
    ap.add_argument("--no-large-solve", action="store_true",
                    help="skip the FP64 / FP32 / FP32+refined solves of the 1024x1024x64 workload")
    ap.add_argument("--graph", action="store_true",
                    help="replay the fixed launch sequences of each iteration from HIP graphs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (reference dispatch for HBM counters)")
    ap.add_argument("--only", choices=["operators", "large-solve"],
                    help="for profiler runs: only the operator table at 1024x1024x64 (after a 256 MiB copy), "
                         "or only one FP32 solve of that workload (30 iterations, after the autotuner)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_12497_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.only == "operators":
        def calibration_copy():
            src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        # every operator: one warm-up launch, then 3 timed ones, right after the copy
        print(json.dumps(operators_large(B, torch, reps=3, before_ops=calibration_copy)), flush=True)
        return
    if a.only == "large-solve":
        from synth import cfg_large1024
        wl = cfg_large1024()
        stack, plan, u_true, b, delta = gpu_data(wl, B, torch)
        p = wl.params
        for dt in (torch.float32, torch.float64):
            log(f"large autotune {dt}: {plan.autotune(dt)}")
        t0 = time.perf_counter()
        r = B.solve_joint(plan, b, delta, u_true=u_true, op_dtype="f32", ell=p["ell"], k_max=30, tau=p["tau"],
                          n_sweeps=p["n_sweeps"], alpha=p["alpha"], eps=p["eps"], eta=p["eta"],
                          delta_r=p["delta_r"])
        torch.cuda.synchronize()
        print(json.dumps({"seconds": time.perf_counter() - t0, "iters": r.iters, "rre": r.rre[-1],
                          "counts": r.counts}), flush=True)
        return
    wl = make_workload()
    stack, plan, u_true, b, delta = gpu_data(wl, B, torch)
    ctx = plan.ctx
    prm = solve_params(wl, "f32", graph=a.graph)
    log(f"workload {wl.name}: n={plan.n} m={plan.m} params={prm}")
    if not a.no_autotune:  # tile shapes of this plan's stencil kernels, once, before any timing
        for dt in (torch.float32, torch.float64):
            log(f"autotune {dt}: {plan.autotune(dt)}")

    def step():
        return B.solve_joint(plan, b, delta, u_true=u_true, **prm)

    if a.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    for i in range(a.warmup):
        r = step()
        log(f"warmup {i}: iters={r.iters} rre={r.rre[-1]:.5f}")
    ctx.profile_kernel(a.profile_kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for i in range(a.steps):
        res.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_launch, k_ms, k_bytes, k_flops = ctx.kernel_timing()
    ctx.profile_kernel(None)
    ms_step = (t1 - t0) * 1e3 / a.steps
    r = res[-1]
    mv = r.counts["A"] + r.counts["At"] + r.counts["L"]
    value = mv * a.steps / (t1 - t0)
    log(f"timed {a.steps} solves: {ms_step:.2f} ms/solve, {mv} matvecs/solve, rre={r.rre[-1]:.5f}, "
        f"{a.profile_kernel}: {n_launch} launches {k_ms:.2f} ms")

    # roofline of the profiled kernel: its algorithmic work over its launches in the timed
    # region (HIP events on the library's stream), against the bound its arithmetic
    # intensity selects
    roof = None
    if n_launch and k_ms > 0 and a.profile_kernel in COMPUTE:
        unit, peak_tf = COMPUTE[a.profile_kernel]
        sec = k_ms * 1e-3
        intensity = k_flops / max(k_bytes, 1.0)
        ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
        traffic = measured_traffic(a.profile_kernel)
        common = {"kernel": a.profile_kernel, "launches": n_launch, "avg_launch_us": round(k_ms * 1e3 / n_launch, 3),
                  "bytes_per_launch": round(k_bytes / n_launch), "flops_per_launch": round(k_flops / n_launch),
                  "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(ridge, 2),
                  "traffic": traffic}
        if intensity < ridge:
            ach = k_bytes / sec / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), **common}
        else:
            ach = k_flops / sec / 1e12
            roof = {"bound": unit, "achieved": round(ach, 2), "peak": peak_tf, "unit": "TFLOP/s",
                    "frac": round(ach / peak_tf, 4), **common}

    # time to solution at a fixed relative error: FP32 operators vs FP64 operators
    tts = None
    if not a.no_tts:
        ref = B.solve_joint(plan, b, delta, u_true=u_true, **solve_params(wl, "f64", graph=a.graph))
        target = ref.rre[-1] * 1.001
        tts = {"rre_target": target, "k_max": prm["k_max"] + 15}
        for op in ("f64", "f32", "f32+refine"):
            kw = solve_params(wl, op.split("+")[0], graph=a.graph)
            kw["k_max"] = prm["k_max"] + 15
            kw["rre_target"] = target
            if op.endswith("refine"):
                kw["refine_iters"] = REFINE_ITERS
            B.solve_joint(plan, b, delta, u_true=u_true, **kw)
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                rr = B.solve_joint(plan, b, delta, u_true=u_true, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            tts[op] = {"seconds": float(np.median(ts)), "iters": rr.iters, "rre": rr.rre[-1],
                       "reached": bool(rr.rre[-1] <= target)}
        log(f"time to solution: {tts}")

    large = None
    if not a.no_large:
        large = operators_large(B, torch)
        log(f"operators at 1024x1024x64: {large['kernels']}")

    ragged = None
    if not a.no_ragged:
        ragged = ragged_blur(B, torch)

    agrad = None
    if not a.no_autograd:
        agrad = autograd_step(B, torch)

    big = None
    if not a.no_large_solve:
        big = large_solve(B, torch)

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(wl)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "A+At+L(v) matvecs/s in the MMGKS-OF joint solve (FP32 operators, FP64 Krylov)",
        "value": round(value, 1),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operators + f64 krylov",
        "data": "synthetic",
        "config": {"workload": "ellipse128x128x16: 3 translating ellipses, 30 angles/frame (+6 deg/frame), "
                               "181 bins, 2% noise; solve ell=10, 30 MM iterations, flow every 10 (200 HS sweeps)",
                   "n_pixels": plan.n, "n_data": plan.m, "matvecs_per_step": mv, "rre": r.rre[-1]},
        "roofline": roof,
        "time_to_solution": tts,
        "cpu_baseline": cpu,
        "operators_large": large,
    }
    if ragged is not None:
        out["ragged_blur"] = ragged
    if agrad is not None:
        out["autograd"] = agrad
    if big is not None:
        out["time_to_solution_large"] = big
    print(json.dumps(out))


if __name__ == "__main__":
    main()
