"""Benchmark of the MMGKS-OF hot path on one MI355X.

Workload (headline): 1024x1024 pixels x 64 frames, 12 ellipses moving with real
velocities in [-2, 2] px/frame and rotating up to 3 deg/frame, 90 parallel-beam angles
per frame shifted by the golden angle from frame to frame, 1449 detector bins, 2%
Gaussian noise (synthetic, seeded).  One step is one complete joint solve (MMGKS-OF,
Alg. 1): Golub-Kahan start (ell = 10), 30 outer MM iterations, Horn-Schunck flow update
(100 sweeps) every 10 iterations, with FP32 operator applications and the FP64
generalized-Krylov projection, Gram matrices, projected solve and discrepancy principle.
Inputs are resident on the GPU before the timed region starts.  `value` counts the
applications of H, H^T and L(v) (each flow direction of L or L^T once) per second of
whole-solve wall time.

Printed JSON fields beyond the driver's contract:
  roofline         the dominant kernel of the solve (largest summed HIP-event time):
                   its algorithmic bytes (or flops) / its mean launch time over the timed
                   region, against the HBM or compute peak its arithmetic intensity selects
  kernel_share     summed HIP-event time per solve of the candidate kernels
  time_to_solution FP64-operator, FP32-operator and FP32 + FP64-refined solves to one RRE
  cpu_baseline     the FP64 oracle's operators on the host, on a bounded sample, extrapolated
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
    "gemv": ("alu", 78.6),
    "gemv_mdot": ("alu", 78.6),
}
# The committed HBM-traffic summary of a kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE runs) and
# the source file it was measured on: traffic is reported only while that source is unchanged.
TRAFFIC = {
    "wgram": ("profiles/wgram_large1024_traffic.txt", "paper_2501_12497_amd/csrc/k_krylov.hip"),
    "gemv": ("profiles/gemv_large1024_traffic.txt", "paper_2501_12497_amd/csrc/k_krylov.hip"),
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
# candidate kernels for the roofline line: the projector pair, the weighted Gram and the
# passes over the Krylov basis (every other kernel of the solve is far smaller)
# the library runs up to 6 Horn-Schunck sweeps per launch (one launch is timed)
HS_SWEEPS_PER_LAUNCH = 6
CANDIDATES = ("wgram", "radon_fwd", "radon_adj", "gemv", "mdot", "gemv_mdot", "flow_adj", "hs_multi")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
        "hs_multi": lambda: B.flow_update(stack, u, w, alpha=0.1, n_sweeps=HS_SWEEPS_PER_LAUNCH, delta_r=1),
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
            ent["sweeps_per_launch"] = HS_SWEEPS_PER_LAUNCH
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


def solve_kw(p, k_max, op, graph=False, **extra):
    kw = dict(ell=p["ell"], k_max=k_max, tau=p["tau"], n_sweeps=p["n_sweeps"], alpha=p["alpha"], eps=p["eps"],
              eta=p["eta"], delta_r=p["delta_r"], op_dtype=op, use_graph=1 if graph else 0)
    kw.update(extra)
    return kw


def roofline_of(name, n_launch, k_ms, k_bytes, k_flops):
    """Roofline object of a kernel from its HIP-event time and algorithmic work."""
    if not (n_launch and k_ms > 0 and name in COMPUTE):
        return None
    unit, peak_tf = COMPUTE[name]
    sec = k_ms * 1e-3
    intensity = k_flops / max(k_bytes, 1.0)
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    common = {"kernel": name, "launches": n_launch, "avg_launch_us": round(k_ms * 1e3 / n_launch, 3),
              "bytes_per_launch": round(k_bytes / n_launch), "flops_per_launch": round(k_flops / n_launch),
              "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(ridge, 2)}
    traffic = measured_traffic(name)
    if intensity < ridge:
        ach = k_bytes / sec / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, **common}
    ach = k_flops / sec / 1e12
    return {"bound": unit, "achieved": round(ach, 2), "peak": peak_tf, "unit": "TFLOP/s",
            "frac": round(ach / peak_tf, 4), "traffic": traffic, **common}


def kernel_shares(ctx, step, names):
    """Summed HIP-event time (ms) of each named kernel over one call of step()."""
    out = {}
    for name in names:
        ctx.profile_kernel(name)
        step()
        n, ms, _, _ = ctx.kernel_timing()
        ctx.profile_kernel(None)
        if n:
            out[name] = {"launches": n, "ms": round(ms, 3)}
    return out


def tts(B, torch, plan, b, delta, u_true, p, k_ref, k_cap, reps=1, graph=False):
    """Time to solution at a fixed relative error: the target is the RRE of the FP64-operator
    solve after k_ref iterations (x 1.01); FP64, FP32 and FP32 + FP64-refined solves run to
    it (at most k_cap iterations), timed by the wall clock of solve_joint (median of reps,
    after an untimed run that also allocates the workspaces).  The refined solve runs its
    last REFINE_ITERS iterations with FP64 operators and is given k_max = (iterations the
    FP32 solve needed) + 1, so that its FP64 phase starts REFINE_ITERS - 1 iterations before
    the FP32 solve reached the target; it is an error if no FP64 iteration ran."""
    ref = B.solve_joint(plan, b, delta, u_true=u_true, **solve_kw(p, k_ref, "f64", graph))
    target = ref.rre[-1] * 1.01
    out = {"k_ref": k_ref, "k_cap": k_cap, "rre_target": target}

    def run(kw):
        B.solve_joint(plan, b, delta, u_true=u_true, **kw)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = B.solve_joint(plan, b, delta, u_true=u_true, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return r, float(np.median(ts))

    for name, op in (("f64", "f64"), ("f32", "f32")):
        r, sec = run(solve_kw(p, k_cap, op, graph, rre_target=target))
        out[name] = {"seconds": sec, "iters": r.iters, "rre": r.rre[-1], "reached": bool(r.rre[-1] <= target)}
        log(f"tts {name}: {out[name]}")
    k_max = out["f32"]["iters"] + 1
    r, sec = run(solve_kw(p, k_max, "f32", graph, rre_target=target, refine_iters=REFINE_ITERS))
    k_sw = max(0, k_max - REFINE_ITERS)
    n64 = max(0, r.iters - k_sw)
    out["f32+refine"] = {"seconds": sec, "iters": r.iters, "rre": r.rre[-1], "reached": bool(r.rre[-1] <= target),
                         "k_max": k_max, "refine_iters": REFINE_ITERS, "fp32_iters": min(r.iters, k_sw),
                         "fp64_iters": n64, "rre_vs_f64": r.rre[-1] - out["f64"]["rre"]}
    log(f"tts f32+refine: {out['f32+refine']}")
    if n64 == 0:
        raise RuntimeError("the FP32 + FP64-refined solve ran no FP64 iteration")
    return out


def cpu_baseline_large(wl, counts, n_frames_sample=2):
    """The FP64 oracle's operators on a bounded sample of the 1024x1024x64 workload, scaled
    to the whole stack and to the operator mix of one GPU solve: H and H^T on the first
    n_frames_sample frames with all their angles (the projector is a sum over frames, so its
    time is linear in them), L(v) and L(v)^T in one direction on the pairs of those frames
    (linear in pairs).  Rate = applications in one GPU solve / the oracle's extrapolated time for them.
    Only operator time is counted (none of the solve's Krylov or flow work), so the rate
    favours the CPU."""
    from oracle import forward, regops
    from synth import smooth_flow_coarse
    s = wl.seqs[0]
    n_t, ny, nx = s.n_t, s.ny, s.nx
    na = s.angles.shape[1]
    u = s.u_true
    f = n_frames_sample
    ang = s.angles[:f]
    v = smooth_flow_coarse(f - 1, nx, seed=11, coarse=16, vmax=3.0)
    t0 = time.perf_counter()
    bb = forward.radon_fwd(u[:f], ang, s.n_bins)
    t1 = time.perf_counter()
    forward.radon_adj(bb, ang, ny, nx)
    t2 = time.perf_counter()
    rr = regops.flow_fwd(u[:f], v, 1)
    t3 = time.perf_counter()
    regops.flow_adj(rr, v, f, 1)
    t4 = time.perf_counter()
    t_A, t_At = (t1 - t0) * n_t / f, (t2 - t1) * n_t / f
    t_L, t_Lt = (t3 - t2) * (n_t - 1) / (f - 1), (t4 - t3) * (n_t - 1) / (f - 1)
    # L counts the forward and the adjoint applications together; take their mean per use
    t_solve = counts["A"] * t_A + counts["At"] * t_At + counts["L"] * 0.5 * (t_L + t_Lt)
    n_mv = counts["A"] + counts["At"] + counts["L"]
    return {"value": n_mv / t_solve, "unit": "matvecs/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle (NumPy, one thread) on the 1024x1024x64 workload: H and H^T on frames 0-{f - 1} "
                      f"with all {na} angles ({t1 - t0:.1f} s, {t2 - t1:.1f} s), L(v) and L(v)^T on their "
                      f"{f - 1} pair(s) ({t3 - t2:.2f} s, {t4 - t3:.2f} s), extrapolated linearly to {n_t} frames "
                      f"and {n_t - 1} pairs (per stack application: H {t_A:.0f} s, H^T {t_At:.0f} s, "
                      f"L {t_L:.1f} s, L^T {t_Lt:.1f} s) and weighted by one GPU solve's {counts['A']} H, "
                      f"{counts['At']} H^T and {counts['L']} L/L^T applications; operator time only",
            "seconds_per_stack_application": {"A": t_A, "At": t_At, "L": t_L, "Lt": t_Lt}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k-max", type=int, default=30, help="outer MM iterations of the headline solve")
    ap.add_argument("--profile-kernel", default=None,
                    help="roofline kernel (default: the largest summed time among the candidates)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution legs")
    ap.add_argument("--no-small", action="store_true", help="skip the 128x128x16 solves")
    ap.add_argument("--no-large", action="store_true", help="skip the operator table at 1024x1024x64")
    ap.add_argument("--no-autotune", action="store_true", help="use the default tile shapes")
    ap.add_argument("--no-ragged", action="store_true", help="skip the batched-deblurring (40 sequences) solves")
    ap.add_argument("--no-autograd", action="store_true", help="skip the autograd forward/backward timing")
    ap.add_argument("--graph", action="store_true",
                    help="replay the fixed launch sequences of each iteration from HIP graphs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device copy first (reference dispatch for HBM counters)")
    ap.add_argument("--only", choices=["operators", "headline"],
                    help="for profiler runs: only the operator table at 1024x1024x64 (after a 256 MiB copy), "
                         "or only the headline solves (no other leg)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_12497_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    def calibration_copy():
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")

    if a.only == "operators":
        # every operator: one warm-up launch, then 3 timed ones, right after the copy
        print(json.dumps(operators_large(B, torch, reps=3, before_ops=calibration_copy)), flush=True)
        return
    if a.only == "headline":
        a.no_tts = a.no_small = a.no_large = a.no_ragged = a.no_autograd = a.no_cpu_baseline = True

    from synth import cfg_large1024
    wl = cfg_large1024()
    stack, plan, u_true, b, delta = gpu_data(wl, B, torch)
    ctx = plan.ctx
    p = wl.params
    prm = solve_kw(p, a.k_max, "f32", a.graph)
    log(f"workload {wl.name}: n={plan.n} m={plan.m} params={prm}")
    if not a.no_autotune:  # tile shapes of this plan's stencil kernels, once, before any timing
        for dt in (torch.float32, torch.float64):
            log(f"autotune {dt}: {plan.autotune(dt)}")

    def step():
        r = B.solve_joint(plan, b, delta, u_true=u_true, **prm)
        return r

    if a.copy_calibration:
        calibration_copy()
    for i in range(a.warmup):
        r = step()
        torch.cuda.synchronize()
        log(f"warmup {i}: iters={r.iters} rre={r.rre[-1]:.5f}")
    # the dominant kernel: summed HIP-event time per solve of each candidate (untimed solves)
    shares = None
    prof = a.profile_kernel
    if prof is None:
        shares = kernel_shares(ctx, step, CANDIDATES)
        prof = max(shares, key=lambda k: shares[k]["ms"])
        log(f"kernel shares per solve: {shares}; roofline kernel: {prof}")
    ctx.profile_kernel(prof)
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
        f"{prof}: {n_launch} launches {k_ms:.2f} ms")
    roof = roofline_of(prof, n_launch, k_ms, k_bytes, k_flops)

    big_tts = None
    if not a.no_tts:
        big_tts = tts(B, torch, plan, b, delta, u_true, p, k_ref=30, k_cap=40, graph=a.graph)
        free, total = torch.cuda.mem_get_info()
        big_tts["hbm_used_gb"] = round((total - free) / 1e9, 1)

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline_large(wl, r.counts)
        log(f"cpu baseline: {cpu}")
    del plan
    torch.cuda.empty_cache()

    small = None
    if not a.no_small:
        from synth import cfg_ellipse128
        ws = cfg_ellipse128()
        _, splan, su, sb, sdelta = gpu_data(ws, B, torch)
        if not a.no_autotune:
            for dt in (torch.float32, torch.float64):
                splan.autotune(dt)
        sp = ws.params
        skw = solve_kw(sp, sp["k_max"], "f32", a.graph)
        B.solve_joint(splan, sb, sdelta, u_true=su, **skw)
        torch.cuda.synchronize()
        ts = []
        for _ in range(10):
            t_0 = time.perf_counter()
            sr = B.solve_joint(splan, sb, sdelta, u_true=su, **skw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t_0)
        sec = float(np.median(ts))
        smv = sr.counts["A"] + sr.counts["At"] + sr.counts["L"]
        small = {"workload": "ellipse128x128x16: 3 translating ellipses, 30 angles/frame (+6 deg/frame), 181 bins, "
                             "2% noise; ell=10, 30 MM iterations, flow every 10 (200 HS sweeps)",
                 "seconds_per_solve": sec, "matvecs_per_solve": smv, "matvecs_per_s": smv / sec, "rre": sr.rre[-1]}
        # the paper's iteration budget (Sec. 5: ell = 10, 200 iterations, flow every 20): the
        # projected problems grow to 209 columns
        kw200 = solve_kw(sp, 200, "f32", a.graph, tau=20)
        B.solve_joint(splan, sb, sdelta, u_true=su, **kw200)
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        r200 = B.solve_joint(splan, sb, sdelta, u_true=su, **kw200)
        torch.cuda.synchronize()
        sec200 = time.perf_counter() - t_0
        mv200 = r200.counts["A"] + r200.counts["At"] + r200.counts["L"]
        small["solve_200_iterations"] = {"seconds": sec200, "iters": r200.iters, "n_cols": r200.n_cols,
                                         "rre": r200.rre[-1], "matvecs": mv200, "matvecs_per_s": mv200 / sec200,
                                         "tau": 20}
        if not a.no_tts:
            small["time_to_solution"] = tts(B, torch, splan, sb, sdelta, su, sp, k_ref=sp["k_max"],
                                            k_cap=sp["k_max"] + 15, reps=3, graph=a.graph)
        log(f"small: {small}")
        del splan

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
        "config": {"workload": "large1024x1024x64: 12 ellipses moving (real velocities in [-2,2] px/frame) and "
                               "rotating (up to 3 deg/frame), 90 parallel-beam angles/frame shifted by the golden "
                               f"angle, 1449 bins, 2% noise; solve ell=10, {a.k_max} MM iterations, flow every "
                               f"{p['tau']} ({p['n_sweeps']} HS sweeps)",
                   "n_pixels": stack.n, "n_data": int(b.numel()), "matvecs_per_step": mv, "rre": r.rre[-1],
                   "iters": r.iters},
        "roofline": roof,
        "kernel_share": shares,
        "time_to_solution": big_tts,
        "cpu_baseline": cpu,
        "small_ellipse128": small,
        "operators_large": large,
    }
    if ragged is not None:
        out["ragged_blur"] = ragged
    if agrad is not None:
        out["autograd"] = agrad
    print(json.dumps(out))


if __name__ == "__main__":
    main()
