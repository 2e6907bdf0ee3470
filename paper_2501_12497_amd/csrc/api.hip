// extern "C" entry points: argument checks, error translation, dispatch to launchers.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"
#include "krylov.h"
#include "solver.h"
#include "tune.h"

namespace mmof {
const char* last_error_cstr();
void radon_plan_init(Ctx& c, Plan& p, const double* cs);  // cs: the host copy of the trig table
}  // namespace mmof

using namespace mmof;

#define MMOF_VERSION_STRING "mmof-gfx950 0.1.0"

template <class F>
static int guarded(Ctx* c, F&& f) {
    try {
        int rc = f();
        return rc;
    } catch (const Error& e) {
        set_last_error(e.what());
        if (c) c->last_error = e.what();
        if (e.code == MMOF_ERR_HIP) (void)hipGetLastError();  // do not leave it for the next call
        return e.code;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        if (c) c->last_error = e.what();
        return MMOF_ERR_HIP;
    } catch (...) {
        set_last_error("unknown error");
        return MMOF_ERR_HIP;
    }
}

static void need(const void* p, const char* what) {
    MMOF_CHECK(p != nullptr, MMOF_ERR_INVALID, std::string(what) + " is NULL");
}

static void need_dt(int dt) {
    MMOF_CHECK(dt == MMOF_F32 || dt == MMOF_F64, MMOF_ERR_DTYPE, "dtype must be MMOF_F32 or MMOF_F64");
}

extern "C" {

const char* mmof_version(void) { return MMOF_VERSION_STRING; }

const char* mmof_last_error(mmof_ctx ctx) {
    (void)ctx;
    return last_error_cstr();
}

int mmof_create(mmof_ctx* out, void* hip_stream) {
    return guarded(nullptr, [&] {
        need(out, "out");
        *out = nullptr;
        std::unique_ptr<mmof_ctx_s> c(new mmof_ctx_s());
        MMOF_HIP(hipGetDevice(&c->device));
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
            c->cu_count = cus;
        c->stream = static_cast<hipStream_t>(hip_stream);
        noalloc_init(c->device);  // this device's address of the allocation-free Gram's scratch
        *out = c.release();
        return MMOF_OK;
    });
}

int mmof_destroy(mmof_ctx ctx) {
    return guarded(nullptr, [&] {
        if (!ctx) return MMOF_OK;
        (void)hipStreamSynchronize(ctx->stream);
        delete ctx;
        return MMOF_OK;
    });
}

int mmof_set_stream(mmof_ctx ctx, void* hip_stream) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        ctx->stream = static_cast<hipStream_t>(hip_stream);
        return MMOF_OK;
    });
}

// ------------------------------------------------------------------ plans

static int plan_projector(mmof_ctx ctx, const mmof_stack* stack, const int32_t* n_angles, const int32_t* n_bins,
                          const double* angles_rad, int kind, double dso, double dsd, double du, mmof_plan* out) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need(stack, "stack");
        need(n_angles, "n_angles");
        need(n_bins, "n_bins");
        need(angles_rad, "angles_rad");
        need(out, "out");
        *out = nullptr;
        std::unique_ptr<mmof_plan_s> p(new mmof_plan_s());
        p->ctx = ctx;
        p->kind = kind;
        p->geom_own = make_geom(stack, ctx->stream);
        p->geom = p->geom_own.get();
        p->n = p->geom->n;
        if (kind == 2) {
            MMOF_CHECK(std::isfinite(dso) && std::isfinite(dsd) && std::isfinite(du) && du > 0 && dsd > dso,
                       MMOF_ERR_INVALID, "fan beam needs du > 0 and dsd > dso");
            for (int s = 0; s < stack->n_seq; ++s)
                MMOF_CHECK(dso > 0.5 * std::hypot((double)stack->nx[s], (double)stack->ny[s]) + 2.0, MMOF_ERR_INVALID,
                           "fan beam: the source must lie outside every frame (dso > half diagonal + 2)");
            p->fan_dso = dso;
            p->fan_dsd = dsd;
            p->fan_du = du;
        }
        int64_t n_trig = 0;
        for (int s = 0; s < stack->n_seq; ++s) {
            MMOF_CHECK(n_angles[s] >= 1 && n_bins[s] >= 1, MMOF_ERR_SHAPE, "n_angles and n_bins must be >= 1");
            p->n_ang.push_back(n_angles[s]);
            p->n_bins.push_back(n_bins[s]);
            n_trig += (int64_t)stack->n_t[s] * n_angles[s];
        }
        std::vector<double> cs(2 * n_trig);
        for (int64_t i = 0; i < n_trig; ++i) {
            MMOF_CHECK(std::isfinite(angles_rad[i]), MMOF_ERR_NONFINITE, "angle is not finite");
            cs[2 * i] = std::cos(angles_rad[i]);
            cs[2 * i + 1] = std::sin(angles_rad[i]);
        }
        p->d_trig.ensure(sizeof(double) * cs.size());
        MMOF_HIP(hipMemcpyAsync(p->d_trig.ptr, cs.data(), sizeof(double) * cs.size(), hipMemcpyHostToDevice,
                                ctx->stream));
        radon_plan_init(*ctx, *p, cs.data());  // synchronizes the stream
        if (kind == 2) fan_plan_init(*ctx, *p);
        *out = p.release();
        return MMOF_OK;
    });
}

int mmof_plan_radon(mmof_ctx ctx, const mmof_stack* stack, const int32_t* n_angles, const int32_t* n_bins,
                    const double* angles_rad, mmof_plan* out) {
    return plan_projector(ctx, stack, n_angles, n_bins, angles_rad, 0, 0.0, 0.0, 0.0, out);
}

int mmof_plan_fan(mmof_ctx ctx, const mmof_stack* stack, const int32_t* n_angles, const int32_t* n_bins,
                  const double* angles_rad, double dso, double dsd, double du, mmof_plan* out) {
    return plan_projector(ctx, stack, n_angles, n_bins, angles_rad, 2, dso, dsd, du, out);
}

int mmof_plan_blur(mmof_ctx ctx, const mmof_stack* stack, int32_t ksize, double sigma, mmof_plan* out) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need(stack, "stack");
        need(out, "out");
        *out = nullptr;
        MMOF_CHECK(ksize >= 1 && ksize <= 15 && (ksize % 2) == 1, MMOF_ERR_INVALID, "ksize must be odd, 1..15");
        MMOF_CHECK(sigma > 0 && std::isfinite(sigma), MMOF_ERR_INVALID, "sigma must be > 0");
        std::unique_ptr<mmof_plan_s> p(new mmof_plan_s());
        p->ctx = ctx;
        p->kind = 1;
        p->geom_own = make_geom(stack, ctx->stream);
        p->geom = p->geom_own.get();
        p->n = p->geom->n;
        p->m = p->geom->n;
        p->ksize = ksize;
        p->sigma = sigma;
        const int r = ksize / 2;
        std::vector<double> k1(ksize);
        double s = 0.0;
        for (int i = -r; i <= r; ++i) s += (k1[i + r] = std::exp(-(double)(i * i) / (2.0 * sigma * sigma)));
        for (auto& v : k1) v /= s;
        p->d_k1.ensure(sizeof(double) * ksize);
        MMOF_HIP(hipMemcpyAsync(p->d_k1.ptr, k1.data(), sizeof(double) * ksize, hipMemcpyHostToDevice, ctx->stream));
        MMOF_HIP(hipStreamSynchronize(ctx->stream));
        *out = p.release();
        return MMOF_OK;
    });
}

int mmof_plan_destroy(mmof_plan plan) {
    return guarded(nullptr, [&] {
        if (!plan) return MMOF_OK;
        (void)hipStreamSynchronize(plan->ctx->stream);
        delete plan;
        return MMOF_OK;
    });
}

int mmof_plan_sizes(mmof_plan plan, int64_t* n, int64_t* m) {
    return guarded(nullptr, [&] {
        need(plan, "plan");
        if (n) *n = plan->n;
        if (m) *m = plan->m;
        return MMOF_OK;
    });
}

int mmof_autotune(mmof_plan plan, mmof_dtype dt, char* report, int32_t report_len) {
    return guarded(plan ? plan->ctx : nullptr, [&] {
        need(plan, "plan");
        need_dt(dt);
        const std::string rep = autotune(*plan, dt);
        if (report && report_len > 0) {
            const size_t k = std::min<size_t>(rep.size(), (size_t)report_len - 1);
            std::memcpy(report, rep.data(), k);
            report[k] = 0;
        }
        return MMOF_OK;
    });
}

int mmof_set_tile(mmof_plan plan, const char* kernel, mmof_dtype dt, int32_t choice) {
    return guarded(plan ? plan->ctx : nullptr, [&] {
        need(plan, "plan");
        need(kernel, "kernel");
        need_dt(dt);
        set_tile(*plan, kernel, dt, choice);
        return MMOF_OK;
    });
}

int mmof_apply_A(mmof_plan plan, mmof_dtype dt, const void* u, void* b) {
    return guarded(plan ? plan->ctx : nullptr, [&] {
        need(plan, "plan");
        need_dt(dt);
        need(u, "u");
        need(b, "b");
        if (plan->kind == 0)
            launch_radon_fwd(*plan->ctx, *plan, dt, u, b);
        else if (plan->kind == 2)
            launch_fan_fwd(*plan->ctx, *plan, dt, u, b);
        else
            launch_blur(*plan->ctx, *plan, dt, u, b);
        return MMOF_OK;
    });
}

int mmof_apply_At(mmof_plan plan, mmof_dtype dt, const void* b, void* u) {
    return guarded(plan ? plan->ctx : nullptr, [&] {
        need(plan, "plan");
        need_dt(dt);
        need(u, "u");
        need(b, "b");
        if (plan->kind == 0)
            launch_radon_adj(*plan->ctx, *plan, dt, b, u);
        else if (plan->kind == 2)
            launch_fan_adj(*plan->ctx, *plan, dt, b, u);
        else
            launch_blur(*plan->ctx, *plan, dt, b, u);
        return MMOF_OK;
    });
}

// ------------------------------------------------------------------ regularisation operators

int mmof_apply_grad(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int transpose, const void* wx,
                    const void* wy, void* u, void* gx, void* gy) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(u, "u");
        need(gx, "gx");
        need(gy, "gy");
        Geom& g = ctx->geom(stack);
        if (transpose)
            launch_grad_adj(*ctx, g, dt, gx, gy, wx, wy, u, false);
        else
            launch_grad_fwd(*ctx, g, dt, u, wx, wy, gx, gy);
        return MMOF_OK;
    });
}

int mmof_apply_flow_op(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int mode, int direction, int interp,
                       const void* u, const void* v, const void* in, void* out) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(v, "v");
        need(out, "out");
        MMOF_CHECK(direction == 1 || direction == -1, MMOF_ERR_INVALID, "direction must be +1 or -1");
        MMOF_CHECK(interp == MMOF_INTERP_BILINEAR || interp == MMOF_INTERP_ROUND, MMOF_ERR_INVALID, "bad interp");
        Geom& g = ctx->geom(stack);
        MMOF_CHECK(g.n_pairs >= 1, MMOF_ERR_SHAPE, "flow operators need sequences with >= 2 frames");
        switch (mode) {
            case MMOF_FLOW_FWD:
                need(u, "u");
                launch_flow_fwd(*ctx, g, dt, direction, interp, u, v, out);
                break;
            case MMOF_FLOW_ADJ:
                need(in, "in");
                launch_flow_adj(*ctx, g, dt, direction, interp, in, v, out, false, nullptr);
                break;
            case MMOF_FLOW_DV:
                need(u, "u");
                need(in, "in");
                launch_flow_dv(*ctx, g, dt, direction, interp, u, v, in, out);
                break;
            default:
                throw Error(MMOF_ERR_INVALID, "mode must be MMOF_FLOW_FWD, _ADJ or _DV");
        }
        return MMOF_OK;
    });
}

int mmof_mm_weights(mmof_ctx ctx, mmof_dtype dt, int64_t n, const void* nu, double eps, void* w2) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        MMOF_CHECK(n >= 0, MMOF_ERR_SHAPE, "n must be >= 0");
        MMOF_CHECK(eps > 0, MMOF_ERR_INVALID, "eps must be > 0");
        if (n == 0) return MMOF_OK;
        need(nu, "nu");
        need(w2, "w2");
        launch_mm_weights(*ctx, dt, n, nu, eps, w2);
        return MMOF_OK;
    });
}

// ------------------------------------------------------------------ optical flow

int mmof_of_derivs(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u, void* I, int32_t delta_r) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(u, "u");
        need(I, "I");
        Geom& g = ctx->geom(stack);
        MMOF_CHECK(delta_r >= 1 && delta_r < g.max_nx && delta_r < g.max_ny, MMOF_ERR_INVALID, "bad delta_r");
        for (int s = 0; s < g.n_seq; ++s)
            MMOF_CHECK(delta_r < g.nx[s] && delta_r < g.ny[s], MMOF_ERR_INVALID, "delta_r must be < frame size");
        launch_of_derivs(*ctx, g, dt, u, I, delta_r);
        return MMOF_OK;
    });
}

// The flow calls: checks, workspaces in the context, flow_update_core, the reverse flow.
static int flow_call(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u, void* v, void* v_rev,
                     int32_t delta_r, int32_t scale, const FlowMethod& fm, double* lambdas) {
    {
        need(ctx, "ctx");
        need_dt(dt);
        need(u, "u");
        need(v, "v");
        Geom& g = ctx->geom(stack);
        scale = resolve_flow_scale(g, scale);
        check_flow_frames(g, scale, delta_r);
        if (fm.solver == 1) check_gks_frames(g, scale, fm.ell, fm.n_iter);
        if (g.n_pairs == 0) return MMOF_OK;
        const size_t es = dt == MMOF_F32 ? 4 : 8;
        Geom* gs = scale > 1 ? &reduced_geom(*ctx, g, scale) : nullptr;
        const Geom& gw = gs ? *gs : g;
        FlowWork w;
        w.I = ctx->work("fu_I", es * 3 * gw.pair_px);
        w.tmp = ctx->work("fu_tmp", es * 2 * gw.pair_px);
        if (gs) {
            w.us = ctx->work("fu_us", es * gw.n);
            w.vs = ctx->work("fu_vs", es * 2 * gw.pair_px);
        }
        if (fm.solver == 1) w.gks = gks_work(*ctx, gw, fm, "fu_gks_");
        flow_update_core(*ctx, g, gs, dt, u, v, scale, delta_r, fm, w);
        if (v_rev) launch_reverse_flow(*ctx, g, dt, v, v_rev, nullptr);
        if (lambdas && fm.solver == 1) {
            MMOF_HIP(hipMemcpyAsync(lambdas, w.gks.lam, sizeof(double) * gw.n_pairs * fm.n_iter,
                                    hipMemcpyDeviceToHost, ctx->stream));
            MMOF_HIP(hipStreamSynchronize(ctx->stream));
        }
        return MMOF_OK;
    }
}

int mmof_flow_update_scaled(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u, void* v,
                            void* v_rev, double alpha, int32_t n_sweeps, int32_t delta_r, int32_t scale) {
    return guarded(ctx, [&] {
        MMOF_CHECK(alpha > 0 && std::isfinite(alpha), MMOF_ERR_INVALID, "alpha must be > 0");
        MMOF_CHECK(n_sweeps >= 0, MMOF_ERR_INVALID, "n_sweeps must be >= 0");
        FlowMethod fm;
        fm.solver = 0;
        fm.gamma = alpha * alpha;
        fm.n_sweeps = n_sweeps;
        return flow_call(ctx, stack, dt, u, v, v_rev, delta_r, scale, fm, nullptr);
    });
}

int mmof_flow_solve_of(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u, void* v, void* v_rev,
                       int32_t delta_r, int32_t ell, int32_t n_iter, double fixed_lambda, int32_t scale, int32_t pq,
                       double eps, double* lambdas) {
    return guarded(ctx, [&] {
        MMOF_CHECK(fixed_lambda >= 0 && std::isfinite(fixed_lambda), MMOF_ERR_INVALID, "fixed_lambda must be >= 0");
        MMOF_CHECK(pq == 1 || pq == 2, MMOF_ERR_INVALID, "pq must be 1 or 2");
        MMOF_CHECK(pq == 2 || (eps > 0 && std::isfinite(eps)), MMOF_ERR_INVALID, "eps must be > 0");
        FlowMethod fm;
        fm.solver = 1;
        fm.ell = ell;
        fm.n_iter = n_iter;
        fm.fixed_lambda = fixed_lambda;
        fm.of_p = pq;
        fm.of_eps = eps;
        return flow_call(ctx, stack, dt, u, v, v_rev, delta_r, scale, fm, lambdas);
    });
}

int mmof_flow_solve_gks(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u, void* v, void* v_rev,
                        int32_t delta_r, int32_t ell, int32_t n_iter, double fixed_lambda, int32_t scale,
                        double* lambdas) {
    return mmof_flow_solve_of(ctx, stack, dt, u, v, v_rev, delta_r, ell, n_iter, fixed_lambda, scale, 2, 0.0,
                              lambdas);
}

int mmof_flow_update(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u, void* v, void* v_rev,
                     double alpha, int32_t n_sweeps, int32_t delta_r) {
    return mmof_flow_update_scaled(ctx, stack, dt, u, v, v_rev, alpha, n_sweeps, delta_r, 1);
}

int mmof_reverse_flow(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* v, void* v_rev) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(v, "v");
        need(v_rev, "v_rev");
        Geom& g = ctx->geom(stack);
        launch_reverse_flow(*ctx, g, dt, v, v_rev, nullptr);
        return MMOF_OK;
    });
}

// ------------------------------------------------------------------ solve

void mmof_solve_defaults(mmof_solve_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->ell = 10;
    p->k_max = 20;
    p->tau = 1;
    p->n_sweeps = 200;
    p->delta_r = 1;
    p->use_flow = 1;
    p->use_reverse = 1;
    p->interp = MMOF_INTERP_BILINEAR;
    p->op_dtype = MMOF_F64;
    p->refine_iters = 0;
    p->eps = 1e-3;
    p->eta = 1.01;
    p->alpha = 0.1;
    p->fixed_lambda = 0.0;
    p->rre_target = 0.0;
    p->u_true = nullptr;
    p->use_graph = 0;
    p->flow_scale = 1;
    p->flow_solver = MMOF_FLOW_HS;
    p->of_ell = 10;
    p->of_iters = 20;
    p->reg = MMOF_REG_PSI;
    p->reorth = MMOF_REORTH_IMPLICIT;
}

int mmof_solve_joint(mmof_plan A, const void* b, double noise_norm, const mmof_solve_params* p, void* u_inout,
                     void* v_out, void* v_rev_out, mmof_report* rep) {
    return guarded(A ? A->ctx : nullptr, [&] {
        need(A, "plan");
        need(b, "b");
        need(p, "params");
        need(u_inout, "u_inout");
        MMOF_CHECK(std::isfinite(noise_norm) && noise_norm >= 0, MMOF_ERR_INVALID, "noise_norm must be >= 0");
        MMOF_CHECK(p->interp == MMOF_INTERP_BILINEAR || p->interp == MMOF_INTERP_ROUND, MMOF_ERR_INVALID, "bad interp");
        MMOF_CHECK(p->reg >= MMOF_REG_PSI && p->reg <= MMOF_REG_GS, MMOF_ERR_INVALID, "bad regulariser");
        MMOF_CHECK(p->reorth == MMOF_REORTH_AUTO || p->reorth == MMOF_REORTH_TWICE ||
                       p->reorth == MMOF_REORTH_IMPLICIT,
                   MMOF_ERR_INVALID, "bad reorth");
        if (p->use_flow) {
            const int f = resolve_flow_scale(*A->geom, p->flow_scale);
            check_flow_frames(*A->geom, f, p->delta_r);
            MMOF_CHECK(p->flow_solver == MMOF_FLOW_HS || p->flow_solver == MMOF_FLOW_GKS, MMOF_ERR_INVALID,
                       "bad flow_solver");
            if (p->flow_solver == MMOF_FLOW_GKS) check_gks_frames(*A->geom, f, p->of_ell, p->of_iters);
        }
        int rc = solve_joint(*A, static_cast<const double*>(b), noise_norm, *p, static_cast<double*>(u_inout), v_out,
                             v_rev_out, rep);
        if (rep) rep->status = rc;
        return rc;
    });
}

// ------------------------------------------------------------------ projected-problem steps

int mmof_weighted_gram(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X, int64_t ld, const void* nu,
                       double eps, double* G, int32_t ldg) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(X, "X");
        need(G, "G");
        MMOF_CHECK(n >= 1 && K >= 1 && K <= KMAX && ld >= n && ldg >= K, MMOF_ERR_SHAPE, "bad Gram sizes");
        MMOF_CHECK(!nu || eps > 0, MMOF_ERR_INVALID, "eps must be > 0");
        double* w = nullptr;
        if (nu) {
            w = static_cast<double*>(ctx->work("gram_w", sizeof(double) * (size_t)n));
            if (dt == MMOF_F32)
                mm_weights_f64<float>(*ctx, n, (const float*)nu, eps, w);
            else
                mm_weights_f64<double>(*ctx, n, (const double*)nu, eps, w);
        }
        if (dt == MMOF_F32)
            wgram<float>(*ctx, n, K, (const float*)X, ld, w, G, ldg);
        else
            wgram<double>(*ctx, n, K, (const double*)X, ld, w, G, ldg);
        return MMOF_OK;
    });
}

int mmof_weighted_gram_noalloc(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X, int64_t ld,
                               const void* nu, double eps, double* G, int32_t ldg) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(X, "X");
        need(G, "G");
        MMOF_CHECK(n >= 1 && K >= 1 && K <= KMAX_SMALL && ld >= n && ldg >= K, MMOF_ERR_SHAPE, "bad Gram sizes");
        MMOF_CHECK(!nu || (eps > 0 && std::isfinite(eps)), MMOF_ERR_INVALID, "eps must be > 0");
        if (dt == MMOF_F32)
            wgram_noalloc<float>(*ctx, n, K, (const float*)X, ld, (const float*)nu, eps, G, ldg);
        else
            wgram_noalloc<double>(*ctx, n, K, (const double*)X, ld, (const double*)nu, eps, G, ldg);
        return MMOF_OK;
    });
}

int mmof_apply_tdiff(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int transpose, const void* in,
                     void* out) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(in, "in");
        need(out, "out");
        Geom& g = ctx->geom(stack);
        launch_tdiff(*ctx, g, dt, transpose != 0, in, out, false);
        return MMOF_OK;
    });
}

int mmof_reg_weights(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int reg, int64_t n_rows, const void* nu,
                     double eps, double* w2) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(nu, "nu");
        need(w2, "w2");
        MMOF_CHECK(reg >= MMOF_REG_PSI && reg <= MMOF_REG_GS, MMOF_ERR_INVALID, "bad regulariser");
        MMOF_CHECK(eps > 0 && std::isfinite(eps), MMOF_ERR_INVALID, "eps must be > 0");
        Geom& g = ctx->geom(stack);
        MMOF_CHECK(n_rows >= g.gx_len + g.gy_len, MMOF_ERR_SHAPE, "n_rows is below the gradient rows of the stack");
        if (dt == MMOF_F32)
            mm_weights_f64<float>(*ctx, n_rows, (const float*)nu, eps, w2);
        else
            mm_weights_f64<double>(*ctx, n_rows, (const double*)nu, eps, w2);
        if (reg == MMOF_REG_ISO || reg == MMOF_REG_GS) launch_group_weights(*ctx, g, dt, reg, nu, eps, w2);
        return MMOF_OK;
    });
}

int mmof_block_dot(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X, int64_t ld, const double* y,
                   double* out) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(X, "X");
        need(y, "y");
        need(out, "out");
        MMOF_CHECK(n >= 1 && K >= 1 && K <= KMAX && ld >= n, MMOF_ERR_SHAPE, "bad block sizes");
        if (dt == MMOF_F32)
            mdot<float, double>(*ctx, n, K, (const float*)X, ld, y, 1.0, out);
        else
            mdot<double, double>(*ctx, n, K, (const double*)X, ld, y, 1.0, out);
        return MMOF_OK;
    });
}

int mmof_block_combine(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X, int64_t ld,
                       const double* z, double alpha, const double* y, double beta, double* out) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need_dt(dt);
        need(X, "X");
        need(z, "z");
        need(out, "out");
        MMOF_CHECK(n >= 1 && K >= 1 && K <= KMAX && ld >= n, MMOF_ERR_SHAPE, "bad block sizes");
        if (dt == MMOF_F32)
            gemv_fused<float, float>(*ctx, n, K, (const float*)X, ld, z, alpha, y, beta, out, nullptr, nullptr,
                                     nullptr);
        else
            gemv_fused<double, double>(*ctx, n, K, (const double*)X, ld, z, alpha, y, beta, out, nullptr, nullptr,
                                       nullptr);
        return MMOF_OK;
    });
}

int mmof_reorth(mmof_ctx ctx, int64_t n, int32_t K, const double* Q, int64_t ld, double* x, double* sq,
                int32_t mode) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need(Q, "Q");
        need(x, "x");
        need(sq, "sq");
        MMOF_CHECK(n >= 1 && K >= 1 && K <= KMAX && ld >= n, MMOF_ERR_SHAPE, "bad block sizes");
        MMOF_CHECK(mode == MMOF_REORTH_AUTO || mode == MMOF_REORTH_TWICE, MMOF_ERR_INVALID, "bad reorth mode");
        double* h = static_cast<double*>(ctx->work("cgs2_h", sizeof(double) * (KMAX + 1)));
        if (mode == MMOF_REORTH_AUTO) {
            cgs_once(*ctx, n, K, Q, ld, x, sq, h);
            return MMOF_OK;
        }
        double* y = static_cast<double*>(ctx->work("cgs2_y", sizeof(double) * (size_t)n));
        mdot<double, double>(*ctx, n, K, Q, ld, x, 1.0, h);
        if (K <= KMAX_SMALL) {
            gemv_mdot(*ctx, n, K, Q, ld, h, x, y, h);
        } else {
            gemv_fused<double, double>(*ctx, n, K, Q, ld, h, -1.0, x, 1.0, y, nullptr, nullptr, nullptr);
            mdot<double, double>(*ctx, n, K, Q, ld, y, 1.0, h);
        }
        gemv_fused<double, double>(*ctx, n, K, Q, ld, h, -1.0, y, 1.0, x, nullptr, nullptr, sq);
        return MMOF_OK;
    });
}

int mmof_cgs2(mmof_ctx ctx, int64_t n, int32_t K, const double* Q, int64_t ld, double* x, double* sq) {
    return mmof_reorth(ctx, n, K, Q, ld, x, sq, MMOF_REORTH_TWICE);
}

int mmof_basis_extend(mmof_ctx ctx, int64_t n, int32_t K, const double* Vs, int64_t ld, double* r, double* T,
                      double* sq) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need(Vs, "Vs");
        need(r, "r");
        need(T, "T");
        need(sq, "sq");
        MMOF_CHECK(n >= 1 && K >= 1 && K < KMAX && ld >= n, MMOF_ERR_SHAPE, "bad block sizes");
        double* h = static_cast<double*>(ctx->work("cgs2_h", sizeof(double) * (KMAX + 1)));
        basis_extend(*ctx, n, K, Vs, ld, r, T, h, sq);
        return MMOF_OK;
    });
}

int mmof_projected_solve(mmof_ctx ctx, int32_t K, const double* GA, const double* GT, const double* d,
                         const double* sc, double fixed_lambda, double* z, double* res) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        need(GA, "GA");
        need(GT, "GT");
        need(d, "d");
        need(sc, "sc");
        need(z, "z");
        need(res, "res");
        small_solve(*ctx, K, GA, GT, d, sc, fixed_lambda, z, res);
        return MMOF_OK;
    });
}

// ------------------------------------------------------------------ measurement

int mmof_profile_kernel(mmof_ctx ctx, const char* kernel_name) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        MMOF_HIP(hipStreamSynchronize(ctx->stream));
        for (auto& e : ctx->timer.events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        ctx->timer.events.clear();
        ctx->timer.launches = 0;
        ctx->timer.total_ms = 0.0;
        ctx->timer.bytes = ctx->timer.flops = 0.0;
        ctx->timer.name = kernel_name ? kernel_name : "";
        return MMOF_OK;
    });
}

int mmof_kernel_timing(mmof_ctx ctx, int64_t* launches, double* total_ms, double* alg_bytes, double* alg_flops) {
    return guarded(ctx, [&] {
        need(ctx, "ctx");
        MMOF_HIP(hipStreamSynchronize(ctx->stream));
        for (auto& e : ctx->timer.events) {
            float ms = 0.f;
            MMOF_HIP(hipEventElapsedTime(&ms, e.first, e.second));
            ctx->timer.total_ms += ms;
            ctx->timer.launches += 1;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        ctx->timer.events.clear();
        if (launches) *launches = ctx->timer.launches;
        if (total_ms) *total_ms = ctx->timer.total_ms;
        if (alg_bytes) *alg_bytes = ctx->timer.bytes;
        if (alg_flops) *alg_flops = ctx->timer.flops;
        return MMOF_OK;
    });
}

}  // extern "C"
