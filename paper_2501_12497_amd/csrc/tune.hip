// Tile-shape autotuner of the stencil kernels.  For a plan's stack and a dtype it times every
// candidate of blur (blur plans), the projector's angle grouping (Radon plans), Psi, Psi^T,
// L(v) and L(v)^T on scratch buffers of the stack's sizes (HIP events on the context's
// stream, a warm-up launch then TUNE_REPS timed launches per candidate) and records the
// fastest candidate in the plan's geometry, where the launchers find it.  The stencil
// candidates compute the same values (the per-pixel arithmetic and summation order do not
// depend on the tile shape); the projector's angle groups split a ray's rows differently,
// which changes its sum by rounding only.
#include <cstdio>
#include <string>
#include <vector>

#include "kernels.h"
#include "krylov.h"
#include "tune.h"

namespace mmof {

static constexpr int TUNE_REPS = 5;

template <class F>
static float time_launches(Ctx& c, F&& launch) {
    launch();  // warm-up (also builds the candidate's tile list outside the timed region)
    hipEvent_t a, b;
    MMOF_HIP(hipEventCreate(&a));
    MMOF_HIP(hipEventCreate(&b));
    MMOF_HIP(hipEventRecord(a, c.stream));
    for (int r = 0; r < TUNE_REPS; ++r) launch();
    MMOF_HIP(hipEventRecord(b, c.stream));
    MMOF_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    MMOF_HIP(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / TUNE_REPS;
}

template <class F>
static int pick(Ctx& c, Geom& g, const char* name, int dt, int n_cand, const TileShape* shapes, F&& launch,
                std::string& report) {
    // (shapes: the tile of each candidate, for the report)
    int best = 0;
    float best_ms = 0.f;
    for (int k = 0; k < n_cand; ++k) {
        const float ms = time_launches(c, [&] { launch(k); });
        if (k == 0 || ms < best_ms) {
            best = k;
            best_ms = ms;
        }
    }
    g.tuned[std::string(name) + (dt == MMOF_F32 ? "/f32" : "/f64")] = best;
    char buf[128];
    std::snprintf(buf, sizeof buf, "%s=%dx%d%s(%.1fus) ", name, shapes[best].tw, shapes[best].th,
                  shapes[best].persistent ? "p" : "", best_ms * 1e3);
    report += buf;
    return best;
}

// The stack-level operator calls of the context (Psi, L(v), ...) use the context's cached
// geometry of the stack, not the plan's copy: the plan's choices are mirrored there.
static void share_choices(Plan& P) {
    Geom& pg = *P.geom;
    const mmof_stack s{pg.n_seq, pg.n_t.data(), pg.ny.data(), pg.nx.data()};
    Geom& g = P.ctx->geom(&s);  // (created if the context has not seen the stack yet)
    if (&g != &pg) g.tuned = pg.tuned;
}

std::string autotune(Plan& P, int dt) {
    Ctx& c = *P.ctx;
    Geom& g = *P.geom;
    const size_t es = dt == MMOF_F32 ? 4 : 8;
    // scratch operands: a smooth-free zero image and zero flows (displacement radius 1)
    void* u = c.work("tune_u", es * (size_t)g.n);
    void* o = c.work("tune_o", es * (size_t)g.n);
    void* gx = c.work("tune_gx", es * (size_t)std::max<int64_t>(g.gx_len, 1));
    void* gy = c.work("tune_gy", es * (size_t)std::max<int64_t>(g.gy_len, 1));
    const int64_t P2 = std::max<int64_t>(2 * g.pair_px, 1);
    void* v = c.work("tune_v", es * (size_t)P2);
    void* r = c.work("tune_r", es * (size_t)std::max<int64_t>(g.pair_px, 1));
    int32_t* rad = static_cast<int32_t*>(c.work("tune_rad", 256));
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        fill_zero<T>(c, g.n, (T*)u);
        fill_zero<T>(c, P2, (T*)v);
        fill_zero<T>(c, std::max<int64_t>(g.pair_px, 1), (T*)r);
    });
    std::string rep;
    if (P.kind == 1)
        pick(c, g, "blur", dt, kBlurCandidates, kBlurShapes, [&](int k) { launch_blur(c, P, dt, u, o, k); }, rep);
    if (P.kind == 0) {
        // angle groups of 1, 2, 4, 8 per workgroup, reported as "<angles>x<row blocks>"
        static const TileShape groups[] = {{1, 8, 0}, {2, 4, 0}, {4, 2, 0}, {8, 1, 0}};
        void* sino = c.work("tune_b", es * (size_t)std::max<int64_t>(P.m, 1));
        pick(c, g, "radon_fwd", dt, kRadonCandidates, groups,
             [&](int k) { launch_radon_fwd(c, P, dt, u, sino, k); }, rep);
    }
    std::vector<TileShape> gsh, fsh;
    for (int k = 0; k < kGradCandidates; ++k) gsh.push_back(grad_tile(g, k));
    for (int k = 0; k < kFlowCandidates; ++k) fsh.push_back(flow_tile(g, k));
    pick(c, g, "grad_fwd", dt, kGradCandidates, gsh.data(),
         [&](int k) { launch_grad_fwd(c, g, dt, u, nullptr, nullptr, gx, gy, k); }, rep);
    pick(c, g, "grad_adj", dt, kGradCandidates, gsh.data(),
         [&](int k) { launch_grad_adj(c, g, dt, gx, gy, nullptr, nullptr, o, false, k); }, rep);
    if (g.n_pairs > 0) {
        launch_flow_radius(c, g, dt, v, rad);
        pick(c, g, "flow_fwd", dt, kFlowCandidates, fsh.data(),
             [&](int k) { launch_flow_fwd(c, g, dt, +1, MMOF_INTERP_BILINEAR, u, v, r, k); }, rep);
        pick(c, g, "flow_adj", dt, kFlowAdjCandidates, kFlowAdjShapes,
             [&](int k) { launch_flow_adj(c, g, dt, +1, MMOF_INTERP_BILINEAR, r, v, o, true, rad, k); }, rep);
    }
    MMOF_HIP(hipStreamSynchronize(c.stream));
    share_choices(P);
    if (!rep.empty()) rep.pop_back();
    return rep;
}

void set_tile(Plan& P, const std::string& kernel, int dt, int choice) {
    int n = kernel == "blur" ? kBlurCandidates
            : kernel == "radon_fwd" ? kRadonCandidates
            : (kernel == "grad_fwd" || kernel == "grad_adj") ? kGradCandidates
            : kernel == "flow_fwd" ? kFlowCandidates
            : kernel == "flow_adj" ? kFlowAdjCandidates
                                   : 0;
    MMOF_CHECK(n > 0, MMOF_ERR_INVALID, "unknown tunable kernel '" + kernel + "'");
    MMOF_CHECK(choice >= 0 && choice < n, MMOF_ERR_INVALID, "tile candidate out of range for " + kernel);
    P.geom->tuned[kernel + (dt == MMOF_F32 ? "/f32" : "/f64")] = choice;
    share_choices(P);
}

}  // namespace mmof
