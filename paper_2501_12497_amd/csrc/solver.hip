// MMGKS-OF driver (Alg. 1): flow update every tau iterations, MM weights, projected
// Gram matrices, discrepancy-principle lambda, u = V z, residual of the weighted normal
// equations, CGS2 against V, subspace growth.  All work runs on the context's stream;
// the host reads back one small report per iteration.
//
// Precision: operator applications (H, H^T, Theta, Theta^T, flow update) run in TX
// (float or double); the Krylov basis V, the Golub-Kahan start, all inner products,
// the Gram matrices, the projected solve and lambda are FP64.  H V and Theta V are kept
// in TX (they are operator outputs) and are accumulated in FP64.
//
// Theta = [Psi; L_t; M-bar(v); M-bar'(v')] (the blocks the regulariser and the flow use) is
// stored row block after row block:
// [gx (all frames) | gy (all frames) | temporal differences | forward flow rows | reverse flow rows].
// The MM weights are per row (l1) or per group of rows (IsoTV, GS: Sec. 5, table of methods).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "kernels.h"
#include "krylov.h"
#include "solver.h"

namespace mmof {

// One phase of a solve: outer iterations [k_begin, k_end) in one operator precision.
// A phase that starts from a previous one takes over its Krylov basis (K_in columns of the
// shared FP64 workspace) and its flows (converted to this phase's precision).
struct Phase {
    int k_begin = 0, k_end = 0;
    bool final = true;             // the last phase: no subspace growth after its last iteration
    int K_in = 0;                  // 0: start with Golub-Kahan
    bool start_only = false;       // build the Golub-Kahan basis V and return
    int start_av = 0;              // columns j < start_av of H V come from the Golub-Kahan start's
                                   // FP64 products (kept in the shared FP64 workspace)
    const void* v_in = nullptr;    // flows of the previous phase (NULL: zero flows)
    const void* vr_in = nullptr;
    int in_dt = MMOF_F32;
    int out_dt = MMOF_F32;         // dtype of v_out / v_rev_out
};

struct PhaseOut {
    int status = 0, K = 0, iters = 0;
    bool stopped = false;          // RRE target reached or breakdown
    const void* flow_v = nullptr;
    const void* flow_vr = nullptr;
};

// Destroys a HIP event when the scope ends.
struct EventGuard {
    hipEvent_t e = nullptr;
    ~EventGuard() {
        if (e) (void)hipEventDestroy(e);
    }
};

template <class TX>
struct Solver {
    Ctx& c;
    Plan& P;
    Geom& g;
    const mmof_solve_params& p;
    int dt;
    int64_t n, m, R, oGX, oGY, oTD, oRF, oRR;
    int Kcap;
    bool flow;
    bool tdiff;  // Theta holds the temporal differences L_t (AnisoTV, IsoTV)
    mmof_report* rep;

    // workspace
    double *V, *U, *r, *tmp_n, *tmp_m, *GA, *GT, *dvec, *z, *h, *sc, *res, *scal;
    double* AVs;  // H v_j of the Golub-Kahan start (FP64, columns 0 .. ell-2)
    // implicit basis (MMOF_REORTH_IMPLICIT): V = Vs T with the stored columns Vs (the buffer V)
    // and T unit upper triangular; G_H, d and G_T are formed for Vs (GAs, ds, GTs) and mapped
    // to V (GA, dvec, GT) before each projected solve, and u = V z = Vs (T z) (zt = T z).
    // Otherwise Vs = V, T = I: GAs, ds and GTs alias GA, dvec and GT, and zt is a copy of z.
    // zt_prev keeps the previous projected solve's coefficients (the iterate a stop returns
    // when the next solve was already queued).
    bool implicit = false;
    double *Tb = nullptr, *GAs = nullptr, *GTs = nullptr, *ds = nullptr, *zt = nullptr, *zt_prev = nullptr;
    TX *AV, *TV, *u_op, *vin_n, *vin_m, *out_n, *out_n2, *nu, *yR, *yW, *flow_v, *flow_vr, *flow_tmp, *I;
    // FP32 operators with flows: every column of V also in the operator precision (V32, its
    // rounding, written where the column is formed), which the rebuild of Theta V's flow rows
    // reads instead of the FP64 columns
    bool col_op = false;
    TX* V32 = nullptr;
    TX* col_in(int j) { return col_op ? V32 + (int64_t)j * n : vin_n; }
    // flow on reduced frames: their geometry (owned by the plan), frames and flow
    int fscale = 1;
    Geom* gs = nullptr;
    TX *flow_us = nullptr, *flow_vs = nullptr;
    FlowMethod fm;
    GksWork gks;
    double* w2;  // FP64 MM weights of the rows of Theta
    int32_t *rad_v, *rad_vr;
    double* host;  // pinned report staging

    Solver(Ctx& c_, Plan& P_, const mmof_solve_params& p_, mmof_report* rep_)
        : c(c_), P(P_), g(*P_.geom), p(p_), rep(rep_) {
        dt = std::is_same<TX, float>::value ? MMOF_F32 : MMOF_F64;
        n = P.n;
        m = P.m;
        flow = p.use_flow != 0;
        tdiff = p.reg == MMOF_REG_ANISO || p.reg == MMOF_REG_ISO;
        oGX = 0;
        oGY = g.gx_len;
        oTD = g.gx_len + g.gy_len;
        oRF = oTD + (tdiff ? g.pair_px : 0);
        oRR = oRF + (flow ? g.pair_px : 0);
        R = oRR + ((flow && p.use_reverse) ? g.pair_px : 0);
        Kcap = p.ell + p.k_max - 1;
        fscale = resolve_flow_scale(g, p.flow_scale);
        fm.solver = p.flow_solver;
        fm.n_sweeps = p.n_sweeps;
        fm.ell = p.of_ell;
        fm.n_iter = p.of_iters;
        implicit = p.reorth == MMOF_REORTH_IMPLICIT;
        if (flow && fscale > 1) {
            auto& r = P.reduced[fscale];
            if (!r) r = make_reduced_geom(g, fscale, c.stream);
            gs = r.get();
        }
    }

    // FP64 buffers (the Krylov state) are shared by both operator precisions, so an FP32
    // phase can hand its basis to an FP64 refinement phase; operator-precision buffers are
    // kept apart per precision.
    template <class T>
    T* ws(const char* name, int64_t count) {
        const char* tag = std::is_same<T, TX>::value && !std::is_same<TX, double>::value ? "solve_f_" : "solve_";
        return static_cast<T*>(c.work(std::string(tag) + name, sizeof(T) * (size_t)std::max<int64_t>(count, 1)));
    }
    TX* wsx(const char* name, int64_t count) {
        return static_cast<TX*>(c.work(std::string(std::is_same<TX, float>::value ? "solve_f_" : "solve_d_") + name,
                                       sizeof(TX) * (size_t)std::max<int64_t>(count, 1)));
    }

    // full = false: only what the Golub-Kahan start needs
    void alloc(bool full) {
        V = ws<double>("V", (int64_t)Kcap * n);
        U = ws<double>("U", (int64_t)(p.ell + 1) * m);
        AVs = ws<double>("AVs", (int64_t)std::max(1, p.ell - 1) * m);
        r = ws<double>("r", n);
        tmp_m = ws<double>("tmp_m", m);
        h = ws<double>("h", KMAX + 1);
        sc = ws<double>("sc", 8);
        scal = ws<double>("scal", 24);
        vin_n = wsx("vin_n", n);
        vin_m = wsx("vin_m", m);
        out_n = wsx("out_n", n);
        host = static_cast<double*>(c.pinned(64 * sizeof(double)));
        fill_zero<double>(c, 24, scal);
        if (!full) return;
        tmp_n = ws<double>("tmp_n", n);
        GA = ws<double>("GA", KLD * KLD);
        GT = ws<double>("GT", KLD * KLD);
        dvec = ws<double>("dvec", KMAX);
        z = ws<double>("z", KMAX);
        res = ws<double>("res", 8);
        zt = ws<double>("zt", KMAX);
        zt_prev = ws<double>("zt_prev", KMAX);
        if (implicit) {
            Tb = ws<double>("T", (int64_t)KLD * KLD);
            GAs = ws<double>("GAs", KLD * KLD);
            GTs = ws<double>("GTs", KLD * KLD);
            ds = ws<double>("ds", KMAX);
        } else {
            GAs = GA;
            GTs = GT;
            ds = dvec;
        }
        AV = wsx("AV", (int64_t)Kcap * m);
        TV = wsx("TV", (int64_t)Kcap * R);
        col_op = flow && std::is_same<TX, float>::value;
        if (col_op) V32 = wsx("V32", (int64_t)Kcap * n);
        u_op = wsx("u_op", n);
        out_n2 = wsx("out_n2", n);
        nu = wsx("nu", R);
        yR = wsx("yR", R);
        yW = wsx("yW", R);
        w2 = ws<double>("w2", R);
        flow_v = wsx("flow_v", 2 * g.pair_px);
        flow_vr = wsx("flow_vr", 2 * g.pair_px);
        const Geom& gw = gs ? *gs : g;  // frames the flow sweeps run on
        flow_tmp = wsx("flow_tmp", 2 * gw.pair_px);
        I = wsx("I", 3 * gw.pair_px);
        if (gs) {
            flow_us = wsx("flow_us", gs->n);
            flow_vs = wsx("flow_vs", 2 * gs->pair_px);
        }
        if (flow && fm.solver == MMOF_FLOW_GKS) gks = gks_work(c, gw, fm, "solve_gks_");
        rad_v = ws<int32_t>("rad_v", 64);
        rad_vr = ws<int32_t>("rad_vr", 64);
    }

    // ---------------------------------------------------------------- operators (TX)
    void A(const TX* in, TX* out) {
        if (P.kind == 0)
            launch_radon_fwd(c, P, dt, in, out);
        else if (P.kind == 2)
            launch_fan_fwd(c, P, dt, in, out);
        else
            launch_blur(c, P, dt, in, out);
        if (rep) rep->n_A++;
    }
    void At(const TX* in, TX* out) {
        if (P.kind == 0)
            launch_radon_adj(c, P, dt, in, out);
        else if (P.kind == 2)
            launch_fan_adj(c, P, dt, in, out);
        else
            launch_blur(c, P, dt, in, out);
        if (rep) rep->n_At++;
    }
    void theta_flow(const TX* in, TX* out) {
        if (!flow) return;
        launch_flow_fwd(c, g, dt, +1, p.interp, in, flow_v, out + oRF);
        if (p.use_reverse) launch_flow_fwd(c, g, dt, -1, p.interp, in, flow_vr, out + oRR);
        if (rep) rep->n_L += p.use_reverse ? 2 : 1;
    }
    void theta(const TX* in, TX* out) {
        launch_grad_fwd(c, g, dt, in, nullptr, nullptr, out + oGX, out + oGY);
        if (tdiff) launch_tdiff(c, g, dt, false, in, out + oTD, false);
        theta_flow(in, out);
        if (rep) rep->n_theta++;
    }
    // theta(in, out) and, in the same kernels, its rows weighted by the MM weights of nu_
    // (1/sqrt(nu^2 + eps^2)) into outw: the residual's W Theta u without a pass of its own
    // (per-row weights from nu, no temporal-difference rows)
    void theta_weighted(const TX* in, TX* out, const TX* nu_, TX* outw) {
        const double eps2 = p.eps * p.eps;
        RowWeighting gw;
        gw.nu_a = nu_ + oGX;
        gw.m_a = outw + oGX;
        gw.nu_b = nu_ + oGY;
        gw.m_b = outw + oGY;
        gw.eps2 = eps2;
        launch_grad_fwd(c, g, dt, in, nullptr, nullptr, out + oGX, out + oGY, -1, &gw);
        if (flow) {
            RowWeighting fw;
            fw.nu_a = nu_ + oRF;
            fw.m_a = outw + oRF;
            fw.eps2 = eps2;
            launch_flow_fwd(c, g, dt, +1, p.interp, in, flow_v, out + oRF, -1, &fw);
            if (p.use_reverse) {
                RowWeighting rw;
                rw.nu_a = nu_ + oRR;
                rw.m_a = outw + oRR;
                rw.eps2 = eps2;
                launch_flow_fwd(c, g, dt, -1, p.interp, in, flow_vr, out + oRR, -1, &rw);
            }
            if (rep) rep->n_L += p.use_reverse ? 2 : 1;
        }
        if (rep) rep->n_theta++;
    }
    // out = Theta^T in; with res (only when flows are on: the last flow adjoint forms it), the
    // residual res->out = res->x + lambda out instead of out.  Returns whether it was formed.
    bool thetaT(const TX* in, TX* out, const ResidualOut* res = nullptr) {
        launch_grad_adj(c, g, dt, in + oGX, in + oGY, nullptr, nullptr, out, false);
        if (tdiff) launch_tdiff(c, g, dt, true, in + oTD, out, true);
        bool formed = false;
        if (flow) {
            launch_flow_adj(c, g, dt, +1, p.interp, in + oRF, flow_v, out, true, rad_v, -1,
                            p.use_reverse ? nullptr : res);
            if (p.use_reverse) launch_flow_adj(c, g, dt, -1, p.interp, in + oRR, flow_vr, out, true, rad_vr, -1, res);
            if (rep) rep->n_L += p.use_reverse ? 2 : 1;
            formed = res != nullptr;
        }
        if (rep) rep->n_thetaT++;
        return formed;
    }

    // FP64 MM weights of the rows of Theta u: per row, then per group for IsoTV and GS.  Per-row
    // weights of a Gram with at most KMAX_SMALL columns are not stored: wsrc = nu_, and the
    // Gram and the residual form each weight 1/sqrt(nu^2 + eps^2) from it (the buffer would
    // cost a pass of 12 bytes per row and 4 more bytes per row in each of its two readers).
    const TX* wsrc = nullptr;
    void weights(const TX* nu_, double* w, int Kg) {
        const bool grouped = p.reg == MMOF_REG_ISO || p.reg == MMOF_REG_GS;
        if (!grouped && Kg <= KMAX_SMALL) {
            wsrc = nu_;
            return;
        }
        wsrc = nullptr;
        mm_weights_f64<TX>(c, R, nu_, p.eps, w);
        if (grouped) launch_group_weights(c, g, dt, p.reg, nu_, p.eps, w);
    }
    // G_T = (P Theta V)^T (P Theta V) for the first Kg columns, with the weights of weights()
    void gram_theta(int Kg, const TX* TV_, const double* w, double* GT_) {
        if (wsrc)
            wgram_nu<TX>(c, R, Kg, TV_, R, wsrc, p.eps, GT_, KLD);
        else
            wgram<TX>(c, R, Kg, TV_, R, w, GT_, KLD);
    }

    // ---------------------------------------------------------------- graphs
    // Runs body, a launch sequence whose launches depend only on `key`: eagerly on its first
    // use (which also creates its tile lists and workspaces), captured into a graph and
    // launched on its second, replayed from the plan's cache afterwards.  The report
    // counters the body increments are added again on every replay; kernels inside a graph
    // are not event-timed.
    template <class F>
    void replayable(const std::string& key, F&& body) {
        if (!p.use_graph) {
            body();
            return;
        }
        auto it = P.graphs.find(key);
        if (it != P.graphs.end()) {
            MMOF_HIP(hipGraphLaunch(it->second.exec, c.stream));
            if (rep) {
                rep->n_A += it->second.dA;
                rep->n_At += it->second.dAt;
                rep->n_theta += it->second.dTheta;
                rep->n_thetaT += it->second.dThetaT;
                rep->n_L += it->second.dL;
            }
            return;
        }
        if (P.graph_seen[key]++ == 0) {
            body();
            return;
        }
        mmof_report before{};
        if (rep) before = *rep;
        if (!c.capture_stream) MMOF_HIP(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking));
        // the launchers use c.stream: point it at the capture stream while the body records
        hipGraph_t gr = nullptr;
        const hipStream_t launch_stream = c.stream;
        MMOF_HIP(hipStreamBeginCapture(c.capture_stream, hipStreamCaptureModeThreadLocal));
        c.stream = c.capture_stream;
        c.capturing = true;
        try {
            body();
        } catch (...) {
            c.capturing = false;
            c.stream = launch_stream;
            (void)hipStreamEndCapture(c.capture_stream, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            (void)hipGetLastError();
            throw;
        }
        c.capturing = false;
        c.stream = launch_stream;
        MMOF_HIP(hipStreamEndCapture(c.capture_stream, &gr));
        CachedGraph cg;
        const hipError_t e = hipGraphInstantiate(&cg.exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        MMOF_CHECK(e == hipSuccess, MMOF_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        if (rep) {
            cg.dA = rep->n_A - before.n_A;
            cg.dAt = rep->n_At - before.n_At;
            cg.dTheta = rep->n_theta - before.n_theta;
            cg.dThetaT = rep->n_thetaT - before.n_thetaT;
            cg.dL = rep->n_L - before.n_L;
        }
        P.graphs[key] = cg;
        MMOF_HIP(hipGraphLaunch(cg.exec, c.stream));
    }
    std::string graph_key(const char* what) const {
        char buf[1024];
        std::snprintf(buf, sizeof buf,
                      "%s|%d|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%d|%d|%d|%d|%a|%lld|%lld", what, dt,
                      (void*)u_op, (void*)I, (void*)flow_v, (void*)flow_tmp, (void*)flow_vr, (void*)rad_v,
                      (void*)rad_vr, (void*)vin_m, (void*)out_n, (void*)out_n2, (void*)w2, (void*)r, (void*)scal,
                      (void*)flow_us, (void*)flow_vs, p.interp, p.use_reverse, p.n_sweeps, p.delta_r, fscale,
                      p.alpha, (long long)n, (long long)R);
        std::snprintf(buf + std::strlen(buf), sizeof buf - std::strlen(buf), "|reg%d", p.reg);
        if (fm.solver == MMOF_FLOW_GKS) {
            std::snprintf(buf + std::strlen(buf), sizeof buf - std::strlen(buf), "|gks|%d|%d|%p|%p|%p|%p|%p", fm.ell,
                          fm.n_iter, (void*)gks.V, (void*)gks.U, (void*)gks.S, (void*)gks.R, (void*)gks.lam);
        }
        std::string key(buf);
        for (const auto& t : g.tuned) key += "|" + t.first + "=" + std::to_string(t.second);  // tile lists used
        return key;
    }

    // ---------------------------------------------------------------- Krylov helpers (FP64)
    void norm_into(int64_t len, const double* x, double* out) {  // out = ||x||^2
        mdot<double, double>(c, len, 1, x, len, x, 1.0, out);
    }
    // x <- x - Q (Q^T x) (Q has k columns of length len), once more when the first pass
    // removed most of x (MMOF_REORTH_AUTO) or always (MMOF_REORTH_TWICE); sq[0] = ||x||^2
    // afterwards
    void reorth(int64_t len, const double* Q, int k, double* x, double* sq) {
        if (k <= 0) {
            norm_into(len, x, sq);
            return;
        }
        if (p.reorth != MMOF_REORTH_TWICE) {
            cgs_once(c, len, k, Q, len, x, sq, h);
            return;
        }
        // h = Q^T x; y = x - Q h and h = Q^T y in one pass over Q; x = y - Q h with ||x||^2
        double* y = static_cast<double*>(c.work("reorth_y", sizeof(double) * (size_t)std::max<int64_t>(len, 1)));
        mdot<double, double>(c, len, k, Q, len, x, 1.0, h);
        if (k <= KMAX_SMALL) {
            gemv_mdot(c, len, k, Q, len, h, x, y, h);
        } else {
            // (beyond the fused pass's register budget: the two steps as separate passes)
            gemv_fused<double, double>(c, len, k, Q, len, h, -1.0, x, 1.0, y, nullptr, nullptr, nullptr);
            mdot<double, double>(c, len, k, Q, len, y, 1.0, h);
        }
        gemv_fused<double, double>(c, len, k, Q, len, h, -1.0, y, 1.0, x, nullptr, nullptr, sq);
    }

    // H v_j, the row/column j of G_H, d_j = (H v_j)^T b and Theta v_j; col_in(j) already holds
    // v_j in TX when have_vin.  For j < start_av, H v_j is the Golub-Kahan start's FP64 product
    // (rounded to TX) instead of a new application of H.
    void add_column(int j, bool have_vin, int start_av = 0) {
        TX* vj = col_in(j);
        if (!have_vin) convert<double, TX>(c, n, V + (int64_t)j * n, vj);
        TX* avj = AV + (int64_t)j * m;
        if (j < start_av)
            convert<double, TX>(c, m, AVs + (int64_t)j * m, avj);
        else
            A(vj, avj);
        gram_row<TX>(c, m, j, AV, m, b, GAs, KLD, ds + j);
        theta(vj, TV + (int64_t)j * R);
    }

    // The Gram matrices and d of the true basis from those of the stored columns, the
    // projected solve, and the coefficients of u = V z in the stored columns.
    void projected(int Kg) {
        if (implicit) {
            basis_gram(c, Kg, Tb, GAs, ds, GA, dvec);
            basis_gram(c, Kg, Tb, GTs, nullptr, GT, nullptr);
        }
        small_solve(c, Kg, GA, GT, dvec, sc, p.fixed_lambda, z, scal + 8, sc + 2);
        std::swap(zt, zt_prev);
        if (implicit)
            basis_coef(c, Kg, Tb, z, zt);
        else
            MMOF_HIP(hipMemcpyAsync(zt, z, sizeof(double) * (size_t)Kg, hipMemcpyDeviceToDevice, c.stream));
    }
    // The new direction r against the basis of K columns: ||r'||^2 into sq; r' / ||r'|| becomes
    // column K of V (explicit passes) or of Vs (implicit basis: r' = r, T gets column K).
    void extend(int K, double* sq) {
        if (implicit)
            basis_extend(c, n, K, V, n, r, Tb, h, sq);
        else
            reorth(n, V, K, r, sq);
    }

    const double* b = nullptr;

    // With MMOF_DUMP_PROJECTED=<path>, a failed projected solve writes K, G_H, G_T, d and the
    // scalars (binary doubles) for offline inspection.
    void dump_projected(int K) {
        const char* path = std::getenv("MMOF_DUMP_PROJECTED");
        if (!path) return;
        std::vector<double> buf(2 * KLD * KLD + KMAX + 8);
        (void)hipStreamSynchronize(c.stream);
        (void)hipMemcpy(buf.data(), GA, sizeof(double) * KLD * KLD, hipMemcpyDeviceToHost);
        (void)hipMemcpy(buf.data() + KLD * KLD, GT, sizeof(double) * KLD * KLD, hipMemcpyDeviceToHost);
        (void)hipMemcpy(buf.data() + 2 * KLD * KLD, dvec, sizeof(double) * KMAX, hipMemcpyDeviceToHost);
        (void)hipMemcpy(buf.data() + 2 * KLD * KLD + KMAX, sc, sizeof(double) * 3, hipMemcpyDeviceToHost);
        if (FILE* f = std::fopen(path, "wb")) {
            const double kk = K;
            std::fwrite(&kk, sizeof(double), 1, f);
            std::fwrite(buf.data(), sizeof(double), buf.size(), f);
            std::fclose(f);
        }
    }

    PhaseOut run(const double* b_, double delta, double* u_io, void* v_out, void* vr_out, const Phase& ph) {
        b = b_;
        MMOF_CHECK(Kcap >= 1 && Kcap <= KMAX, MMOF_ERR_SHAPE,
                   "ell + k_max - 1 must be in [1, " + std::to_string(KMAX) + "]");
        MMOF_CHECK(p.ell >= 1 && p.k_max >= 1 && p.tau >= 1, MMOF_ERR_INVALID, "ell, k_max, tau must be >= 1");
        MMOF_CHECK(!flow || p.n_sweeps >= 0, MMOF_ERR_INVALID, "n_sweeps must be >= 0");
        MMOF_CHECK(p.eps > 0 && p.alpha > 0 && p.eta > 0, MMOF_ERR_INVALID, "eps, alpha, eta must be > 0");
        alloc(!ph.start_only);
        // scalars: sc[0] = ||b||^2, sc[1] = (eta delta)^2, sc[2] = previous lambda
        norm_into(m, b, sc);
        set_scalar(c, sc + 1, (p.eta * delta) * (p.eta * delta));
        if (ph.k_begin == 0) set_scalar(c, sc + 2, 0.0);  // a later phase keeps the previous lambda

        // ||H^T b|| for the breakdown test
        convert<double, TX>(c, m, b, vin_m);
        At(vin_m, out_n);
        mdot<TX, TX>(c, n, 1, out_n, n, out_n, 1.0, scal + 4);
        // RRE denominator
        if (p.u_true) norm_into(n, p.u_true, scal + 5);
        // squared norms of the inputs (scal[6], scal[7] are free until the first report): a NaN
        // or an infinity anywhere in b or u_inout makes its norm non-finite
        copy_scalar(c, scal + 6, sc);
        norm_into(n, u_io, scal + 7);
        MMOF_HIP(hipMemcpyAsync(host, scal + 4, 4 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        MMOF_HIP(hipStreamSynchronize(c.stream));
        MMOF_CHECK(std::isfinite(host[2]), MMOF_ERR_NONFINITE, "b holds NaN or Inf (or its norm overflows)");
        MMOF_CHECK(std::isfinite(host[3]), MMOF_ERR_NONFINITE, "u_inout holds NaN or Inf (or its norm overflows)");
        const double atb = std::sqrt(host[0]);
        const double utn = p.u_true ? std::sqrt(host[1]) : 0.0;

        int K = ph.K_in;
        if (K == 0) {
            // ---- Golub-Kahan start: u_1 = b/||b||, ell right vectors, both bases re-orthogonalised
            // scalar slots: scal[0..3] = alpha^2, alpha, beta^2, beta; the normalisations also
            // leave the new vector in the operator precision for the next product
            norm_into(m, b, scal + 12);
            normalize2<TX>(c, m, b, scal + 12, scal + 13, U, vin_m);
            At(vin_m, out_n);
            convert<TX, double>(c, n, out_n, r);
            norm_into(n, r, scal);
            normalize2<TX>(c, n, r, scal, scal + 1, V, vin_n);
            for (int i = 1; i < p.ell; ++i) {
                // w = H v_{i-1} - alpha u_{i-1}; H v_{i-1} is kept as column i-1 of H V
                A(vin_n, vin_m);
                convert<TX, double>(c, m, vin_m, AVs + (int64_t)(i - 1) * m);
                axpy_conv<TX>(c, m, vin_m, U + (int64_t)(i - 1) * m, scal + 1, -1.0, tmp_m);
                reorth(m, U, i, tmp_m, scal + 2);
                normalize2<TX>(c, m, tmp_m, scal + 2, scal + 3, U + (int64_t)i * m, vin_m);
                // v = H^T u_i - beta v_{i-1}
                At(vin_m, out_n);
                axpy_conv<TX>(c, n, out_n, V + (int64_t)(i - 1) * n, scal + 3, -1.0, r);
                reorth(n, V, i, r, scal);
                normalize2<TX>(c, n, r, scal, scal + 1, V + (int64_t)i * n, vin_n);
            }
            K = p.ell;
            if (ph.start_only) {
                MMOF_HIP(hipStreamSynchronize(c.stream));
                PhaseOut out;
                out.K = K;
                return out;
            }
        }

        // ---- state: u^(k), the flows (zero at the start), then H V, G_H, d and Theta V
        convert<double, TX>(c, n, u_io, u_op);
        if (flow) {
            if (!ph.v_in) {
                fill_zero<TX>(c, 2 * g.pair_px, flow_v);
                fill_zero<TX>(c, 2 * g.pair_px, flow_vr);
            } else if (ph.in_dt == MMOF_F32) {
                convert<float, TX>(c, 2 * g.pair_px, (const float*)ph.v_in, flow_v);
                convert<float, TX>(c, 2 * g.pair_px, (const float*)ph.vr_in, flow_vr);
            } else {
                convert<double, TX>(c, 2 * g.pair_px, (const double*)ph.v_in, flow_v);
                convert<double, TX>(c, 2 * g.pair_px, (const double*)ph.vr_in, flow_vr);
            }
            launch_flow_radius(c, g, dt, flow_v, rad_v);
            launch_flow_radius(c, g, dt, flow_vr, rad_vr);
        }
        const int start_av = ph.K_in == 0 ? p.ell - 1 : ph.start_av;
        // the start's columns are orthonormal as stored (a later phase keeps the T it gets)
        if (implicit && ph.k_begin == 0) basis_identity(c, K, Tb);
        for (int j = 0; j < K; ++j) add_column(j, false, start_av);
        int status = 0;
        int iters = 0;
        const double gamma = p.alpha * p.alpha;
        bool stopped = false;
        bool nu_fresh = false;  // nu already holds Theta u^(k) (from the previous residual)
        // report slots: scal[6] = ||u - u_true||^2, scal[7] = ||r||^2, scal[8..11] = lambda,
        // D^2, status, factorizations (written by the projected solve)
        double* res = scal + 8;
        // Steps 2-5 of the next iteration (and the column append that precedes them) change
        // only the solver's own buffers, so they are queued before the host waits for the
        // report of the current iteration: the device keeps working while the host decides
        // whether to stop (a stop discards them; the operator counts they added are taken
        // back).  Not when the next iteration updates the flow (that changes the returned
        // flows) and not while projected systems are being dumped.
        const bool may_queue_ahead = std::getenv("MMOF_DUMP_PROJECTED") == nullptr;
        EventGuard ev_rep;
        MMOF_HIP(hipEventCreateWithFlags(&ev_rep.e, hipEventDisableTiming));
        bool queued = false;  // steps 2-5 of this iteration are already queued
        for (int k = ph.k_begin; k < ph.k_end; ++k) {
            if (!queued) {
                // 1. flow update on u^(k) and rebuild of the flow rows of Theta V
                if (flow && k % p.tau == 0) {
                    replayable(graph_key("flow"), [&] {
                        FlowWork w;
                        w.I = I;
                        w.tmp = flow_tmp;
                        w.us = flow_us;
                        w.vs = flow_vs;
                        w.gks = gks;
                        fm.gamma = gamma;
                        flow_update_core(c, g, gs, dt, u_op, flow_v, fscale, p.delta_r, fm, w);
                        launch_flow_radius(c, g, dt, flow_v, rad_v);
                        if (p.use_reverse) {
                            launch_reverse_flow(c, g, dt, flow_v, flow_vr, rad_v);
                            launch_flow_radius(c, g, dt, flow_vr, rad_vr);
                        }
                    });
                    launch_flow_fwd_cols(c, g, dt, p.interp, col_op ? (const void*)V32 : (const void*)V, col_op, n, K,
                                         flow_v, p.use_reverse ? flow_vr : nullptr, TV, R,
                                         oRF, oRR);
                    if (rep) rep->n_L += (int64_t)K * (p.use_reverse ? 2 : 1);
                    if (rep) rep->n_flow_updates++;
                    nu_fresh = false;
                }
                // 2. nu = Theta u^(k); FP64 weights; weighted Gram of Theta V
                if (!nu_fresh) theta(u_op, nu);
                weights(nu, w2, K);
                gram_theta(K, TV, w2, GTs);
                // 3-5. lambda (discrepancy principle) and z; lambda is kept in sc[2] as the next warm start
                projected(K);
            }
            queued = false;
            // 6. u^(k+1) = V z (the operator copy, ||u - u_true||^2, and the FP64 copy on the phase's
            // last iteration; an earlier stop forms the FP64 copy afterwards)
            const bool write_u = k == ph.k_end - 1;
            gemv_fused<double, TX>(c, n, K, V, n, zt, 1.0, nullptr, 0.0, write_u ? u_io : nullptr, u_op, p.u_true,
                                   p.u_true ? scal + 6 : nullptr);
            const bool last = ph.final && (k == ph.k_end - 1);
            if (!last) {
                // 7. r = H^T (H V z - b) + lambda Theta^T P^2 Theta V z
                gemv_fused<TX, TX>(c, m, K, AV, m, zt, 1.0, b, -1.0, nullptr, vin_m, nullptr, nullptr);
                std::string key = graph_key("residual");
                key += "|" + std::to_string(reinterpret_cast<uintptr_t>(yR)) + "|" +
                       std::to_string(reinterpret_cast<uintptr_t>(yW)) + "|" +
                       std::to_string(reinterpret_cast<uintptr_t>(wsrc));
                replayable(key, [&] {
                    At(vin_m, out_n);
                    if (wsrc && !tdiff) {
                        theta_weighted(u_op, yR, wsrc, yW);
                    } else {
                        theta(u_op, yR);
                        if (wsrc)
                            weight_mul_nu<TX>(c, R, wsrc, p.eps, yR, yW);
                        else
                            weight_mul<TX>(c, R, w2, yR, yW);
                    }
                    ResidualOut ro;
                    ro.x = out_n;
                    ro.lam = res;
                    ro.out = r;
                    if (!thetaT(yW, out_n2, &ro)) residual_combine<TX>(c, n, out_n, out_n2, res, r);
                });
                // 8. r against the basis, ||r'||^2
                extend(K, scal + 7);
                // Theta u^(k+1) is the next iteration's nu unless the flow changes first
                std::swap(nu, yR);
                nu_fresh = true;
            }
            MMOF_HIP(hipMemcpyAsync(host, scal + 6, 6 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
            MMOF_HIP(hipEventRecord(ev_rep.e, c.stream));
            const bool ahead = may_queue_ahead && !last && k + 1 < ph.k_end && !(flow && (k + 1) % p.tau == 0) &&
                               K + 1 <= Kcap;
            mmof_report saved{};
            if (rep) saved = *rep;
            // the coefficients of u^(k+1), whatever is queued next
            const double* zt_k = zt;
            if (ahead) {
                normalize2<TX>(c, n, r, scal + 7, scal + 14, V + (int64_t)K * n, col_in(K));
                add_column(K, true);
                if (!nu_fresh) theta(u_op, nu);
                weights(nu, w2, K + 1);
                gram_theta(K + 1, TV, w2, GTs);
                projected(K + 1);
            }
            // counts of work queued ahead, taken back if the iteration ends the solve
            auto take_back = [&] {
                if (ahead && rep) {
                    rep->n_A = saved.n_A;
                    rep->n_At = saved.n_At;
                    rep->n_theta = saved.n_theta;
                    rep->n_thetaT = saved.n_thetaT;
                    rep->n_L = saved.n_L;
                }
            };
            MMOF_HIP(hipEventSynchronize(ev_rep.e));
            const double rre2 = host[0], rnorm = std::sqrt(std::max(host[1], 0.0));
            const double lam = host[2], D2 = host[3];
            const int st = (int)host[4];
            if (rep) rep->n_factorizations += (int64_t)host[5];
            iters = k + 1;
            if (st == 2) status = std::max(status, (int)MMOF_WARN_DP_CLAMPED);
            if (st == 4) {
                dump_projected(K);
                throw Error(MMOF_ERR_NONFINITE, "projected system is not positive definite (iteration " +
                                                    std::to_string(k) + ", " + std::to_string(K) + " columns)");
            }
            double rre = p.u_true ? std::sqrt(std::max(rre2, 0.0)) / utn : 0.0;
            if (rep && k < rep->capacity) {
                if (rep->lambda) rep->lambda[k] = lam;
                if (rep->resid) rep->resid[k] = std::sqrt(std::max(D2, 0.0));
                if (rep->rre) rep->rre[k] = rre;
                if (rep->dp_status) rep->dp_status[k] = st;
            }
            if (rep) rep->n_cols = K;
            // u^(k+1) in FP64 when the phase stops before its last iteration
            auto finish_u = [&] {
                if (!write_u)
                    gemv_fused<double, TX>(c, n, K, V, n, zt_k, 1.0, nullptr, 0.0, u_io, (TX*)nullptr, nullptr,
                                           nullptr);
            };
            if (p.u_true && p.rre_target > 0 && rre <= p.rre_target) {
                take_back();
                finish_u();
                stopped = true;
                break;
            }
            if (last) {
                if (p.u_true && p.rre_target > 0) status = std::max(status, (int)MMOF_WARN_KMAX);
                break;
            }
            // 9. breakdown or append r/||r||
            if (!(rnorm > 1e-14 * atb)) {
                take_back();
                finish_u();
                status = MMOF_WARN_BREAKDOWN;
                stopped = true;
                break;
            }
            if (!ahead) {
                normalize2<TX>(c, n, r, scal + 7, scal + 14, V + (int64_t)K * n, col_in(K));
                add_column(K, true);
            }
            ++K;
            queued = ahead;
        }
        if (rep) {
            rep->iters = std::max(rep->iters, iters);
            rep->status = std::max(rep->status, status);
        }
        if (ph.final || stopped) {
            const int64_t nv = 2 * g.pair_px;
            for (int q = 0; q < 2 && flow && nv; ++q) {
                void* dst = q == 0 ? v_out : vr_out;
                const TX* src = q == 0 ? flow_v : flow_vr;
                if (!dst) continue;
                if (ph.out_dt == MMOF_F32)
                    convert<TX, float>(c, nv, src, static_cast<float*>(dst));
                else
                    convert<TX, double>(c, nv, src, static_cast<double*>(dst));
            }
        }
        MMOF_HIP(hipStreamSynchronize(c.stream));
        PhaseOut out;
        out.status = status;
        out.K = K;
        out.iters = iters;
        out.stopped = stopped;
        out.flow_v = flow_v;
        out.flow_vr = flow_vr;
        return out;
    }
};

// The Krylov basis (V in FP64; H V and Theta V in each operator precision the solve uses) is
// the bulk of a solve's memory: refuse before anything is allocated when it cannot fit, and
// name the largest basis that would (at 1024 x 1024 x 64 a column takes 0.54 GB of V, 1.1 GB
// of FP32 Theta V and 2.1 GB of FP64 Theta V).
static void check_solve_capacity(Ctx& c, const Plan& P, const mmof_solve_params& p) {
    const Geom& g = *P.geom;
    const bool flow = p.use_flow != 0;
    const size_t n = (size_t)P.n, m = (size_t)P.m;
    const bool tdiff = p.reg == MMOF_REG_ANISO || p.reg == MMOF_REG_ISO;
    const size_t R = (size_t)(g.gx_len + g.gy_len + (tdiff ? g.pair_px : 0) + (flow ? g.pair_px : 0) +
                              ((flow && p.use_reverse) ? g.pair_px : 0));
    const size_t K = (size_t)std::max(1, p.ell + p.k_max - 1);
    const bool f64 = p.op_dtype == MMOF_F64 || p.refine_iters > 0;
    const bool f32 = p.op_dtype == MMOF_F32 && p.refine_iters < p.k_max;
    size_t per_col = sizeof(double) * n;
    size_t grow = c.work_growth("solve_V", sizeof(double) * K * n);
    // the vectors of one iteration: FP64 ones shared by both precisions, the others per precision
    size_t vecs = 0;
    for (const char* nm : {"solve_r", "solve_tmp_n"}) vecs += c.work_growth(nm, sizeof(double) * n);
    if (p.reorth == MMOF_REORTH_TWICE) vecs += c.work_growth("reorth_y", sizeof(double) * n);
    vecs += c.work_growth("solve_w2", sizeof(double) * R) + c.work_growth("solve_AVs", sizeof(double) * p.ell * m);
    auto per_precision = [&](const char* tag, size_t es) {
        const std::string t(tag);
        per_col += es * (m + R);
        grow += c.work_growth(t + "AV", es * K * m) + c.work_growth(t + "TV", es * K * R);
        for (const char* nm : {"u_op", "out_n", "out_n2", "vin_n"}) vecs += c.work_growth(t + nm, es * n);
        for (const char* nm : {"nu", "yR", "yW"}) vecs += c.work_growth(t + nm, es * R);
        if (flow && es == sizeof(float)) {
            // the FP32 copy of V's columns
            per_col += es * n;
            grow += c.work_growth(t + "V32", es * K * n);
        }
    };
    if (f64) per_precision("solve_d_", sizeof(double));
    if (f32) per_precision("solve_f_", sizeof(float));
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return;  // no estimate: the allocations report any failure themselves
    }
    // room for those vectors, the flow buffers and smaller workspaces
    const size_t reserve = vecs + sizeof(double) * 2 * (size_t)g.pair_px * 4 + ((size_t)1 << 30);
    if (grow + reserve <= free_b) return;
    const size_t avail = free_b > reserve ? free_b - reserve : 0;
    char msg[512];
    std::snprintf(msg, sizeof msg,
                  "the Krylov basis of %zu columns needs %.1f GB more device memory (%.2f GB per column); %.1f GB "
                  "are free, so at most about %zu columns (ell + k_max - 1) fit",
                  K, grow / 1e9, per_col / 1e9, free_b / 1e9, avail / std::max<size_t>(per_col, 1));
    throw Error(MMOF_ERR_OOM, msg);
}

int solve_joint(Plan& P, const double* b, double delta, const mmof_solve_params& p, double* u_io, void* v_out,
                void* vr_out, mmof_report* rep) {
    MMOF_CHECK(p.op_dtype == MMOF_F32 || p.op_dtype == MMOF_F64, MMOF_ERR_DTYPE, "op_dtype must be F32 or F64");
    MMOF_CHECK(p.refine_iters >= 0, MMOF_ERR_INVALID, "refine_iters must be >= 0");
    MMOF_CHECK(p.ell >= 1 && p.k_max >= 1 && p.ell + p.k_max - 1 <= KMAX, MMOF_ERR_SHAPE,
               "ell + k_max - 1 must be in [1, " + std::to_string(KMAX) + "]");
    check_solve_capacity(*P.ctx, P, p);
    if (rep) {
        rep->n_A = rep->n_At = rep->n_theta = rep->n_thetaT = rep->n_flow_updates = rep->n_L = 0;
        rep->n_factorizations = 0;
        rep->iters = 0;
        rep->status = 0;
    }
    Phase ph;
    ph.k_end = p.k_max;
    ph.out_dt = p.op_dtype;
    const int k_sw = std::max(0, p.k_max - p.refine_iters);
    if (p.op_dtype == MMOF_F64 || k_sw == 0) {
        Solver<double> s(*P.ctx, P, p, rep);
        return s.run(b, delta, u_io, v_out, vr_out, ph).status;
    }
    // FP32 operators in the MM iterations.  The Golub-Kahan start runs with FP64 operators:
    // its recurrence loses accuracy in the later start vectors in proportion to the operator
    // rounding, and the discrepancy-principle lambda amplifies a perturbed start subspace,
    // while the residual directions appended later are computed afresh in every iteration.
    {
        Phase p0 = ph;
        p0.start_only = true;
        Solver<double> s0(*P.ctx, P, p, rep);
        s0.run(b, delta, u_io, nullptr, nullptr, p0);
    }
    Phase p1 = ph;
    p1.K_in = p.ell;
    p1.start_av = p.ell - 1;
    p1.k_end = k_sw;
    p1.final = p.refine_iters == 0;
    Solver<float> s1(*P.ctx, P, p, rep);
    const PhaseOut o1 = s1.run(b, delta, u_io, v_out, vr_out, p1);
    if (p1.final || o1.stopped) return o1.status;
    // FP64 refinement for iterations [k_sw, k_max), starting from the FP32 phase's basis
    Phase p2 = ph;
    p2.k_begin = k_sw;
    p2.K_in = o1.K;
    p2.start_av = p.ell - 1;
    p2.v_in = o1.flow_v;
    p2.vr_in = o1.flow_vr;
    p2.in_dt = MMOF_F32;
    Solver<double> s2(*P.ctx, P, p, rep);
    const PhaseOut o2 = s2.run(b, delta, u_io, v_out, vr_out, p2);
    return std::max(o1.status, o2.status);
}

}  // namespace mmof
