// Host-side launchers of the HIP kernels (one translation unit per operator family).
#pragma once

#include "common.h"

namespace mmof {

// Tunable stencil kernels take a tile-shape candidate index; -1 uses the geometry's tuned
// choice (candidate 0 until the autotuner has run).
extern const TileShape kBlurShapes[], kGradShapes[], kFlowShapes[], kFlowAdjShapes[];
extern const int kBlurCandidates, kGradCandidates, kFlowCandidates, kFlowAdjCandidates;
// Output tile of candidate `choice` of Psi / Psi^T and of L(v) on geometry g (the vector
// forms, used when every frame width is a multiple of 4, have tiles of their own).
TileShape grad_tile(const Geom& g, int choice);
TileShape flow_tile(const Geom& g, int choice);

// The MM weighting of Theta's rows fused into the kernel that forms them: besides its rows y, the
// kernel writes m = y / sqrt(nu^2 + eps^2) (the weight in FP64, the product rounded to the row
// type, as the separate weighting pass computes it), nu and m laid out like y.  a: the rows of the
// first output (gx, or the flow rows), b: those of the second (gy).
struct RowWeighting {
    const void* nu_a = nullptr;
    void* m_a = nullptr;
    const void* nu_b = nullptr;
    void* m_b = nullptr;
    double eps2 = 0.0;
};

// Psi and Psi^T (eq. L); weights optional; rw: the MM weighting of the rows (may be null).
void launch_grad_fwd(Ctx& c, Geom& g, int dt, const void* u, const void* wx, const void* wy, void* gx, void* gy,
                     int choice = -1, const RowWeighting* rw = nullptr);
void launch_grad_adj(Ctx& c, Geom& g, int dt, const void* gx, const void* gy, const void* wx, const void* wy,
                     void* u, bool accumulate, int choice = -1);

// L(v) = -M-bar (direction +1) / -M-bar' (direction -1) and relatives.
void launch_flow_fwd(Ctx& c, Geom& g, int dt, int direction, int interp, const void* u, const void* v, void* r,
                     int choice = -1, const RowWeighting* rw = nullptr);
// The residual formed where the last Theta^T kernel writes its output: instead of u, the kernel
// writes out = x + lambda u in FP64 (x in the operator precision, lambda on the device), the
// arithmetic of the separate combination pass.
struct ResidualOut {
    const void* x = nullptr;
    const double* lam = nullptr;
    double* out = nullptr;
};
// res (may be null): write the residual instead of u (ResidualOut).
void launch_flow_adj(Ctx& c, Geom& g, int dt, int direction, int interp, const void* r, const void* v, void* u,
                     bool accumulate, const int32_t* d_radius /* device int: floor(max|v|)+1, or null */,
                     int choice = -1, const ResidualOut* res = nullptr);
// Forward (v) and, when vr is not null, reverse (vr) flow rows of Theta for K columns U (FP64,
// or in the operator precision of dt when u_op; leading dimension ldu) in one launch:
// out[j*ldo + oF ...] and out[j*ldo + oR ...], dtype dt.  Both forms give the same values.
void launch_flow_fwd_cols(Ctx& c, Geom& g, int dt, int interp, const void* U, bool u_op, int64_t ldu, int K,
                          const void* v, const void* vr, void* out, int64_t ldo, int64_t oF, int64_t oR);
void launch_flow_dv(Ctx& c, Geom& g, int dt, int direction, int interp, const void* u, const void* v,
                    const void* w, void* gv);
// Device int *d_out = floor(max |v|) + 1 over all pairs (saturating at 1<<20, NaN -> saturate).
void launch_flow_radius(Ctx& c, Geom& g, int dt, const void* v, int32_t* d_out);

// Temporal first difference L_t of the spatio-temporal regularisers: forward r = u(t+1) - u(t)
// per pair ([pairs][ny][nx]); transpose (accumulating into u or overwriting it).
void launch_tdiff(Ctx& c, Geom& g, int dt, bool transpose, const void* in, void* out, bool accumulate);
// MM weights of the grouped rows of Theta (reg MMOF_REG_ISO: per pixel over its horizontal
// and vertical difference; MMOF_REG_GS: per difference location over the frames of its
// sequence): nu holds Theta u from its start (gx rows, then gy rows), w2 (FP64) likewise;
// only the gx and gy rows of w2 are written.
void launch_group_weights(Ctx& c, Geom& g, int dt, int reg, const void* nu, double eps, double* w2);

// App. C derivatives, Horn-Schunck sweeps, reverse flow.
void launch_of_derivs(Ctx& c, Geom& g, int dt, const void* u, void* I, int dr);
// n_sweeps Horn-Schunck sweeps starting from v, several per launch, ping-ponging between
// v and tmp; returns 1 when the result is in tmp, 0 when it is in v.
int launch_hs_sweeps(Ctx& c, Geom& g, int dt, const void* I, void* v, void* tmp, double gamma, int n_sweeps);
void launch_reverse_flow(Ctx& c, Geom& g, int dt, const void* v, void* vr, const int32_t* d_radius);

// Flow on frames reduced by a factor f (Sec. 4.2): the geometry of the stack with every frame
// side ceil(n / f) (cached in the context, or owned), block means of the frames (mode 0) or of the
// flow, divided by f (mode 1), and the reduced flow upscaled bilinearly and multiplied by f.
Geom& reduced_geom(Ctx& c, const Geom& g, int f);
std::unique_ptr<Geom> make_reduced_geom(const Geom& g, int f, hipStream_t st);  // an owned copy
// The factor a requested scale stands for: 0 -> 1, MMOF_FLOW_SCALE_AUTO -> the smallest power
// of two (at most 64) that brings every frame side below 50 pixels, others unchanged.
int resolve_flow_scale(const Geom& g, int f);
// Raises MMOF_ERR_INVALID unless 1 <= f <= 64 and 1 <= dr < every side of the reduced frames.
void check_flow_frames(const Geom& g, int f, int dr);
void launch_box_down(Ctx& c, Geom& g, Geom& gs, int dt, int mode, int f, const void* in, void* out);
void launch_flow_up(Ctx& c, Geom& g, Geom& gs, int dt, int f, const void* vs, void* v);
// Solve-OF (Alg. 2, p = q = 2) per pair on geometry g: GKS with GCV (or a fixed lambda),
// from the derivatives I into the flow v (dtype dt; v's previous content is not used).
// Workspace (FP64): V (ell + n_iter - 1) * 2 * pair_px, U (ell + 1) * pair_px, S and R
// 2 * pair_px each, lam n_pairs * n_iter (the lambda of every iteration, 0 past a breakdown).
struct GksWork {
    double *V = nullptr, *U = nullptr, *S = nullptr, *R = nullptr, *lam = nullptr;
    double* W = nullptr;  // p = q = 1: 5 * pair_px weights
};
int of_gks_capacity();  // largest ell + n_iter - 1
// l1: the p = q = 1 variant (MM weights (x^2 + eps^2)^(-1/2) of the data rows and of the flow
// differences, from the current iterate); needs w.W.
void launch_of_gks(Ctx& c, Geom& g, int dt, const void* I, void* v, int ell, int n_iter, double fixed_lambda,
                   const GksWork& w, bool l1 = false, double eps = 1e-3);

// Raises MMOF_ERR_INVALID unless ell >= 1, n_iter >= 1, ell + n_iter - 1 <= of_gks_capacity(),
// and every (reduced by f) frame has more than ell pixels and fewer than 2^30.
void check_gks_frames(const Geom& g, int f, int ell, int n_iter);
struct FlowMethod;
// Solve-OF workspaces for geometry g (the frames the flow is computed on), named prefix + part
// in the context.
GksWork gks_work(Ctx& c, const Geom& g, const FlowMethod& fm, const std::string& prefix);

// How a flow update computes the flow: Horn-Schunck sweeps warm-started from the current flow
// (solver 0) or Solve-OF (solver 1).
struct FlowMethod {
    int solver = 0;
    double gamma = 0.01;   // HS: alpha^2
    int n_sweeps = 200;    // HS
    int ell = 10, n_iter = 20;
    double fixed_lambda = 0.0;  // Solve-OF: > 0 skips the GCV search
    int of_p = 2;               // Solve-OF: 2 (p = q = 2) or 1 (the smoothed-l1 MM variant)
    double of_eps = 1e-3;       // Solve-OF p = q = 1: smoothing of the l1 terms
};
// Workspace of one flow update: I and tmp sized for the frames the flow is computed on (the
// reduced ones when f > 1), us / vs for the reduced frames and flow (unused when f = 1), gks
// for Solve-OF.
struct FlowWork {
    void *I = nullptr, *tmp = nullptr, *us = nullptr, *vs = nullptr;
    GksWork gks;
};
// Derivatives and the flow (method fm) into v (updated in place), on the frames reduced by f
// (gs = reduced_geom(g, f); f = 1: on the frames themselves, gs unused); graph-safe (no memcpy
// nodes).
void flow_update_core(Ctx& c, Geom& g, Geom* gs, int dt, const void* u, void* v, int f, int dr, const FlowMethod& fm,
                      const FlowWork& w);

// Elementwise.
void launch_mm_weights(Ctx& c, int dt, int64_t n, const void* nu, double eps, void* w2);

// Forward operators.
// choice: angle-group candidate (0..3 = 1, 2, 4, 8 angles per workgroup), -1 = tuned/default
extern const int kRadonCandidates;
void launch_radon_fwd(Ctx& c, Plan& p, int dt, const void* u, void* b, int choice = -1);
void launch_radon_adj(Ctx& c, Plan& p, int dt, const void* b, void* u);
void launch_blur(Ctx& c, Plan& p, int dt, const void* in, void* out, int choice = -1);
void launch_fan_fwd(Ctx& c, Plan& p, int dt, const void* u, void* b);
void launch_fan_adj(Ctx& c, Plan& p, int dt, const void* b, void* u);
// Builds the frame table, trig table users and tile lists of a projector plan (radon or fan);
// the trig table must already be in p.d_trig.
void radon_plan_init(Ctx& c, Plan& p, const double* cs);  // cs: the host copy of the trig table
void fan_plan_init(Ctx& c, Plan& p);  // the per-ray table of a fan-beam plan (after radon_plan_init)

}  // namespace mmof
