/*
 * mmof.h -- C ABI of the MI355X (gfx950) MMGKS-OF hot-path library.
 *
 * The library applies the space-time operators of joint image reconstruction and
 * motion estimation (Okunola, Pasha, Kilmer, Freitag, "Efficient dynamic image
 * reconstruction with motion estimation") and runs the alternating
 * majorization-minimization / generalized-Krylov solve (MMGKS-OF, Alg. 1) on one GPU.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Images are stacks of frames stored [t][y][x] (x fastest), sequences one after
 *    another ("packed"); a stack is described by mmof_stack.  Frames are 0-based.
 *  - Flows are [pair][2][y][x] (component 0 = x, 1 = y), one pair per consecutive
 *    frame pair (t, t+1) of each sequence, pairs packed sequence after sequence.
 *    The reverse flow s'(t+1) of the paper is stored at the pair index t.
 *  - Array arguments are DEVICE pointers owned by the caller, contiguous and
 *    naturally aligned for their dtype.  The library never frees them and does not
 *    keep them after the call returns (work is enqueued asynchronously on the
 *    context's stream; the caller keeps buffers alive until the stream reaches it).
 *  - Host structs and host arrays passed in are copied; the caller keeps ownership.
 *  - Every entry point returns an int status: 0 = OK, < 0 = error (nothing useful
 *    was written), > 0 = completed with a warning.  No C++ exception crosses the ABI.
 *    mmof_last_error() returns the message of the most recent failure.
 *  - A context is bound to one HIP stream and is not thread-safe; use one context
 *    per host thread/stream.
 */
#ifndef MMOF_H
#define MMOF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define MMOF_OK 0
#define MMOF_ERR_INVALID (-1)     /* null pointer, bad enum, bad parameter value     */
#define MMOF_ERR_SHAPE (-2)       /* inconsistent sizes (stack, plan, capacity)      */
#define MMOF_ERR_DTYPE (-3)       /* unsupported dtype for this call                 */
#define MMOF_ERR_HIP (-4)         /* HIP runtime error (launch, copy, device)        */
#define MMOF_ERR_OOM (-5)         /* device workspace allocation failed              */
#define MMOF_ERR_NONFINITE (-6)   /* NaN/Inf found in an input that is checked       */
#define MMOF_WARN_KMAX 1          /* solve: k_max reached before the RRE target      */
#define MMOF_WARN_DP_CLAMPED 2    /* solve: discrepancy principle clamped lambda     */
#define MMOF_WARN_BREAKDOWN 3     /* solve: Krylov breakdown (residual vanished)     */

typedef enum { MMOF_F32 = 0, MMOF_F64 = 1 } mmof_dtype;

/* apply_flow_op modes */
#define MMOF_FLOW_FWD 0   /* out = L(v) u                         (r: [pairs][ny][nx])   */
#define MMOF_FLOW_ADJ 1   /* out = L(v)^T in                      (u: [frames][ny][nx])  */
#define MMOF_FLOW_DV 2    /* out = (d (L(v)u) / d v)^T in         (g: [pairs][2][ny][nx]) */
/* warp interpolation */
#define MMOF_INTERP_BILINEAR 0
#define MMOF_INTERP_ROUND 1
/* flow scale picked from the frame sizes (mmof_flow_update_scaled) */
#define MMOF_FLOW_SCALE_AUTO (-1)
/* flow solvers of the joint solve */
#define MMOF_FLOW_HS 0
#define MMOF_FLOW_GKS 1
/* regularisers of the joint solve (Sec. 5, table of methods); each with the motion rows when
 * use_flow is set (the -OF variants) */
#define MMOF_REG_PSI 0     /* M:  Theta = [Psi], l1 on every row                             */
#define MMOF_REG_ANISO 1   /* D1 AnisoTV: Theta = [Psi; L_t], l1 on every row                 */
#define MMOF_REG_ISO 2     /* D2 IsoTV: [Psi; L_t], a pixel's two spatial differences grouped */
#define MMOF_REG_GS 3      /* D3 GS: [Psi], each difference location grouped over the frames  */
/* reorthogonalisation of the new Krylov vector against the basis (Sec. 4.1: the vector is
 * orthogonal to the basis in exact arithmetic, and is reorthogonalised in floating point) */
#define MMOF_REORTH_AUTO 0   /* one classical Gram-Schmidt pass, a second one only when the   */
                             /* first keeps less than 1/sqrt(2) of the norm (Kahan's test)   */
#define MMOF_REORTH_TWICE 1  /* always two passes                                            */
#define MMOF_REORTH_IMPLICIT 2  /* joint solve: each new direction is stored as computed and     */
                                /* its components along the basis are carried in a triangular    */
                                /* factor T of the basis (V = Vs T), from the one pass Vs^T r     */
                                /* that the inner products need anyway; an explicit pass where r  */
                                /* keeps less than 1/sqrt(2) of its norm; the start as AUTO       */

typedef struct mmof_ctx_s* mmof_ctx;
typedef struct mmof_plan_s* mmof_plan;

/* A batch of image sequences (ragged sizes allowed).  Host arrays of n_seq entries. */
typedef struct {
    int32_t n_seq;
    const int32_t* n_t;   /* frames per sequence, >= 1 (flow calls need >= 2) */
    const int32_t* ny;    /* rows per frame, 2 .. 65535                       */
    const int32_t* nx;    /* columns per frame, 2 .. 65535                    */
} mmof_stack;

/* ------------------------------------------------------------------ context */

/* Create a context bound to a HIP stream (hipStream_t passed as void*; NULL = the
 * null stream) on the current HIP device.  The context owns its device workspace,
 * plan/tile caches and the autotuner cache. */
int mmof_create(mmof_ctx* out, void* hip_stream);
int mmof_destroy(mmof_ctx ctx);
/* Rebind the context to another stream of the same device. */
int mmof_set_stream(mmof_ctx ctx, void* hip_stream);
/* Message of the last failure on this host thread ("" if none).  ctx may be NULL. */
const char* mmof_last_error(mmof_ctx ctx);
/* Library version string. */
const char* mmof_version(void);

/* ------------------------------------------------------------------ forward operator H */

/* Plan for the per-frame parallel-beam projector H^t (Sec. 2.1: H = blockdiag(H^t)).
 * Model: pixel-driven linear ("hat") weights with unit pixels and unit detector bins,
 *   a_{(theta,j),p} = max(0, 1 - |X_p cos(theta) + Y_p sin(theta) - d_j|),
 *   X_p = x - (nx-1)/2, Y_p = y - (ny-1)/2, d_j = j - (n_bins-1)/2.
 * n_angles, n_bins: per sequence (host arrays of n_seq).  angles_rad: host array of
 * sum_s n_t[s]*n_angles[s] angles, sequence-major then frame-major ([t][k]).
 * Sinograms are stored [frame][angle][bin], sequences packed. */
int mmof_plan_radon(mmof_ctx ctx, const mmof_stack* stack, const int32_t* n_angles,
                    const int32_t* n_bins, const double* angles_rad, mmof_plan* out);

/* Plan for a fan-beam projector with a flat detector (Sec. 5 builds its operators on a flat
 * fan-beam geometry; it states no projector model or distances).  Angle theta: detector
 * axis a = (cos theta, sin theta), central ray e = (-sin theta, cos theta), point source at
 * -dso e from the frame centre, detector line at distance dsd from the source, n_bins bins
 * of width du centred at u_j = (j - (n_bins-1)/2) du; ray j runs from the source along
 * dsd e + u_j a (all lengths in pixel units).  Model: Joseph's method -- a ray with
 * |d_y| >= |d_x| is sampled on every pixel row by linear interpolation between the two
 * pixels around its crossing (pixels outside the frame count as 0), each sample weighted
 * by its path length per row |d| / |d_y|; other rays on the columns.  mmof_apply_At is the
 * exact transpose.  Sizes, angles and layouts as for mmof_plan_radon.  Errors:
 * MMOF_ERR_INVALID unless du > 0, dsd > dso and dso exceeds half the diagonal of every frame
 * by 2 (the source lies outside the frames). */
int mmof_plan_fan(mmof_ctx ctx, const mmof_stack* stack, const int32_t* n_angles,
                  const int32_t* n_bins, const double* angles_rad, double dso, double dsd,
                  double du, mmof_plan* out);
/* Plan for a per-frame Gaussian blur H^t: K(i,j) = exp(-(i^2+j^2)/(2 sigma^2)) / sum,
 * |i|,|j| <= ksize/2 (ksize odd, <= 15), zero boundary, output the size of the input.
 * K is symmetric so H^T applies the same sum. */
int mmof_plan_blur(mmof_ctx ctx, const mmof_stack* stack, int32_t ksize, double sigma, mmof_plan* out);
int mmof_plan_destroy(mmof_plan plan);
/* n = number of pixels, m = number of data entries of the plan's stack. */
int mmof_plan_sizes(mmof_plan plan, int64_t* n, int64_t* m);

/* Tile-shape autotuner of the plan's stencil kernels (blur for blur plans, the angle
 * grouping of the projector for Radon plans, Psi, Psi^T, L(v), L(v)^T): every candidate
 * is timed on the plan's stack in dtype dt (HIP events on the context's stream) and the
 * fastest is used by later launches of the plan (apply_A/At, solve_joint) in that dtype,
 * and by the stack-level operator calls on the plan's context for a stack of the same
 * sizes (apply_grad, apply_flow_op).
 * The stencil candidates compute identical values; the projector's angle groups split the
 * rows of a ray differently, which changes its sums by rounding only.
 * report: host buffer of report_len bytes (or NULL) that receives a NUL-terminated line
 * "kernel=AxB(mean us) ..." (tile width x height, or angles x row blocks for radon_fwd; a
 * trailing "p" marks a persistent launch).  Allocates scratch in the context; synchronizes
 * the stream. */
int mmof_autotune(mmof_plan plan, mmof_dtype dt, char* report, int32_t report_len);
/* Forces tile candidate `choice` (0-based, in the order the autotuner tries them) of a
 * tunable kernel ("blur", "radon_fwd", "grad_fwd", "grad_adj", "flow_fwd", "flow_adj") for the plan
 * in dtype dt.  MMOF_ERR_INVALID for an unknown kernel or an out-of-range choice. */
int mmof_set_tile(mmof_plan plan, const char* kernel, mmof_dtype dt, int32_t choice);

/* b <- H u  (u: n entries, b: m entries, both of dtype dt). */
int mmof_apply_A(mmof_plan plan, mmof_dtype dt, const void* u, void* b);
/* u <- H^T b (overwrites u). */
int mmof_apply_At(mmof_plan plan, mmof_dtype dt, const void* b, void* u);

/* ------------------------------------------------------------------ regularisation operators */

/* Edge-weighted spatial gradient Psi = blockdiag(L), L = [I (x) L_x ; L_y (x) I] with
 * first differences and no boundary rows (Sec. 4.1, eq. L):
 *   gx[t][y][x] = wx * (u[t][y][x+1] - u[t][y][x]),  gx: [frames][ny][nx-1]
 *   gy[t][y][x] = wy * (u[t][y+1][x] - u[t][y][x]),  gy: [frames][ny-1][nx]
 * transpose = 0: u is read, gx/gy are written.
 * transpose = 1: gx/gy are read, u <- Psi^T (w (.) g) is written.
 * wx, wy: optional weights with the layout of gx, gy (NULL = 1). */
int mmof_apply_grad(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int transpose,
                    const void* wx, const void* wy, void* u, void* gx, void* gy);

/* Optical-flow temporal operator L(v) ~ d/dt + v.grad, in the warp form of Sec. 3:
 *   direction +1 (M-bar):  r_t = W(v_t) u_{t+1} - u_t
 *   direction -1 (M-bar'): r_t = W(v_t) u_t - u_{t+1}      (v = reverse flow s')
 * for every pair t of every sequence.  W(v) pulls samples at p + v(p): bilinear
 * weights of the four neighbours with sample coordinates clipped to [0, n-1]
 * (MMOF_INTERP_BILINEAR), or the nearest pixel, ties to even, clipped
 * (MMOF_INTERP_ROUND, eq. m_matrix).  L(v) = -M-bar(s) of the paper.
 *   mode FWD: out (r, [pairs][ny][nx]) <- L(v) u;                     `in` unused
 *   mode ADJ: out (u, [frames][ny][nx]) <- L(v)^T in (in: r-shaped);  `u` unused
 *   mode DV : out (g, [pairs][2][ny][nx]) <- (d(L(v)u)/dv)^T in (in: r-shaped);
 *             per pixel the bilinear-interpolant gradient times in; 0 on clipped
 *             axes; the cell [floor(x'), floor(x')+1] at integer x'; 0 for ROUND.
 * The adjoint is a deterministic gather (no atomics): repeated calls are bitwise equal. */
int mmof_apply_flow_op(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int mode,
                       int direction, int interp, const void* u, const void* v,
                       const void* in, void* out);

/* Temporal first difference L_t of the spatio-temporal regularisers (Sec. 5, table of methods:
 * the mode-3 product U x_3 L_t):
 *   transpose = 0: out (r, [pairs][ny][nx]) <- u(t+1) - u(t) for every pair of every sequence;
 *   transpose = 1: out (u, [frames][ny][nx]) <- L_t^T in, i.e. in(t-1) - in(t) with the terms
 *                  of missing pairs left out (overwrites out). */
int mmof_apply_tdiff(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int transpose, const void* in,
                     void* out);

/* MM weights of the rows of Theta for regulariser reg (MMOF_REG_*; eq. QuadraticMajorantQ with
 * groups): nu (dtype dt, n_rows entries) is Theta u in the joint solve's row order, starting with
 * the gx rows ([frames][ny][nx-1]) and the gy rows ([frames][ny-1][nx]) of the stack; w2 (device
 * FP64, n_rows) receives 1 / sqrt(||nu_g||^2 + eps^2) for every row, g its group: a row of its
 * own for MMOF_REG_PSI and MMOF_REG_ANISO and for every row after the gy rows; for MMOF_REG_ISO a
 * pixel's horizontal and vertical difference; for MMOF_REG_GS a difference location's entries in
 * all frames of its sequence.  MMOF_ERR_SHAPE unless n_rows >= the gx and gy rows of the stack. */
int mmof_reg_weights(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, int reg, int64_t n_rows,
                     const void* nu, double eps, double* w2);

/* MM weights of Sec. 4.1.1: w2 = diag(P_eps^2) = 1 / sqrt(nu^2 + eps^2), n entries. */
int mmof_mm_weights(mmof_ctx ctx, mmof_dtype dt, int64_t n, const void* nu, double eps, void* w2);

/* ------------------------------------------------------------------ optical flow */

/* App. C image derivatives for every pair (t, t+1): I [pairs][3][ny][nx] = (I_x, I_y, I_t),
 *   I_x = 1/(2dr+1) sum_{j=-dr..dr} (u_t(y+j, x+dr) - u_t(y+j, x-dr)) / (2dr),  I_y alike,
 *   I_t = 1/(2dr+1)^2 sum_box (u_{t+1} - u_t),
 * with half-sample-symmetric mirroring at the borders; 1 <= delta_r < min(ny, nx). */
int mmof_of_derivs(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u,
                   void* I, int32_t delta_r);

/* Horn-Schunck flow update for eq. of_reg with p = q = 2 (gamma = alpha^2):
 * n_sweeps exact 2x2 block-Jacobi sweeps for
 *   min sum (I_x s_x + I_y s_y + I_t)^2 + gamma (||D s_x||^2 + ||D s_y||^2),
 *   s_new = sbar - g (g.sbar + I_t) / (gamma d_p + |g|^2),
 * warm-started from v (in/out, [pairs][2][ny][nx]).  If v_rev is not NULL it
 * receives the reverse flow of v (mmof_reverse_flow). */
int mmof_flow_update(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u,
                     void* v, void* v_rev, double alpha, int32_t n_sweeps, int32_t delta_r);

/* The same flow update computed on frames reduced by `scale` (Sec. 4.2 suggests cheaper
 * flow estimates; Sec. 5 reports flows computed on downscaled frames).  With f = scale:
 *   1. u_s = f x f block means of every frame of u, v_s = block means of v divided by f
 *      (reduced sides ceil(n / f); a block at the right or bottom border averages its
 *      in-frame pixels);
 *   2. the derivatives and n_sweeps Horn-Schunck sweeps of mmof_flow_update on (u_s, v_s);
 *   3. v(y, x) = f * bilinear sample of v_s at ((x + 1/2)/f - 1/2, (y + 1/2)/f - 1/2),
 *      the position clamped to the reduced grid.
 * scale = 1 (or 0) is mmof_flow_update.  scale = MMOF_FLOW_SCALE_AUTO picks the smallest
 * power of two that brings every frame side below 50 pixels (Sec. 5 reduces the frames by 2
 * or 4 to below 50 x 50), at most 64.  Arguments, layouts and ownership as there; errors:
 * MMOF_ERR_INVALID unless 1 <= scale <= 64 and 1 <= delta_r < every reduced frame side.
 * Workspaces of the reduced frames live in the context. */
int mmof_flow_update_scaled(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u,
                            void* v, void* v_rev, double alpha, int32_t n_sweeps, int32_t delta_r,
                            int32_t scale);

/* Solve-OF (Alg. 2) with p = q = 2, the paper's own flow solver: for every pair, with the
 * App. C derivatives (delta_r) and Y = [diag(I_x) diag(I_y)], b = -I_t, L = blockdiag(D, D)
 * (D: the first differences of mmof_apply_grad), the flow minimising
 *   ||Y s - b||^2 + lambda ||L s||^2          (eq. subproblem_motion_estimation_redefined)
 * by GKS (MMGKS with unit weights): `ell` Golub-Kahan steps on Y from b (both bases
 * re-orthogonalised), then `n_iter` projected solves; before each, lambda minimises the GCV
 * functional (eq. gcv_functional) of the projected solution V z,
 *   G(lambda) = ||Y V z - b||^2 / (m - trace(M^-1 (Y V)^T Y V))^2,
 *   M = (Y V)^T Y V + lambda (L V)^T L V, m = pixels of the pair,
 * over x = log10 lambda by a grid search (32 points over c + [-12, 12], c = log10(||Y V||_F^2 /
 * ||L V||_F^2), then 5 refinements of 8 points over [x* - h, x* + h], h the previous spacing;
 * in increasing x a point wins only when it lowers G by more than a relative 1e-9);
 * fixed_lambda > 0 skips the search.  Between solves the
 * basis grows by the residual Y^T(Y s - b) + lambda L^T L s orthogonalised twice against it;
 * the solve stops early when that residual vanishes (<= 1e-14 ||Y^T b||); Y^T b = 0 gives
 * s = 0.  v [pairs][2][ny][nx] receives the flow (its previous content is not used); v_rev,
 * if not NULL, the reverse flow of v.  scale > 1 computes on frames reduced as in
 * mmof_flow_update_scaled (no warm start is reduced).  lambdas, if not NULL, is a HOST array
 * [pairs][n_iter] that receives every lambda (0 after an early stop); the call then waits for
 * the stream.  Arithmetic in FP64 (the derivatives in dt).  Errors: MMOF_ERR_INVALID unless
 * ell >= 1, n_iter >= 1, ell + n_iter - 1 <= 32, fixed_lambda >= 0, every frame (reduced) has
 * more than ell and fewer than 2^30 pixels, and delta_r and scale are as for
 * mmof_flow_update_scaled.  Workspace (context-owned): about (2 (ell + n_iter) + 5) doubles
 * per pixel of the pairs. */
int mmof_flow_solve_gks(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u,
                        void* v, void* v_rev, int32_t delta_r, int32_t ell, int32_t n_iter,
                        double fixed_lambda, int32_t scale, double* lambdas);

/* Solve-OF (Alg. 2) with a choice of norms: pq = 2 is mmof_flow_solve_gks; pq = 1 is the
 * p = q = 1 variant of eq. of_reg_full, MMGKS on ||Y s - b||_1 + lambda ||L s||_1 with each
 * |x| smoothed to sqrt(x^2 + eps^2) and majorized by the weights 1 / phi_eps of the current
 * iterate as for the image problem (eq. QuadraticMajorantQ): at projected solve k the
 * weights come from the iterate s^(k) (s^(0) = 0),
 *   W_d = diag((e^2 + eps^2)^(-1/2)), e = Y s^(k) - b   (data rows),
 *   W_r = diag(((L s^(k))^2 + eps^2)^(-1/2))           (rows of L),
 * and the projected problem, the GCV functional and the residual are those of the weighted
 * problem (Y -> W_d^(1/2) Y, b -> W_d^(1/2) b, L -> W_r^(1/2) L; m stays the pixel count);
 * the basis, start and stopping rule as for pq = 2 (the weighted Gram matrices are formed
 * anew at every solve).  Arguments, output, lambdas and errors as for mmof_flow_solve_gks,
 * plus MMOF_ERR_INVALID unless pq is 1 or 2 and, for pq = 1, eps > 0 (the paper's reading:
 * 1e-3).  Workspace with pq = 1: 5 more doubles per pixel of the pairs. */
int mmof_flow_solve_of(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* u,
                       void* v, void* v_rev, int32_t delta_r, int32_t ell, int32_t n_iter,
                       double fixed_lambda, int32_t scale, int32_t pq, double eps,
                       double* lambdas);

/* Reverse flow (Remark on estimating the reverse optical flow): v_rev at
 * rint(p + v(p)) = -v(p), contributions to one pixel averaged, pixels that receive
 * none set to 0, targets outside the frame dropped. */
int mmof_reverse_flow(mmof_ctx ctx, const mmof_stack* stack, mmof_dtype dt, const void* v,
                      void* v_rev);

/* ------------------------------------------------------------------ joint solve */

typedef struct {
    int32_t ell;          /* Golub-Kahan start dimension (paper: 10)                     */
    int32_t k_max;        /* outer MM iterations (ell + k_max - 1 <= 256)                */
    int32_t tau;          /* flow update when k % tau == 0                               */
    int32_t n_sweeps;     /* Horn-Schunck sweeps per flow update                          */
    int32_t delta_r;      /* derivative box radius                                        */
    int32_t use_flow;     /* 0: Theta = Psi (method M); 1: Theta = [Psi; M-bar(...)]      */
    int32_t use_reverse;  /* 1: also M-bar'(s') with s' from the reverse-flow remark      */
    int32_t interp;       /* MMOF_INTERP_*                                                */
    int32_t op_dtype;     /* MMOF_F32 or MMOF_F64: precision of operator applications     */
    int32_t refine_iters; /* with op_dtype F32: the last refine_iters outer iterations run  */
                          /* with F64 operators on the basis the F32 iterations built      */
                          /* (H V, G_H, d and Theta V recomputed in F64); 0: F32 throughout */
    double eps;           /* MM smoothing (reading: 1e-3)                                 */
    double eta;           /* discrepancy safety factor (reading: 1.01)                    */
    double alpha;         /* Horn-Schunck alpha (gamma = alpha^2)                         */
    double fixed_lambda;  /* > 0: use this lambda instead of the discrepancy principle    */
    double rre_target;    /* > 0 with u_true: stop at the first RRE <= rre_target         */
    const double* u_true; /* device, n doubles, or NULL                                   */
    int32_t use_graph;    /* 1: replay the fixed launch sequences of an iteration (the flow  */
                          /* update and the residual's operator applications) from HIP      */
                          /* graphs captured on their second use and kept in the context    */
    int32_t flow_scale;   /* >= 2: the flow is computed on frames reduced by this factor    */
                          /* and upscaled (mmof_flow_update_scaled); 0 or 1: full frames;    */
                          /* MMOF_FLOW_SCALE_AUTO: the factor that setting picks            */
    int32_t flow_solver;  /* MMOF_FLOW_HS: n_sweeps Horn-Schunck sweeps warm-started from    */
                          /* the last flow (gamma = alpha^2); MMOF_FLOW_GKS: Solve-OF        */
                          /* (mmof_flow_solve_gks, lambda by GCV)                           */
    int32_t of_ell;       /* Solve-OF: Golub-Kahan steps (10)                               */
    int32_t of_iters;     /* Solve-OF: projected solves per flow computation (20)           */
    int32_t reg;          /* MMOF_REG_*: the spatial(-temporal) part of Theta (M by default)  */
    int32_t reorth;       /* MMOF_REORTH_*: reorthogonalisation of each new basis vector      */
                          /* (Golub-Kahan start and MM iterations)                            */
} mmof_solve_params;

typedef struct {
    int32_t iters;        /* outer iterations done                                        */
    int32_t status;       /* same value as the return code                                */
    int32_t n_cols;       /* Krylov basis size of the last projected solve                */
    int32_t capacity;     /* entries available in the host arrays below                   */
    double* lambda;       /* host [capacity] or NULL: lambda^(k)                          */
    double* resid;        /* host [capacity] or NULL: ||H u^(k+1) - b||                   */
    double* rre;          /* host [capacity] or NULL: RRE(u^(k+1)) if u_true given        */
    int32_t* dp_status;   /* host [capacity] or NULL: 0 root found, 2 clamped             */
    int64_t n_A, n_At, n_theta, n_thetaT, n_flow_updates;  /* operator application counts */
    int64_t n_L;          /* applications of L(v) or L(v)^T, one per flow direction      */
    int64_t n_factorizations; /* Cholesky factorizations in the projected solves          */
} mmof_report;

/* MMGKS-OF (Alg. 1) for min ||H u - b||^2 + lambda ||Theta u||_1 with the flow
 * re-estimated every tau iterations; p->reg selects the regulariser variant of the method
 * family (Sec. 5: M, D1 AnisoTV, D2 IsoTV, D3 GS; Theta's rows [gx | gy | L_t | forward flow |
 * reverse flow] as present), its groups entering the smoothed norm and the MM weights as in
 * mmof_reg_weights.  b: device FP64 [m]; noise_norm: ||e|| for the
 * discrepancy principle; u_inout: device FP64 [n] (initial estimate in, solution out);
 * v_out, v_rev_out: device flows of dtype op_dtype (either may be NULL); rep may be NULL.
 * Krylov vectors, Gram matrices, the projected solve and lambda are FP64 on the GPU.
 * A batch of several sequences is ONE problem: one objective over the packed stack, one
 * Krylov basis and one lambda (the discrepancy principle of Sec. 4.1.3 applied to the
 * stacked data), so noise_norm is the norm of the noise of the whole stack,
 * sqrt(sum_s ||e_s||^2).  Independent problems with a lambda each are independent calls
 * (one plan per sequence; several contexts on several streams run them concurrently).
 * Errors: MMOF_ERR_NONFINITE when b or u_inout holds NaN or Inf (checked on the device
 * before the first iteration); MMOF_ERR_SHAPE when ell + k_max - 1 exceeds the Krylov
 * capacity. */
int mmof_solve_joint(mmof_plan A, const void* b, double noise_norm, const mmof_solve_params* p,
                     void* u_inout, void* v_out, void* v_rev_out, mmof_report* rep);
/* Fill p with the defaults (ell 10, k_max 20, tau 1, 200 sweeps, delta_r 1, flow on,
 * reverse on, bilinear, F64 operators, eps 1e-3, eta 1.01, alpha 0.1, MMOF_REORTH_IMPLICIT). */
void mmof_solve_defaults(mmof_solve_params* p);

/* ------------------------------------------------------------------ projected-problem steps */

/* Weighted Gram matrix of a block of K columns (Sec. 4.1.1: R^T R of the thin QR of
 * P Theta V, eq. QR):  G = X^T diag(w2) X with w2 = 1/sqrt(nu^2 + eps^2) (nu NULL: w2 = 1).
 * X: device, K columns of length n in dtype dt, column j at X + j*ld; nu: device, n entries
 * of dtype dt or NULL.  G: device FP64, K x K row-major with leading dimension ldg.
 * 1 <= K <= 256 (the paper runs up to 200 iterations from ell = 10 start vectors, Sec. 5).
 * Accumulation is FP64 on the matrix cores; every entry is the sum over all n rows in a
 * fixed order (run to run reproducible), and G is exactly symmetric. */
int mmof_weighted_gram(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X, int64_t ld,
                       const void* nu, double eps, double* G, int32_t ldg);

/* mmof_weighted_gram for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same G, with the weights
 * formed inside the kernel from nu and the per-workgroup partial sums held in a fixed
 * library-owned device array of 5 MiB per GPU (kept until the process ends; looked up once per
 * device when a context is created).  No hipMalloc, hipFree or allocating library call is made.
 * Arguments, layouts and limits as for mmof_weighted_gram (1 <= K <= 64); the K x K entries
 * of G are written (entries K..ldg-1 of a row are not touched).  Every call on one GPU uses the
 * same array, which keeps the last call's partials: calls that overlap in time on one device
 * (from several streams or host threads) race on it and must be serialized by the caller.
 * The result equals mmof_weighted_gram's up to the order of the FP64 partial sums. */
int mmof_weighted_gram_noalloc(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X,
                               int64_t ld, const void* nu, double eps, double* G, int32_t ldg);

/* The passes over the Krylov basis of a GKS step (Alg. 1), exported so they can be checked on
 * their own at full length.  X, Q: device, K columns of length n, column j at X + j*ld
 * (1 <= K <= 256, ld >= n; 64-bit offsets, so K*ld may exceed 2^31); accumulation in FP64.
 *   mmof_block_dot:     out[j] = X_j^T y (X in dt, y device FP64 [n], out device FP64 [K]);
 *                       each inner product summed over row chunks in a fixed order.
 *   mmof_block_combine: out = alpha X z + beta y (z device FP64 [K]; y device FP64 [n] or
 *                       NULL, may alias out; out device FP64 [n]) -- u = V z and the CGS updates.
 *   mmof_cgs2:          x <- x - Q (Q^T x), twice (classical Gram-Schmidt with one
 *                       reorthogonalisation, the residual step of Alg. 1), Q FP64, x device FP64
 *                       [n] in/out; sq device FP64 [1] receives ||x||^2 afterwards.  The
 *                       context holds two workspace vectors (n and 256 doubles).
 *   mmof_reorth:        the same with a choice of passes (MMOF_REORTH_*): MMOF_REORTH_TWICE
 *                       is mmof_cgs2; MMOF_REORTH_AUTO makes one pass and a second one only
 *                       when the first kept less than 1/sqrt(2) of ||x|| (the test is taken on
 *                       the device; the second pass's launches then return at once).  The
 *                       joint solve reorthogonalises its new basis vectors this way
 *                       (mmof_solve_params.reorth).  MMOF_ERR_INVALID for another mode
 *                       (MMOF_REORTH_IMPLICIT is a property of the solve's basis). */
int mmof_block_dot(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X, int64_t ld,
                   const double* y, double* out);
int mmof_block_combine(mmof_ctx ctx, mmof_dtype dt, int64_t n, int32_t K, const void* X, int64_t ld,
                       const double* z, double alpha, const double* y, double beta, double* out);
int mmof_cgs2(mmof_ctx ctx, int64_t n, int32_t K, const double* Q, int64_t ld, double* x, double* sq);
int mmof_reorth(mmof_ctx ctx, int64_t n, int32_t K, const double* Q, int64_t ld, double* x, double* sq,
                int32_t mode);
/* One step of the implicit basis of the joint solve (MMOF_REORTH_IMPLICIT): the orthonormal
 * basis is V = Vs T with Vs the K stored columns (device FP64, column-major [K][ld]) and T unit
 * upper triangular (device FP64 [256][256], column-major: T[j * 256 + i] = T(i, j), column j =
 * the coefficients of v_j in Vs; rows below the diagonal are not read).  With g = V^T r and
 * rho^2 = ||r||^2 - ||g||^2: writes sq[0] = rho^2 and column K of T, e_K - T g / rho, so that
 * the new basis vector is v_K = r / rho - V g / rho when r / rho is stored as column K of Vs.
 * When r keeps less than 1/sqrt(2) of its norm outside span(V), r (device FP64 [n], in/out)
 * is first replaced by r - V g (one explicit pass; r is otherwise left as it is).  Reads Vs
 * once (twice on the explicit path).  1 <= K <= 255. */
int mmof_basis_extend(mmof_ctx ctx, int64_t n, int32_t K, const double* Vs, int64_t ld, double* r, double* T,
                      double* sq);

/* Projected solve of MMGKS (eq. minKryov2) with the discrepancy principle (Sec. 4.1.3):
 * (G_H + lambda G_T) z = d, lambda such that ||b||^2 - d^T z - lambda z^T G_T z = target.
 * 1 <= K <= 256.  GA, GT: device FP64 K x K (leading dimension 256, symmetric; only the first
 * K rows and columns are read); d: device FP64 [K];
 * sc: device FP64 {||b||^2, target = (eta delta)^2, previous lambda or 0};
 * fixed_lambda > 0 skips the root search.  Writes z (device FP64 [K]) and
 * res (device FP64 [4]) = {lambda, discrepancy^2, status 0 root / 2 clamped / 4 failure,
 * number of Cholesky factorizations}. */
int mmof_projected_solve(mmof_ctx ctx, int32_t K, const double* GA, const double* GT, const double* d,
                         const double* sc, double fixed_lambda, double* z, double* res);

/* ------------------------------------------------------------------ measurement */

/* Time every launch of the named kernel with HIP events on the context's stream
 * (name NULL or "" switches timing off; names: radon_fwd, radon_adj, blur, grad_fwd,
 * grad_adj, flow_fwd, flow_adj, flow_dv, of_derivs, hs_multi, reverse_flow, mdot, wgram,
 * small_solve).  mmof_kernel_timing returns the number of timed launches, their summed
 * duration in milliseconds and their summed algorithmic work (bytes that must move, each
 * input read and each output written once; flops the method needs), and synchronizes the
 * stream.  Any output pointer may be NULL. */
int mmof_profile_kernel(mmof_ctx ctx, const char* kernel_name);
int mmof_kernel_timing(mmof_ctx ctx, int64_t* launches, double* total_ms, double* alg_bytes, double* alg_flops);

#ifdef __cplusplus
}
#endif
#endif /* MMOF_H */
