// Solve-OF (Alg. 2), p = q = 2 and p = q = 1: per frame pair, the flow s minimising
//   ||Y s + u_t||^2 + lambda ||L s||^2,  Y = [diag(I_x) diag(I_y)],  L = blockdiag(D, D)
// (eq. subproblem_motion_estimation_redefined) by the generalized Krylov subspace method
// (MMGKS with unit weights): ell Golub-Kahan steps on Y from b = -u_t, then n_iter projected
// solves, each with lambda chosen by generalized cross-validation (eq. gcv_functional) on the
// projected solution and the basis grown by the orthogonalised residual.
//
// One workgroup per pair runs the whole solve in FP64: the basis and the Golub-Kahan left
// vectors live in global memory (workspace of the caller), the Gram matrices (Y V)^T Y V and
// (L V)^T L V, (Y V)^T b and the per-wave factorizations of the GCV search in LDS.  The Gram
// matrices grow by one row per iteration; Y V and L V are never stored (Y is diagonal per
// pixel and L a two-point stencil, so their entries are formed from V on the fly).
//
// GCV: G(lambda) = ||Y V z - b||^2 / (m - trace(M^-1 G_Y))^2 with M = G_Y + lambda G_L and
// m the pixels of the pair; the numerator is ||b||^2 - 2 z.d + z^T G_Y z.  The search over
// x = log10 lambda: 32 points evenly over c + [-12, 12], c = log10(tr G_Y / tr G_L), then 5
// refinements of 8 points evenly over [x* - h, x* + h] around the best point so far (h the
// previous spacing); scanned in increasing x, a point wins only when it lowers G by more than
// a relative 1e-9 (closer values are ties, the earlier point stays, so that the choice does
// not depend on rounding where G is flat); a factorization that fails gives G = inf.  Every wave of the workgroup evaluates one point
// at a time (Cholesky of M in LDS, lanes = rows; the K columns of G_Y and d solved together,
// lanes = columns).
//
// The p = q = 1 variant (MMGKS on the smoothed l1 norms of the data rows and of the flow
// differences): before every projected solve the weights of the current iterate are formed
// per pixel (one data weight, four edge weights stored at an edge's left / upper pixel), the
// weighted Gram matrices, d and b^T W_d b are built from scratch, and GCV, z and the residual
// are those of the weighted problem.
#include "dev.h"
#include "kernels.h"

namespace mmof {

namespace {

constexpr int GK_THREADS = 512;
constexpr int GK_WAVES = GK_THREADS / 64;
constexpr int GK_KC = 32;         // basis capacity (ell + n_iter - 1)
constexpr int GK_P = GK_KC + 1;   // padded LDS row stride of the factorization buffers
constexpr int GK_GRID0 = 32, GK_REFINE = 5, GK_GRIDR = 8;
constexpr double GK_SPAN = 12.0;
constexpr double GK_TIE = 1e-9;   // relative improvement of G a later grid point needs to win
constexpr int GK_G = 4;           // Gram columns per pass
constexpr int GK_NR = 2 * GK_G + 1;  // values per workgroup sum of a Gram pass
constexpr int GK_RMAX = GK_NR > 8 ? GK_NR : 8;  // largest workgroup sum

struct GksLds {
    double GA[GK_KC * GK_KC];     // (Y V)^T Y V
    double GL[GK_KC * GK_KC];     // (L V)^T L V
    double d[GK_KC];              // (Y V)^T b
    double z[GK_KC];
    double z0[GK_KC];             // the unregularised projected solution G_Y^-1 d
    double h[GK_KC];              // Gram-Schmidt coefficients
    double M[GK_WAVES][GK_KC * GK_P];
    double X[GK_WAVES][GK_KC * GK_P];
    double part[GK_WAVES * GK_RMAX];
    double tot[GK_RMAX];
    double gval[GK_GRID0], gxv[GK_GRID0];
};

// Orders a wave's LDS writes before its later LDS reads by other lanes of the same wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;  // identical on every lane (each butterfly step adds the same two values)
}

// Workgroup sums of a[0..NV): fixed order (lanes by butterfly, then waves in order); the
// totals land in s.tot[0..NV) and in a.
template <int NV>
__device__ void wg_sum(double (&a)[NV], GksLds& s) {
    static_assert(NV <= GK_RMAX, "workgroup sum too wide");
    __syncthreads();  // earlier readers of s.tot are done
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double v = wave_sum(a[j]);
        if (lane == 0) s.part[w * NV + j] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = s.part[threadIdx.x];
        for (int q = 1; q < GK_WAVES; ++q) t += s.part[q * NV + threadIdx.x];
        s.tot[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) a[j] = s.tot[j];
}

__device__ double wg_norm(const double* x, int64_t len, GksLds& s) {
    double a[1] = {0.0};
    for (int64_t p = threadIdx.x; p < len; p += GK_THREADS) a[0] += x[p] * x[p];
    wg_sum<1>(a, s);
    return sqrt(a[0]);
}

// x <- x - Q (Q^T x), twice, against columns 0..ncols-1 of Q (column stride len).
__device__ void reorth(const double* Q, int64_t len, int ncols, double* x, GksLds& s) {
    for (int pass = 0; pass < 2; ++pass) {
        for (int c0 = 0; c0 < ncols; c0 += 8) {
            double a[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) a[c] = 0.0;
            for (int64_t p = threadIdx.x; p < len; p += GK_THREADS) {
                const double xv = x[p];
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (c0 + c < ncols) a[c] += Q[(int64_t)(c0 + c) * len + p] * xv;
            }
            wg_sum<8>(a, s);
            if (threadIdx.x < 8 && c0 + (int)threadIdx.x < ncols) s.h[c0 + threadIdx.x] = s.tot[threadIdx.x];
        }
        __syncthreads();
        for (int64_t p = threadIdx.x; p < len; p += GK_THREADS) {
            double acc = 0.0;
            for (int c = 0; c < ncols; ++c) acc += s.h[c] * Q[(int64_t)c * len + p];
            x[p] -= acc;
        }
        __syncthreads();
    }
}

// Y v, the x- and y-differences of both components of v at pixel p (0 past the last
// column / row).
struct PixVals {
    double y, dxx, dxy, dyx, dyy;
};

template <class T>
__device__ __forceinline__ PixVals pix_vals(const double* v, int n, int nx, int p, bool hx, bool hy, T ix, T iy) {
    const double vx = v[p], vy = v[n + p];
    PixVals r;
    r.y = (double)ix * vx + (double)iy * vy;
    r.dxx = hx ? v[p + 1] - vx : 0.0;
    r.dxy = hx ? v[n + p + 1] - vy : 0.0;
    r.dyx = hy ? v[p + nx] - vx : 0.0;
    r.dyy = hy ? v[n + p + nx] - vy : 0.0;
    return r;
}

// Row j of the Gram matrices (against columns 0..j) and d[j]; with W (the p = q = 1 variant)
// every data row is weighted by W[p] and every difference by its edge weight W[n + 4p + e].
template <class T>
__device__ void gram_row(int j, const double* V, int n, int nx, int ny, const T* Ix, const T* Iy, const T* It,
                         GksLds& s, const double* W) {
    const int64_t N = 2 * (int64_t)n;
    const double* vj = V + (int64_t)j * N;
    for (int i0 = 0; i0 <= j; i0 += GK_G) {
        double a[GK_NR];
#pragma unroll
        for (int c = 0; c < GK_NR; ++c) a[c] = 0.0;
        for (int p = threadIdx.x; p < n; p += GK_THREADS) {
            const int x = p % nx, y = p / nx;
            const bool hx = x + 1 < nx, hy = y + 1 < ny;
            const T ix = Ix[p], iy = Iy[p];
            PixVals J = pix_vals(vj, n, nx, p, hx, hy, ix, iy);
            if (W) {  // weighted copies of the new column's values
                const double* we = W + n + 4 * (int64_t)p;
                J.y *= W[p];
                J.dxx *= we[0];
                J.dxy *= we[1];
                J.dyx *= we[2];
                J.dyy *= we[3];
            }
            if (i0 == 0) a[2 * GK_G] += J.y * -(double)It[p];
#pragma unroll
            for (int c = 0; c < GK_G; ++c) {
                if (i0 + c <= j) {
                    const PixVals Q = pix_vals(V + (int64_t)(i0 + c) * N, n, nx, p, hx, hy, ix, iy);
                    a[c] += Q.y * J.y;
                    a[GK_G + c] += Q.dxx * J.dxx + Q.dyx * J.dyx + Q.dxy * J.dxy + Q.dyy * J.dyy;
                }
            }
        }
        wg_sum<GK_NR>(a, s);
        if (threadIdx.x < GK_G && i0 + (int)threadIdx.x <= j) {
            const int i = i0 + threadIdx.x;
            s.GA[i * GK_KC + j] = s.GA[j * GK_KC + i] = s.tot[threadIdx.x];
            s.GL[i * GK_KC + j] = s.GL[j * GK_KC + i] = s.tot[GK_G + threadIdx.x];
        }
        if (i0 == 0 && threadIdx.x == 0) s.d[j] = s.tot[2 * GK_G];
    }
    __syncthreads();
}

// G(lambda) on the calling wave; with zout, also writes z (lanes < K) unless the factorization
// fails (G = inf).  The numerator: with rho0 = ||Y V z0 - b||^2 >= 0 (z0 = s.z0 solving the
// unregularised projected normal equations), ||Y V z - b||^2 = rho0 + (z - z0)^T G_Y (z - z0)
// exactly, a sum of non-negative terms; with rho0 < 0, ||b||^2 - 2 z.d + z^T G_Y z.
__device__ double gcv_eval(int K, double lam, double bb, double rho0, double m, GksLds& s, double* zout) {
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    double* M = s.M[w];
    double* X = s.X[w];
    for (int e = lane; e < K * K; e += 64) {
        const int i = e / K, k = e % K;
        M[i * GK_P + k] = fma(lam, s.GL[i * GK_KC + k], s.GA[i * GK_KC + k]);
    }
    wave_sync();
    // Cholesky M = R R^T in place (lower), lane i owns row i
    for (int j = 0; j < K; ++j) {
        const double mjj = M[j * GK_P + j];
        if (!(mjj > 0.0) || !isfinite(mjj)) return INFINITY;  // same value on every lane
        const double ljj = sqrt(mjj);
        double lij = 0.0;
        if (lane > j && lane < K) lij = M[lane * GK_P + j] / ljj;
        wave_sync();
        if (lane > j && lane < K) M[lane * GK_P + j] = lij;
        if (lane == j) M[j * GK_P + j] = ljj;
        wave_sync();
        if (lane > j && lane < K)
            for (int k = j + 1; k <= lane; ++k) M[lane * GK_P + k] -= lij * M[k * GK_P + j];
        wave_sync();
    }
    // columns c < K: M^-1 G_Y e_c; column K: z = M^-1 d (lane c owns column c of X)
    if (lane <= K) {
        for (int r = 0; r < K; ++r) {
            double y = lane < K ? s.GA[r * GK_KC + lane] : s.d[r];
            for (int k = 0; k < r; ++k) y -= M[r * GK_P + k] * X[k * GK_P + lane];
            X[r * GK_P + lane] = y / M[r * GK_P + r];
        }
        for (int r = K - 1; r >= 0; --r) {
            double x = X[r * GK_P + lane];
            for (int k = r + 1; k < K; ++k) x -= M[k * GK_P + r] * X[k * GK_P + lane];
            X[r * GK_P + lane] = x / M[r * GK_P + r];
        }
    }
    wave_sync();
    const double t = wave_sum(lane < K ? X[lane * GK_P + lane] : 0.0);
    double rho;
    if (rho0 >= 0.0) {
        double dgd = 0.0;
        if (lane < K) {
            double gd = 0.0;
            for (int k = 0; k < K; ++k) gd += s.GA[lane * GK_KC + k] * (X[k * GK_P + K] - s.z0[k]);
            dgd = (X[lane * GK_P + K] - s.z0[lane]) * gd;
        }
        rho = rho0 + fmax(wave_sum(dgd), 0.0);
    } else {
        double zd = 0.0, zgz = 0.0;
        if (lane < K) {
            const double zi = X[lane * GK_P + K];
            double gz = 0.0;
            for (int k = 0; k < K; ++k) gz += s.GA[lane * GK_KC + k] * X[k * GK_P + K];
            zd = zi * s.d[lane];
            zgz = zi * gz;
        }
        zd = wave_sum(zd);
        zgz = wave_sum(zgz);
        rho = fmax(bb - 2.0 * zd + zgz, 0.0);
    }
    if (zout && lane < K) zout[lane] = X[lane * GK_P + K];
    const double den = (m - t) * (m - t);
    const double g = den > 0.0 ? rho / den : INFINITY;
    return isfinite(g) ? g : INFINITY;
}

// The GCV minimiser (every thread returns the same value).
__device__ double gcv_search(int K, double bb, double rho0, double m, GksLds& s) {
    double tA = 0.0, tL = 0.0;
    for (int i = 0; i < K; ++i) {
        tA += s.GA[i * GK_KC + i];
        tL += s.GL[i * GK_KC + i];
    }
    const double c = log10(fmax(tA, 1e-300) / fmax(tL, 1e-300));
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    double best_g = INFINITY, best_x = c;
    double h = 2.0 * GK_SPAN / (GK_GRID0 - 1);
    for (int stage = 0; stage <= GK_REFINE; ++stage) {
        const int npt = stage == 0 ? GK_GRID0 : GK_GRIDR;
        const double lo = stage == 0 ? c - GK_SPAN : best_x - h;
        const double step2 = stage == 0 ? 2.0 * GK_SPAN : 2.0 * h;
        const int den = npt - 1;
        for (int p = w; p < npt; p += GK_WAVES) {
            const double x = lo + step2 * p / den;
            const double g = gcv_eval(K, pow(10.0, x), bb, rho0, m, s, nullptr);
            if (lane == 0) {
                s.gval[p] = g;
                s.gxv[p] = x;
            }
        }
        __syncthreads();
        for (int p = 0; p < npt; ++p)
            if (s.gval[p] < best_g * (1.0 - GK_TIE)) {
                best_g = s.gval[p];
                best_x = s.gxv[p];
            }
        __syncthreads();
        if (stage > 0) h = 2.0 * h / (GK_GRIDR - 1);
    }
    return pow(10.0, best_x);
}

template <class T>
__global__ __launch_bounds__(GK_THREADS) void k_of_gks(const Tile* __restrict__ pairs,
                                                       const FrameInfo* __restrict__ frames,
                                                       const T* __restrict__ I, T* __restrict__ vout,
                                                       double* __restrict__ Vw, double* __restrict__ Uw,
                                                       double* __restrict__ Sw, double* __restrict__ Rw,
                                                       double* __restrict__ lam_out, int ell, int n_iter, int kc,
                                                       double fixed_lambda, double* __restrict__ Ww, double eps) {
    __shared__ GksLds s;
    const FrameInfo f = frames[pairs[blockIdx.x].frame];
    const int nx = f.nx, ny = f.ny, n = nx * ny;
    const int64_t N = 2 * (int64_t)n;
    const T* Ix = I + 3 * f.pair_off;
    const T* Iy = Ix + n;
    const T* It = Iy + n;
    double* V = Vw + (int64_t)kc * 2 * f.pair_off;   // column j: V + j N
    double* U = Uw + (int64_t)(ell + 1) * f.pair_off;  // column j: U + j n
    double* sv = Sw + 2 * f.pair_off;
    double* r = Rw + 2 * f.pair_off;
    double* lam = lam_out + (int64_t)blockIdx.x * n_iter;
    // p = q = 1: weights of the current iterate, W[p] for the data row and W[n + 4p + e] for
    // the differences (e: x of s_x, x of s_y, y of s_x, y of s_y) (null: p = q = 2)
    double* W = Ww ? Ww + 5 * f.pair_off : nullptr;
    T* vo = vout + 2 * f.pair_off;
    const int tid = threadIdx.x;
    for (int k = tid; k < n_iter; k += GK_THREADS) lam[k] = 0.0;

    // ||b||^2 and ||Y^T b||^2, b = -I_t
    double a2[2] = {0.0, 0.0};
    for (int p = tid; p < n; p += GK_THREADS) {
        const double bt = -(double)It[p];
        const double gx = (double)Ix[p] * bt, gy = (double)Iy[p] * bt;
        a2[0] += bt * bt;
        a2[1] += gx * gx + gy * gy;
    }
    wg_sum<2>(a2, s);
    const double bb = a2[0], atb = sqrt(a2[1]);
    if (atb == 0.0) {
        for (int64_t p = tid; p < N; p += GK_THREADS) vo[p] = T(0);
        return;
    }

    // ell Golub-Kahan steps, both bases re-orthogonalised
    double beta = sqrt(bb);
    for (int p = tid; p < n; p += GK_THREADS) U[p] = -(double)It[p] / beta;
    double a1[1] = {0.0};
    for (int p = tid; p < n; p += GK_THREADS) {
        const double gx = (double)Ix[p] * U[p], gy = (double)Iy[p] * U[p];
        a1[0] += gx * gx + gy * gy;
    }
    wg_sum<1>(a1, s);
    double alpha = sqrt(a1[0]);
    for (int p = tid; p < n; p += GK_THREADS) {
        V[p] = (double)Ix[p] * U[p] / alpha;
        V[n + p] = (double)Iy[p] * U[p] / alpha;
    }
    for (int i = 1; i <= ell; ++i) {
        double* ui = U + (int64_t)i * n;
        const double* up = U + (int64_t)(i - 1) * n;
        const double* vp = V + (int64_t)(i - 1) * N;
        for (int p = tid; p < n; p += GK_THREADS)
            ui[p] = ((double)Ix[p] * vp[p] + (double)Iy[p] * vp[n + p]) - alpha * up[p];
        __syncthreads();
        reorth(U, n, i, ui, s);
        beta = wg_norm(ui, n, s);
        for (int p = tid; p < n; p += GK_THREADS) ui[p] = ui[p] / beta;
        if (i == ell) break;
        double* vi = V + (int64_t)i * N;
        for (int p = tid; p < n; p += GK_THREADS) {
            vi[p] = (double)Ix[p] * ui[p] - beta * vp[p];
            vi[n + p] = (double)Iy[p] * ui[p] - beta * vp[n + p];
        }
        __syncthreads();
        reorth(V, N, i, vi, s);
        alpha = wg_norm(vi, N, s);
        for (int64_t p = tid; p < N; p += GK_THREADS) vi[p] = vi[p] / alpha;
        __syncthreads();  // element n + p of vi is read next by the thread of pixel p
    }
    __syncthreads();

    // generalized Krylov iterations
    int K = ell;
    if (!W)
        for (int j = 0; j < K; ++j) gram_row(j, V, n, nx, ny, Ix, Iy, It, s, (const double*)nullptr);
    else
        for (int64_t p = tid; p < N; p += GK_THREADS) sv[p] = 0.0;  // s^(0)
    const double m = (double)n;
    double bbw = bb;  // b^T W_d b
    for (int k = 0; k < n_iter; ++k) {
        if (W) {
            // weights of the iterate s^(k), then the weighted Gram matrices from scratch
            __syncthreads();
            double a1w[1] = {0.0};
            for (int p = tid; p < n; p += GK_THREADS) {
                const int x = p % nx, y = p / nx;
                const double sx = sv[p], sy = sv[n + p];
                const double e = (double)Ix[p] * sx + (double)Iy[p] * sy + (double)It[p];
                const double wd = 1.0 / sqrt(e * e + eps * eps);
                W[p] = wd;
                const double bt = (double)It[p];
                a1w[0] += wd * bt * bt;
                double* we = W + n + 4 * (int64_t)p;
                const double gxx = x + 1 < nx ? sv[p + 1] - sx : 0.0, gxy = x + 1 < nx ? sv[n + p + 1] - sy : 0.0;
                const double gyx = y + 1 < ny ? sv[p + nx] - sx : 0.0, gyy = y + 1 < ny ? sv[n + p + nx] - sy : 0.0;
                we[0] = x + 1 < nx ? 1.0 / sqrt(gxx * gxx + eps * eps) : 0.0;
                we[1] = x + 1 < nx ? 1.0 / sqrt(gxy * gxy + eps * eps) : 0.0;
                we[2] = y + 1 < ny ? 1.0 / sqrt(gyx * gyx + eps * eps) : 0.0;
                we[3] = y + 1 < ny ? 1.0 / sqrt(gyy * gyy + eps * eps) : 0.0;
            }
            wg_sum<1>(a1w, s);
            bbw = a1w[0];
            __syncthreads();
            for (int j = 0; j < K; ++j) gram_row(j, V, n, nx, ny, Ix, Iy, It, s, (const double*)W);
        }
        double lk = fixed_lambda;
        if (!(fixed_lambda > 0.0)) {
            // rho0 = ||Y V z0 - b||^2 from a pass over the pixels (< 0 when G_Y is singular)
            double st[1] = {0.0};
            if (tid < 64) {
                const double g0 = gcv_eval(K, 0.0, bbw, -1.0, m, s, s.z0);
                st[0] = tid == 0 ? g0 : 0.0;
            }
            wg_sum<1>(st, s);  // every thread learns whether z0 exists
            double rho0 = -1.0;
            if (isfinite(st[0])) {
                double e2[1] = {0.0};
                for (int p = tid; p < n; p += GK_THREADS) {
                    double acc = 0.0;
                    for (int j = 0; j < K; ++j) {
                        const double* vj = V + (int64_t)j * N;
                        acc += s.z0[j] * ((double)Ix[p] * vj[p] + (double)Iy[p] * vj[n + p]);
                    }
                    const double e = acc + (double)It[p];
                    e2[0] += (W ? W[p] : 1.0) * e * e;
                }
                wg_sum<1>(e2, s);
                rho0 = e2[0];
            }
            lk = gcv_search(K, bbw, rho0, m, s);
        }
        if (tid == 0) lam[k] = lk;
        if (tid < 64) (void)gcv_eval(K, lk, bbw, -1.0, m, s, s.z);
        __syncthreads();
        for (int64_t p = tid; p < N; p += GK_THREADS) {
            double acc = 0.0;
            for (int j = 0; j < K; ++j) acc += s.z[j] * V[(int64_t)j * N + p];
            sv[p] = acc;
        }
        if (k == n_iter - 1) break;
        __syncthreads();
        // r = Y^T W_d (Y s - b) + lambda L^T W_r L s (W = I for p = q = 2)
        for (int p = tid; p < n; p += GK_THREADS) {
            const int x = p % nx, y = p / nx;
            const double sx = sv[p], sy = sv[n + p];
            double e = (double)Ix[p] * sx + (double)Iy[p] * sy + (double)It[p];
            double lx = 0.0, ly = 0.0;
            // L^T W_r L s: every edge (p, q) adds w_pq (s(p) - s(q)), its weight stored at the
            // edge's left / upper end (all ones for p = q = 2)
            const double* wp = W ? W + n + 4 * (int64_t)p : nullptr;
            if (x > 0) {
                const double* wq = W ? W + n + 4 * (int64_t)(p - 1) : nullptr;
                lx += (W ? wq[0] : 1.0) * (sx - sv[p - 1]);
                ly += (W ? wq[1] : 1.0) * (sy - sv[n + p - 1]);
            }
            if (x + 1 < nx) {
                lx += (W ? wp[0] : 1.0) * (sx - sv[p + 1]);
                ly += (W ? wp[1] : 1.0) * (sy - sv[n + p + 1]);
            }
            if (y > 0) {
                const double* wq = W ? W + n + 4 * (int64_t)(p - nx) : nullptr;
                lx += (W ? wq[2] : 1.0) * (sx - sv[p - nx]);
                ly += (W ? wq[3] : 1.0) * (sy - sv[n + p - nx]);
            }
            if (y + 1 < ny) {
                lx += (W ? wp[2] : 1.0) * (sx - sv[p + nx]);
                ly += (W ? wp[3] : 1.0) * (sy - sv[n + p + nx]);
            }
            if (W) e *= W[p];
            r[p] = (double)Ix[p] * e + lk * lx;
            r[n + p] = (double)Iy[p] * e + lk * ly;
        }
        __syncthreads();
        reorth(V, N, K, r, s);
        const double nr = wg_norm(r, N, s);
        if (nr <= 1e-14 * atb) break;  // breakdown: keep the last s
        double* vk = V + (int64_t)K * N;
        for (int64_t p = tid; p < N; p += GK_THREADS) vk[p] = r[p] / nr;
        __syncthreads();
        ++K;
        if (!W) gram_row(K - 1, V, n, nx, ny, Ix, Iy, It, s, (const double*)nullptr);
    }
    __syncthreads();
    for (int64_t p = tid; p < N; p += GK_THREADS) vo[p] = (T)sv[p];
}

}  // namespace

int of_gks_capacity() { return GK_KC; }

void check_gks_frames(const Geom& g, int f, int ell, int n_iter) {
    MMOF_CHECK(ell >= 1 && n_iter >= 1 && ell + n_iter - 1 <= GK_KC, MMOF_ERR_INVALID,
               "need ell >= 1, n_iter >= 1, ell + n_iter - 1 <= " + std::to_string(GK_KC));
    for (int s = 0; s < g.n_seq; ++s) {
        if (g.n_t[s] < 2) continue;
        const int64_t n = (int64_t)((g.ny[s] + f - 1) / f) * ((g.nx[s] + f - 1) / f);
        MMOF_CHECK(n > ell && n < ((int64_t)1 << 30), MMOF_ERR_INVALID,
                   "Solve-OF needs frames of more than ell and fewer than 2^30 pixels");
    }
}

GksWork gks_work(Ctx& c, const Geom& g, const FlowMethod& fm, const std::string& prefix) {
    const int64_t P = std::max<int64_t>(g.pair_px, 1);
    GksWork w;
    w.V = static_cast<double*>(c.work(prefix + "V", sizeof(double) * (size_t)(fm.ell + fm.n_iter - 1) * 2 * P));
    w.U = static_cast<double*>(c.work(prefix + "U", sizeof(double) * (size_t)(fm.ell + 1) * P));
    w.S = static_cast<double*>(c.work(prefix + "S", sizeof(double) * 2 * (size_t)P));
    w.R = static_cast<double*>(c.work(prefix + "R", sizeof(double) * 2 * (size_t)P));
    w.lam = static_cast<double*>(
        c.work(prefix + "lam", sizeof(double) * (size_t)std::max<int64_t>(g.n_pairs, 1) * fm.n_iter));
    if (fm.of_p == 1) w.W = static_cast<double*>(c.work(prefix + "W", sizeof(double) * 5 * (size_t)P));
    return w;
}

void launch_of_gks(Ctx& c, Geom& g, int dt, const void* I, void* v, int ell, int n_iter, double fixed_lambda,
                   const GksWork& w, bool l1, double eps) {
    MMOF_CHECK(!l1 || (w.W && eps > 0 && std::isfinite(eps)), MMOF_ERR_INVALID, "p = q = 1 needs eps > 0");
    if (g.n_pairs == 0) return;
    const int kc = ell + n_iter - 1;
    MMOF_CHECK(ell >= 1 && n_iter >= 1 && kc <= GK_KC, MMOF_ERR_INVALID,
               "need ell >= 1, n_iter >= 1, ell + n_iter - 1 <= " + std::to_string(GK_KC));
    // one tile per pair: the list of pairs
    const TileList& tl = g.tile_list(c.stream, 65535, 65535, true);
    MMOF_CHECK(tl.count == g.n_pairs, MMOF_ERR_SHAPE, "pair list");
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "of_gks", sizeof(T) * 5.0 * g.pair_px, 0.0);
        hipLaunchKernelGGL(k_of_gks<T>, dim3((unsigned)tl.count), dim3(GK_THREADS), 0, c.stream, tl.buf.as<Tile>(),
                           g.dframes(), (const T*)I, (T*)v, w.V, w.U, w.S, w.R, w.lam, ell, n_iter, kc, fixed_lambda,
                           l1 ? w.W : nullptr, eps);
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
