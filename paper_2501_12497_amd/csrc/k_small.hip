// Small projected problem of MMGKS (eq. minKryov2) and the discrepancy principle
// (Sec. 4.1.3), in FP64 on one wavefront.
//
// With G_H = (HV)^T(HV), G_T = (P Theta V)^T (P Theta V) and d = (HV)^T b, the projected
// normal equations read (G_H + lambda G_T) z = d and the discrepancy of u = V z is
//   D(lambda)^2 = ||H V z - b||^2 = ||b||^2 - d^T z - lambda z^T G_T z.
// lambda solves D(lambda) = eta*delta.  D^2 increases with lambda; its derivative is
//   dD^2/dlambda = 2 lambda w^T (G_H + lambda G_T)^{-1} w,   w = G_T z.
// The root is bracketed in mu = log10(lambda) on [-12, 12] + log10(tr G_H / tr G_T)
// (the ends are taken when the root lies outside) and found by Newton steps in mu,
// safeguarded by bisection of the bracket.  Each evaluation factors
// G_H + lambda G_T by Cholesky in LDS.
#include "dev.h"
#include "krylov.h"

namespace mmof {

static constexpr int KP = KMAX_SMALL + 1;  // padded row length (odd: no LDS bank aliasing)

struct SmallLds {
    double A[KMAX_SMALL][KP];
    double T[KMAX_SMALL][KP];
    double M[KMAX_SMALL][KP];
    double d[KMAX_SMALL], z[KMAX_SMALL], w[KMAX_SMALL], y[KMAX_SMALL];
};

// Cholesky of M (lower, in place); returns false on a non-positive pivot.
__device__ bool chol(SmallLds& s, int K) {
    const int lane = threadIdx.x;
    for (int k = 0; k < K; ++k) {
        const double piv = s.M[k][k];
        if (!(piv > 0.0)) return false;
        const double lkk = sqrt(piv);
        __syncthreads();
        for (int i = k + lane; i < K; i += 64) s.M[i][k] = (i == k) ? lkk : s.M[i][k] / lkk;
        __syncthreads();
        for (int i = k + 1 + lane; i < K; i += 64) {
            const double lik = s.M[i][k];
            for (int j = k + 1; j <= i; ++j) s.M[i][j] -= lik * s.M[j][k];
        }
        __syncthreads();
    }
    return true;
}

// Solve L L^T x = b with the factor in s.M; b is read from `in`, x is written to `out`
// (both LDS vectors, may alias).
__device__ void chol_solve(SmallLds& s, int K, const double* in, double* out) {
    const int lane = threadIdx.x;
    for (int i = lane; i < K; i += 64) s.y[i] = in[i];
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        const double yk = s.y[k] / s.M[k][k];
        __syncthreads();
        for (int i = k + 1 + lane; i < K; i += 64) s.y[i] -= s.M[i][k] * yk;
        if (lane == 0) s.y[k] = yk;
        __syncthreads();
    }
    for (int k = K - 1; k >= 0; --k) {
        const double xk = s.y[k] / s.M[k][k];
        __syncthreads();
        for (int i = lane; i < k; i += 64) s.y[i] -= s.M[k][i] * xk;
        if (lane == 0) s.y[k] = xk;
        __syncthreads();
    }
    for (int i = lane; i < K; i += 64) out[i] = s.y[i];
    __syncthreads();
}

__device__ double dot_lds(const double* a, const double* b, int K) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < K; i += 64) acc += a[i] * b[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    return acc;  // all lanes hold the same value
}

// One evaluation at lambda: z, D^2 and (optionally) dD^2/dmu.  Returns false if the
// Cholesky factorization failed.
__device__ bool evaluate(SmallLds& s, int K, double lam, double bb, bool deriv, double& D2, double& dD2) {
    const int lane = threadIdx.x;
    for (int i = lane; i < K; i += 64)
        for (int j = 0; j <= i; ++j) s.M[i][j] = s.A[i][j] + lam * s.T[i][j];
    __syncthreads();
    if (!chol(s, K)) return false;
    chol_solve(s, K, s.d, s.z);
    for (int i = lane; i < K; i += 64) {
        double acc = 0.0;
        for (int j = 0; j < K; ++j) acc += s.T[i][j] * s.z[j];
        s.w[i] = acc;
    }
    __syncthreads();
    const double dz = dot_lds(s.d, s.z, K);
    const double zTz = dot_lds(s.z, s.w, K);
    D2 = bb - dz - lam * zTz;
    dD2 = 0.0;
    if (deriv) {
        // dD^2/dmu = ln(10) * lambda * 2 lambda w^T M^{-1} w
        __shared__ double sv[KMAX_SMALL];
        for (int i = lane; i < K; i += 64) sv[i] = s.w[i];
        __syncthreads();
        chol_solve(s, K, sv, sv);
        const double wMw = dot_lds(s.w, sv, K);
        dD2 = 2.302585092994046 * 2.0 * lam * lam * wMw;
    }
    return true;
}

__global__ __launch_bounds__(64) void k_small_solve(int K, const double* __restrict__ GA, const double* __restrict__ GT,
                                                    const double* __restrict__ dvec, const double* __restrict__ sc,
                                                    double fixed_lambda, double* __restrict__ zout,
                                                    double* __restrict__ res) {
    __shared__ SmallLds s;
    const int lane = threadIdx.x;
    for (int i = lane; i < K; i += 64) {
        for (int j = 0; j < K; ++j) {
            s.A[i][j] = GA[(int64_t)i * KMAX_SMALL + j];
            s.T[i][j] = GT[(int64_t)i * KMAX_SMALL + j];
        }
        s.d[i] = dvec[i];
    }
    __syncthreads();
    const double bb = sc[0], target = sc[1];
    double D2 = 0.0, dD2 = 0.0;
    double lam;
    int status = 0;
    if (fixed_lambda > 0.0) {
        lam = fixed_lambda;
        if (!evaluate(s, K, lam, bb, false, D2, dD2)) status = 4;
    } else {
        double trA = 0.0, trT = 0.0;
        for (int i = 0; i < K; ++i) {
            trA += s.A[i][i];
            trT += s.T[i][i];
        }
        const double shift = log10(trA / fmax(trT, 1e-300));
        double lo = -12.0 + shift, hi = 12.0 + shift;
        bool ok_lo = evaluate(s, K, pow(10.0, lo), bb, false, D2, dD2);
        if (ok_lo && D2 > target) {
            lam = pow(10.0, lo);
            status = 2;
        } else {
            bool ok_hi = evaluate(s, K, pow(10.0, hi), bb, false, D2, dD2);
            if (ok_hi && D2 < target) {
                lam = pow(10.0, hi);
                status = 2;
            } else {
                double mu = 0.5 * (lo + hi);
                const double prev = sc[2];
                if (prev > 0.0) {
                    const double m = log10(prev);
                    if (m > lo && m < hi) mu = m;
                }
                for (int it = 0; it < 200; ++it) {
                    const bool ok = evaluate(s, K, pow(10.0, mu), bb, true, D2, dD2);
                    const double f = ok ? D2 - target : -target;
                    if (f < 0.0)
                        lo = mu;
                    else
                        hi = mu;
                    // stop at the rounding level of D^2 or of mu
                    if (ok && fabs(f) <= 1e-14 * bb) break;
                    if (hi - lo <= 1e-14 * fmax(1.0, fabs(mu))) break;
                    double nmu = (ok && dD2 > 0.0) ? mu - f / dD2 : 0.5 * (lo + hi);
                    if (!(nmu > lo && nmu < hi)) nmu = 0.5 * (lo + hi);
                    if (fabs(nmu - mu) <= 1e-14 * fmax(1.0, fabs(mu))) break;
                    mu = nmu;
                }
                lam = pow(10.0, mu);
                if (!evaluate(s, K, lam, bb, false, D2, dD2)) status = 4;
            }
        }
    }
    for (int i = lane; i < K; i += 64) zout[i] = status == 4 ? 0.0 : s.z[i];
    if (lane == 0) {
        res[0] = lam;
        res[1] = D2;
        res[2] = (double)status;
    }
}

void small_solve(Ctx& c, int K, const double* GA, const double* GT, const double* d, const double* sc,
                 double fixed_lambda, double* z, double* res) {
    MMOF_CHECK(K >= 1 && K <= KMAX_SMALL, MMOF_ERR_SHAPE, "Krylov basis size out of range");
    ScopedTime st(&c, "small_solve");
    hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(64), 0, c.stream, K, GA, GT, d, sc, fixed_lambda, z, res);
    MMOF_LAUNCH_CHECK();
}

}  // namespace mmof
