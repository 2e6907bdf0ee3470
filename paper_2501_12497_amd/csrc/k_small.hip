// Small projected problem of MMGKS (eq. minKryov2) and the discrepancy principle
// (Sec. 4.1.3), in FP64 on one wavefront.
//
// With G_H = (HV)^T(HV), G_T = (P Theta V)^T (P Theta V) and d = (HV)^T b, the projected
// normal equations read (G_H + lambda G_T) z = d and the discrepancy of u = V z is
//   D(lambda)^2 = ||H V z - b||^2 = ||b||^2 - d^T z - lambda z^T G_T z.
// lambda solves D(lambda) = eta*delta.  D^2 increases with lambda; its derivative is
//   dD^2/dlambda = 2 lambda w^T (G_H + lambda G_T)^{-1} w,   w = G_T z.
// The root is bracketed in mu = log10(lambda) on [-12, 12] + log10(tr G_H / tr G_T)
// (an end is taken when the root lies beyond it) and found by Newton steps in mu,
// safeguarded by bisection of the bracket, starting from the previous lambda.
//
// One lane owns one row (K <= 64).  Each evaluation factors M = G_H + lambda G_T with a
// left-looking Cholesky (the inner products only read LDS, so they pipeline) and solves
// with the factor held in LDS and the right-hand side in registers, broadcasting the
// pivot entries with readlane.
#include "dev.h"
#include "krylov.h"

// Optional per-iteration trace (a probe build can define it; no-op in the library).
#ifndef MMOF_SMALL_TRACE
#define MMOF_SMALL_TRACE(it, mu, e, f, lo, hi)
#endif

namespace mmof {

static constexpr int KP = KMAX_SMALL + 1;  // padded row length (odd: no LDS bank aliasing)

struct SmallLds {
    double A[KMAX_SMALL][KP];
    double T[KMAX_SMALL][KP];
    double L[KMAX_SMALL][KP];
    double invd[KMAX_SMALL];
};

__device__ __forceinline__ double bcast(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave sum whose result is bitwise identical in every lane: the root finder branches on
// it, and a butterfly alone is not lane-symmetric once the compiler fuses the first add
// with the product that feeds it.  Lane 0's sum is broadcast.
__device__ __forceinline__ double wave_sum64(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return bcast(v, 0);
}

// Left-looking Cholesky of M = A + lam T into s.L (lower) and s.invd; false on a
// non-positive pivot (uniform across the wave).
__device__ bool chol(SmallLds& s, int K, double lam) {
    const int i = threadIdx.x;
    for (int k = 0; k < K; ++k) {
        double dot = 0.0;
        if (i >= k && i < K) {
#pragma unroll 8
            for (int j = 0; j < k; ++j) dot += s.L[i][j] * s.L[k][j];
        }
        const double mik = (i < K) ? s.A[i][k] + lam * s.T[i][k] - dot : 0.0;
        const double piv = bcast(mik, k);
        if (!(piv > 0.0)) return false;
        const double lkk = sqrt(piv);
        const double inv = 1.0 / lkk;
        if (i > k && i < K) s.L[i][k] = mik * inv;
        if (i == k) {
            s.L[k][k] = lkk;
            s.invd[k] = inv;
        }
        __syncthreads();
    }
    return true;
}

// x = M^{-1} b with the factor in s.L; b and x are per-lane registers (row i = lane).
__device__ double chol_solve(SmallLds& s, int K, double b) {
    const int i = threadIdx.x;
    double y = b;
    for (int k = 0; k < K; ++k) {  // L y = b
        const double yk = bcast(y, k) * s.invd[k];
        if (i == k) y = yk;
        if (i > k && i < K) y -= s.L[i][k] * yk;
    }
    for (int k = K - 1; k >= 0; --k) {  // L^T x = y
        const double xk = bcast(y, k) * s.invd[k];
        if (i == k) y = xk;
        if (i < k) y -= s.L[k][i] * xk;
    }
    return i < K ? y : 0.0;
}

// (T z)_i for the lane's row, z distributed one entry per lane.
__device__ double matvec_T(SmallLds& s, int K, double z) {
    const int i = threadIdx.x;
    double acc = 0.0;
    for (int j = 0; j < K; ++j) {
        const double zj = bcast(z, j);
        if (i < K) acc += s.T[i][j] * zj;
    }
    return acc;
}

struct Eval {
    bool ok;
    double D2, dD2, z;  // z: this lane's entry
};

__device__ Eval evaluate(SmallLds& s, int K, double lam, double bb, double d, bool deriv, int& nfac) {
    Eval e{false, 0.0, 0.0, 0.0};
    ++nfac;
    if (!chol(s, K, lam)) return e;
    e.ok = true;
    e.z = chol_solve(s, K, d);
    const double w = matvec_T(s, K, e.z);
    const double dz = wave_sum64(d * e.z);
    const double zw = wave_sum64(e.z * w);
    e.D2 = bb - dz - lam * zw;
    if (deriv) {
        const double q = chol_solve(s, K, w);
        e.dD2 = 2.302585092994046 * 2.0 * lam * lam * wave_sum64(w * q);
    }
    return e;
}

__global__ __launch_bounds__(64) void k_small_solve(int K, const double* __restrict__ GA, const double* __restrict__ GT,
                                                    const double* __restrict__ dvec, const double* __restrict__ sc,
                                                    double fixed_lambda, double* __restrict__ zout,
                                                    double* __restrict__ res, double* __restrict__ lam_out) {
    __shared__ SmallLds s;
    const int i = threadIdx.x;
    // coalesced loads: each instruction moves one contiguous row of the 64-wide matrices
    for (int r = 0; r < K; ++r) {
        const double ga = GA[(int64_t)r * KMAX_SMALL + i];
        const double gt = GT[(int64_t)r * KMAX_SMALL + i];
        if (i < K) {
            s.A[r][i] = ga;
            s.T[r][i] = gt;
        }
    }
    const double d = i < K ? dvec[i] : 0.0;
    __syncthreads();
    const double bb = sc[0], target = sc[1];
    double lam = fixed_lambda;
    int status = 0;
    int nfac = 0;
    Eval e{false, 0.0, 0.0, 0.0};
    if (fixed_lambda > 0.0) {
        e = evaluate(s, K, lam, bb, d, false, nfac);
    } else {
        const double trA = wave_sum64(i < K ? s.A[i][i] : 0.0);
        const double trT = wave_sum64(i < K ? s.T[i][i] : 0.0);
        const double shift = log10(trA / fmax(trT, 1e-300));
        const double LO = -12.0 + shift, HI = 12.0 + shift;
        double lo = LO, hi = HI;
        bool lo_checked = false, hi_checked = false;
        double mu = 0.5 * (lo + hi);
        const double prev = sc[2];
        if (prev > 0.0) {
            const double m = log10(prev);
            if (m > lo && m < hi) mu = m;
        }
        // Newton in mu inside the bracket [lo, hi].  An end of the search interval is only
        // evaluated when a step would leave through it: an interior root proves, by
        // monotonicity of D^2, that neither end needs clamping.
        for (int it = 0; it < 200; ++it) {
            e = evaluate(s, K, pow(10.0, mu), bb, d, true, nfac);
            const double f = e.ok ? e.D2 - target : -target;
            MMOF_SMALL_TRACE(it, mu, e, f, lo, hi);
            if (f < 0.0)
                lo = mu;
            else
                hi = mu;
            if (e.ok && fabs(f) <= 1e-13 * bb) break;  // rounding level of D^2
            double nmu = (e.ok && e.dD2 > 0.0) ? mu - f / e.dD2 : 0.5 * (lo + hi);
            if (!(nmu > lo && nmu < hi)) {
                if (f < 0.0 && !hi_checked && hi == HI) {
                    hi_checked = true;
                    const Eval eh = evaluate(s, K, pow(10.0, HI), bb, d, false, nfac);
                    if (eh.ok && eh.D2 < target) {
                        e = eh;
                        mu = HI;
                        status = 2;
                        break;
                    }
                }
                if (f > 0.0 && !lo_checked && lo == LO) {
                    lo_checked = true;
                    const Eval el = evaluate(s, K, pow(10.0, LO), bb, d, false, nfac);
                    if (el.ok && el.D2 > target) {
                        e = el;
                        mu = LO;
                        status = 2;
                        break;
                    }
                }
                nmu = 0.5 * (lo + hi);
            }
            if (fabs(nmu - mu) <= 1e-11 * fmax(1.0, fabs(mu)) || hi - lo <= 1e-14 * fmax(1.0, fabs(mu))) {
                mu = nmu;
                e = evaluate(s, K, pow(10.0, mu), bb, d, false, nfac);
                break;
            }
            mu = nmu;
        }
        lam = pow(10.0, mu);
    }
    if (!e.ok) status = 4;
    if (i < K) zout[i] = e.ok ? e.z : 0.0;
    if (i == 0) {
        res[0] = lam;
        res[1] = e.D2;
        res[2] = (double)status;
        res[3] = (double)nfac;
        if (lam_out) lam_out[0] = lam;
    }
}

void small_solve(Ctx& c, int K, const double* GA, const double* GT, const double* d, const double* sc,
                 double fixed_lambda, double* z, double* res, double* lam_out) {
    MMOF_CHECK(K >= 1 && K <= KMAX_SMALL, MMOF_ERR_SHAPE, "Krylov basis size out of range");
    ScopedTime st(&c, "small_solve");
    hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(64), 0, c.stream, K, GA, GT, d, sc, fixed_lambda, z, res,
                       lam_out);
    MMOF_LAUNCH_CHECK();
}

}  // namespace mmof
