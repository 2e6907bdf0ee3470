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
// K <= 64: one wavefront.  Each evaluation factors M = G_H + lambda G_T with a blocked
// Cholesky (registers and matrix cores), then solves with the factor: the right-hand side is one entry
// per lane and each step broadcasts the finished entry with readlane.  D^2 and its
// derivative only need forward solves (d^T z = ||L^{-1} d||^2, w^T M^{-1} w = ||L^{-1} w||^2)
// plus one backward solve for z.
// 64 < K <= 256: four wavefronts, thread i owning row i; the factor lives in an L2-resident
// global workspace (too large for the LDS at these sizes), built and used in 16-column
// blocks: the wave holding a diagonal block factors it with readlane broadcasts, the other
// waves form their panel rows from it through the LDS, and every thread updates its own row
// of the trailing matrix; the triangular solves go block by block the same way (one barrier
// per block).  The root search is the same for both.
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

typedef double dbl4 __attribute__((ext_vector_type(4)));

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps r <- r (3 - x r^2) / 2
// (each step squares the relative error), a short dependency chain on the pivot path.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * r, r, 1.0);
        r = fma(0.5 * r, e, r);
    }
    return r;
}

// Blocked Cholesky of M = A + lam T into the lower triangle of s.L, in 16-column block
// columns (rows and columns K..16*ceil(K/16)-1 are padded with the identity).  Lane i owns
// row i.  A block column is loaded into registers and factored right-looking there (the
// pivot and the finished column entries are broadcast with readlane), written back, and
// the trailing lower blocks are updated on the FP64 matrix cores:
// M_{I,J'} -= L_{I,J} L_{J',J}^T with v_mfma_f64_16x16x4f64 (lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; the 16x16 result is D[l/16 + 4v][l%16] in four doubles per lane).
// Returns false on a non-positive pivot (uniform across the wave); on success *inv holds
// 1 / L[lane][lane].
__device__ bool chol(SmallLds& s, int K, double lam, double* inv) {
    const int i = threadIdx.x;
    const int nbk = (K + 15) >> 4;
    const int KP = nbk << 4;
    // M = A + lam T with the identity on the padded diagonal (A and T are zero outside
    // K x K); whole rows, without branches, so the LDS loads of 16 columns go out together
    const double pad = i >= K ? 1.0 : 0.0;
    for (int c0 = 0; c0 < KP; c0 += 16) {
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int c = c0 + cc;
            s.L[i][c] = fma(lam, s.T[i][c], s.A[i][c]) + (i == c ? pad : 0.0);
        }
    }
    __syncthreads();
    double my_inv = 0.0;
    for (int J = 0; J < nbk; ++J) {
        const int c0 = J << 4;
        double a[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double v = s.L[i][c0 + c];  // (every row is in the array: loads without branches)
            a[c] = (i >= c0 + c && i < KP) ? v : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double piv = bcast(a[c], c0 + c);
            if (!(piv > 0.0)) return false;
            const double r = rsqrt_nr(piv);
            const double l = a[c] * r;  // L[i][c0+c] for rows below the pivot, L[c0+c][c0+c] on its lane
            a[c] = l;
            if (i == c0 + c) my_inv = r;
#pragma unroll
            for (int c2 = c + 1; c2 < 16; ++c2) a[c2] -= l * bcast(l, c0 + c2);
        }
        // (the entries above the diagonal become zero; nothing reads them)
#pragma unroll
        for (int c = 0; c < 16; ++c) s.L[i][c0 + c] = a[c];
        __syncthreads();
        // trailing update of the lower blocks (I, J'), J < J' <= I
        const int lr = i & 15, lk = i >> 4;
        for (int Jp = J + 1; Jp < nbk; ++Jp) {
            for (int I = Jp; I < nbk; ++I) {
                dbl4 acc;
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] = s.L[(I << 4) + lk + 4 * v][(Jp << 4) + lr];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double av = -s.L[(I << 4) + lr][c0 + 4 * q + lk];
                    const double bv = s.L[(Jp << 4) + lr][c0 + 4 * q + lk];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) s.L[(I << 4) + lk + 4 * v][(Jp << 4) + lr] = acc[v];
            }
        }
        __syncthreads();
    }
    *inv = my_inv;
    return true;
}

// The solves below walk the columns in groups of four with the next group's LDS entries
// loaded ahead, so the LDS latency overlaps the broadcast chain.  The walk runs up to K
// rounded up to 4 (at most the padded size of the factor): a step j >= K changes nothing,
// since entry j of the right-hand side is zero and the rows it would update lie outside
// [0, K).

// y = L^{-1} b (one entry per lane)
__device__ double fwd_solve(const SmallLds& s, int K, double inv, double b) {
    const int i = threadIdx.x;
    const int row = min(i, KMAX_SMALL - 1);
    const int K4 = (K + 3) & ~3;
    double y = i < K ? b : 0.0;
    double l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) l[q] = s.L[row][q];
    for (int j = 0; j < K4; j += 4) {
        double nl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) nl[q] = s.L[row][min(j + 4 + q, KMAX_SMALL)];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jj = j + q;
            const double yj = bcast(y * inv, jj);
            const double upd = fma(-l[q], yj, y);
            y = (i == jj) ? yj : ((i > jj && i < K) ? upd : y);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) l[q] = nl[q];
    }
    return i < K ? y : 0.0;
}

// z = L^{-T} y
__device__ double bwd_solve(const SmallLds& s, int K, double inv, double y) {
    const int i = threadIdx.x;
    const int col = min(i, KMAX_SMALL - 1);
    const int K4 = (K + 3) & ~3;
    double z = i < K ? y : 0.0;
    double l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) l[q] = s.L[K4 - 1 - q][col];
    for (int j = K4 - 1; j >= 0; j -= 4) {
        double nl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) nl[q] = s.L[max(j - 4 - q, 0)][col];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jj = j - q;
            const double zj = bcast(z * inv, jj);
            const double upd = fma(-l[q], zj, z);
            z = (i == jj) ? zj : ((i < jj && i < K) ? upd : z);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) l[q] = nl[q];
    }
    return i < K ? z : 0.0;
}

// (T z)_i for the lane's row, z distributed one entry per lane (T is zero outside K x K).
__device__ double matvec_T(const SmallLds& s, int K, double z) {
    const int i = threadIdx.x;
    const int row = min(i, KMAX_SMALL - 1);
    const int K4 = (K + 3) & ~3;
    double acc = 0.0;
    for (int j = 0; j < K4; j += 4) {
        double t[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) t[q] = s.T[row][j + q];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += t[q] * bcast(z, j + q);
    }
    return i < K ? acc : 0.0;
}

struct Eval {
    bool ok;
    double D2, dD2, z;  // z: this lane's entry
};

__device__ Eval evaluate(SmallLds& s, int K, double lam, double bb, double d, bool deriv, int& nfac) {
    Eval e{false, 0.0, 0.0, 0.0};
    ++nfac;
    double inv;
    if (!chol(s, K, lam, &inv)) return e;
    e.ok = true;
    const double y = fwd_solve(s, K, inv, d);
    e.z = bwd_solve(s, K, inv, y);
    const double w = matvec_T(s, K, e.z);
    const double dz = wave_sum64(y * y);  // d^T z = ||L^{-1} d||^2
    const double zw = wave_sum64(e.z * w);
    e.D2 = bb - dz - lam * zw;
    if (deriv) {
        const double q = fwd_solve(s, K, inv, w);  // w^T M^{-1} w = ||L^{-1} w||^2
        e.dD2 = 2.302585092994046 * 2.0 * lam * lam * wave_sum64(q * q);
    }
    return e;
}

// The discrepancy-principle root in mu = log10(lambda) (or the fixed lambda), given
// ev(lambda, with_derivative) -> Eval and the traces of G_H and G_T (all three uniform across
// the threads of the solve).  Leaves the last accepted evaluation in e, lambda in lam and
// 0 (root) / 2 (clamped to an end of the bracket) in status.
template <class EV>
__device__ void dp_root(EV&& ev, double trA, double trT, double target, double bb, double prev, double fixed_lambda,
                        Eval& e, double& lam, int& status) {
    if (fixed_lambda > 0.0) {
        e = ev(lam, false);
        return;
    }
    const double shift = log10(trA / fmax(trT, 1e-300));
    const double LO = -12.0 + shift, HI = 12.0 + shift;
    double lo = LO, hi = HI;
    bool lo_checked = false, hi_checked = false;
    double mu = 0.5 * (lo + hi);
    if (prev > 0.0) {
        const double m = log10(prev);
        if (m > lo && m < hi) mu = m;
    }
    // Newton in mu inside the bracket [lo, hi].  An end of the search interval is only
    // evaluated when a step would leave through it: an interior root proves, by
    // monotonicity of D^2, that neither end needs clamping.
    for (int it = 0; it < 200; ++it) {
        e = ev(pow(10.0, mu), true);
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
                const Eval eh = ev(pow(10.0, HI), false);
                if (eh.ok && eh.D2 < target) {
                    e = eh;
                    mu = HI;
                    status = 2;
                    break;
                }
            }
            if (f > 0.0 && !lo_checked && lo == LO) {
                lo_checked = true;
                const Eval el = ev(pow(10.0, LO), false);
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
            // converged to ~1e-11 in log10(lambda): keep the evaluation at mu (its z and
            // D^2 differ from those at the root by the same relative amount) unless it failed
            if (!e.ok) {
                mu = nmu;
                e = ev(pow(10.0, mu), false);
            }
            break;
        }
        mu = nmu;
    }
    lam = pow(10.0, mu);
}

__global__ __launch_bounds__(64) void k_small_solve(int K, const double* __restrict__ GA, const double* __restrict__ GT,
                                                    const double* __restrict__ dvec, const double* __restrict__ sc,
                                                    double fixed_lambda, double* __restrict__ zout,
                                                    double* __restrict__ res, double* __restrict__ lam_out) {
    __shared__ SmallLds s;
    const int i = threadIdx.x;
    // coalesced loads: each instruction moves one contiguous row of the 64-wide matrices;
    // entries outside K x K are zero
    for (int r = 0; r < KMAX_SMALL; ++r) {
        double ga = 0.0, gt = 0.0;
        if (r < K) {
            ga = GA[(int64_t)r * KLD + i];
            gt = GT[(int64_t)r * KLD + i];
        }
        s.A[r][i] = i < K ? ga : 0.0;
        s.T[r][i] = i < K ? gt : 0.0;
    }
    const double d = i < K ? dvec[i] : 0.0;
    __syncthreads();
    const double bb = sc[0], target = sc[1];
    double lam = fixed_lambda;
    int status = 0;
    int nfac = 0;
    Eval e{false, 0.0, 0.0, 0.0};
    const double trA = fixed_lambda > 0.0 ? 0.0 : wave_sum64(i < K ? s.A[i][i] : 0.0);
    const double trT = fixed_lambda > 0.0 ? 0.0 : wave_sum64(i < K ? s.T[i][i] : 0.0);
    dp_root([&](double l, bool deriv) { return evaluate(s, K, l, bb, d, deriv, nfac); }, trA, trT, target, bb, sc[2],
            fixed_lambda, e, lam, status);
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

// ----------------------------------------------------------------------------- 64 < K <= 256

static constexpr int BIG_T = KMAX;   // threads of the multi-wave solve: thread i owns row i

struct BigLds {
    double P[KMAX][17];   // panel rows L[i][c0..c0+15] of the current block column (padded)
    double D[16][17];     // the diagonal block L_JJ
    double inv_d[16];     // 1 / L_JJ diagonal
    double vec[KMAX];     // finished entries of a triangular solve / the vector of a product
    double red[BIG_T / 64];
    int fail;
};

// Sum over the workgroup, bitwise identical in every thread (wave sums broadcast from lane
// 0, then the wave totals added in a fixed order from the LDS).
__device__ __forceinline__ double block_sum_uniform(BigLds& s, double v) {
    v = wave_sum64(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < BIG_T / 64; ++w) r += s.red[w];
    return r;
}

// Cholesky of M = A + lam T (A, T row-major with leading dimension KLD, symmetric) into the
// lower triangle of Lg (column-major: L[r][c] at Lg[c * KLD + r]).  Returns false, uniformly,
// on a non-positive pivot; on success inv = 1 / L[i][i] for this thread's row.
__device__ bool chol_big(BigLds& s, double* __restrict__ Lg, const double* __restrict__ A,
                         const double* __restrict__ T, int K, double lam, double& inv) {
    const int i = threadIdx.x;
    const bool mine = i < K;
    const int lane = i & 63, wave = i >> 6;
    // (every thread is past the previous factorization's reads of Lg and s.fail)
    __syncthreads();
    // M (lower triangle and the diagonal; A[i][c] = A[c][i] is read along row c: coalesced)
    if (mine)
        for (int c = 0; c <= i; ++c) Lg[(int64_t)c * KLD + i] = fma(lam, T[(int64_t)c * KLD + i], A[(int64_t)c * KLD + i]);
    if (i == 0) s.fail = 0;
    __syncthreads();
    double my_inv = 0.0;
    const int nbk = (K + 15) >> 4;
    for (int J = 0; J < nbk; ++J) {
        const int c0 = J << 4;
        const int nc = min(16, K - c0);
        const int w0 = c0 >> 6;   // the wave holding rows c0 .. c0 + 15
        double a[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] = (mine && c < nc && i >= c0 + c) ? Lg[(int64_t)(c0 + c) * KLD + i] : 0.0;
        if (wave == w0) {
            // right-looking factorization of the block column in registers: the pivot and the
            // finished entries of the diagonal rows come from their lanes (readlane)
            // (fully unrolled with guards: a register array indexed by a loop bound known only at
            // run time would be placed in scratch memory)
            bool ok = true;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                if (c < nc && ok) {
                    const double piv = bcast(a[c], (c0 + c) & 63);
                    if (!(piv > 0.0)) {
                        ok = false;   // uniform: the pivot is broadcast
                    } else {
                        const double r = rsqrt_nr(piv);
                        const double l = a[c] * r;
                        a[c] = l;
                        if (i == c0 + c) my_inv = r;
#pragma unroll
                        for (int c2 = c + 1; c2 < 16; ++c2)
                            if (c2 < nc) a[c2] -= l * bcast(l, (c0 + c2) & 63);
                    }
                }
            }
            if (!ok) {
                if (lane == 0) s.fail = 1;
            } else if (i >= c0 && i < c0 + nc) {
#pragma unroll
                for (int c = 0; c < 16; ++c) s.D[i - c0][c] = (c <= i - c0) ? a[c] : 0.0;
                s.inv_d[i - c0] = my_inv;
            }
        }
        __syncthreads();
        if (s.fail) return false;
        if (wave != w0 && mine && i >= c0 + 16) {
            // panel rows of the other waves: a_i L_JJ^{-T}, the same operations in the same order
            // as the in-wave factorization performs on its own rows
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                if (c < nc) {
                    double v = a[c];
#pragma unroll
                    for (int c2 = 0; c2 < 16; ++c2)
                        if (c2 < c) v -= a[c2] * s.D[c][c2];
                    a[c] = v * s.inv_d[c];
                }
            }
        }
        if (mine && i >= c0) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                if (c < nc) {
                    const double v = (i >= c0 + c) ? a[c] : 0.0;
                    Lg[(int64_t)(c0 + c) * KLD + i] = v;
                    s.P[i][c] = v;
                }
            }
        }
        __syncthreads();
        // trailing update of this thread's row: M[i][j] -= sum_c L[i][c0+c] L[j][c0+c], c0+16 <= j <= i,
        // four columns j at a time (independent sums), each sum in column order
        if (mine && i >= c0 + 16) {
            int j = c0 + 16;
            for (; j + 3 <= i; j += 4) {
                double m[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) m[q] = Lg[(int64_t)(j + q) * KLD + i];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c < nc) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) m[q] -= a[c] * s.P[j + q][c];
                    }
#pragma unroll
                for (int q = 0; q < 4; ++q) Lg[(int64_t)(j + q) * KLD + i] = m[q];
            }
            for (; j <= i; ++j) {
                double m = Lg[(int64_t)j * KLD + i];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c < nc) m -= a[c] * s.P[j][c];
                Lg[(int64_t)j * KLD + i] = m;
            }
        }
        __syncthreads();
    }
    inv = my_inv;
    return true;
}

// y = L^{-1} b, one entry per thread; block by block: the wave of a diagonal block solves its
// 16 entries with readlane broadcasts and publishes them, then every row below subtracts the
// block's contribution (the subtractions of a row in column order, as in the one-wave solve).
__device__ double fwd_big(BigLds& s, const double* __restrict__ Lg, int K, double inv, double b) {
    const int i = threadIdx.x;
    const bool mine = i < K;
    const int wave = i >> 6;
    double y = mine ? b : 0.0;
    __syncthreads();
    const int nbk = (K + 15) >> 4;
    for (int J = 0; J < nbk; ++J) {
        const int c0 = J << 4;
        const int nc = min(16, K - c0);
        if (wave == (c0 >> 6)) {
            double l[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) l[c] = (mine && c < nc && i > c0 + c) ? Lg[(int64_t)(c0 + c) * KLD + i] : 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                if (c < nc) {
                    const double yc = bcast(y * inv, (c0 + c) & 63);
                    if (i == c0 + c)
                        y = yc;
                    else if (i > c0 + c && i < c0 + nc)
                        y = fma(-l[c], yc, y);
                }
            }
            if (i >= c0 && i < c0 + nc) s.vec[i] = y;
        }
        __syncthreads();
        if (mine && i >= c0 + 16) {
            double l[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) l[c] = c < nc ? Lg[(int64_t)(c0 + c) * KLD + i] : 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < nc) y = fma(-l[c], s.vec[c0 + c], y);
        }
    }
    return mine ? y : 0.0;
}

// z = L^{-T} y, blocks from the last one up; a row reads the entries of its own column of L.
__device__ double bwd_big(BigLds& s, const double* __restrict__ Lg, int K, double inv, double y) {
    const int i = threadIdx.x;
    const bool mine = i < K;
    const int wave = i >> 6;
    double z = mine ? y : 0.0;
    __syncthreads();
    const int nbk = (K + 15) >> 4;
    for (int J = nbk - 1; J >= 0; --J) {
        const int c0 = J << 4;
        const int nc = min(16, K - c0);
        if (wave == (c0 >> 6)) {
            double l[16];   // L[c0 + c][i] for c0 + c > i
#pragma unroll
            for (int c = 0; c < 16; ++c) l[c] = (mine && c < nc && c0 + c > i) ? Lg[(int64_t)i * KLD + c0 + c] : 0.0;
#pragma unroll
            for (int c = 15; c >= 0; --c) {
                if (c < nc) {
                    const double zc = bcast(z * inv, (c0 + c) & 63);
                    if (i == c0 + c)
                        z = zc;
                    else if (i >= c0 && i < c0 + c)
                        z = fma(-l[c], zc, z);
                }
            }
            if (i >= c0 && i < c0 + nc) s.vec[i] = z;
        }
        __syncthreads();
        if (mine && i < c0) {
            double l[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) l[c] = c < nc ? Lg[(int64_t)i * KLD + c0 + c] : 0.0;
#pragma unroll
            for (int c = 15; c >= 0; --c)
                if (c < nc) z = fma(-l[c], s.vec[c0 + c], z);
        }
    }
    return mine ? z : 0.0;
}

__device__ Eval evaluate_big(BigLds& s, double* __restrict__ Lg, const double* __restrict__ GA,
                             const double* __restrict__ GT, int K, double lam, double bb, double d, bool deriv,
                             int& nfac) {
    const int i = threadIdx.x;
    Eval e{false, 0.0, 0.0, 0.0};
    ++nfac;
    double inv = 0.0;
    if (!chol_big(s, Lg, GA, GT, K, lam, inv)) return e;
    e.ok = true;
    const double y = fwd_big(s, Lg, K, inv, d);
    e.z = bwd_big(s, Lg, K, inv, y);
    // w = T z (T symmetric: row i read along column i, coalesced)
    __syncthreads();
    s.vec[i] = e.z;
    __syncthreads();
    double w = 0.0;
    if (i < K)
        for (int j = 0; j < K; ++j) w += GT[(int64_t)j * KLD + i] * s.vec[j];
    const double dz = block_sum_uniform(s, y * y);
    const double zw = block_sum_uniform(s, e.z * w);
    e.D2 = bb - dz - lam * zw;
    if (deriv) {
        const double q = fwd_big(s, Lg, K, inv, w);
        e.dD2 = 2.302585092994046 * 2.0 * lam * lam * block_sum_uniform(s, q * q);
    }
    return e;
}

__global__ __launch_bounds__(BIG_T) void k_small_solve_big(int K, const double* __restrict__ GA,
                                                           const double* __restrict__ GT,
                                                           const double* __restrict__ dvec,
                                                           const double* __restrict__ sc, double fixed_lambda,
                                                           double* __restrict__ Lg, double* __restrict__ zout,
                                                           double* __restrict__ res, double* __restrict__ lam_out) {
    __shared__ BigLds s;
    const int i = threadIdx.x;
    const double d = i < K ? dvec[i] : 0.0;
    const double bb = sc[0], target = sc[1];
    double lam = fixed_lambda;
    int status = 0;
    int nfac = 0;
    Eval e{false, 0.0, 0.0, 0.0};
    double trA = 0.0, trT = 0.0;
    if (!(fixed_lambda > 0.0)) {
        trA = block_sum_uniform(s, i < K ? GA[(int64_t)i * KLD + i] : 0.0);
        trT = block_sum_uniform(s, i < K ? GT[(int64_t)i * KLD + i] : 0.0);
    }
    dp_root([&](double l, bool deriv) { return evaluate_big(s, Lg, GA, GT, K, l, bb, d, deriv, nfac); }, trA, trT,
            target, bb, sc[2], fixed_lambda, e, lam, status);
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
    MMOF_CHECK(K >= 1 && K <= KMAX, MMOF_ERR_SHAPE, "Krylov basis size out of range");
    ScopedTime st(&c, "small_solve");
    if (K <= KMAX_SMALL) {
        hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(64), 0, c.stream, K, GA, GT, d, sc, fixed_lambda, z, res,
                           lam_out);
    } else {
        double* Lg = static_cast<double*>(c.work("small_L", sizeof(double) * (size_t)KLD * KLD));
        hipLaunchKernelGGL(k_small_solve_big, dim3(1), dim3(BIG_T), 0, c.stream, K, GA, GT, d, sc, fixed_lambda, Lg,
                           z, res, lam_out);
    }
    MMOF_LAUNCH_CHECK();
}

}  // namespace mmof
