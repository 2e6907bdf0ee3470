// FP64 generalized-Krylov machinery of MMGKS (Sec. 4.1.1, Alg. 1): inner products
// against a block of columns, column combinations, weighted Gram matrices of the
// projected operators, and the small projected solve with the discrepancy principle.
//
// Column blocks are stored column-major ([K][ld], each column contiguous) in the
// operator precision TX (float or double); all accumulation is in double.  Every
// reduction is two-stage with a fixed order, so results are bitwise reproducible.
#include "dev.h"
#include "krylov.h"

namespace mmof {

static constexpr int KB = 256;          // threads per block for the streaming kernels
static constexpr int MAX_PART = 1024;   // max partial blocks of a reduction

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block sum of one value per thread (256 threads), result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* s4) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s4[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    return r;
}

template <class TI, class TO>
__global__ void k_convert(int64_t n, const TI* __restrict__ in, TO* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (TO)in[i];
}

// part[b][j] = sum_{i in chunk b} X_j[i] * y[i]
template <class TX, class TY>
__global__ __launch_bounds__(KB) void k_mdot_part(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                  const TY* __restrict__ y, double* __restrict__ part) {
    __shared__ double s4[4];
    const int64_t nb = gridDim.x;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int j = 0; j < K; ++j) {
        const TX* xj = X + (int64_t)j * ld;
        double acc = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += KB) acc += (double)xj[i] * (double)y[i];
        const double s = block_sum(acc, s4);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * K + j] = s;
    }
}

// out[j] = alpha * sum_b part[b][j]  (fixed-order tree over b); one block per j.
__global__ __launch_bounds__(KB) void k_mdot_final(int nb, int K, const double* __restrict__ part, double alpha,
                                                   double* __restrict__ out) {
    __shared__ double s4[4];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += KB) acc += part[(int64_t)b * K + j];
    const double s = block_sum(acc, s4);
    if (threadIdx.x == 0) out[j] = alpha * s;
}

// out[i] = beta * out[i] + alpha * sum_j X_j[i] * h[j]   (h on the device)
template <class TX>
__global__ __launch_bounds__(KB) void k_gemv_cols(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                  const double* __restrict__ h, double alpha, double beta,
                                                  double* __restrict__ out) {
    __shared__ double sh[KMAX_SMALL];
    for (int j = threadIdx.x; j < K; j += KB) sh[j] = h[j];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
        double acc = 0.0;
        for (int j = 0; j < K; ++j) acc += (double)X[(int64_t)j * ld + i] * sh[j];
        out[i] = (beta == 0.0 ? 0.0 : beta * out[i]) + alpha * acc;
    }
}

// Weighted Gram, stage 1: part[b] (K x K, upper blocks) = X^T diag(w2) X over chunk b,
// w2 = 1/sqrt(nu^2 + eps^2) (or 1 when nu is null).  Rows are staged in LDS as double;
// each thread owns a 4x4 block of the Gram for a slice of the staged rows.
static constexpr int GCH = 32;  // rows staged per step
template <class TX>
__global__ __launch_bounds__(KB) void k_wgram_part(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                   const TX* __restrict__ nu, double eps2,
                                                   double* __restrict__ part) {
    __shared__ double sx[GCH][KMAX_SMALL + 1];
    __shared__ double sred[(KMAX_SMALL / 4) * (KMAX_SMALL / 4 + 1) / 2 * 16];
    const int nb4 = (K + 3) / 4;
    const int npairs = nb4 * (nb4 + 1) / 2;
    const int groups = max(1, KB / npairs);
    const int tid = threadIdx.x;
    const int pair = tid % npairs, grp = tid / npairs;
    const bool active = tid < npairs * groups;
    // block pair -> (bi, bj), bi <= bj
    int bi = 0, bj = 0;
    {
        int p = pair, row = 0;
        while (p >= nb4 - row) {
            p -= nb4 - row;
            ++row;
        }
        bi = row;
        bj = row + p;
    }
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

    const int64_t nbk = gridDim.x;
    const int64_t chunk = ((n + nbk - 1) / nbk + GCH - 1) / GCH * GCH;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int64_t r0 = lo; r0 < hi; r0 += GCH) {
        __syncthreads();
        // stage rows r0..r0+GCH of every column (weights folded into a copy below)
        for (int e = tid; e < GCH * K; e += KB) {
            const int j = e / GCH, r = e % GCH;
            const int64_t i = r0 + r;
            sx[r][j] = (i < hi) ? (double)X[(int64_t)j * ld + i] : 0.0;
        }
        for (int j = K + tid; j < 4 * nb4; j += KB)
            for (int r = 0; r < GCH; ++r) sx[r][j] = 0.0;
        __syncthreads();
        if (active) {
            for (int r = grp; r < GCH; r += groups) {
                const int64_t i = r0 + r;
                if (i >= hi) break;
                double w = 1.0;
                if (nu) {
                    const double a = (double)nu[i];
                    w = 1.0 / sqrt(a * a + eps2);
                }
                double xa[4], xb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    xa[a] = sx[r][4 * bi + a] * w;
                    xb[a] = sx[r][4 * bj + a];
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * xb[b];
            }
        }
    }
    // reduce the row groups into group 0 through LDS, highest group first (fixed order)
    for (int g = groups - 1; g >= 1; --g) {
        __syncthreads();
        if (active && grp == g) {
#pragma unroll
            for (int e = 0; e < 16; ++e) sred[pair * 16 + e] = acc[e / 4][e % 4];
        }
        __syncthreads();
        if (active && grp == 0) {
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[e / 4][e % 4] += sred[pair * 16 + e];
        }
    }
    if (active && grp == 0) {
        double* out = part + (int64_t)blockIdx.x * KMAX_SMALL * KMAX_SMALL;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int ii = 4 * bi + a, jj = 4 * bj + b;
                if (ii < K && jj < K) out[(int64_t)ii * KMAX_SMALL + jj] = acc[a][b];
            }
    }
}

// Weighted Gram, stage 2: G[i][j] = sum_b part[b][i][j] for i <= j (block order), mirrored.
__global__ __launch_bounds__(KB) void k_wgram_final(int nb, int K, const double* __restrict__ part,
                                                    double* __restrict__ G, int ldg) {
    for (int e = blockIdx.x * KB + threadIdx.x; e < K * K; e += gridDim.x * KB) {
        const int i = e / K, j = e % K;
        if (i > j) continue;
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) acc += part[(int64_t)b * KMAX_SMALL * KMAX_SMALL + (int64_t)i * KMAX_SMALL + j];
        G[(int64_t)i * ldg + j] = acc;
        G[(int64_t)j * ldg + i] = acc;
    }
}

// Scale x by 1/s[0] when s[0] > thr, else leave a zero column; s holds ||x||.
__global__ void k_normalize(int64_t n, const double* __restrict__ x, const double* __restrict__ nrm, double thr,
                            double* __restrict__ out) {
    const double s = nrm[0];
    const double inv = s > thr ? 1.0 / s : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = x[i] * inv;
}

// out = a*x + b*y (doubles; x, y may alias out)
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, const double* y, double* out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// out = x + lam[0] * y where x, y are in the operator precision TX.
template <class TX>
__global__ void k_residual_combine(int64_t n, const TX* __restrict__ x, const TX* __restrict__ y,
                                   const double* __restrict__ lam, double* __restrict__ out) {
    const double l = lam[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)x[i] + l * (double)y[i];
}

// y[i] = w2(nu[i]) * x[i] in TX, w2 = 1/sqrt(nu^2 + eps^2).
template <class TX>
__global__ void k_weight_apply(int64_t n, const TX* __restrict__ nu, double eps2, const double* __restrict__ x,
                               TX* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)nu[i];
        y[i] = (TX)(x[i] / sqrt(a * a + eps2));
    }
}

// diff = x - y (doubles), for RRE
__global__ void k_sub(int64_t n, const double* __restrict__ x, const double* __restrict__ y, double* __restrict__ d) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = x[i] - y[i];
}

template <class T>
__global__ void k_fill_zero(int64_t n, T* __restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

__global__ void k_set_scalar(double* p, double v) { *p = v; }
__global__ void k_sqrt_scalar(const double* in, double* out) { *out = sqrt(fmax(*in, 0.0)); }
__global__ void k_copy_scalar(double* dst, const double* src) { *dst = *src; }

// y += sign * s[0] * x
__global__ void k_axpy_dev(int64_t n, const double* __restrict__ x, double* __restrict__ y,
                           const double* __restrict__ s, double sign) {
    const double a = sign * s[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

// G[j][i] = G[i][j] = h[i] for i <= j
__global__ void k_put_rowcol(double* __restrict__ G, int ldg, int j, const double* __restrict__ h) {
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        G[(int64_t)j * ldg + i] = h[i];
        G[(int64_t)i * ldg + j] = h[i];
    }
}

// y = w2(nu) * x in TX
template <class TX>
__global__ void k_weight_mul(int64_t n, const TX* __restrict__ nu, double eps2, const TX* __restrict__ x,
                             TX* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)nu[i];
        y[i] = (TX)((double)x[i] / sqrt(a * a + eps2));
    }
}

// ------------------------------------------------------------------------ host launchers

template <class T>
void fill_zero(Ctx& c, int64_t n, T* p) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_zero<T>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, p);
    MMOF_LAUNCH_CHECK();
}
template void fill_zero<float>(Ctx&, int64_t, float*);
template void fill_zero<double>(Ctx&, int64_t, double*);

void set_scalar(Ctx& c, double* p, double v) {
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, c.stream, p, v);
    MMOF_LAUNCH_CHECK();
}
void sqrt_scalar(Ctx& c, const double* in, double* out) {
    hipLaunchKernelGGL(k_sqrt_scalar, dim3(1), dim3(1), 0, c.stream, in, out);
    MMOF_LAUNCH_CHECK();
}
void copy_scalar(Ctx& c, double* dst, const double* src) {
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c.stream, dst, src);
    MMOF_LAUNCH_CHECK();
}
void axpy_dev(Ctx& c, int64_t n, const double* x, double* y, const double* s, double sign) {
    hipLaunchKernelGGL(k_axpy_dev, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, x, y, s, sign);
    MMOF_LAUNCH_CHECK();
}
void put_rowcol(Ctx& c, double* G, int ldg, int j, const double* h) {
    hipLaunchKernelGGL(k_put_rowcol, dim3(1), dim3(64), 0, c.stream, G, ldg, j, h);
    MMOF_LAUNCH_CHECK();
}
template <class TX>
void weight_mul(Ctx& c, int64_t n, const TX* nu, double eps, const TX* x, TX* y) {
    hipLaunchKernelGGL(k_weight_mul<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, nu, eps * eps, x, y);
    MMOF_LAUNCH_CHECK();
}
template void weight_mul<float>(Ctx&, int64_t, const float*, double, const float*, float*);
template void weight_mul<double>(Ctx&, int64_t, const double*, double, const double*, double*);


int mdot_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(MAX_PART, cdiv(n, 2048))); }

template <class TX, class TY>
void mdot(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TY* y, double alpha, double* out) {
    if (K <= 0) return;
    const int nb = mdot_blocks(n);
    MMOF_CHECK(K <= KMAX_SMALL, MMOF_ERR_SHAPE, "too many columns for a block inner product");
    double* part = static_cast<double*>(c.work("mdot_part", sizeof(double) * (size_t)MAX_PART * KMAX_SMALL));
    hipLaunchKernelGGL((k_mdot_part<TX, TY>), dim3(nb), dim3(KB), 0, c.stream, n, K, X, ld, y, part);
    MMOF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mdot_final, dim3(K), dim3(KB), 0, c.stream, nb, K, part, alpha, out);
    MMOF_LAUNCH_CHECK();
}
template void mdot<float, double>(Ctx&, int64_t, int, const float*, int64_t, const double*, double, double*);
template void mdot<double, double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double, double*);
template void mdot<float, float>(Ctx&, int64_t, int, const float*, int64_t, const float*, double, double*);

template <class TX>
void gemv_cols(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* h, double alpha, double beta,
               double* out) {
    MMOF_CHECK(K <= KMAX_SMALL, MMOF_ERR_SHAPE, "too many Krylov columns");
    if (K <= 0) {
        if (beta != 1.0) {
            hipLaunchKernelGGL(k_axpby, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, beta, (const double*)out,
                               0.0, (const double*)out, out);
            MMOF_LAUNCH_CHECK();
        }
        return;
    }
    hipLaunchKernelGGL(k_gemv_cols<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, K, X, ld, h, alpha, beta,
                       out);
    MMOF_LAUNCH_CHECK();
}
template void gemv_cols<float>(Ctx&, int64_t, int, const float*, int64_t, const double*, double, double, double*);
template void gemv_cols<double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double, double, double*);

template <class TX>
void wgram(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TX* nu, double eps, double* G, int ldg) {
    MMOF_CHECK(K <= KMAX_SMALL, MMOF_ERR_SHAPE, "too many Krylov columns");
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(512, cdiv(n, 4096)));
    double* part = static_cast<double*>(c.work("wgram_part", sizeof(double) * (size_t)512 * KMAX_SMALL * KMAX_SMALL));
    {
        ScopedTime st(&c, "wgram");
        hipLaunchKernelGGL(k_wgram_part<TX>, dim3(nb), dim3(KB), 0, c.stream, n, K, X, ld, nu, eps * eps, part);
        MMOF_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_wgram_final, dim3((unsigned)cdiv((int64_t)K * K, KB)), dim3(KB), 0, c.stream, nb, K, part,
                       G, ldg);
    MMOF_LAUNCH_CHECK();
}
template void wgram<float>(Ctx&, int64_t, int, const float*, int64_t, const float*, double, double*, int);
template void wgram<double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double, double*, int);

template <class TI, class TO>
void convert(Ctx& c, int64_t n, const TI* in, TO* out) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_convert<TI, TO>), grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, in, out);
    MMOF_LAUNCH_CHECK();
}
template void convert<double, float>(Ctx&, int64_t, const double*, float*);
template void convert<float, double>(Ctx&, int64_t, const float*, double*);
template void convert<double, double>(Ctx&, int64_t, const double*, double*);
template void convert<float, float>(Ctx&, int64_t, const float*, float*);

void normalize(Ctx& c, int64_t n, const double* x, const double* nrm, double thr, double* out) {
    hipLaunchKernelGGL(k_normalize, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, x, nrm, thr, out);
    MMOF_LAUNCH_CHECK();
}

void axpby(Ctx& c, int64_t n, double a, const double* x, double b, const double* y, double* out) {
    hipLaunchKernelGGL(k_axpby, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, a, x, b, y, out);
    MMOF_LAUNCH_CHECK();
}

template <class TX>
void residual_combine(Ctx& c, int64_t n, const TX* x, const TX* y, const double* lam, double* out) {
    hipLaunchKernelGGL(k_residual_combine<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, x, y, lam, out);
    MMOF_LAUNCH_CHECK();
}
template void residual_combine<float>(Ctx&, int64_t, const float*, const float*, const double*, double*);
template void residual_combine<double>(Ctx&, int64_t, const double*, const double*, const double*, double*);

template <class TX>
void weight_apply(Ctx& c, int64_t n, const TX* nu, double eps, const double* x, TX* y) {
    hipLaunchKernelGGL(k_weight_apply<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, nu, eps * eps, x, y);
    MMOF_LAUNCH_CHECK();
}
template void weight_apply<float>(Ctx&, int64_t, const float*, double, const double*, float*);
template void weight_apply<double>(Ctx&, int64_t, const double*, double, const double*, double*);

void sub(Ctx& c, int64_t n, const double* x, const double* y, double* d) {
    hipLaunchKernelGGL(k_sub, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, x, y, d);
    MMOF_LAUNCH_CHECK();
}

}  // namespace mmof
