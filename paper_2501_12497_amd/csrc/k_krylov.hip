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

// FP64 MM weights w2 = 1/sqrt(nu^2 + eps^2) of the rows of Theta.
template <class TX>
__global__ void k_mm_weights_f64(int64_t n, const TX* __restrict__ nu, double eps2, double* __restrict__ w) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)nu[i];
        w[i] = 1.0 / sqrt(a * a + eps2);
    }
}

template <class TI, class TO>
__global__ void k_convert(int64_t n, const TI* __restrict__ in, TO* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (TO)in[i];
}

// part[b][j] = sum_{i in chunk b} X_j[i] * y[i]; eight columns per pass over the chunk.
template <class TX, class TY>
__global__ __launch_bounds__(KB) void k_mdot_part(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                  const TY* __restrict__ y, double* __restrict__ part) {
    __shared__ double s8[4][8];
    const int64_t nb = gridDim.x;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j0 = 0; j0 < K; j0 += 8) {
        const int nj = min(8, K - j0);
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += KB) {
            const double yi = (double)y[i];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nj) acc[q] += (double)X[(int64_t)(j0 + q) * ld + i] * yi;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = wave_sum(acc[q]);
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) s8[w][q] = acc[q];
        }
        __syncthreads();
        if (threadIdx.x < nj)
            part[(int64_t)blockIdx.x * K + j0 + threadIdx.x] =
                (s8[0][threadIdx.x] + s8[1][threadIdx.x]) + (s8[2][threadIdx.x] + s8[3][threadIdx.x]);
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

// Weighted Gram G = X^T diag(w2) X (K <= 64), w2 = 1/sqrt(nu^2 + eps^2) (1 when nu is null),
// on the FP64 matrix cores: v_mfma_f64_16x16x4f64 multiplies a 16x4 block of X^T by a
// 4x16 block of diag(w2) X.  Lane l supplies A[l%16][l/16] and B[l/16][l%16], which here
// are the same entry X[16g + l%16][r0 + l/16] (times w2 for B); the 16x16 result sits in
// four doubles per lane, D[l/16 + 4v][l%16] (layout checked on the device).  Each wave keeps the upper blocks of the
// (K/16)^2 block grid for its rows; stage 1 writes one partial Gram per workgroup.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <class TX>
struct GramStep {
    TX x[4][4];   // [row group u][column group g]
    double w[4];  // row weights
};

template <class TX>
__device__ __forceinline__ void gram_load(GramStep<TX>& st, const TX* __restrict__ X, int64_t ld,
                                          const double* __restrict__ w, int64_t r0, int64_t hi, int K, int G,
                                          int lane) {
    const int c = lane & 15;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t r = r0 + 4 * u + (lane >> 4);
        const bool inr = r < hi;
        st.w[u] = inr ? (w ? w[r] : 1.0) : 0.0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int col = 16 * g + c;
            st.x[u][g] = (g < G && col < K && inr) ? X[(int64_t)col * ld + r] : TX(0);
        }
    }
}

template <class TX>
__global__ __launch_bounds__(KB) void k_wgram_part(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                   const double* __restrict__ w, double* __restrict__ part) {
    __shared__ double sred[2][10][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int G = (K + 15) >> 4;
    dbl4 acc[10];
#pragma unroll
    for (int p = 0; p < 10; ++p) acc[p] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int64_t nbk = gridDim.x;
    const int64_t chunk = ((n + nbk - 1) / nbk + 63) / 64 * 64;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    // Each wave takes 4 groups of 4 rows per step (16 rows), the block 64 rows per step.
    // The next step's loads are issued before the current step's MFMAs.
    GramStep<TX> cur, nxt;
    int64_t r0 = lo + 16 * wave;
    if (r0 < hi) gram_load(cur, X, ld, w, r0, hi, K, G, lane);
    for (; r0 < hi; r0 += 64) {
        if (r0 + 64 < hi) gram_load(nxt, X, ld, w, r0 + 64, hi, K, G, lane);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double wu = cur.w[u];
            double a[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) a[g] = (double)cur.x[u][g];
            int p = 0;
#pragma unroll
            for (int gi = 0; gi < 4; ++gi)
#pragma unroll
                for (int gj = gi; gj < 4; ++gj, ++p)
                    if (gj < G) acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[gi], a[gj] * wu, acc[p], 0, 0, 0);
        }
        cur = nxt;
    }
    // combine the four waves in a fixed order: (w2, w3) into (w0, w1), then w1 into w0
    if (wave >= 2) {
#pragma unroll
        for (int p = 0; p < 10; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) sred[wave - 2][p][v][lane] = acc[p][v];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int p = 0; p < 10; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[p][v] += sred[wave][p][v][lane];
    }
    __syncthreads();
    if (wave == 1) {
#pragma unroll
        for (int p = 0; p < 10; ++p)
#pragma unroll
            for (int v = 0; v < 4; ++v) sred[0][p][v][lane] = acc[p][v];
    }
    __syncthreads();
    if (wave == 0) {
        double* out = part + (int64_t)blockIdx.x * KMAX_SMALL * KMAX_SMALL;
        int p = 0;
#pragma unroll
        for (int gi = 0; gi < 4; ++gi)
#pragma unroll
            for (int gj = gi; gj < 4; ++gj, ++p) {
                if (gj >= G) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ii = 16 * gi + (lane >> 4) + 4 * v, jj = 16 * gj + (lane & 15);
                    if (ii < K && jj < K) out[(int64_t)ii * KMAX_SMALL + jj] = acc[p][v] + sred[0][p][v][lane];
                }
            }
    }
}

// Weighted Gram, stage 2: G[i][j] = sum_b part[b][entry].  Four entries per workgroup, one
// wavefront per entry: lane l sums partials l, l+64, ... and the wave combines them with a
// fixed butterfly.
__global__ __launch_bounds__(KB) void k_wgram_final(int nb, int K, const double* __restrict__ part,
                                                    double* __restrict__ G, int ldg) {
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (e >= K * K) return;
    const int i = e / K, j = e % K;
    // upper-block storage: the entry lives at (i, j) if its block is upper, else at (j, i)
    const bool up = (i >> 4) <= (j >> 4);
    const int ii = up ? i : j, jj = up ? j : i;
    const double* src = part + (int64_t)ii * KMAX_SMALL + jj;
    double acc = 0.0;
    for (int b = lane; b < nb; b += 64) acc += src[(int64_t)b * KMAX_SMALL * KMAX_SMALL];
    acc = wave_sum(acc);
    if (lane == 0) G[(int64_t)i * ldg + j] = acc;
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

// y = w * x in TX (w: FP64 MM weights)
template <class TX>
__global__ void k_weight_mul(int64_t n, const double* __restrict__ w, const TX* __restrict__ x, TX* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (TX)((double)x[i] * w[i]);
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
void weight_mul(Ctx& c, int64_t n, const double* w, const TX* x, TX* y) {
    hipLaunchKernelGGL(k_weight_mul<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, w, x, y);
    MMOF_LAUNCH_CHECK();
}
template void weight_mul<float>(Ctx&, int64_t, const double*, const float*, float*);
template void weight_mul<double>(Ctx&, int64_t, const double*, const double*, double*);


int mdot_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(MAX_PART, cdiv(n, 1024))); }

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
void mm_weights_f64(Ctx& c, int64_t n, const TX* nu, double eps, double* w) {
    hipLaunchKernelGGL(k_mm_weights_f64<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, nu, eps * eps, w);
    MMOF_LAUNCH_CHECK();
}
template void mm_weights_f64<float>(Ctx&, int64_t, const float*, double, double*);
template void mm_weights_f64<double>(Ctx&, int64_t, const double*, double, double*);

template <class TX>
void wgram(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* w, double* G, int ldg) {
    MMOF_CHECK(K >= 1 && K <= KMAX_SMALL, MMOF_ERR_SHAPE, "too many Krylov columns");
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(256, cdiv(n, 1024)));
    double* part = static_cast<double*>(c.work("wgram_part", sizeof(double) * (size_t)256 * KMAX_SMALL * KMAX_SMALL));
    {
        ScopedTime st(&c, "wgram");
        hipLaunchKernelGGL(k_wgram_part<TX>, dim3(nb), dim3(KB), 0, c.stream, n, K, X, ld, w, part);
        MMOF_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_wgram_final, dim3((unsigned)cdiv((int64_t)K * K, 4)), dim3(KB), 0, c.stream, nb, K, part,
                       G, ldg);
    MMOF_LAUNCH_CHECK();
}
template void wgram<float>(Ctx&, int64_t, int, const float*, int64_t, const double*, double*, int);
template void wgram<double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double*, int);

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
