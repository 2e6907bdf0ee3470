// FP64 generalized-Krylov machinery of MMGKS (Sec. 4.1.1, Alg. 1): inner products
// against a block of columns, column combinations, weighted Gram matrices of the
// projected operators, and the small projected solve with the discrepancy principle.
//
// Column blocks are stored column-major ([K][ld], each column contiguous) in the
// operator precision TX (float or double); all accumulation is in double.  Every
// reduction is two-stage with a fixed order, so results are bitwise reproducible.
#include <mutex>

#include "dev.h"
#include "krylov.h"

namespace mmof {

static constexpr int KB = 256;          // threads per block for the streaming kernels
static constexpr int MAX_PART = 8192;   // max row chunks of a block inner product
static constexpr int MAX_GEMV_PART = 32768;   // max workgroups of a column combination

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

// sum_j X[j][i] h[j] in column order; the loads go out in groups of 8 (all in flight
// together) ahead of the sequential sum.
template <class TX>
__device__ __forceinline__ double dot_row(const TX* __restrict__ X, int64_t ld, int64_t i, int K,
                                          const double* __restrict__ h) {
    double acc = 0.0;
    for (int j0 = 0; j0 < K; j0 += 8) {
        double q[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) q[t] = j0 + t < K ? (double)X[(int64_t)(j0 + t) * ld + i] : 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (j0 + t < K) acc += q[t] * h[j0 + t];
    }
    return acc;
}

// dot_row for the rows i and i + 1 at once: one 2-element load per column (element-aligned,
// which global loads accept, so any ld qualifies); each row's sum in column order as in dot_row.
// The columns are streamed once, so their loads are marked nontemporal (measured at 67M rows
// x 11..39 FP64 columns: 5.6-5.7 TB/s against 5.0-5.3 TB/s with ordinary loads).
template <class TX>
__device__ __forceinline__ void dot_row2(const TX* __restrict__ X, int64_t ld, int64_t i, int K,
                                         const double* __restrict__ h, double& a0, double& a1) {
    typedef TX V2 __attribute__((ext_vector_type(2), aligned(sizeof(TX))));
    a0 = 0.0;
    a1 = 0.0;
    for (int j0 = 0; j0 < K; j0 += 8) {
        V2 q[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            q[t] = j0 + t < K ? __builtin_nontemporal_load(reinterpret_cast<const V2*>(X + (int64_t)(j0 + t) * ld + i))
                              : V2{TX(0), TX(0)};
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (j0 + t < K) {
                a0 += (double)q[t].x * h[j0 + t];
                a1 += (double)q[t].y * h[j0 + t];
            }
    }
}

// FP64 MM weights w2 = 1/sqrt(nu^2 + eps^2) of the rows of Theta.
template <class TX>
__global__ void k_mm_weights_f64(int64_t n, const TX* __restrict__ nu, double eps2, double* __restrict__ w) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        w[i] = mm_weight((double)nu[i], eps2);
    }
}

template <class TI, class TO>
__global__ void k_convert(int64_t n, const TI* __restrict__ in, TO* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (TO)in[i];
}

// Row chunk bx and column group gy (8 columns) of a block inner-product workgroup.  The grid is
// one-dimensional, 8 * ceil(nb / 8) * ng workgroups (nb row chunks, ng column groups).  The
// dispatcher deals workgroups to the eight XCDs in turn (workgroup L runs on XCD L % 8), and
// the ng groups of one row chunk take consecutive slots of one XCD, so they run close together
// and read y through that XCD's L2 once from HBM.  False for the padding of the last round.
__device__ __forceinline__ bool mdot_tile(int nb, int ng, int& bx, int& gy) {
    const int L = (int)blockIdx.x, x = L & 7, s = L >> 3;
    bx = (s / ng) * 8 + x;
    gy = s % ng;
    return bx < nb;
}

// Inner products of K columns (and of one extra FP64 column xe, when given) with y, over nb
// row chunks (grid: mdot_tile); part[j * nb + b] receives chunk b's sum for column j.  (A
// single-launch completion by the last workgroup would need a device-scope release per
// workgroup, which writes back the XCD's L2; a second small launch is cheaper.)
// skip (may be null): when *skip is non-zero the launch does nothing (this and the other
// kernels of a conditional pass read the decision on the device).
template <class TX, class TY>
__global__ __launch_bounds__(KB) void k_mdot(int64_t n, int K, int nbc, const TX* __restrict__ X, int64_t ld,
                                             const TY* __restrict__ y, const double* __restrict__ xe,
                                             double* __restrict__ part, const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double s8[4][8];
    const int Kt = K + (xe ? 1 : 0);
    int bx, gy;
    if (!mdot_tile(nbc, (Kt + 7) / 8, bx, gy)) return;
    const int64_t nb = nbc;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t lo = bx * chunk, hi = min(n, lo + chunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j0 = gy * 8;
    const int nj = min(8, Kt - j0);
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += KB) {
        const double yi = (double)y[i];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = j0 + q;
            if (q < nj) acc[q] += (j < K ? (double)X[(int64_t)j * ld + i] : xe[i]) * yi;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) s8[w][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < nj)
        part[(int64_t)(j0 + threadIdx.x) * nb + bx] =
            (s8[0][threadIdx.x] + s8[1][threadIdx.x]) + (s8[2][threadIdx.x] + s8[3][threadIdx.x]);
}

// k_mdot with two rows per lane (chunks of an even number of rows; 2-element loads of the
// columns, of y and of xe); a chunk with an odd row count ends with one single row.  The K
// columns are streamed once and their loads are marked nontemporal, so that they do not
// evict y, which the other column groups of the chunk read from L2 (measured at 67M rows x
// 11..39 FP64 columns: 6.5-7.1 TB/s, against 5.3-5.7 TB/s with a two-dimensional grid and
// ordinary loads).
template <class TX, class TY>
__global__ __launch_bounds__(KB) void k_mdot2(int64_t n, int K, int nbc, const TX* __restrict__ X, int64_t ld,
                                              const TY* __restrict__ y, const double* __restrict__ xe,
                                              double* __restrict__ part, const int* __restrict__ skip) {
    if (skip && *skip) return;
    // (element-aligned: global multi-word loads accept it, so any ld and any column qualify)
    typedef TX VX __attribute__((ext_vector_type(2), aligned(sizeof(TX))));
    typedef TY VY __attribute__((ext_vector_type(2), aligned(sizeof(TY))));
    typedef double VD __attribute__((ext_vector_type(2), aligned(sizeof(double))));
    __shared__ double s8[4][8];
    const int Kt = K + (xe ? 1 : 0);
    int bx, gy;
    if (!mdot_tile(nbc, (Kt + 7) / 8, bx, gy)) return;
    const int64_t nb = nbc;
    const int64_t chunk = 2 * ((n + 2 * nb - 1) / (2 * nb));
    const int64_t lo = bx * chunk, hi = min(n, lo + chunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j0 = gy * 8;
    const int nj = min(8, Kt - j0);
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    for (int64_t i = lo + 2 * (int64_t)threadIdx.x; i < hi; i += 2 * KB) {
        if (i + 1 < hi) {
            const VY yv = *reinterpret_cast<const VY*>(y + i);
            const double y0 = (double)yv.x, y1 = (double)yv.y;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + q;
                if (q < nj) {
                    double x0, x1;
                    if (j < K) {
                        const VX xv = __builtin_nontemporal_load(reinterpret_cast<const VX*>(X + (int64_t)j * ld + i));
                        x0 = (double)xv.x;
                        x1 = (double)xv.y;
                    } else {
                        const VD xv = *reinterpret_cast<const VD*>(xe + i);
                        x0 = xv.x;
                        x1 = xv.y;
                    }
                    acc[q] += x0 * y0;
                    acc[q] += x1 * y1;
                }
            }
        } else {
            const double yi = (double)y[i];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + q;
                if (q < nj) acc[q] += (j < K ? (double)X[(int64_t)j * ld + i] : xe[i]) * yi;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) s8[w][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < nj)
        part[(int64_t)(j0 + threadIdx.x) * nb + bx] =
            (s8[0][threadIdx.x] + s8[1][threadIdx.x]) + (s8[2][threadIdx.x] + s8[3][threadIdx.x]);
}

// Sums of the chunk partials part[j * nb + b] in a fixed order, one workgroup of 256 threads per
// column j (grid Kt): thread t sums chunks t, t + 256, ... in eight interleaved running sums
// (the eight loads of a step in flight together) combined in a fixed order, then the
// workgroup's fixed-order sum:
//   G == null: out[j] = alpha * s_j (j < Kt)
//   G != null: G[row][j] = G[j][row] = s_j for j < Kt - 1 and dj[0] = s_{Kt-1}.
__global__ __launch_bounds__(KB) void k_mdot_final(int nb, int Kt, const double* __restrict__ part, double alpha,
                                                   double* __restrict__ out, double* __restrict__ G, int ldg,
                                                   int row, double* __restrict__ dj, const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double s4[4];
    const int j = blockIdx.x;
    const double* __restrict__ pj = part + (int64_t)j * nb;
    double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b0 = threadIdx.x; b0 < nb; b0 += 8 * KB) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + KB * u;
            if (b < nb) a8[u] += pj[b];
        }
    }
    const double a = block_sum(((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7])), s4);
    if (threadIdx.x == 0) {
        if (!G)
            out[j] = alpha * a;
        else if (j < Kt - 1) {
            G[(int64_t)row * ldg + j] = a;
            G[(int64_t)j * ldg + row] = a;
        } else {
            dj[0] = a;
        }
    }
}

// out[i] = beta * out[i] + alpha * sum_j X_j[i] * h[j]   (h on the device)
template <class TX>
__global__ __launch_bounds__(KB) void k_gemv_cols(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                  const double* __restrict__ h, double alpha, double beta,
                                                  double* __restrict__ out) {
    __shared__ double sh[KMAX];
    for (int j = threadIdx.x; j < K; j += KB) sh[j] = h[j];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
        const double acc = dot_row(X, ld, i, K, sh);
        out[i] = (beta == 0.0 ? 0.0 : beta * out[i]) + alpha * acc;
    }
}

// v_i = alpha * sum_j X_j[i] h[j] + beta * y[i]; stores v (FP64) and/or its rounding to TO,
// and optionally the workgroup's partial of sum (v_i - cv_i)^2 (sum v_i^2 without cv) in
// part[blockIdx.x].  y and out_d may alias.
template <class TX, class TO>
__global__ __launch_bounds__(KB) void k_gemv_fused(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                   const double* __restrict__ h, double alpha, const double* y,
                                                   double beta, double* out_d, TO* __restrict__ out_t,
                                                   const double* __restrict__ cv, double* __restrict__ part,
                                                   const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double sh[KMAX];
    __shared__ double s4[4];
    for (int j = threadIdx.x; j < K; j += KB) sh[j] = h[j];
    __syncthreads();
    double e2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x; i < n; i += (int64_t)gridDim.x * KB) {
        const double acc = dot_row(X, ld, i, K, sh);
        const double v = alpha * acc + (y ? beta * y[i] : 0.0);
        if (out_d) out_d[i] = v;
        if (out_t) out_t[i] = (TO)v;
        if (part) {
            const double e = cv ? v - cv[i] : v;
            e2 += e * e;
        }
    }
    if (!part) return;
    const double bs = block_sum(e2, s4);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// k_gemv_fused with two rows per lane (dot_row2); n odd leaves one single row.  Each
// workgroup walks one contiguous chunk of rows (a multiple of 2 KB rows), so that each column
// is read as sequential runs (a grid-strided walk measured 10% slower); many short chunks
// (2048 rows) beat few long ones (5.7 against 5.5 TB/s with 8192-row chunks at 67M rows).
template <class TX, class TO>
__global__ __launch_bounds__(KB) void k_gemv_fused2(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                    const double* __restrict__ h, double alpha, const double* y,
                                                    double beta, double* out_d, TO* __restrict__ out_t,
                                                    const double* __restrict__ cv, double* __restrict__ part,
                                                    const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double sh[KMAX];
    __shared__ double s4[4];
    for (int j = threadIdx.x; j < K; j += KB) sh[j] = h[j];
    __syncthreads();
    double e2 = 0.0;
    auto finish = [&](int64_t i, double acc) {
        const double v = alpha * acc + (y ? beta * y[i] : 0.0);
        if (out_d) out_d[i] = v;
        if (out_t) out_t[i] = (TO)v;
        if (part) {
            const double e = cv ? v - cv[i] : v;
            e2 += e * e;
        }
    };
    const int64_t nb = gridDim.x;
    const int64_t chunk = 2 * KB * ((n + 2 * KB * nb - 1) / (2 * KB * nb));
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    for (int64_t i = lo + 2 * (int64_t)threadIdx.x; i < hi; i += 2 * KB) {
        if (i + 1 < hi) {
            double a0, a1;
            dot_row2(X, ld, i, K, sh, a0, a1);
            finish(i, a0);
            finish(i + 1, a1);
        } else {
            finish(i, dot_row(X, ld, i, K, sh));
        }
    }
    if (!part) return;
    const double bs = block_sum(e2, s4);
    if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// y = x - Q h and the chunk partials of Q^T y, reading Q once (y must not alias x).  The
// four waves of a workgroup split the columns (wave w owns columns w*CPW .. w*CPW+CPW-1)
// and walk the workgroup's row chunk 64 rows at a time: each wave forms its columns' part
// of (Q h)_i for its lane's row and keeps its Q entries in registers; the four parts are
// added through LDS in a fixed order, every wave forms the same y_i = x_i - (Q h)_i, and
// the wave then accumulates its columns' products with y_i.  CPW >= ceil(K / 4).
template <int CPW>
__global__ __launch_bounds__(KB) void k_gemv_mdot(int64_t n, int K, const double* __restrict__ Q, int64_t ld,
                                                  const double* __restrict__ h, const double* __restrict__ x,
                                                  double* __restrict__ y, double* __restrict__ part) {
    __shared__ double sp[2][4][64];  // per-row parts of Q h, double-buffered
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int jw = w * CPW;
    double hw[CPW], acc[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        hw[c] = jw + c < K ? h[jw + c] : 0.0;
        acc[c] = 0.0;
    }
    const int64_t nb = gridDim.x;
    const int64_t chunk = (n + nb - 1) / nb;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    int buf = 0;
    for (int64_t i0 = lo; i0 < hi; i0 += 64, buf ^= 1) {
        const int64_t i = i0 + lane;
        const bool in = i < hi;
        double q[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) q[c] = (in && jw + c < K) ? Q[(int64_t)(jw + c) * ld + i] : 0.0;
        const double xi = in ? x[i] : 0.0;
        double sw = 0.0;
#pragma unroll
        for (int c = 0; c < CPW; ++c) sw += q[c] * hw[c];
        sp[buf][w][lane] = sw;
        __syncthreads();
        const double s = (sp[buf][0][lane] + sp[buf][1][lane]) + (sp[buf][2][lane] + sp[buf][3][lane]);
        const double v = xi - s;
        if (w == 0 && in) y[i] = v;
#pragma unroll
        for (int c = 0; c < CPW; ++c) acc[c] += q[c] * v;
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const double a = wave_sum(acc[c]);
        if (lane == 0 && jw + c < K) part[(int64_t)(jw + c) * gridDim.x + blockIdx.x] = a;
    }
}

// out[0] = sum of nb partials in a fixed order: thread t of 1024 sums t, t + 1024, ... in eight
// interleaved running sums (the eight loads of a step in flight together) combined in a fixed
// order, then the waves' sums in wave order.
__global__ __launch_bounds__(1024) void k_sum_final(int nb, const double* __restrict__ part, double* __restrict__ out,
                                                   const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double s16[16];
    double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b0 = threadIdx.x; b0 < nb; b0 += 8 * 1024) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (b0 + 1024 * u < nb) a8[u] += part[b0 + 1024 * u];
    }
    double a = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) s16[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += s16[w];
        out[0] = t;
    }
}

// s = sqrt(s2[0]); out_d = x / s, out_t = (TO)(x / s) (zero when s = 0); s1[0] = s.
template <class TO>
__global__ void k_normalize2(int64_t n, const double* x, const double* __restrict__ s2, double* __restrict__ s1,
                             double* out_d, TO* __restrict__ out_t) {
    const double s = sqrt(fmax(s2[0], 0.0));
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    if (s1 && blockIdx.x == 0 && threadIdx.x == 0) s1[0] = s;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[i] * inv;
        if (out_d) out_d[i] = v;
        if (out_t) out_t[i] = (TO)v;
    }
}

// out = (double)in + sign * s[0] * q
template <class TX>
__global__ void k_axpy_conv(int64_t n, const TX* __restrict__ in, const double* __restrict__ q,
                            const double* __restrict__ s, double sign, double* __restrict__ out) {
    const double a = sign * s[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i] + a * q[i];
}

// Weighted Gram G = X^T diag(w) X (w = 1 when null) on the FP64 matrix cores: up to 40
// columns on the 4x4x4 form below (k_wgram_quad), 41..64 columns and the diagonal tiles of
// wider bases on the 16x16x4 form (k_wgram_part), the tiles above them by k_wgram_rect.
// v_mfma_f64_16x16x4f64 multiplies a 16x4 block A by a 4x16 block B: lane l supplies
// A[l%16][l/16] and B[l/16][l%16], and the 16x16 result sits in four doubles per lane,
// D[l/16 + 4v][l%16].  Here A[i][k] = X[row_k][16gi + i] and B[k][j] = w[row_k] X[row_k][16gj + j]
// for the column blocks gi <= gj, so one instruction adds four rows to a 16x16 block.
//
// A wave takes 16 rows per step: lane group q = l/16 owns rows r0 + 4q .. r0 + 4q + 3 and
// reads them with one 16-byte (float) or two 16-byte (double) loads per column block,
// so a load instruction covers 64 contiguous bytes of each of 16 columns; the k-th MFMA
// of the step uses row r0 + 4q + k in lane group q.  The next step's loads are issued
// before the current step's MFMAs.  Stage 1 leaves one partial per workgroup (the waves
// are combined in LDS in a fixed order); stage 2 sums the partials in a fixed order.
typedef double dbl4 __attribute__((ext_vector_type(4)));

static constexpr int GRAM_WAVES = 16;      // most waves per stage-1 workgroup (8 for G >= 3: registers)
static constexpr int GRAM_BLOCKS = 1024;   // most stage-1 workgroups (partials)
static constexpr int GRAM_PAIRS = 10;      // upper blocks of a 4x4 block grid
static constexpr int GRAM_SLAB = 64;       // partial entries per stage-2 workgroup

template <class TX, int G>
struct GramRows {
    TX x[G][4];    // [column block][row k]
    double w[4];
};

// Weight of one row: read from w (NU = false), or formed from nu by mm_weight, the weights of
// k_mm_weights_f64 (NU = true; wv then points to nu in TX).
template <class TX, bool NU>
__device__ __forceinline__ double row_weight(const void* __restrict__ wv, int64_t r, double eps2) {
    if constexpr (NU) {
        return mm_weight((double)static_cast<const TX*>(wv)[r], eps2);
    } else {
        return static_cast<const double*>(wv)[r];
    }
}

// Rows r0 + 4q + k (k < 4) of column blocks g < G for this lane; rows at or beyond n and
// columns at or beyond K read as zero.  VEC: the four rows are loaded with one vector load
// (element-aligned X suffices; rows r0 + 4q + 3 < n).  The row weights come
// from w (NU = false; null: 1) or from nu (NU = true, see row_weight).
template <class TX, int G, bool VEC, bool NU = false>
__device__ __forceinline__ void gram_rows(GramRows<TX, G>& st, const TX* __restrict__ X, int64_t ld,
                                          const void* __restrict__ wv, int64_t n, int K, int64_t r0, int lane,
                                          double eps2 = 0.0) {
    const double* __restrict__ w = static_cast<const double*>(wv);
    const int c = lane & 15;
    const int64_t rb = r0 + 4 * (lane >> 4);
    if (VEC && rb + 3 < n) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int col = 16 * g + c;
            if (col < K) {
                const TX* src = X + (int64_t)col * ld + rb;
                if constexpr (sizeof(TX) == 4) {
                    typedef float F4e __attribute__((ext_vector_type(4), aligned(4)));
                    const F4e v = *reinterpret_cast<const F4e*>(src);
                    st.x[g][0] = v.x;
                    st.x[g][1] = v.y;
                    st.x[g][2] = v.z;
                    st.x[g][3] = v.w;
                } else {
                    struct alignas(16) D2 {
                        double a, b;
                    };
                    const D2 v0 = *reinterpret_cast<const D2*>(src);
                    const D2 v1 = *reinterpret_cast<const D2*>(src + 2);
                    st.x[g][0] = v0.a;
                    st.x[g][1] = v0.b;
                    st.x[g][2] = v1.a;
                    st.x[g][3] = v1.b;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) st.x[g][k] = TX(0);
            }
        }
        if constexpr (NU) {
#pragma unroll
            for (int k = 0; k < 4; ++k) st.w[k] = row_weight<TX, true>(wv, rb + k, eps2);
        } else if (w) {
            const double2 w0 = *reinterpret_cast<const double2*>(w + rb);
            const double2 w1 = *reinterpret_cast<const double2*>(w + rb + 2);
            st.w[0] = w0.x;
            st.w[1] = w0.y;
            st.w[2] = w1.x;
            st.w[3] = w1.y;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) st.w[k] = 1.0;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t r = rb + k;
        const bool in = r < n;
        if constexpr (NU)
            st.w[k] = in ? row_weight<TX, true>(wv, r, eps2) : 0.0;
        else
            st.w[k] = in ? (w ? w[r] : 1.0) : 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int col = 16 * g + c;
            st.x[g][k] = (in && col < K) ? X[(int64_t)col * ld + r] : TX(0);
        }
    }
}

template <class TX, int G, bool VEC, int W, bool NU = false>
__global__ __launch_bounds__(64 * W) void k_wgram_part(int64_t n, int K, const TX* __restrict__ X,
                                                                int64_t ld, const void* __restrict__ w,
                                                                double eps2, double* __restrict__ part) {
    constexpr int NP = G * (G + 1) / 2;
    __shared__ double sred[W][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    dbl4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = dbl4{0.0, 0.0, 0.0, 0.0};
    // contiguous 16-row steps per wave
    const int64_t steps = (n + 15) / 16;
    const int64_t nw = (int64_t)gridDim.x * W;
    const int64_t gw = (int64_t)blockIdx.x * W + wave;
    const int64_t s_lo = steps * gw / nw, s_hi = steps * (gw + 1) / nw;
    GramRows<TX, G> cur, nxt;
    if (s_lo < s_hi) gram_rows<TX, G, VEC, NU>(cur, X, ld, w, n, K, 16 * s_lo, lane, eps2);
    for (int64_t st = s_lo; st < s_hi; ++st) {
        if (st + 1 < s_hi) gram_rows<TX, G, VEC, NU>(nxt, X, ld, w, n, K, 16 * (st + 1), lane, eps2);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double a[G], bw[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                a[g] = (double)cur.x[g][k];
                bw[g] = a[g] * cur.w[k];
            }
            int p = 0;
#pragma unroll
            for (int gi = 0; gi < G; ++gi)
#pragma unroll
                for (int gj = gi; gj < G; ++gj, ++p)
                    acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[gi], bw[gj], acc[p], 0, 0, 0);
        }
        cur = nxt;
    }
    // combine the waves pair by pair: thread t < 256 sums entry t over the waves in order
    double* out = part + (int64_t)blockIdx.x * (GRAM_PAIRS * 256);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int v = 0; v < 4; ++v) sred[wave][v * 64 + lane] = acc[p][v];
        __syncthreads();
        if (threadIdx.x < 256) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < W; ++q) sum += sred[q][threadIdx.x];
            out[p * 256 + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

// Stage 2: entry e (pair p = e / 256, register slot e % 256) summed over the partials.
// A workgroup takes GRAM_SLAB consecutive entries; its 16 waves split the partials and
// are combined in a fixed order; the upper triangle's entry is written to both triangles.
__global__ __launch_bounds__(1024) void k_wgram_final(int nb, int K, int G, const double* __restrict__ part,
                                                      double* __restrict__ Gm, int ldg) {
    __shared__ double s[16][GRAM_SLAB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = blockIdx.x * GRAM_SLAB + lane;
    double acc = 0.0;
    for (int b = wave; b < nb; b += 16) acc += part[(int64_t)b * (GRAM_PAIRS * 256) + e];
    s[wave][lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) sum += s[q][lane];
    // map (pair, slot) to (i, j)
    const int p = e >> 8, slot = e & 255, v = slot >> 6, l = slot & 63;
    int gi = 0, base = 0;
    while (gi < G && p >= base + (G - gi)) {
        base += G - gi;
        ++gi;
    }
    if (gi >= G) return;
    const int gj = gi + (p - base);
    const int i = 16 * gi + (l >> 4) + 4 * v, j = 16 * gj + (l & 15);
    // a diagonal block holds both (i, j) and (j, i), which round differently: the upper one
    // is written to both triangles, so G is exactly symmetric and every entry has one writer
    if (i <= j && j < K) {
        Gm[(int64_t)i * ldg + j] = sum;
        Gm[(int64_t)j * ldg + i] = sum;
    }
}

// Weighted Gram on the 4x4x4 FP64 MFMA (K <= 4 * GRAM_QUADS).  v_mfma_f64_4x4x4f64 holds four
// independent products of a 4x4 block A by a 4x4 block B: in block b, lane l = 16k + 4b + i
// supplies A[i][k] and lane 16k + 4b + j supplies B[k][j], and the result D[i][j] of block b
// sits in lane 16i + 4b + j.  The four blocks take four different row groups of one 4x4 tile
// of G: with x_r the row r of X, a tile (qa, qb) of column quads qa <= qb gets
// A[i][k] = x_r[4qa + i] and B[k][j] = w_r x_r[4qb + j] for the row r of (block, k), so each
// instruction adds 16 rows to one 4x4 tile and every tile costs 16 multiply-adds per row:
// ceil(K/4)(ceil(K/4)+1)/2 tiles instead of the 16-column blocks' padding (at K = 39, 880
// instead of 1536 per row).
//
// A lane owns row slot s = l/4 and column i = l%4 of each quad: it reads the 16 bytes of rows
// r0 + RPL s .. r0 + RPL s + RPL - 1 (RPL = 4 floats or 2 doubles) of column 4q + i, so a load
// instruction covers 256 contiguous bytes of each of four columns, and a wave step covers
// 16 RPL rows; the step's t-th instructions take row r0 + RPL s + t of every slot.  The next
// step's loads are issued before the current step's MFMAs.  At the end the four row groups of
// a result are summed across lanes (l, l^4, l^8, l^12), the waves of a workgroup in LDS in a
// fixed order, and stage 2 sums the workgroups' partials in a fixed order.
static constexpr int GRAM_QUADS = 10;   // most column quads of the 4x4x4 form (K <= 40)

template <class TX, int NQ>
struct QuadRows {
    static constexpr int RPL = 16 / (int)sizeof(TX);
    TX x[NQ][RPL];    // [column quad][row t]
    double w[RPL];
};

// Row weights of the quad kernels: none (1), read from an FP64 buffer, or formed from nu.
enum QuadWeight { QW_ONE = 0, QW_BUF = 1, QW_NU = 2 };

// This lane's rows rb .. rb + RPL - 1 (rb = r0 + RPL (lane/4)), all below n, of columns
// 4q + lane%4, with 16-byte loads and no branches (X needs only element alignment: global
// multi-word loads accept it, so columns of any leading dimension qualify; w and nu, read at
// rows rb that are multiples of RPL, must be 16-byte aligned).  Columns at or beyond K exist only in the last quad; they read column
// K - 1 instead.  A result D[i][j] involves only column i of the A operand and column j of
// the B operand, so those copies reach only entries with i or j at or beyond K, which stage 2
// never writes.
template <class TX, int NQ, int WK>
__device__ __forceinline__ void quad_load_full(QuadRows<TX, NQ>& st, const TX* __restrict__ X, int64_t ld,
                                               const void* __restrict__ wv, int K, int64_t rb, int ci,
                                               double eps2) {
    constexpr int RPL = QuadRows<TX, NQ>::RPL;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int col = 4 * q + ci;
        const int cl = (q == NQ - 1) ? min(col, K - 1) : col;   // (only the last quad can pass K)
        const TX* src = X + (int64_t)cl * ld + rb;
        typedef TX VR __attribute__((ext_vector_type(RPL), aligned(sizeof(TX))));
        const VR v = __builtin_nontemporal_load(reinterpret_cast<const VR*>(src));
#pragma unroll
        for (int t = 0; t < RPL; ++t) st.x[q][t] = v[t];
    }
    if constexpr (WK == QW_BUF) {
        const double* __restrict__ w = static_cast<const double*>(wv);
#pragma unroll
        for (int t = 0; t < RPL; t += 2) {
            const double2 v = *reinterpret_cast<const double2*>(w + rb + t);
            st.w[t] = v.x;
            st.w[t + 1] = v.y;
        }
    } else if constexpr (WK == QW_NU) {
        // (nu itself: the weights are formed in quad_mfma, after the loads have arrived)
        const TX* __restrict__ nu = static_cast<const TX*>(wv);
        if constexpr (sizeof(TX) == 4) {
            typedef float F4 __attribute__((ext_vector_type(4), aligned(16)));
            const F4 v = __builtin_nontemporal_load(reinterpret_cast<const F4*>(nu + rb));
            st.w[0] = v.x;
            st.w[1] = v.y;
            st.w[2] = v.z;
            st.w[3] = v.w;
        } else {
            const double2 v = *reinterpret_cast<const double2*>(nu + rb);
            st.w[0] = v.x;
            st.w[1] = v.y;
        }
    } else {
#pragma unroll
        for (int t = 0; t < RPL; ++t) st.w[t] = 1.0;
    }
}

// The same rows with one guarded load per element: rows at or beyond n and columns at or beyond
// K read as zero (the ragged last step, and any step of unaligned columns).
template <class TX, int NQ, int WK>
__device__ __forceinline__ void quad_load_guarded(QuadRows<TX, NQ>& st, const TX* __restrict__ X, int64_t ld,
                                                  const void* __restrict__ wv, int64_t n, int K, int64_t rb, int ci,
                                                  double eps2) {
    constexpr int RPL = QuadRows<TX, NQ>::RPL;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int64_t r = rb + t;
        const bool in = r < n;
        if constexpr (WK == QW_NU)
            st.w[t] = in ? (double)static_cast<const TX*>(wv)[r] : 0.0;   // (nu; zero rows stay zero below)
        else if constexpr (WK == QW_BUF)
            st.w[t] = in ? static_cast<const double*>(wv)[r] : 0.0;
        else
            st.w[t] = in ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int col = 4 * q + ci;
            st.x[q][t] = (in && col < K) ? X[(int64_t)col * ld + r] : TX(0);
        }
    }
}

// The MFMAs of one step: every tile (qa <= qb) and row t of the lanes' slots.  QW_NU: st.w holds
// nu, and the row weight 1/sqrt(nu^2 + eps^2) is formed here (a row beyond n has x = 0).
template <class TX, int NQ, int WK>
__device__ __forceinline__ void quad_mfma(const QuadRows<TX, NQ>& st, double* acc, double eps2) {
#pragma unroll
    for (int t = 0; t < QuadRows<TX, NQ>::RPL; ++t) {
        double wt = st.w[t];
        if constexpr (WK == QW_NU) wt = mm_weight(wt, eps2);
        double a[NQ], bw[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            a[q] = (double)st.x[q][t];
            bw[q] = a[q] * wt;
        }
        int p = 0;
#pragma unroll
        for (int qa = 0; qa < NQ; ++qa)
#pragma unroll
            for (int qb = qa; qb < NQ; ++qb, ++p)
                acc[p] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[qa], bw[qb], acc[p], 0, 0, 0);
    }
}

template <class TX, int NQ, bool VEC, int W, int WK>
__global__ __launch_bounds__(64 * W) void k_wgram_quad(int64_t n, int K, const TX* __restrict__ X, int64_t ld,
                                                       const void* __restrict__ w, double eps2,
                                                       double* __restrict__ part) {
    constexpr int RPL = QuadRows<TX, NQ>::RPL;
    constexpr int STEP = 16 * RPL;
    constexpr int NT = NQ * (NQ + 1) / 2;
    __shared__ double sred[W][NT * 16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ci = lane & 3;
    const int64_t slot = RPL * (lane >> 2);
    double acc[NT];
#pragma unroll
    for (int p = 0; p < NT; ++p) acc[p] = 0.0;
    // contiguous steps per wave; steps below n / STEP hold no row at or beyond n
    const int64_t steps = (n + STEP - 1) / STEP;
    const int64_t nw = (int64_t)gridDim.x * W;
    const int64_t gw = (int64_t)blockIdx.x * W + wave;
    const int64_t s_lo = steps * gw / nw, s_hi = steps * (gw + 1) / nw;
    int64_t st = s_lo;
    QuadRows<TX, NQ> A, B;
    if constexpr (VEC) {
        const int64_t f_hi = std::min<int64_t>(s_hi, n / STEP);
        if (st < f_hi) {
            // two buffers in turn: the next step's loads are in flight during this step's MFMAs
            quad_load_full<TX, NQ, WK>(A, X, ld, w, K, STEP * st + slot, ci, eps2);
            // (the scheduling barriers keep each buffer's conversions after the other buffer's
            // MFMAs, so no wait for the loads in flight is placed inside them)
            for (; st + 2 <= f_hi; st += 2) {
                quad_load_full<TX, NQ, WK>(B, X, ld, w, K, STEP * (st + 1) + slot, ci, eps2);
                __builtin_amdgcn_sched_barrier(0);
                quad_mfma<TX, NQ, WK>(A, acc, eps2);
                __builtin_amdgcn_sched_barrier(0);
                const int64_t s2 = std::min<int64_t>(st + 2, f_hi - 1);   // (a repeat load at the end)
                quad_load_full<TX, NQ, WK>(A, X, ld, w, K, STEP * s2 + slot, ci, eps2);
                __builtin_amdgcn_sched_barrier(0);
                quad_mfma<TX, NQ, WK>(B, acc, eps2);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (st < f_hi) {
                quad_mfma<TX, NQ, WK>(A, acc, eps2);
                ++st;
            }
        }
    }
    for (; st < s_hi; ++st) {
        quad_load_guarded<TX, NQ, WK>(A, X, ld, w, n, K, STEP * st + slot, ci, eps2);
        quad_mfma<TX, NQ, WK>(A, acc, eps2);
    }
    // the four row groups of each result, then the waves in order
#pragma unroll
    for (int p = 0; p < NT; ++p) {
        double v = acc[p];
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        if ((lane & 12) == 0) sred[wave][p * 16 + (lane >> 4) * 4 + (lane & 3)] = v;
    }
    __syncthreads();
    double* out = part + (int64_t)blockIdx.x * (NT * 16);
    for (int e = threadIdx.x; e < NT * 16; e += 64 * W) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) sum += sred[q][e];
        out[e] = sum;
    }
}

// Stage 2 of the 4x4x4 form: entry e = 16 p + 4 i + j of tile p (quads qa <= qb in row-major
// order) summed over the partials in a fixed order; G[4qa + i][4qb + j] written to both
// triangles when 4qa + i <= 4qb + j < K (the upper entry of a diagonal tile serves both).
__global__ __launch_bounds__(1024) void k_wgram_final_quad(int nb, int K, int NQ, const double* __restrict__ part,
                                                           double* __restrict__ Gm, int ldg) {
    __shared__ double s[16][GRAM_SLAB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ne = NQ * (NQ + 1) / 2 * 16;
    const int e = blockIdx.x * GRAM_SLAB + lane;
    double acc = 0.0;
    if (e < ne)
        for (int b = wave; b < nb; b += 16) acc += part[(int64_t)b * ne + e];
    s[wave][lane] = acc;
    __syncthreads();
    if (wave != 0 || e >= ne) return;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) sum += s[q][lane];
    const int p = e >> 4;
    int qa = 0, base = 0;
    while (p >= base + (NQ - qa)) {
        base += NQ - qa;
        ++qa;
    }
    const int qb = qa + (p - base);
    const int i = 4 * qa + ((e >> 2) & 3), j = 4 * qb + (e & 3);
    if (i <= j && j < K) {
        Gm[(int64_t)i * ldg + j] = sum;
        Gm[(int64_t)j * ldg + i] = sum;
    }
}

// Off-diagonal tile of a Gram with more than 64 columns: G[I][J] for the column blocks
// I = i0 .. i0 + GI - 1 of XI and J = j0 .. j0 + GJ - 1 of XJ (XI, XJ point at the first
// column of each tile; KI, KJ columns are valid), every block pair (gi, gj) on the matrix
// cores as in k_wgram_part; part[b][gi * GJ + gj][256] receives workgroup b's sums.
static constexpr int GRAM_RECT = 4;   // column blocks per side of an off-diagonal tile

template <class TX, int GI, int GJ, bool VEC, int W>
__global__ __launch_bounds__(64 * W) void k_wgram_rect(int64_t n, int KI, int KJ, const TX* __restrict__ XI,
                                                       const TX* __restrict__ XJ, int64_t ld,
                                                       const double* __restrict__ w, double* __restrict__ part) {
    constexpr int NP = GI * GJ;
    __shared__ double sred[W][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    dbl4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int64_t steps = (n + 15) / 16;
    const int64_t nw = (int64_t)gridDim.x * W;
    const int64_t gw = (int64_t)blockIdx.x * W + wave;
    const int64_t s_lo = steps * gw / nw, s_hi = steps * (gw + 1) / nw;
    GramRows<TX, GI> ci, ni;
    GramRows<TX, GJ> cj, nj;
    if (s_lo < s_hi) {
        gram_rows<TX, GI, VEC>(ci, XI, ld, nullptr, n, KI, 16 * s_lo, lane);
        gram_rows<TX, GJ, VEC>(cj, XJ, ld, w, n, KJ, 16 * s_lo, lane);
    }
    for (int64_t st = s_lo; st < s_hi; ++st) {
        if (st + 1 < s_hi) {
            gram_rows<TX, GI, VEC>(ni, XI, ld, nullptr, n, KI, 16 * (st + 1), lane);
            gram_rows<TX, GJ, VEC>(nj, XJ, ld, w, n, KJ, 16 * (st + 1), lane);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double a[GI], bw[GJ];
#pragma unroll
            for (int g = 0; g < GI; ++g) a[g] = (double)ci.x[g][k];
#pragma unroll
            for (int g = 0; g < GJ; ++g) bw[g] = (double)cj.x[g][k] * cj.w[k];
#pragma unroll
            for (int gi = 0; gi < GI; ++gi)
#pragma unroll
                for (int gj = 0; gj < GJ; ++gj)
                    acc[gi * GJ + gj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[gi], bw[gj], acc[gi * GJ + gj], 0, 0, 0);
        }
        ci = ni;
        cj = nj;
    }
    double* out = part + (int64_t)blockIdx.x * (NP * 256);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int v = 0; v < 4; ++v) sred[wave][v * 64 + lane] = acc[p][v];
        __syncthreads();
        if (threadIdx.x < 256) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < W; ++q) sum += sred[q][threadIdx.x];
            out[p * 256 + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

// Stage 2 of an off-diagonal tile: entry e = (pair gi * GJ + gj, register slot) summed over the
// partials in a fixed order; G[i][j] and G[j][i] (i in the I tile, j in the J tile) written.
__global__ __launch_bounds__(1024) void k_wgram_final_rect(int nb, int GJ, int np, int KI, int KJ, int i0, int j0,
                                                           const double* __restrict__ part, double* __restrict__ Gm,
                                                           int ldg) {
    __shared__ double s[16][GRAM_SLAB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = blockIdx.x * GRAM_SLAB + lane;
    double acc = 0.0;
    if (e < np * 256)
        for (int b = wave; b < nb; b += 16) acc += part[(int64_t)b * (np * 256) + e];
    s[wave][lane] = acc;
    __syncthreads();
    if (wave != 0 || e >= np * 256) return;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) sum += s[q][lane];
    const int p = e >> 8, slot = e & 255, v = slot >> 6, l = slot & 63;
    const int gi = p / GJ, gj = p % GJ;
    const int ri = 16 * gi + (l >> 4) + 4 * v, cj = 16 * gj + (l & 15);
    if (ri < KI && cj < KJ) {
        const int i = i0 + ri, j = j0 + cj;
        Gm[(int64_t)i * ldg + j] = sum;
        Gm[(int64_t)j * ldg + i] = sum;
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

// y = w * x in TX (w: FP64 MM weights)
template <class TX>
__global__ void k_weight_mul(int64_t n, const double* __restrict__ w, const TX* __restrict__ x, TX* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (TX)((double)x[i] * w[i]);
}

// y = x w with w = mm_weight(nu) formed here (the weights of k_mm_weights_f64).
template <class TX>
__global__ void k_weight_mul_nu(int64_t n, const TX* __restrict__ nu, double eps2, const TX* __restrict__ x,
                                TX* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        y[i] = (TX)((double)x[i] * mm_weight((double)nu[i], eps2));
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
void weight_mul(Ctx& c, int64_t n, const double* w, const TX* x, TX* y) {
    hipLaunchKernelGGL(k_weight_mul<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, w, x, y);
    MMOF_LAUNCH_CHECK();
}
template void weight_mul<float>(Ctx&, int64_t, const double*, const float*, float*);
template void weight_mul<double>(Ctx&, int64_t, const double*, const double*, double*);

template <class TX>
void weight_mul_nu(Ctx& c, int64_t n, const TX* nu, double eps, const TX* x, TX* y) {
    hipLaunchKernelGGL(k_weight_mul_nu<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, nu, eps * eps, x, y);
    MMOF_LAUNCH_CHECK();
}
template void weight_mul_nu<float>(Ctx&, int64_t, const float*, double, const float*, float*);
template void weight_mul_nu<double>(Ctx&, int64_t, const double*, double, const double*, double*);


// Two rows per lane (k_mdot2) when every column, y and xe are element-aligned (2-element
// loads need no more).
template <class TX, class TY>
static bool mdot_pairs(const TX* X, int64_t ld, const TY* y, const double* xe) {
    (void)ld;
    return reinterpret_cast<uintptr_t>(X) % sizeof(TX) == 0 && reinterpret_cast<uintptr_t>(y) % sizeof(TY) == 0 &&
           (!xe || reinterpret_cast<uintptr_t>(xe) % sizeof(double) == 0);
}

// row chunks of 8192 rows (32 per thread), but at least 256 chunks (of no fewer than 256
// rows) so that short vectors still spread over the chip; at most MAX_PART chunks
int mdot_blocks(int64_t n) {
    const int64_t nb = std::max<int64_t>(cdiv(n, 8192), std::min<int64_t>(cdiv(n, 256), 256));
    return (int)std::max<int64_t>(1, std::min<int64_t>(MAX_PART, nb));
}

// The block inner products of K columns of X (and of the FP64 column xe, when given) with y
// over nb row chunks, into part (column-major, [Kt][nb]); then their fixed-order sums
// (k_mdot_final: out, or a Gram row and column with dj).
template <class TX, class TY>
static void launch_mdot(Ctx& c, int nb, int64_t n, int K, const TX* X, int64_t ld, const TY* y, const double* xe,
                        double* part, const int* skip) {
    const int Kt = K + (xe ? 1 : 0);
    const dim3 grid((unsigned)(8 * cdiv(nb, 8) * cdiv(Kt, 8)));
    if (mdot_pairs(X, ld, y, xe))
        hipLaunchKernelGGL((k_mdot2<TX, TY>), grid, dim3(KB), 0, c.stream, n, K, nb, X, ld, y, xe, part, skip);
    else
        hipLaunchKernelGGL((k_mdot<TX, TY>), grid, dim3(KB), 0, c.stream, n, K, nb, X, ld, y, xe, part, skip);
    MMOF_LAUNCH_CHECK();
}

static void mdot_final(Ctx& c, int nb, int Kt, const double* part, double alpha, double* out, double* G, int ldg,
                       int row, double* dj, const int* skip) {
    hipLaunchKernelGGL(k_mdot_final, dim3((unsigned)Kt), dim3(KB), 0, c.stream, nb, Kt, part, alpha, out, G, ldg,
                       row, dj, skip);
    MMOF_LAUNCH_CHECK();
}


template <class TX, class TY>
void mdot(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TY* y, double alpha, double* out) {
    if (K <= 0) return;
    const int nb = mdot_blocks(n);
    MMOF_CHECK(K <= KMAX, MMOF_ERR_SHAPE, "too many columns for a block inner product");
    double* part = static_cast<double*>(c.work("mdot_part", sizeof(double) * (size_t)MAX_PART * (KMAX + 1)));
    {
        ScopedTime st(&c, "mdot", (double)n * ((double)sizeof(TX) * K + sizeof(TY)), 2.0 * n * K);
        launch_mdot<TX, TY>(c, nb, n, K, X, ld, y, nullptr, part, nullptr);
    }
    mdot_final(c, nb, K, part, alpha, out, nullptr, 0, 0, nullptr, nullptr);
}
template void mdot<float, double>(Ctx&, int64_t, int, const float*, int64_t, const double*, double, double*);
template void mdot<double, double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double, double*);
template void mdot<float, float>(Ctx&, int64_t, int, const float*, int64_t, const float*, double, double*);

void gemv_mdot(Ctx& c, int64_t n, int K, const double* Q, int64_t ld, const double* h, const double* x, double* y,
               double* hout) {
    MMOF_CHECK(K >= 1 && K <= KMAX_SMALL, MMOF_ERR_SHAPE, "too many columns for the fused CGS pass");
    // chunks of 256 rows (4 steps of the workgroup), at most MAX_PART partials
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(MAX_PART, cdiv(n, 256)));
    double* part = static_cast<double*>(c.work("mdot_part", sizeof(double) * (size_t)MAX_PART * (KMAX + 1)));
    {
        ScopedTime st(&c, "gemv_mdot", (double)n * (8.0 * K + 16.0), 4.0 * n * K);
        auto k = K <= 16 ? k_gemv_mdot<4> : K <= 32 ? k_gemv_mdot<8> : K <= 48 ? k_gemv_mdot<12> : k_gemv_mdot<16>;
        hipLaunchKernelGGL(k, dim3(nb), dim3(KB), 0, c.stream, n, K, Q, ld, h, x, y, part);
        MMOF_LAUNCH_CHECK();
    }
    mdot_final(c, nb, K, part, 1.0, hout, nullptr, 0, 0, nullptr, nullptr);
}

template <class TX>
void gram_row(Ctx& c, int64_t n, int j, const TX* X, int64_t ld, const double* e, double* G, int ldg, double* dj) {
    MMOF_CHECK(j >= 0 && j < KMAX, MMOF_ERR_SHAPE, "too many Krylov columns");
    const int nb = mdot_blocks(n);
    double* part = static_cast<double*>(c.work("mdot_part", sizeof(double) * (size_t)MAX_PART * (KMAX + 1)));
    const TX* xj = X + (int64_t)j * ld;
    launch_mdot<TX, TX>(c, nb, n, j + 1, X, ld, xj, e, part, nullptr);
    mdot_final(c, nb, j + 2, part, 1.0, nullptr, G, ldg, j, dj, nullptr);
}
template void gram_row<float>(Ctx&, int64_t, int, const float*, int64_t, const double*, double*, int, double*);
template void gram_row<double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double*, int, double*);

// gemv_fused; with skip, every launch returns at once when *skip is non-zero on the device
// (timed under the name tname)
template <class TX, class TO>
static void gemv_fused_impl(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* h, double alpha,
                            const double* y, double beta, double* out_d, TO* out_t, const double* cv, double* sq,
                            const int* skip, const char* tname) {
    MMOF_CHECK(K >= 0 && K <= KMAX, MMOF_ERR_SHAPE, "too many Krylov columns");
    if (n == 0) {
        if (sq && !skip) set_scalar(c, sq, 0.0);
        return;
    }
    // two rows per lane when the columns allow 2-element loads (the grid covers row pairs)
    const bool pair = reinterpret_cast<uintptr_t>(X) % sizeof(TX) == 0;
    // pairs: contiguous row chunks of 2048 rows (at least 1024 chunks of no fewer than 2 KB
    // rows, so that short vectors still spread over the chip; at most MAX_GEMV_PART); otherwise
    // a grid-strided walk
    const int64_t nbp = std::max<int64_t>(cdiv(n, 2048), std::min<int64_t>(cdiv(n, 2 * KB), 1024));
    const dim3 grid = pair ? dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(MAX_GEMV_PART, nbp)))
                           : grid_for(n, KB, 2048);
    double* part = sq ? static_cast<double*>(c.work("gemv_part", sizeof(double) * MAX_GEMV_PART)) : nullptr;
    {
        // K columns and y (if any) read, the outputs written, cv read when given
        const double bytes = (double)n * ((double)sizeof(TX) * K + (y ? 8.0 : 0.0) + (out_d ? 8.0 : 0.0) +
                                          (out_t ? (double)sizeof(TO) : 0.0) + (cv ? 8.0 : 0.0));
        // (a conditional launch may do nothing: no work is credited to it)
        ScopedTime st(&c, tname, skip ? 0.0 : bytes, skip ? 0.0 : 2.0 * n * K);
        if (pair)
            hipLaunchKernelGGL((k_gemv_fused2<TX, TO>), grid, dim3(KB), 0, c.stream, n, K, X, ld, h, alpha, y, beta,
                               out_d, out_t, cv, part, skip);
        else
            hipLaunchKernelGGL((k_gemv_fused<TX, TO>), grid, dim3(KB), 0, c.stream, n, K, X, ld, h, alpha, y, beta,
                               out_d, out_t, cv, part, skip);
        MMOF_LAUNCH_CHECK();
    }
    if (sq) {
        hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(1024), 0, c.stream, (int)grid.x, (const double*)part, sq, skip);
        MMOF_LAUNCH_CHECK();
    }
}

template <class TX, class TO>
void gemv_fused(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* h, double alpha, const double* y,
                double beta, double* out_d, TO* out_t, const double* cv, double* sq) {
    gemv_fused_impl<TX, TO>(c, n, K, X, ld, h, alpha, y, beta, out_d, out_t, cv, sq, nullptr, "gemv");
}
template void gemv_fused<double, float>(Ctx&, int64_t, int, const double*, int64_t, const double*, double,
                                        const double*, double, double*, float*, const double*, double*);
template void gemv_fused<double, double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double,
                                         const double*, double, double*, double*, const double*, double*);
template void gemv_fused<float, float>(Ctx&, int64_t, int, const float*, int64_t, const double*, double,
                                       const double*, double, double*, float*, const double*, double*);

// Second-pass test of cgs_once: flag[0] = 1 (skip the second pass) when the first pass kept at
// least 1/sqrt(2) of the norm, ||x'||^2 >= ||x||^2 / 2.
__global__ void k_cgs_keep(const double* __restrict__ xx, const double* __restrict__ sq, int* __restrict__ flag) {
    flag[0] = (sq[0] >= 0.5 * xx[0]) ? 1 : 0;
}

void cgs_once(Ctx& c, int64_t n, int K, const double* Q, int64_t ld, double* x, double* sq, double* h) {
    MMOF_CHECK(K >= 1 && K <= KMAX, MMOF_ERR_SHAPE, "too many Krylov columns");
    const int nb = mdot_blocks(n);
    double* part = static_cast<double*>(c.work("mdot_part", sizeof(double) * (size_t)MAX_PART * (KMAX + 1)));
    int* flag = static_cast<int*>(c.work("cgs_flag", sizeof(int)));
    // h[0..K-1] = Q^T x and h[K] = ||x||^2 (x as the extra column), one pass over Q and x
    auto dots = [&](const double* xe, const int* skip, const char* tname) {
        const int Kt = K + (xe ? 1 : 0);
        {
            ScopedTime st(&c, tname, skip ? 0.0 : (double)n * (8.0 * K + 8.0), skip ? 0.0 : 2.0 * n * Kt);
            launch_mdot<double, double>(c, nb, n, K, Q, ld, (const double*)x, xe, part, skip);
        }
        mdot_final(c, nb, Kt, part, 1.0, h, nullptr, 0, 0, nullptr, skip);
    };
    dots(x, nullptr, "mdot");
    // x <- x - Q h in place (each row read before it is written), ||x||^2 into sq
    gemv_fused_impl<double, double>(c, n, K, Q, ld, h, -1.0, x, 1.0, x, (double*)nullptr, nullptr, sq, nullptr,
                                    "gemv");
    hipLaunchKernelGGL(k_cgs_keep, dim3(1), dim3(1), 0, c.stream, (const double*)(h + K), (const double*)sq, flag);
    MMOF_LAUNCH_CHECK();
    // the second pass, carried out only where the test asks for it
    dots(nullptr, flag, "cgs_second");
    gemv_fused_impl<double, double>(c, n, K, Q, ld, h, -1.0, x, 1.0, x, (double*)nullptr, nullptr, sq, flag,
                                    "cgs_second");
}

// ---------------------------------------------------------------- implicit basis
// The true basis is V = Vs T with Vs the stored columns and T unit upper triangular
// (column-major, leading dimension KLD: T(i, j) = T[j * KLD + i], column j = the coefficients
// of v_j in Vs).  One workgroup of KB threads; K <= KMAX.

// g = T^T h (g_i = sum_{k <= i} T(k, i) h_k), into LDS, and its squared norm (thread 0).
__device__ double basis_coeffs(int K, const double* __restrict__ T, const double* __restrict__ h, double* g,
                               double* s4) {
    double e2 = 0.0;
    for (int i = threadIdx.x; i < K; i += KB) {
        const double* ti = T + (int64_t)i * KLD;
        double a = 0.0;
        for (int k = 0; k < i; ++k) a = fma(ti[k], h[k], a);
        a += h[i];  // T(i, i) = 1
        g[i] = a;
        e2 = fma(a, a, e2);
    }
    return block_sum(e2, s4);  // (also orders the writes of g before any later read)
}

// keep[0] = 1 when ||r||^2 - ||g||^2 >= ||r||^2 / 2 (r keeps at least 1/sqrt(2) of its norm
// outside the basis: no explicit pass); otherwise keep[0] = 0 and hc = T g, the coefficients
// in Vs of the part of r along the basis.
__global__ __launch_bounds__(KB) void k_basis_check(int K, const double* __restrict__ T,
                                                    const double* __restrict__ h, const double* __restrict__ rr2,
                                                    double* __restrict__ hc, int* __restrict__ keep) {
    __shared__ double g[KMAX];
    __shared__ double s4[4];
    __shared__ int need;
    const double G2 = basis_coeffs(K, T, h, g, s4);
    if (threadIdx.x == 0) {
        need = !(rr2[0] - G2 >= 0.5 * rr2[0]);
        keep[0] = need ? 0 : 1;
    }
    __syncthreads();
    if (!need) return;
    for (int k = threadIdx.x; k < K; k += KB) {
        double a = g[k];  // T(k, k) = 1
        for (int i = k + 1; i < K; ++i) a = fma(T[(int64_t)i * KLD + k], g[i], a);
        hc[k] = a;
    }
}

// Appends column K of T for a new stored column vs_K = r / rho: g = T^T h with h = Vs^T r,
// rho^2 = ||r||^2 - ||g||^2 (written to sq[0]), T(:, K) = e_K - T g / rho, so that
// v_K = vs_K - V g / rho = (r - V V^T r) / rho.
__global__ __launch_bounds__(KB) void k_basis_append(int K, double* __restrict__ T, const double* __restrict__ h,
                                                     const double* __restrict__ rr2, double* __restrict__ sq) {
    __shared__ double g[KMAX];
    __shared__ double s4[4];
    __shared__ double inv;
    const double G2 = basis_coeffs(K, T, h, g, s4);
    if (threadIdx.x == 0) {
        const double rho2 = fmax(rr2[0] - G2, 0.0);
        sq[0] = rho2;
        inv = rho2 > 0.0 ? 1.0 / sqrt(rho2) : 0.0;
    }
    __syncthreads();
    double* tK = T + (int64_t)K * KLD;
    for (int k = threadIdx.x; k <= K; k += KB) {
        if (k == K) {
            tK[k] = 1.0;
            continue;
        }
        double a = g[k];
        for (int i = k + 1; i < K; ++i) a = fma(T[(int64_t)i * KLD + k], g[i], a);
        tK[k] = -a * inv;
    }
}

// W(a, j) = sum_{b <= j} Gs(a, b) T(b, j) for a, j < K (one thread per entry).
__global__ __launch_bounds__(KB) void k_basis_right(int K, const double* __restrict__ Gs, int ldg,
                                                    const double* __restrict__ T, double* __restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (e >= (int64_t)K * K) return;
    const int a = (int)(e % K), j = (int)(e / K);
    const double* tj = T + (int64_t)j * KLD;
    double s = Gs[(int64_t)a * ldg + j];  // T(j, j) = 1
    for (int b = 0; b < j; ++b) s = fma(Gs[(int64_t)a * ldg + b], tj[b], s);
    W[(int64_t)j * KLD + a] = s;
}

// G(i, j) = G(j, i) = sum_{a <= i} T(a, i) W(a, j) for i <= j < K, and (d != null)
// d_i = sum_{a <= i} T(a, i) ds_a.
__global__ __launch_bounds__(KB) void k_basis_left(int K, const double* __restrict__ T, const double* __restrict__ W,
                                                   double* __restrict__ G, int ldg, const double* __restrict__ ds,
                                                   double* __restrict__ d) {
    const int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (e < (int64_t)K * K) {
        const int i = (int)(e % K), j = (int)(e / K);
        if (i <= j) {
            const double* ti = T + (int64_t)i * KLD;
            const double* wj = W + (int64_t)j * KLD;
            double s = wj[i];
            for (int a = 0; a < i; ++a) s = fma(ti[a], wj[a], s);
            G[(int64_t)i * ldg + j] = s;
            G[(int64_t)j * ldg + i] = s;
        }
    }
    if (d && blockIdx.x == 0) {
        for (int i = threadIdx.x; i < K; i += KB) {
            const double* ti = T + (int64_t)i * KLD;
            double s = ds[i];
            for (int a = 0; a < i; ++a) s = fma(ti[a], ds[a], s);
            d[i] = s;
        }
    }
}

// zt = T z (zt_k = sum_{i >= k} T(k, i) z_i).
__global__ __launch_bounds__(KB) void k_basis_coef(int K, const double* __restrict__ T, const double* __restrict__ z,
                                                   double* __restrict__ zt) {
    for (int k = threadIdx.x; k < K; k += KB) {
        double a = z[k];
        for (int i = k + 1; i < K; ++i) a = fma(T[(int64_t)i * KLD + k], z[i], a);
        zt[k] = a;
    }
}

__global__ void k_basis_eye(int K0, double* __restrict__ T) {
    // columns 0 .. K0-1 of the identity (the rest of T is written as columns are appended)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)K0 * KLD;
         e += (int64_t)gridDim.x * blockDim.x)
        T[e] = (e % KLD) == (e / KLD) ? 1.0 : 0.0;
}

void basis_identity(Ctx& c, int K0, double* T) {
    if (K0 <= 0) return;
    hipLaunchKernelGGL(k_basis_eye, grid_for((int64_t)K0 * KLD, KB, 1024), dim3(KB), 0, c.stream, K0, T);
    MMOF_LAUNCH_CHECK();
}

void basis_extend(Ctx& c, int64_t n, int K, const double* Vs, int64_t ld, double* r, double* T, double* h,
                  double* sq) {
    MMOF_CHECK(K >= 1 && K < KMAX, MMOF_ERR_SHAPE, "too many Krylov columns");
    const int nb = mdot_blocks(n);
    double* part = static_cast<double*>(c.work("mdot_part", sizeof(double) * (size_t)MAX_PART * (KMAX + 1)));
    int* keep = static_cast<int*>(c.work("cgs_flag", sizeof(int)));
    double* hc = static_cast<double*>(c.work("basis_hc", sizeof(double) * KMAX));
    auto dots = [&](const double* xe, const int* skip, const char* tname) {
        const int Kt = K + (xe ? 1 : 0);
        {
            ScopedTime st(&c, tname, skip ? 0.0 : (double)n * (8.0 * K + 8.0), skip ? 0.0 : 2.0 * n * Kt);
            launch_mdot<double, double>(c, nb, n, K, Vs, ld, (const double*)r, xe, part, skip);
        }
        mdot_final(c, nb, Kt, part, 1.0, h, nullptr, 0, 0, nullptr, skip);
    };
    // h = Vs^T r and h[K] = ||r||^2 in one pass
    dots(r, nullptr, "mdot");
    hipLaunchKernelGGL(k_basis_check, dim3(1), dim3(KB), 0, c.stream, K, (const double*)T, (const double*)h,
                       (const double*)(h + K), hc, keep);
    MMOF_LAUNCH_CHECK();
    // where r lies mostly in the basis: r <- r - V V^T r explicitly (||r||^2 into h[K]) and
    // h = Vs^T r again; these launches return at once otherwise
    gemv_fused_impl<double, double>(c, n, K, Vs, ld, hc, -1.0, r, 1.0, r, (double*)nullptr, nullptr, h + K, keep,
                                    "cgs_second");
    dots(nullptr, keep, "cgs_second");
    hipLaunchKernelGGL(k_basis_append, dim3(1), dim3(KB), 0, c.stream, K, T, (const double*)h,
                       (const double*)(h + K), sq);
    MMOF_LAUNCH_CHECK();
}

void basis_gram(Ctx& c, int K, const double* T, const double* Gs, const double* ds, double* G, double* d) {
    if (K <= 0) return;
    double* W = static_cast<double*>(c.work("basis_W", sizeof(double) * KLD * KLD));
    const unsigned nb = (unsigned)cdiv((int64_t)K * K, KB);
    hipLaunchKernelGGL(k_basis_right, dim3(nb), dim3(KB), 0, c.stream, K, Gs, KLD, T, W);
    MMOF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_basis_left, dim3(nb), dim3(KB), 0, c.stream, K, T, (const double*)W, G, KLD, ds, d);
    MMOF_LAUNCH_CHECK();
}

void basis_coef(Ctx& c, int K, const double* T, const double* z, double* zt) {
    if (K <= 0) return;
    hipLaunchKernelGGL(k_basis_coef, dim3(1), dim3(KB), 0, c.stream, K, T, z, zt);
    MMOF_LAUNCH_CHECK();
}

template <class TO>
void normalize2(Ctx& c, int64_t n, const double* x, const double* s2, double* s1, double* out_d, TO* out_t) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_normalize2<TO>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, x, s2, s1, out_d, out_t);
    MMOF_LAUNCH_CHECK();
}
template void normalize2<float>(Ctx&, int64_t, const double*, const double*, double*, double*, float*);
template void normalize2<double>(Ctx&, int64_t, const double*, const double*, double*, double*, double*);

template <class TX>
void axpy_conv(Ctx& c, int64_t n, const TX* in, const double* q, const double* s, double sign, double* out) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_axpy_conv<TX>, grid_for(n, KB, 8192), dim3(KB), 0, c.stream, n, in, q, s, sign, out);
    MMOF_LAUNCH_CHECK();
}
template void axpy_conv<float>(Ctx&, int64_t, const float*, const double*, const double*, double, double*);
template void axpy_conv<double>(Ctx&, int64_t, const double*, const double*, const double*, double, double*);

template <class TX>
void gemv_cols(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* h, double alpha, double beta,
               double* out) {
    MMOF_CHECK(K <= KMAX, MMOF_ERR_SHAPE, "too many Krylov columns");
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

template <class TX, int G, bool VEC, bool NU>
static void wgram_launch(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const void* w, double eps2,
                         double* part, int max_blocks, int& nb) {
    // 16 waves per workgroup where the registers allow (4 per SIMD, to overlap the loads with
    // the matrix-core work), about 16 16-row steps per wave, at most max_blocks partials
    constexpr int W = (sizeof(TX) == 4 && G <= 2) ? 16 : 8;
    const int64_t steps = (n + 15) / 16;
    nb = (int)std::max<int64_t>(1, std::min<int64_t>(max_blocks, cdiv(steps, 16 * W)));
    hipLaunchKernelGGL((k_wgram_part<TX, G, VEC, W, NU>), dim3(nb), dim3(64 * W), 0, c.stream, n, K, X, ld, w, eps2,
                       part);
}

template <class TX, int G, bool NU>
static void wgram_launch_g(Ctx& c, int& nb, bool vec, int64_t n, int K, const TX* X, int64_t ld, const void* w,
                           double eps2, double* part, int max_blocks) {
    if constexpr (sizeof(TX) == 4) {
        if (vec) {
            wgram_launch<TX, G, true, NU>(c, n, K, X, ld, w, eps2, part, max_blocks, nb);
            return;
        }
    }
    wgram_launch<TX, G, false, NU>(c, n, K, X, ld, w, eps2, part, max_blocks, nb);
}

template <class TX, int NQ, bool NU>
static void wgram_quad_launch(Ctx& c, bool vec, int64_t n, int K, const TX* X, int64_t ld, const void* w,
                              double eps2, double* part, int max_blocks, int& nb) {
    // four waves per workgroup (the largest forms hold one wave per SIMD: 294 registers at
    // 10 FP32 quads), at least 16 steps per wave, at most max_blocks partials
    constexpr int W = 4;
    constexpr int STEP = 16 * QuadRows<TX, NQ>::RPL;
    const int64_t steps = (n + STEP - 1) / STEP;
    nb = (int)std::max<int64_t>(1, std::min<int64_t>(max_blocks, cdiv(steps, 16 * W)));
    constexpr int WN = NU ? QW_NU : QW_BUF;
    if (vec) {
        if (NU || w)
            hipLaunchKernelGGL((k_wgram_quad<TX, NQ, true, W, WN>), dim3(nb), dim3(64 * W), 0, c.stream, n, K, X, ld,
                               w, eps2, part);
        else
            hipLaunchKernelGGL((k_wgram_quad<TX, NQ, true, W, QW_ONE>), dim3(nb), dim3(64 * W), 0, c.stream, n, K, X,
                               ld, w, eps2, part);
    } else {
        if (NU || w)
            hipLaunchKernelGGL((k_wgram_quad<TX, NQ, false, W, WN>), dim3(nb), dim3(64 * W), 0, c.stream, n, K, X,
                               ld, w, eps2, part);
        else
            hipLaunchKernelGGL((k_wgram_quad<TX, NQ, false, W, QW_ONE>), dim3(nb), dim3(64 * W), 0, c.stream, n, K,
                               X, ld, w, eps2, part);
    }
}

// K <= 4 GRAM_QUADS: stage 1 on the 4x4x4 form, then its fixed-order stage 2 into G.
template <class TX, bool NU>
static void wgram_quad_stages(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const void* w, double eps2,
                              double* G, int ldg, double* part, int max_blocks, bool timed) {
    constexpr int RPL = QuadRows<TX, 1>::RPL;
    const int NQ = (K + 3) / 4;
    (void)RPL;
    const bool vec = (reinterpret_cast<uintptr_t>(X) % sizeof(TX) == 0) &&
                     (!w || reinterpret_cast<uintptr_t>(w) % 16 == 0);
    int nb = 1;
    {
        // K columns and the row weights (8 bytes from w, the size of TX from nu, none when null)
        const double wb = NU ? (double)sizeof(TX) : (w ? 8.0 : 0.0);
        ScopedTime st(timed ? &c : nullptr, "wgram", (double)n * ((double)sizeof(TX) * K + wb),
                      (double)n * K * (K + 1));
        switch (NQ) {
            case 1: wgram_quad_launch<TX, 1, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 2: wgram_quad_launch<TX, 2, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 3: wgram_quad_launch<TX, 3, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 4: wgram_quad_launch<TX, 4, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 5: wgram_quad_launch<TX, 5, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 6: wgram_quad_launch<TX, 6, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 7: wgram_quad_launch<TX, 7, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 8: wgram_quad_launch<TX, 8, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            case 9: wgram_quad_launch<TX, 9, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
            default: wgram_quad_launch<TX, GRAM_QUADS, NU>(c, vec, n, K, X, ld, w, eps2, part, max_blocks, nb); break;
        }
        MMOF_LAUNCH_CHECK();
    }
    const int ne = NQ * (NQ + 1) / 2 * 16;
    hipLaunchKernelGGL(k_wgram_final_quad, dim3((unsigned)cdiv((int64_t)ne, GRAM_SLAB)), dim3(1024), 0, c.stream, nb,
                       K, NQ, part, G, ldg);
    MMOF_LAUNCH_CHECK();
}

// Stage 1 for 1..4 column blocks, then the fixed-order stage 2 into G.
template <class TX, bool NU>
static void wgram_stages(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const void* w, double eps2, double* G,
                         int ldg, double* part, int max_blocks, bool timed) {
    if (K <= 4 * GRAM_QUADS) {
        wgram_quad_stages<TX, NU>(c, n, K, X, ld, w, eps2, G, ldg, part, max_blocks, timed);
        return;
    }
    const int Gb = (K + 15) / 16;
    const int np = Gb * (Gb + 1) / 2;
    int nb = 1;  // stage-1 workgroups (partials), set by the launch
    // (vector loads for FP32 columns; FP64 columns load a double per row, which keeps the
    // row buffers in registers; the vector path also reads w with 16-byte loads)
    const bool vec = sizeof(TX) == 4 && (reinterpret_cast<uintptr_t>(X) % 4 == 0) &&
                     (NU || !w || reinterpret_cast<uintptr_t>(w) % 16 == 0);
    {
        const double wb = NU ? (double)sizeof(TX) : (w ? 8.0 : 0.0);
        ScopedTime st(timed ? &c : nullptr, "wgram", (double)n * ((double)sizeof(TX) * K + wb),
                      (double)n * K * (K + 1));
        switch (Gb) {
            case 1: wgram_launch_g<TX, 1, NU>(c, nb, vec, n, K, X, ld, w, eps2, part, max_blocks); break;
            case 2: wgram_launch_g<TX, 2, NU>(c, nb, vec, n, K, X, ld, w, eps2, part, max_blocks); break;
            case 3: wgram_launch_g<TX, 3, NU>(c, nb, vec, n, K, X, ld, w, eps2, part, max_blocks); break;
            default: wgram_launch_g<TX, 4, NU>(c, nb, vec, n, K, X, ld, w, eps2, part, max_blocks); break;
        }
        MMOF_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_wgram_final, dim3((unsigned)cdiv((int64_t)np * 256, GRAM_SLAB)), dim3(1024), 0, c.stream,
                       nb, K, Gb, part, G, ldg);
    MMOF_LAUNCH_CHECK();
}

template <class TX>
void wgram(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* w, double* G, int ldg) {
    MMOF_CHECK(K >= 1 && K <= KMAX, MMOF_ERR_SHAPE, "too many Krylov columns");
    constexpr int RP = GRAM_RECT * GRAM_RECT;
    double* part = static_cast<double*>(
        c.work("wgram_part", sizeof(double) * (size_t)GRAM_BLOCKS * std::max(GRAM_PAIRS, RP) * 256));
    if (K <= 64) {
        wgram_stages<TX, false>(c, n, K, X, ld, w, 0.0, G, ldg, part, GRAM_BLOCKS, true);
        return;
    }
    // more than 64 columns: tiles of 64 x 64 entries -- the diagonal tiles by the kernel above,
    // the tiles above them by k_wgram_rect, one partial buffer reused tile after tile (stream order)
    const int nsb = (K + 63) / 64;
    const bool vec = sizeof(TX) == 4 && (reinterpret_cast<uintptr_t>(X) % 4 == 0) &&
                     (!w || reinterpret_cast<uintptr_t>(w) % 16 == 0);
    for (int a = 0; a < nsb; ++a) {
        const int Ka = std::min(64, K - 64 * a);
        wgram_stages<TX, false>(c, n, Ka, X + (int64_t)64 * a * ld, ld, w, 0.0, G + (int64_t)64 * a * ldg + 64 * a,
                                ldg, part, GRAM_BLOCKS, true);
        for (int b2 = a + 1; b2 < nsb; ++b2) {
            const int Kb = std::min(64, K - 64 * b2);
            constexpr int W = sizeof(TX) == 4 ? 8 : 4;   // (FP64 rows need twice the registers)
            const int64_t steps = (n + 15) / 16;
            const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(GRAM_BLOCKS, cdiv(steps, 16 * W)));
            const TX* XI = X + (int64_t)64 * a * ld;
            const TX* XJ = X + (int64_t)64 * b2 * ld;
            {
                ScopedTime st(&c, "wgram", (double)n * ((double)sizeof(TX) * (Ka + Kb) + 8.0),
                              2.0 * (double)n * Ka * Kb);
                if (vec)
                    hipLaunchKernelGGL((k_wgram_rect<TX, GRAM_RECT, GRAM_RECT, sizeof(TX) == 4, W>), dim3(nb),
                                       dim3(64 * W), 0, c.stream, n, Ka, Kb, XI, XJ, ld, w, part);
                else
                    hipLaunchKernelGGL((k_wgram_rect<TX, GRAM_RECT, GRAM_RECT, false, W>), dim3(nb), dim3(64 * W),
                                       0, c.stream, n, Ka, Kb, XI, XJ, ld, w, part);
                MMOF_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_wgram_final_rect, dim3((unsigned)cdiv((int64_t)RP * 256, GRAM_SLAB)), dim3(1024), 0,
                               c.stream, nb, GRAM_RECT, RP, Ka, Kb, 64 * a, 64 * b2, (const double*)part, G, ldg);
            MMOF_LAUNCH_CHECK();
        }
    }
}
template void wgram<float>(Ctx&, int64_t, int, const float*, int64_t, const double*, double*, int);
template void wgram<double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double*, int);

template <class TX>
void wgram_nu(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TX* nu, double eps, double* G, int ldg) {
    MMOF_CHECK(K >= 1 && K <= KMAX_SMALL, MMOF_ERR_SHAPE, "too many Krylov columns for weights formed from nu");
    constexpr int RP = GRAM_RECT * GRAM_RECT;
    double* part = static_cast<double*>(
        c.work("wgram_part", sizeof(double) * (size_t)GRAM_BLOCKS * std::max(GRAM_PAIRS, RP) * 256));
    wgram_stages<TX, true>(c, n, K, X, ld, nu, eps * eps, G, ldg, part, GRAM_BLOCKS, true);
}
template void wgram_nu<float>(Ctx&, int64_t, int, const float*, int64_t, const float*, double, double*, int);
template void wgram_nu<double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double, double*, int);

// ------------------------------------------------------------------------ allocation-free Gram
//
// The Gram of a column block for callers that cannot allocate device memory: the stage-1
// partials live in this file-scope array, one copy per GPU (its address on each device is
// looked up once, at context creation, with hipGetSymbolAddress; the host-side name of the
// array is never passed to a kernel), and the MM weights are formed inside the kernel from nu
// instead of in an n-entry buffer.  Every call on one GPU uses the same array: calls that
// overlap in time on one device (several streams, several host threads) race on it.
static constexpr int NOALLOC_BLOCKS = 256;   // at most 256 stage-1 workgroups
static constexpr size_t NOALLOC_DOUBLES = (size_t)NOALLOC_BLOCKS * GRAM_PAIRS * 256;   // 5 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

static constexpr int NOALLOC_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEV] = {};

void noalloc_init(int device) {
    MMOF_CHECK(device >= 0 && device < NOALLOC_MAX_DEV, MMOF_ERR_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    int cur = -1;
    MMOF_HIP(hipGetDevice(&cur));
    MMOF_CHECK(cur == device, MMOF_ERR_INVALID, "scratch lookup needs the device current");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    MMOF_CHECK(e == hipSuccess && ptr, MMOF_ERR_HIP,
               std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<double*>(ptr);
}

size_t noalloc_scratch_bytes() { return sizeof(double) * NOALLOC_DOUBLES; }

template <class TX>
void wgram_noalloc(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TX* nu, double eps, double* G,
                   int ldg) {
    MMOF_CHECK(K >= 1 && K <= KMAX_SMALL, MMOF_ERR_SHAPE, "too many Krylov columns");
    MMOF_CHECK(c.device >= 0 && c.device < NOALLOC_MAX_DEV && g_scratch_ptr[c.device], MMOF_ERR_INVALID,
               "the context was created without the scratch lookup");
    double* part = g_scratch_ptr[c.device];
    if (nu)
        wgram_stages<TX, true>(c, n, K, X, ld, nu, eps * eps, G, ldg, part, NOALLOC_BLOCKS, false);
    else
        wgram_stages<TX, false>(c, n, K, X, ld, nullptr, 0.0, G, ldg, part, NOALLOC_BLOCKS, false);
}
template void wgram_noalloc<float>(Ctx&, int64_t, int, const float*, int64_t, const float*, double, double*, int);
template void wgram_noalloc<double>(Ctx&, int64_t, int, const double*, int64_t, const double*, double, double*,
                                    int);

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
