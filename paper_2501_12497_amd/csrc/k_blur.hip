// Per-frame Gaussian blur with zero boundary, K = k1 k1^T (k1 normalised to unit sum, so
// sum K = 1).  Because K(i,j) = K(-i,-j) the transpose applies the same sum, so one
// kernel serves H and H^T.  Separable: a horizontal then a vertical pass over an LDS
// tile of outputs plus a halo of ksize/2 on every side (tile shape chosen per geometry).
#include "dev.h"
#include "kernels.h"

namespace mmof {

static constexpr int BRMAX = 7;

// TW x TH output tile per workgroup of 256 threads.  PERS: a grid of a few workgroups per
// CU loops over the tile list (persistent launch); otherwise one workgroup per tile.
template <class T, int TW, int TH, bool PERS>
__global__ __launch_bounds__(256) void k_blur(const Tile* __restrict__ tiles, int64_t n_tiles,
                                              const FrameInfo* __restrict__ fr, const double* __restrict__ k1d,
                                              int r, const T* __restrict__ in, T* __restrict__ out) {
    __shared__ T s_in[TH + 2 * BRMAX][TW + 2 * BRMAX];
    __shared__ T s_h[TH + 2 * BRMAX][TW];
    __shared__ T s_k[2 * BRMAX + 1];
    if (threadIdx.x < 2 * r + 1) s_k[threadIdx.x] = (T)k1d[threadIdx.x];
    const int64_t step = PERS ? gridDim.x : n_tiles;
    for (int64_t ti = PERS ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x); ti < n_tiles; ti += step) {
        const Tile tl = tiles[ti];
        const FrameInfo f = fr[tl.frame];
        const int nx = f.nx, ny = f.ny;
        const T* src = in + f.off;
        const int hw = TW + 2 * r, hh = TH + 2 * r;
        __syncthreads();  // LDS of the previous tile is free
        for (int i = threadIdx.x; i < hw * hh; i += 256) {
            const int ly = i / hw, lx = i % hw;
            const int y = tl.y0 - r + ly, x = tl.x0 - r + lx;
            s_in[ly][lx] = (y >= 0 && y < ny && x >= 0 && x < nx) ? src[(int64_t)y * nx + x] : T(0);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < TW * hh; i += 256) {
            const int ly = i / TW, lx = i % TW;
            T acc = T(0);
            for (int j = 0; j <= 2 * r; ++j) acc += s_k[j] * s_in[ly][lx + j];
            s_h[ly][lx] = acc;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < TW * TH; i += 256) {
            const int ly = i / TW, lx = i % TW;
            const int y = tl.y0 + ly, x = tl.x0 + lx;
            if (y >= ny || x >= nx) continue;
            T acc = T(0);
            for (int k = 0; k <= 2 * r; ++k) acc += s_k[k] * s_h[ly + k][lx];
            out[f.off + (int64_t)y * nx + x] = acc;
        }
    }
}

// The same sums with the radius R compiled in (the 9-tap case): both passes are unrolled and
// a thread forms 4 outputs from one register copy of the 4 + 2R inputs they share (a row
// segment in the horizontal pass, a column segment in the vertical one), so a tap costs
// one FMA and the LDS reads drop from 2R + 1 to (4 + 2R) / 4 per output.  Per output the
// taps are added in the order of k_blur, so the values are identical.
template <class T, int TW, int TH, bool PERS, int R>
__global__ __launch_bounds__(256) void k_blur_r(const Tile* __restrict__ tiles, int64_t n_tiles,
                                                const FrameInfo* __restrict__ fr, const double* __restrict__ k1d,
                                                const T* __restrict__ in, T* __restrict__ out) {
    constexpr int HW = TW + 2 * R, HH = TH + 2 * R;
    static_assert(TW % 4 == 0 && TH % 4 == 0, "tiles split into 4-output segments");
    __shared__ T s_in[HH][HW + 1];
    __shared__ T s_h[HH][TW + 1];
    T kk[2 * R + 1];
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) kk[j] = (T)k1d[j];
    const int64_t step = PERS ? gridDim.x : n_tiles;
    for (int64_t ti = PERS ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x); ti < n_tiles; ti += step) {
        const Tile tl = tiles[ti];
        const FrameInfo f = fr[tl.frame];
        const int nx = f.nx, ny = f.ny;
        const T* src = in + f.off;
        __syncthreads();  // LDS of the previous tile is free
        for (int i = threadIdx.x; i < HW * HH; i += 256) {
            const int ly = i / HW, lx = i % HW;
            const int y = tl.y0 - R + ly, x = tl.x0 - R + lx;
            s_in[ly][lx] = (y >= 0 && y < ny && x >= 0 && x < nx) ? src[(int64_t)y * nx + x] : T(0);
        }
        __syncthreads();
        // horizontal pass: row ly, outputs lx0 .. lx0 + 3
        for (int i = threadIdx.x; i < (TW / 4) * HH; i += 256) {
            const int ly = i / (TW / 4), lx0 = 4 * (i % (TW / 4));
            T v[4 + 2 * R];
#pragma unroll
            for (int c = 0; c < 4 + 2 * R; ++c) v[c] = s_in[ly][lx0 + c];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j <= 2 * R; ++j) acc += kk[j] * v[q + j];
                s_h[ly][lx0 + q] = acc;
            }
        }
        __syncthreads();
        // vertical pass: column lx, outputs ly0 .. ly0 + 3
        for (int i = threadIdx.x; i < TW * (TH / 4); i += 256) {
            const int lx = i % TW, ly0 = 4 * (i / TW);
            T v[4 + 2 * R];
#pragma unroll
            for (int c = 0; c < 4 + 2 * R; ++c) v[c] = s_h[ly0 + c][lx];
            const int x = tl.x0 + lx;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int y = tl.y0 + ly0 + q;
                T acc = T(0);
#pragma unroll
                for (int k = 0; k <= 2 * R; ++k) acc += kk[k] * v[q + k];
                if (y < ny && x < nx) out[f.off + (int64_t)y * nx + x] = acc;
            }
        }
    }
}

const TileShape kBlurShapes[] = {{64, 16, 0}, {32, 32, 0}, {128, 8, 0}, {32, 16, 0}, {64, 16, 1}};
const int kBlurCandidates = sizeof(kBlurShapes) / sizeof(kBlurShapes[0]);

void launch_blur(Ctx& c, Plan& p, int dt, const void* in, void* out, int choice) {
    Geom& g = *p.geom;
    if (choice < 0) choice = g.choice("blur", dt);
    MMOF_CHECK(choice >= 0 && choice < kBlurCandidates, MMOF_ERR_INVALID, "blur tile candidate out of range");
    const TileShape sh = kBlurShapes[choice];
    const TileList& tl = g.tile_list(c.stream, sh.tw, sh.th, false);
    if (tl.count == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "blur", 2.0 * sizeof(T) * g.n, 4.0 * p.ksize * g.n);
        const int64_t grid = sh.persistent ? std::min<int64_t>(tl.count, (int64_t)c.cu_count * 4) : tl.count;
        if (p.ksize == 9) {
            auto k = choice == 0 ? k_blur_r<T, 64, 16, false, 4>
                     : choice == 1 ? k_blur_r<T, 32, 32, false, 4>
                     : choice == 2 ? k_blur_r<T, 128, 8, false, 4>
                     : choice == 3 ? k_blur_r<T, 32, 16, false, 4>
                                   : k_blur_r<T, 64, 16, true, 4>;
            hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), 0, c.stream, tl.buf.as<Tile>(), tl.count,
                               g.dframes(), p.d_k1.as<double>(), (const T*)in, (T*)out);
        } else {
            auto k = choice == 0 ? k_blur<T, 64, 16, false>
                     : choice == 1 ? k_blur<T, 32, 32, false>
                     : choice == 2 ? k_blur<T, 128, 8, false>
                     : choice == 3 ? k_blur<T, 32, 16, false>
                                   : k_blur<T, 64, 16, true>;
            hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), 0, c.stream, tl.buf.as<Tile>(), tl.count,
                               g.dframes(), p.d_k1.as<double>(), p.ksize / 2, (const T*)in, (T*)out);
        }
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
