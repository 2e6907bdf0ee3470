// Per-frame Gaussian blur with zero boundary, K = k1 k1^T (k1 normalised to unit sum, so
// sum K = 1).  Because K(i,j) = K(-i,-j) the transpose applies the same sum, so one
// kernel serves H and H^T.  Separable: a horizontal then a vertical pass over an LDS
// tile of 64x16 outputs plus a halo of ksize/2 on every side.
#include "dev.h"
#include "kernels.h"

namespace mmof {

static constexpr int BTX = 64, BTY = 16, BRMAX = 7;

template <class T>
__global__ __launch_bounds__(256) void k_blur(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                              const double* __restrict__ k1d, int r, const T* __restrict__ in,
                                              T* __restrict__ out) {
    __shared__ T s_in[BTY + 2 * BRMAX][BTX + 2 * BRMAX];
    __shared__ T s_h[BTY + 2 * BRMAX][BTX];
    __shared__ T s_k[2 * BRMAX + 1];
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int nx = f.nx, ny = f.ny;
    const T* src = in + f.off;
    if (threadIdx.x < 2 * r + 1) s_k[threadIdx.x] = (T)k1d[threadIdx.x];
    const int hw = BTX + 2 * r, hh = BTY + 2 * r;
    for (int i = threadIdx.x; i < hw * hh; i += 256) {
        const int ly = i / hw, lx = i % hw;
        const int y = tl.y0 - r + ly, x = tl.x0 - r + lx;
        s_in[ly][lx] = (y >= 0 && y < ny && x >= 0 && x < nx) ? src[(int64_t)y * nx + x] : T(0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < BTX * hh; i += 256) {
        const int ly = i / BTX, lx = i % BTX;
        T acc = T(0);
        for (int j = 0; j <= 2 * r; ++j) acc += s_k[j] * s_in[ly][lx + j];
        s_h[ly][lx] = acc;
    }
    __syncthreads();
    const int lx = threadIdx.x % BTX;
    for (int ly = threadIdx.x / BTX; ly < BTY; ly += 256 / BTX) {
        const int y = tl.y0 + ly, x = tl.x0 + lx;
        if (y >= ny || x >= nx) continue;
        T acc = T(0);
        for (int i = 0; i <= 2 * r; ++i) acc += s_k[i] * s_h[ly + i][lx];
        out[f.off + (int64_t)y * nx + x] = acc;
    }
}

void launch_blur(Ctx& c, Plan& p, int dt, const void* in, void* out) {
    Geom& g = *p.geom;
    const TileList& tl = g.tile_list(c.stream, BTX, BTY, false);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "blur", 2.0 * sizeof(T) * g.n, 4.0 * p.ksize * g.n);
        hipLaunchKernelGGL(k_blur<T>, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(),
                           g.dframes(), p.d_k1.as<double>(), p.ksize / 2, (const T*)in, (T*)out);
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
