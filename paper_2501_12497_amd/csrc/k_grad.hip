// Psi = blockdiag(L), L = [I (x) L_x ; L_y (x) I] (first differences, no boundary rows),
// optionally weighted row by row, and its transpose, over tiles of every frame in the
// packed stack (tile shape chosen per geometry).
#include "dev.h"
#include "kernels.h"

namespace mmof {

// A GTW x GTH tile per workgroup of 256 threads; each thread owns RPT = GTW * GTH / 256
// consecutive rows of one column, so the row below is loaded once and reused.
template <class T, int GTW, int GTH>
__global__ __launch_bounds__(256) void k_grad_fwd(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                  const T* __restrict__ u, const T* __restrict__ wx,
                                                  const T* __restrict__ wy, T* __restrict__ gx, T* __restrict__ gy) {
    constexpr int RPT = GTW * GTH / 256;
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % GTW);
    const int y0 = tl.y0 + (int)(threadIdx.x / GTW) * RPT;
    if (x >= f.nx || y0 >= f.ny) return;
    const int nx = f.nx, ny = f.ny;
    const T* uf = u + f.off;
    T c = uf[(int64_t)y0 * nx + x];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int y = y0 + k;
        if (y >= ny) break;
        const int64_t p = (int64_t)y * nx + x;
        if (x < nx - 1) {
            const int64_t o = f.gx_off + (int64_t)y * (nx - 1) + x;
            T d = uf[p + 1] - c;
            gx[o] = wx ? wx[o] * d : d;
        }
        T below = T(0);
        if (y < ny - 1) {
            below = uf[p + nx];
            const int64_t o = f.gy_off + p;
            T d = below - c;
            gy[o] = wy ? wy[o] * d : d;
        }
        c = below;
    }
}

template <class T, int GTW, int GTH>
__global__ __launch_bounds__(256) void k_grad_adj(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                  const T* __restrict__ gx, const T* __restrict__ gy,
                                                  const T* __restrict__ wx, const T* __restrict__ wy,
                                                  T* __restrict__ u, int accumulate) {
    constexpr int RPT = GTW * GTH / 256;
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % GTW);
    const int y0 = tl.y0 + (int)(threadIdx.x / GTW) * RPT;
    if (x >= f.nx || y0 >= f.ny) return;
    const int nx = f.nx, ny = f.ny;
    const int64_t ry = f.gy_off;
    // gy of the row above the first row
    T up = T(0);
    if (y0 > 0) {
        const int64_t o = ry + (int64_t)(y0 - 1) * nx + x;
        up = wy ? wy[o] * gy[o] : gy[o];
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int y = y0 + k;
        if (y >= ny) break;
        const int64_t rx = f.gx_off + (int64_t)y * (nx - 1);  // row y of gx
        T acc = T(0);
        if (x > 0) {
            const int64_t o = rx + x - 1;
            acc += wx ? wx[o] * gx[o] : gx[o];
        }
        if (x < nx - 1) {
            const int64_t o = rx + x;
            acc -= wx ? wx[o] * gx[o] : gx[o];
        }
        if (y > 0) acc += up;
        T here = T(0);
        if (y < ny - 1) {
            const int64_t o = ry + (int64_t)y * nx + x;
            here = wy ? wy[o] * gy[o] : gy[o];
            acc -= here;
        }
        up = here;
        const int64_t p = f.off + (int64_t)y * nx + x;
        u[p] = accumulate ? u[p] + acc : acc;
    }
}

const TileShape kGradShapes[] = {{64, 16, 0}, {64, 8, 0}, {64, 4, 0}, {32, 32, 0}};
const int kGradCandidates = sizeof(kGradShapes) / sizeof(kGradShapes[0]);

template <class T>
static auto grad_fwd_kernel(int choice) {
    return choice == 0 ? k_grad_fwd<T, 64, 16>
           : choice == 1 ? k_grad_fwd<T, 64, 8>
           : choice == 2 ? k_grad_fwd<T, 64, 4>
                         : k_grad_fwd<T, 32, 32>;
}
template <class T>
static auto grad_adj_kernel(int choice) {
    return choice == 0 ? k_grad_adj<T, 64, 16>
           : choice == 1 ? k_grad_adj<T, 64, 8>
           : choice == 2 ? k_grad_adj<T, 64, 4>
                         : k_grad_adj<T, 32, 32>;
}

void launch_grad_fwd(Ctx& c, Geom& g, int dt, const void* u, const void* wx, const void* wy, void* gx, void* gy,
                     int choice) {
    if (choice < 0) choice = g.choice("grad_fwd", dt, 2);
    MMOF_CHECK(choice >= 0 && choice < kGradCandidates, MMOF_ERR_INVALID, "grad tile candidate out of range");
    const TileShape sh = kGradShapes[choice];
    const TileList& tl = g.tile_list(c.stream, sh.tw, sh.th, false);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "grad_fwd", 3.0 * sizeof(T) * g.n, 2.0 * g.n);
        hipLaunchKernelGGL(grad_fwd_kernel<T>(choice), dim3((unsigned)tl.count), dim3(256), 0, c.stream,
                           tl.buf.as<Tile>(), g.dframes(), (const T*)u, (const T*)wx, (const T*)wy, (T*)gx, (T*)gy);
        MMOF_LAUNCH_CHECK();
    });
}

void launch_grad_adj(Ctx& c, Geom& g, int dt, const void* gx, const void* gy, const void* wx, const void* wy,
                     void* u, bool accumulate, int choice) {
    if (choice < 0) choice = g.choice("grad_adj", dt, 2);
    MMOF_CHECK(choice >= 0 && choice < kGradCandidates, MMOF_ERR_INVALID, "grad tile candidate out of range");
    const TileShape sh = kGradShapes[choice];
    const TileList& tl = g.tile_list(c.stream, sh.tw, sh.th, false);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "grad_adj", 3.0 * sizeof(T) * g.n, 3.0 * g.n);
        hipLaunchKernelGGL(grad_adj_kernel<T>(choice), dim3((unsigned)tl.count), dim3(256), 0, c.stream,
                           tl.buf.as<Tile>(), g.dframes(), (const T*)gx, (const T*)gy, (const T*)wx, (const T*)wy,
                           (T*)u, accumulate ? 1 : 0);
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
