// Psi = blockdiag(L), L = [I (x) L_x ; L_y (x) I] (first differences, no boundary rows),
// optionally weighted row by row, and its transpose, over tiles of every frame in the
// packed stack (tile shape chosen per geometry).
#include "dev.h"
#include "kernels.h"

namespace mmof {

// A GTW x GTH tile per workgroup of 256 threads; each thread owns RPT = GTW * GTH / 256
// consecutive rows of one column, so the row below is loaded once and reused.
// mx, my (may be null): gx and gy weighted by the MM weights of nux, nuy (RowWeighting).
template <class T, int GTW, int GTH>
__global__ __launch_bounds__(256) void k_grad_fwd(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                  const T* __restrict__ u, const T* __restrict__ wx,
                                                  const T* __restrict__ wy, T* __restrict__ gx, T* __restrict__ gy,
                                                  const T* __restrict__ nux, const T* __restrict__ nuy,
                                                  T* __restrict__ mx, T* __restrict__ my, double eps2) {
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
            d = wx ? wx[o] * d : d;
            gx[o] = d;
            if (mx) mx[o] = mm_weighted(d, nux[o], eps2);
        }
        T below = T(0);
        if (y < ny - 1) {
            below = uf[p + nx];
            const int64_t o = f.gy_off + p;
            T d = below - c;
            d = wy ? wy[o] * d : d;
            gy[o] = d;
            if (my) my[o] = mm_weighted(d, nuy[o], eps2);
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

// Vector form, for stacks whose frame widths are multiples of 4: each thread owns 4
// consecutive pixels of RPT consecutive rows, so image and gy rows move as whole 16-byte
// (FP32) or 2 x 16-byte (FP64) accesses and every wave keeps 4x more bytes in flight than
// with one pixel per lane.  A row of the tile is LW lanes (4*LW pixels) wide.  gx rows
// (stride nx-1) are not 4-aligned: the forward kernel realigns its gx values across lanes
// and stores aligned vectors; the adjoint reads gx as single values.  The pixel right of a
// thread's four (forward) or the gx value left of them (adjoint) comes from the neighbouring
// lane, or from memory at the edge of a lane row.  Values and summation order equal those
// of the scalar kernels above.
template <class T, int LW, int RPT>
__global__ __launch_bounds__(256) void k_grad_fwd4(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                   const T* __restrict__ u, const T* __restrict__ wx,
                                                   const T* __restrict__ wy, T* __restrict__ gx, T* __restrict__ gy,
                                                   const T* __restrict__ nux, const T* __restrict__ nuy,
                                                   T* __restrict__ mx, T* __restrict__ my, double eps2) {
    // the MM-weighted copies of four aligned values and of one value (mx, my may be null)
    auto mw4 = [&](T* m, const T* nu, int64_t o, const Quad<T>& q) {
        const Quad<T> nq = ld4(nu + o);
        Quad<T> r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r.v[i] = mm_weighted(q.v[i], nq.v[i], eps2);
        st4(m + o, r);
    };
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int lx = (int)(threadIdx.x % LW);
    const int x = tl.x0 + 4 * lx;
    const int y0 = tl.y0 + (int)(threadIdx.x / LW) * RPT;
    const int nx = f.nx, ny = f.ny;
    if (x >= nx || y0 >= ny) return;  // x < nx implies x + 3 < nx
    const T* uf = u + f.off;
    Quad<T> c = ld4(uf + (int64_t)y0 * nx + x);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int y = y0 + k;
        if (y >= ny) break;
        const int64_t p = (int64_t)y * nx + x;
        // pixel x + 4: the next lane's first pixel (same row, live whenever x + 4 < nx)
        T right = __shfl_down(c.v[0], 1);
        if (lx == LW - 1 && x + 4 < nx) right = uf[p + 4];
        T d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = (j < 3 ? c.v[j + 1] : right) - c.v[j];
        // The lane row's n_el gx values start at element B of gx (rows of nx - 1 values, so B
        // is rarely 4-aligned): lane lx stores the aligned 4 values from element
        // B + t0 + 4 lx on, taking the ones past its own from the next lane; the t0 values
        // before the first aligned element and the short tail go out singly.
        const int64_t B = f.gx_off + (int64_t)y * (nx - 1) + tl.x0;
        const int n_el = min(4 * LW, nx - 1 - tl.x0);
        const int t0 = (int)((4 - (B & 3)) & 3);
        T sh[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) sh[j] = __shfl_down(d[j], 1);
        Quad<T> g;  // values of elements B + t0 + 4 lx + i
        if (t0 == 0) g = Quad<T>{{d[0], d[1], d[2], d[3]}};
        else if (t0 == 1) g = Quad<T>{{d[1], d[2], d[3], sh[0]}};
        else if (t0 == 2) g = Quad<T>{{d[2], d[3], sh[0], sh[1]}};
        else g = Quad<T>{{d[3], sh[0], sh[1], sh[2]}};
        const int e0 = t0 + 4 * lx;  // first element of the lane's aligned group
        if (e0 + 3 < n_el) {
            if (wx) {
                const Quad<T> w = ld4(wx + B + e0);
#pragma unroll
                for (int i = 0; i < 4; ++i) g.v[i] = w.v[i] * g.v[i];
            }
            st4(gx + B + e0, g);
            if (mx) mw4(mx, nux, B + e0, g);
        } else if (e0 < n_el) {  // the tail (fewer than 4 values)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (e0 + i < n_el) {
                    const T val = wx ? wx[B + e0 + i] * g.v[i] : g.v[i];
                    gx[B + e0 + i] = val;
                    if (mx) mx[B + e0 + i] = mm_weighted(val, nux[B + e0 + i], eps2);
                }
        }
        if (lx == 0) {  // the head, before the first aligned element
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (i < t0 && i < n_el) {
                    const T val = wx ? wx[B + i] * d[i] : d[i];
                    gx[B + i] = val;
                    if (mx) mx[B + i] = mm_weighted(val, nux[B + i], eps2);
                }
        }
        Quad<T> below = zero4<T>();
        if (y < ny - 1) {
            below = ld4(uf + p + nx);
            const int64_t og = f.gy_off + p;
            Quad<T> d;
#pragma unroll
            for (int j = 0; j < 4; ++j) d.v[j] = below.v[j] - c.v[j];
            if (wy) {
                const Quad<T> w = ld4(wy + og);
#pragma unroll
                for (int j = 0; j < 4; ++j) d.v[j] = w.v[j] * d.v[j];
            }
            st4(gy + og, d);
            if (my) mw4(my, nuy, og, d);
        }
        c = below;
    }
}

template <class T, int LW, int RPT>
__global__ __launch_bounds__(256) void k_grad_adj4(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                   const T* __restrict__ gx, const T* __restrict__ gy,
                                                   const T* __restrict__ wx, const T* __restrict__ wy,
                                                   T* __restrict__ u, int accumulate) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int lx = (int)(threadIdx.x % LW);
    const int x = tl.x0 + 4 * lx;
    const int y0 = tl.y0 + (int)(threadIdx.x / LW) * RPT;
    const int nx = f.nx, ny = f.ny;
    if (x >= nx || y0 >= ny) return;
    const int64_t ry = f.gy_off;
    auto wgy = [&](int64_t o) {
        Quad<T> q = ld4(gy + o);
        if (wy) {
            const Quad<T> w = ld4(wy + o);
#pragma unroll
            for (int j = 0; j < 4; ++j) q.v[j] = w.v[j] * q.v[j];
        }
        return q;
    };
    // weighted gy of the row above the first row
    Quad<T> up = zero4<T>();
    if (y0 > 0) up = wgy(ry + (int64_t)(y0 - 1) * nx + x);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int y = y0 + k;
        if (y >= ny) break;
        const int64_t rx = f.gx_off + (int64_t)y * (nx - 1) + x;  // gx at (x, y)
        T g[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            g[j] = T(0);
            if (j < 3 || x + 4 < nx) g[j] = wx ? wx[rx + j] * gx[rx + j] : gx[rx + j];
        }
        // gx at x - 1: the previous lane's last value (same row), or memory at a lane-row edge
        T left = __shfl_up(g[3], 1);
        if (lx == 0) left = x > 0 ? (wx ? wx[rx - 1] * gx[rx - 1] : gx[rx - 1]) : T(0);
        Quad<T> here = zero4<T>();
        if (y < ny - 1) here = wgy(ry + (int64_t)y * nx + x);
        const int64_t p = f.off + (int64_t)y * nx + x;
        Quad<T> out = accumulate ? ld4(u + p) : zero4<T>();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T acc = T(0);
            if (x + j > 0) acc += j == 0 ? left : g[j - 1];
            if (x + j < nx - 1) acc -= g[j];
            if (y > 0) acc += up.v[j];
            if (y < ny - 1) acc -= here.v[j];
            out.v[j] = accumulate ? out.v[j] + acc : acc;
        }
        st4(u + p, out);
        up = here;
    }
}

const TileShape kGradShapes[] = {{64, 16, 0}, {64, 8, 0}, {64, 4, 0}, {32, 32, 0}};
const int kGradCandidates = sizeof(kGradShapes) / sizeof(kGradShapes[0]);
// vector-form candidates: lanes per tile row, rows per thread, waves per workgroup
struct Grad4Shape {
    int lw, rpt, nw;
    int tw() const { return 4 * lw; }
    int th() const { return 64 * nw / lw * rpt; }
};
static const Grad4Shape kGrad4Shapes[] = {{64, 1, 4}, {64, 2, 4}, {32, 1, 2}, {32, 1, 4}};
static_assert(sizeof(kGrad4Shapes) / sizeof(kGrad4Shapes[0]) == sizeof(kGradShapes) / sizeof(kGradShapes[0]),
              "both forms offer the same number of tile candidates");

TileShape grad_tile(const Geom& g, int choice) {
    return g.vec4 ? TileShape{kGrad4Shapes[choice].tw(), kGrad4Shapes[choice].th(), 0} : kGradShapes[choice];
}

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
template <class T>
static auto grad_fwd4_kernel(int choice) {
    return choice == 0 ? k_grad_fwd4<T, 64, 1>
           : choice == 1 ? k_grad_fwd4<T, 64, 2>
                         : k_grad_fwd4<T, 32, 1>;  // candidates 2 and 3 differ in waves only
}
template <class T>
static auto grad_adj4_kernel(int choice) {
    return choice == 0 ? k_grad_adj4<T, 64, 1>
           : choice == 1 ? k_grad_adj4<T, 64, 2>
                         : k_grad_adj4<T, 32, 1>;
}

void launch_grad_fwd(Ctx& c, Geom& g, int dt, const void* u, const void* wx, const void* wy, void* gx, void* gy,
                     int choice, const RowWeighting* rw) {
    if (choice < 0) choice = g.choice("grad_fwd", dt, 2);
    MMOF_CHECK(choice >= 0 && choice < kGradCandidates, MMOF_ERR_INVALID, "grad tile candidate out of range");
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        // u read, gx and gy written, weights read when given; with rw also nu read and the
        // weighted rows written
        const double per_row = (rw ? 3.0 : 1.0);
        const double bytes = sizeof(T) * ((double)g.n + (per_row + (wx ? 1.0 : 0.0)) * g.gx_len +
                                          (per_row + (wy ? 1.0 : 0.0)) * g.gy_len);
        ScopedTime st(&c, "grad_fwd", bytes, (wx ? 2.0 : 1.0) * g.gx_len + (wy ? 2.0 : 1.0) * g.gy_len);
        const T* nux = rw ? (const T*)rw->nu_a : nullptr;
        const T* nuy = rw ? (const T*)rw->nu_b : nullptr;
        T* mx = rw ? (T*)rw->m_a : nullptr;
        T* my = rw ? (T*)rw->m_b : nullptr;
        const double eps2 = rw ? rw->eps2 : 0.0;
        if (g.vec4 && aligned_to(4 * sizeof(T), {u, wx, wy, gx, gy, nux, nuy, mx, my})) {
            const Grad4Shape sh = kGrad4Shapes[choice];
            const TileList& tl = g.tile_list(c.stream, sh.tw(), sh.th(), false);
            hipLaunchKernelGGL(grad_fwd4_kernel<T>(choice), dim3((unsigned)tl.count), dim3(64 * sh.nw), 0, c.stream,
                               tl.buf.as<Tile>(), g.dframes(), (const T*)u, (const T*)wx, (const T*)wy, (T*)gx,
                               (T*)gy, nux, nuy, mx, my, eps2);
        } else {
            const TileShape sh = kGradShapes[choice];
            const TileList& tl = g.tile_list(c.stream, sh.tw, sh.th, false);
            hipLaunchKernelGGL(grad_fwd_kernel<T>(choice), dim3((unsigned)tl.count), dim3(256), 0, c.stream,
                               tl.buf.as<Tile>(), g.dframes(), (const T*)u, (const T*)wx, (const T*)wy, (T*)gx,
                               (T*)gy, nux, nuy, mx, my, eps2);
        }
        MMOF_LAUNCH_CHECK();
    });
}

void launch_grad_adj(Ctx& c, Geom& g, int dt, const void* gx, const void* gy, const void* wx, const void* wy,
                     void* u, bool accumulate, int choice) {
    if (choice < 0) choice = g.choice("grad_adj", dt, 2);
    MMOF_CHECK(choice >= 0 && choice < kGradCandidates, MMOF_ERR_INVALID, "grad tile candidate out of range");
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        // gx and gy (and weights) read, u written (and read when accumulating)
        const double bytes =
            sizeof(T) * ((accumulate ? 2.0 : 1.0) * g.n + (wx ? 2.0 : 1.0) * g.gx_len + (wy ? 2.0 : 1.0) * g.gy_len);
        ScopedTime st(&c, "grad_adj", bytes, 3.0 * g.n);
        if (g.vec4 && aligned_to(4 * sizeof(T), {u, gy, wy})) {
            const Grad4Shape sh = kGrad4Shapes[choice];
            const TileList& tl = g.tile_list(c.stream, sh.tw(), sh.th(), false);
            hipLaunchKernelGGL(grad_adj4_kernel<T>(choice), dim3((unsigned)tl.count), dim3(64 * sh.nw), 0, c.stream,
                               tl.buf.as<Tile>(), g.dframes(), (const T*)gx, (const T*)gy, (const T*)wx,
                               (const T*)wy, (T*)u, accumulate ? 1 : 0);
        } else {
            const TileShape sh = kGradShapes[choice];
            const TileList& tl = g.tile_list(c.stream, sh.tw, sh.th, false);
            hipLaunchKernelGGL(grad_adj_kernel<T>(choice), dim3((unsigned)tl.count), dim3(256), 0, c.stream,
                               tl.buf.as<Tile>(), g.dframes(), (const T*)gx, (const T*)gy, (const T*)wx,
                               (const T*)wy, (T*)u, accumulate ? 1 : 0);
        }
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
