// Optical-flow subproblem kernels: App. C image derivatives, Horn-Schunck block-Jacobi
// sweeps for the p = q = 2 flow energy (eq. of_reg), the reverse-flow estimate of the
// Remark in Sec. 3, and the MM weights of Sec. 4.1.1.
#include "dev.h"
#include "kernels.h"

namespace mmof {

static constexpr int OTW = 64, OTH = 4;

// I [pair][3][ny][nx] = (I_x, I_y, I_t) with box radius dr and mirrored borders.
template <class T>
__global__ __launch_bounds__(256) void k_of_derivs(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                   const T* __restrict__ u, T* __restrict__ I, int dr) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % OTW);
    const int y = tl.y0 + (int)(threadIdx.x / OTW);
    if (x >= f.nx || y >= f.ny) return;
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const T* a = u + f.off;   // frame t
    const T* b = a + np;      // frame t+1
    T Ix = T(0), Iy = T(0), It = T(0);
    const int xp = mirror(x + dr, nx), xm = mirror(x - dr, nx);
    const int yp = mirror(y + dr, ny), ym = mirror(y - dr, ny);
    for (int j = -dr; j <= dr; ++j) {
        const int yj = mirror(y + j, ny), xj = mirror(x + j, nx);
        Ix += a[(int64_t)yj * nx + xp] - a[(int64_t)yj * nx + xm];
        Iy += a[(int64_t)yp * nx + xj] - a[(int64_t)ym * nx + xj];
        for (int k = -dr; k <= dr; ++k) {
            const int64_t o = (int64_t)yj * nx + mirror(x + k, nx);
            It += b[o] - a[o];
        }
    }
    const T box = T(2 * dr + 1);
    const int64_t p = (int64_t)y * nx + x;
    T* Ip = I + 3 * f.pair_off;
    Ip[p] = Ix / (box * T(2 * dr));
    Ip[np + p] = Iy / (box * T(2 * dr));
    Ip[2 * np + p] = It / (box * box);
}

// One exact 2x2 block-Jacobi sweep: sbar = mean of in-image 4-neighbours,
// s = sbar - g (g.sbar + I_t) / (gamma d + |g|^2).
template <class T>
__global__ __launch_bounds__(256) void k_hs_sweep(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                  const T* __restrict__ I, const T* __restrict__ vin,
                                                  T* __restrict__ vout, T gamma) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % OTW);
    const int y = tl.y0 + (int)(threadIdx.x / OTW);
    if (x >= f.nx || y >= f.ny) return;
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const int64_t p = (int64_t)y * nx + x;
    const T* sx = vin + 2 * f.pair_off;
    const T* sy = sx + np;
    T ax = T(0), ay = T(0);
    int d = 0;
    // neighbour order: y-1, y+1, x-1, x+1
    if (y > 0) { ax += sx[p - nx]; ay += sy[p - nx]; ++d; }
    if (y < ny - 1) { ax += sx[p + nx]; ay += sy[p + nx]; ++d; }
    if (x > 0) { ax += sx[p - 1]; ay += sy[p - 1]; ++d; }
    if (x < nx - 1) { ax += sx[p + 1]; ay += sy[p + 1]; ++d; }
    const T dd = T(d);
    ax /= dd;
    ay /= dd;
    const T* Ip = I + 3 * f.pair_off;
    const T gx = Ip[p], gy = Ip[np + p], gt = Ip[2 * np + p];
    const T k = (gx * ax + gy * ay + gt) / (gamma * dd + gx * gx + gy * gy);
    T* o = vout + 2 * f.pair_off;
    o[p] = ax - gx * k;
    o[np + p] = ay - gy * k;
}

// Reverse flow: target q gathers, in raster order of the sources p, every p with
// rint(p + v(p)) == q; the result is minus the mean of their velocities (0 if none).
template <class T>
__global__ __launch_bounds__(256) void k_reverse_flow(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                      const T* __restrict__ v, T* __restrict__ vr,
                                                      const int32_t* __restrict__ d_radius) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int qx = tl.x0 + (int)(threadIdx.x % OTW);
    const int qy = tl.y0 + (int)(threadIdx.x / OTW);
    if (qx >= f.nx || qy >= f.ny) return;
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const T* vx = v + 2 * f.pair_off;
    const T* vy = vx + np;
    const int R = *d_radius;
    T ax = T(0), ay = T(0);
    int cnt = 0;
    const int py_lo = max(qy - R, 0), py_hi = min(qy + R, ny - 1);
    const int px_lo = max(qx - R, 0), px_hi = min(qx + R, nx - 1);
    for (int py = py_lo; py <= py_hi; ++py)
        for (int px = px_lo; px <= px_hi; ++px) {
            const int64_t p = (int64_t)py * nx + px;
            const T a = vx[p], b = vy[p];
            if (!(fabs(a) < T(1048576)) || !(fabs(b) < T(1048576))) continue;
            if (rint_shift(px, a) != qx || rint_shift(py, b) != qy) continue;
            ax -= a;
            ay -= b;
            ++cnt;
        }
    const int64_t q = (int64_t)qy * nx + qx;
    T* o = vr + 2 * f.pair_off;
    o[q] = cnt ? ax / T(cnt) : T(0);
    o[np + q] = cnt ? ay / T(cnt) : T(0);
}

template <class T>
__global__ void k_mm_weights(int64_t n, const T* __restrict__ nu, T eps2, T* __restrict__ w2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T a = nu[i];
        w2[i] = T(1) / sqrt(a * a + eps2);
    }
}

void launch_of_derivs(Ctx& c, Geom& g, int dt, const void* u, void* I, int dr) {
    if (g.n_pairs == 0) return;
    const TileList& tl = g.tile_list(c.stream, OTW, OTH, true);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "of_derivs");
        hipLaunchKernelGGL(k_of_derivs<T>, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(),
                           g.dframes(), (const T*)u, (T*)I, dr);
        MMOF_LAUNCH_CHECK();
    });
}

void launch_hs_sweep(Ctx& c, Geom& g, int dt, const void* I, const void* vin, void* vout, double gamma) {
    if (g.n_pairs == 0) return;
    const TileList& tl = g.tile_list(c.stream, OTW, OTH, true);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "hs_sweep");
        hipLaunchKernelGGL(k_hs_sweep<T>, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(),
                           g.dframes(), (const T*)I, (const T*)vin, (T*)vout, (T)gamma);
        MMOF_LAUNCH_CHECK();
    });
}

void launch_reverse_flow(Ctx& c, Geom& g, int dt, const void* v, void* vr, const int32_t* d_radius) {
    if (g.n_pairs == 0) return;
    int32_t* rad = const_cast<int32_t*>(d_radius);
    if (!rad) {
        rad = static_cast<int32_t*>(c.work("rev_radius", 256));
        launch_flow_radius(c, g, dt, v, rad);
    }
    const TileList& tl = g.tile_list(c.stream, OTW, OTH, true);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "reverse_flow");
        hipLaunchKernelGGL(k_reverse_flow<T>, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(),
                           g.dframes(), (const T*)v, (T*)vr, rad);
        MMOF_LAUNCH_CHECK();
    });
}

void launch_mm_weights(Ctx& c, int dt, int64_t n, const void* nu, double eps, void* w2) {
    if (n == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        hipLaunchKernelGGL(k_mm_weights<T>, grid_for(n, 256), dim3(256), 0, c.stream, n, (const T*)nu,
                           (T)(eps * eps), (T*)w2);
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
