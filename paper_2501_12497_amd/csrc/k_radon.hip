// Parallel-beam projector H^t (hat model, unit pixels and bins) and its transpose.
//
//   (H u)_{theta,j} = sum_p max(0, 1 - |X_p cos(theta) + Y_p sin(theta) - d_j|) u_p
//
// Forward (ray-driven gather, one lane per detector bin): for |cos| >= |sin| the ray
// crosses every row y once; inside row y the pixels with non-zero weight sit within
// 1/|cos| of xs(y) = cx + (d_j - Y sin)/cos, and their weight is 1 - |cos| |x - xs|.
// Steep angles use the same loop over the columns of a transposed copy of the frame,
// so every lane of a wavefront walks contiguous memory.  Transpose (pixel-driven
// gather, one lane per pixel): each angle contributes (1-f) b[j0] + f b[j0+1] with
// j0 + f = tau_p + (n_d-1)/2.  Sample positions are formed in double; the weights are
// evaluated in the operator's precision.
#include "dev.h"
#include "kernels.h"

namespace mmof {

struct RadonFrame {
    int64_t u_off;     // pixel offset of the frame
    int64_t sino_off;  // offset of its sinogram [n_ang][n_bins]
    int64_t trig_off;  // index of its first angle in the trig table
    int32_t n_ang, n_bins, ny, nx;
};

struct RayTile {
    int32_t frame, angle, bin0, pad;
};

static constexpr int RTW = 64, RTH = 4;  // pixel tiles of the transpose

// Per-frame transpose uT[f][x][y] = u[f][y][x] through a 32x33 LDS tile.
template <class T>
__global__ __launch_bounds__(256) void k_transpose_frames(const Tile* __restrict__ tiles,
                                                          const RadonFrame* __restrict__ rf, const T* __restrict__ u,
                                                          T* __restrict__ ut) {
    __shared__ T s[32][33];
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[tl.frame];
    const int lx = threadIdx.x % 32, ly = threadIdx.x / 32;  // 32 x 8
    for (int r = ly; r < 32; r += 8) {
        const int y = tl.y0 + r, x = tl.x0 + lx;
        if (y < f.ny && x < f.nx) s[r][lx] = u[f.u_off + (int64_t)y * f.nx + x];
    }
    __syncthreads();
    for (int r = ly; r < 32; r += 8) {
        const int x = tl.x0 + r, y = tl.y0 + lx;
        if (y < f.ny && x < f.nx) ut[f.u_off + (int64_t)x * f.ny + y] = s[lx][r];
    }
}

// One workgroup per (frame, angle, 64 bins): lane = bin, the four waves walk disjoint
// quarters of the rows and their partial sums are added in a fixed order.
template <class T>
__global__ __launch_bounds__(256) void k_radon_fwd(const RayTile* __restrict__ rays, int64_t n_rays,
                                                   const RadonFrame* __restrict__ rf, const double2* __restrict__ trig,
                                                   const T* __restrict__ u, const T* __restrict__ ut,
                                                   T* __restrict__ b) {
    __shared__ T part[4][64];
    const int64_t wid = xcd_remap(blockIdx.x, gridDim.x);
    const RayTile rt = rays[wid];
    const RadonFrame f = rf[rt.frame];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = rt.bin0 + lane;
    const double2 cs = trig[f.trig_off + rt.angle];
    const double c = cs.x, s = cs.y;
    const double cx = 0.5 * (f.nx - 1), cy = 0.5 * (f.ny - 1);
    const double dj = (double)j - 0.5 * (f.n_bins - 1);
    // Row walk over (rows, cols) = (ny, nx) of u, or over (nx, ny) of the transpose.
    const bool steep = fabs(s) > fabs(c);
    const double a = steep ? s : c;              // coefficient of the in-row coordinate
    const double bb = steep ? c : s;             // coefficient of the row coordinate
    const int nrow = steep ? f.nx : f.ny, ncol = steep ? f.ny : f.nx;
    const double crow = steep ? cx : cy, ccol = steep ? cy : cx;
    const T* img = (steep ? ut : u) + f.u_off;
    // position of the ray centre in row r: xs(r) = ccol + (dj - (r - crow) bb) / a
    const double xs0 = ccol + (dj + crow * bb) / a;
    const double step = -bb / a;
    const T aa = (T)fabs(a);
    const int q = (nrow + 3) >> 2;
    const int r_lo = wave * q, r_hi = min(nrow, r_lo + q);
    T acc = T(0);
    if (j < f.n_bins) {
        for (int r = r_lo; r < r_hi; ++r) {
            const double xs = fma((double)r, step, xs0);
            const double fl = floor(xs);
            const int xi = (int)fl;
            const T fr = (T)(xs - fl);
            const T* row = img + (int64_t)r * ncol;
#pragma unroll
            for (int k = -1; k <= 2; ++k) {
                const int x = xi + k;
                if (x < 0 || x >= ncol) continue;
                const T w = T(1) - aa * fabs((T)k - fr);
                if (w > T(0)) acc += w * row[x];
            }
        }
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && j < f.n_bins)
        b[f.sino_off + (int64_t)rt.angle * f.n_bins + j] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

template <class T>
__global__ __launch_bounds__(256) void k_radon_adj(const Tile* __restrict__ tiles, const RadonFrame* __restrict__ rf,
                                                   const double2* __restrict__ trig, const T* __restrict__ b,
                                                   T* __restrict__ u) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % RTW);
    const int y = tl.y0 + (int)(threadIdx.x / RTW);
    if (x >= f.nx || y >= f.ny) return;
    const double X = x - 0.5 * (f.nx - 1), Y = y - 0.5 * (f.ny - 1);
    const double cd = 0.5 * (f.n_bins - 1);
    const T* sino = b + f.sino_off;
    T acc = T(0);
    for (int k = 0; k < f.n_ang; ++k) {
        const double2 cs = trig[f.trig_off + k];
        const double pos = fma(X, cs.x, fma(Y, cs.y, cd));
        const double fl = floor(pos);
        const int j0 = (int)fl;
        const T fr = (T)(pos - fl);
        const T* row = sino + (int64_t)k * f.n_bins;
        if (j0 >= 0 && j0 < f.n_bins) acc += (T(1) - fr) * row[j0];
        if (j0 + 1 >= 0 && j0 + 1 < f.n_bins) acc += fr * row[j0 + 1];
    }
    u[f.u_off + (int64_t)y * f.nx + x] = acc;
}

// ----------------------------------------------------------------------------- host side

void radon_plan_init(Ctx& c, Plan& p) {
    Geom& g = *p.geom;
    std::vector<RadonFrame> rfs;
    std::vector<RayTile> rays;
    std::vector<Tile> px, tr;
    int64_t sino = 0, trig = 0;
    for (int64_t fi = 0; fi < g.n_frames; ++fi) {
        const FrameInfo& fr = g.frames[fi];
        RadonFrame r{};
        r.u_off = fr.off;
        r.sino_off = sino;
        r.trig_off = trig;
        r.n_ang = p.n_ang[fr.seq];
        r.n_bins = p.n_bins[fr.seq];
        r.ny = fr.ny;
        r.nx = fr.nx;
        rfs.push_back(r);
        p.sino_off.push_back(sino);
        for (int k = 0; k < r.n_ang; ++k)
            for (int j0 = 0; j0 < r.n_bins; j0 += 64) rays.push_back(RayTile{(int32_t)fi, k, j0, 0});
        for (int y0 = 0; y0 < fr.ny; y0 += RTH)
            for (int x0 = 0; x0 < fr.nx; x0 += RTW) px.push_back(Tile{(int32_t)fi, y0, x0, 0});
        for (int y0 = 0; y0 < fr.ny; y0 += 32)
            for (int x0 = 0; x0 < fr.nx; x0 += 32) tr.push_back(Tile{(int32_t)fi, y0, x0, 0});
        sino += (int64_t)r.n_ang * r.n_bins;
        trig += r.n_ang;
        p.radon_flops += 4.0 * (double)fr.ny * fr.nx * r.n_ang;
    }
    p.m = sino;
    p.d_rinfo.ensure(sizeof(RadonFrame) * rfs.size());
    MMOF_HIP(hipMemcpyAsync(p.d_rinfo.ptr, rfs.data(), sizeof(RadonFrame) * rfs.size(), hipMemcpyHostToDevice, c.stream));
    p.n_rays = (int64_t)rays.size();
    p.d_rays.ensure(sizeof(RayTile) * std::max<size_t>(rays.size(), 1));
    if (!rays.empty())
        MMOF_HIP(hipMemcpyAsync(p.d_rays.ptr, rays.data(), sizeof(RayTile) * rays.size(), hipMemcpyHostToDevice,
                                c.stream));
    p.n_tiles_a = (int64_t)px.size();
    p.d_tiles_a.ensure(sizeof(Tile) * px.size());
    MMOF_HIP(hipMemcpyAsync(p.d_tiles_a.ptr, px.data(), sizeof(Tile) * px.size(), hipMemcpyHostToDevice, c.stream));
    p.n_tiles_b = (int64_t)tr.size();
    p.d_tiles_b.ensure(sizeof(Tile) * tr.size());
    MMOF_HIP(hipMemcpyAsync(p.d_tiles_b.ptr, tr.data(), sizeof(Tile) * tr.size(), hipMemcpyHostToDevice, c.stream));
    MMOF_HIP(hipStreamSynchronize(c.stream));
}

void launch_radon_fwd(Ctx& c, Plan& p, int dt, const void* u, void* b) {
    if (p.n_rays == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        T* ut = static_cast<T*>(c.work("radon_transpose", sizeof(T) * p.n));
        hipLaunchKernelGGL(k_transpose_frames<T>, dim3((unsigned)p.n_tiles_b), dim3(256), 0, c.stream,
                           p.d_tiles_b.as<Tile>(), p.d_rinfo.as<RadonFrame>(), (const T*)u, ut);
        MMOF_LAUNCH_CHECK();
        ScopedTime st(&c, "radon_fwd", (double)sizeof(T) * (p.n + p.m), p.radon_flops);
        hipLaunchKernelGGL(k_radon_fwd<T>, dim3((unsigned)p.n_rays), dim3(256), 0, c.stream,
                           p.d_rays.as<RayTile>(), p.n_rays, p.d_rinfo.as<RadonFrame>(), p.d_trig.as<double2>(),
                           (const T*)u, (const T*)ut, (T*)b);
        MMOF_LAUNCH_CHECK();
    });
}

void launch_radon_adj(Ctx& c, Plan& p, int dt, const void* b, void* u) {
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "radon_adj", (double)sizeof(T) * (p.n + p.m), p.radon_flops);
        hipLaunchKernelGGL(k_radon_adj<T>, dim3((unsigned)p.n_tiles_a), dim3(256), 0, c.stream,
                           p.d_tiles_a.as<Tile>(), p.d_rinfo.as<RadonFrame>(), p.d_trig.as<double2>(), (const T*)b,
                           (T*)u);
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
