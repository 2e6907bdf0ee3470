// Spatio-temporal regulariser pieces of the MMGKS method family (Sec. 5, table of methods):
// the temporal first difference L_t (the mode-3 product U x_3 L_t) and its adjoint, and the
// MM weights of the grouped norms -- IsoTV's per-pixel pairs of spatial differences and GS's
// per-location spatial differences over all frames of a sequence (the l2,1 norm of L_s U).
//
// Every kernel runs over all frames of a ragged stack in one launch: grid.y = frame index
// (the FrameInfo table gives the frame's offsets), grid.x strides over the frame's pixels.
// All are bandwidth kernels (a few flops per element).
#include "dev.h"
#include "kernels.h"

namespace mmof {

static constexpr int RB = 256;   // threads per workgroup
static constexpr int RPT = 4;    // elements per thread per step

// r[pair_off + p] = u[off + ny nx + p] - u[off + p] for the frames that begin a pair.
template <class TX>
__global__ __launch_bounds__(RB) void k_tdiff_fwd(const FrameInfo* __restrict__ frames, const TX* __restrict__ u,
                                                  TX* __restrict__ r) {
    const FrameInfo f = frames[blockIdx.y];
    if (f.t + 1 >= f.n_t) return;
    const int64_t np = (int64_t)f.ny * f.nx;
    const TX* __restrict__ a = u + f.off;
    TX* __restrict__ out = r + f.pair_off;
    for (int64_t p0 = ((int64_t)blockIdx.x * RB + threadIdx.x) * RPT; p0 < np; p0 += (int64_t)gridDim.x * RB * RPT) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t p = p0 + q;
            if (p < np) out[p] = a[np + p] - a[p];
        }
    }
}

// u[off + p] (+)= r_{t-1}[p] (t >= 1) - r_t[p] (t < n_t - 1): the transpose, a gather.
template <class TX>
__global__ __launch_bounds__(RB) void k_tdiff_adj(const FrameInfo* __restrict__ frames, const TX* __restrict__ r,
                                                  TX* __restrict__ u, int accumulate) {
    const int fi = blockIdx.y;
    const FrameInfo f = frames[fi];
    const int64_t np = (int64_t)f.ny * f.nx;
    const TX* __restrict__ prev = f.t >= 1 ? r + frames[fi - 1].pair_off : nullptr;
    const TX* __restrict__ cur = f.t + 1 < f.n_t ? r + f.pair_off : nullptr;
    TX* __restrict__ out = u + f.off;
    for (int64_t p0 = ((int64_t)blockIdx.x * RB + threadIdx.x) * RPT; p0 < np; p0 += (int64_t)gridDim.x * RB * RPT) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int64_t p = p0 + q;
            if (p < np) {
                TX v = TX(0);
                if (prev) v += prev[p];
                if (cur) v -= cur[p];
                out[p] = accumulate ? out[p] + v : v;
            }
        }
    }
}

// IsoTV: the group of pixel (y, x) of a frame holds its horizontal difference (x < nx - 1,
// row of gx) and its vertical one (y < ny - 1, row of gy); both rows get
// w = 1 / sqrt(gx^2 + gy^2 + eps^2) (a missing member counts 0).
template <class TX>
__global__ __launch_bounds__(RB) void k_group_weights_iso(const FrameInfo* __restrict__ frames,
                                                          const TX* __restrict__ nu_gx, const TX* __restrict__ nu_gy,
                                                          double eps2, double* __restrict__ w_gx,
                                                          double* __restrict__ w_gy) {
    const FrameInfo f = frames[blockIdx.y];
    const int64_t np = (int64_t)f.ny * f.nx;
    for (int64_t p = (int64_t)blockIdx.x * RB + threadIdx.x; p < np; p += (int64_t)gridDim.x * RB) {
        const int y = (int)(p / f.nx), x = (int)(p - (int64_t)y * f.nx);
        const bool hx = x + 1 < f.nx, hy = y + 1 < f.ny;
        const int64_t ix = f.gx_off + (int64_t)y * (f.nx - 1) + x;
        const int64_t iy = f.gy_off + (int64_t)y * f.nx + x;
        double s = 0.0;
        if (hx) {
            const double a = (double)nu_gx[ix];
            s += a * a;
        }
        if (hy) {
            const double b = (double)nu_gy[iy];
            s += b * b;
        }
        const double w = 1.0 / sqrt(s + eps2);
        if (hx) w_gx[ix] = w;
        if (hy) w_gy[iy] = w;
    }
}

// GS: the group of a difference location of a sequence holds that difference in every frame
// of the sequence; every member gets w = 1 / sqrt(sum_t g_t^2 + eps^2).  Workgroups of the
// sequence's first frame do the work (the frames of a sequence are consecutive in the table);
// locations are the ny (nx - 1) horizontal ones, then the (ny - 1) nx vertical ones.
template <class TX>
__global__ __launch_bounds__(RB) void k_group_weights_gs(const FrameInfo* __restrict__ frames,
                                                         const TX* __restrict__ nu_gx, const TX* __restrict__ nu_gy,
                                                         double eps2, double* __restrict__ w_gx,
                                                         double* __restrict__ w_gy) {
    const int fi = blockIdx.y;
    const FrameInfo f = frames[fi];
    if (f.t != 0) return;
    const int64_t nlx = (int64_t)f.ny * (f.nx - 1), nly = (int64_t)(f.ny - 1) * f.nx;
    for (int64_t l = (int64_t)blockIdx.x * RB + threadIdx.x; l < nlx + nly; l += (int64_t)gridDim.x * RB) {
        const bool isx = l < nlx;
        const int64_t li = isx ? l : l - nlx;
        const TX* __restrict__ src = isx ? nu_gx : nu_gy;
        double* __restrict__ dst = isx ? w_gx : w_gy;
        double s = 0.0;
        for (int t = 0; t < f.n_t; ++t) {
            const FrameInfo& ft = frames[fi + t];
            const double a = (double)src[(isx ? ft.gx_off : ft.gy_off) + li];
            s += a * a;
        }
        const double w = 1.0 / sqrt(s + eps2);
        for (int t = 0; t < f.n_t; ++t) {
            const FrameInfo& ft = frames[fi + t];
            dst[(isx ? ft.gx_off : ft.gy_off) + li] = w;
        }
    }
}

static dim3 frame_grid(const Geom& g, int per_block) {
    const int64_t max_np = (int64_t)g.max_ny * g.max_nx;
    const int64_t bx = std::max<int64_t>(1, std::min<int64_t>(cdiv(max_np, per_block), 4096));
    return dim3((unsigned)bx, (unsigned)g.n_frames);
}

void launch_tdiff(Ctx& c, Geom& g, int dt, bool transpose, const void* in, void* out, bool accumulate) {
    MMOF_CHECK(g.n_frames <= 65535, MMOF_ERR_SHAPE, "too many frames for one launch (at most 65535)");
    const dim3 grid = frame_grid(g, RB * RPT);
    // one read and one write per pair pixel (forward) or per frame pixel (transpose, which
    // reads up to two residuals and, when accumulating, the output)
    const double bytes = transpose ? (double)(2 * g.pair_px + (accumulate ? 2 : 1) * g.n) : 3.0 * (double)g.pair_px;
    const size_t es = dt == MMOF_F32 ? 4 : 8;
    ScopedTime st(&c, transpose ? "tdiff_adj" : "tdiff_fwd", bytes * es, (double)g.pair_px * (transpose ? 2 : 1));
    dispatch(dt, [&](auto z) {
        using TX = decltype(z);
        if (transpose)
            hipLaunchKernelGGL(k_tdiff_adj<TX>, grid, dim3(RB), 0, c.stream, g.dframes(), (const TX*)in, (TX*)out,
                               accumulate ? 1 : 0);
        else
            hipLaunchKernelGGL(k_tdiff_fwd<TX>, grid, dim3(RB), 0, c.stream, g.dframes(), (const TX*)in, (TX*)out);
    });
    MMOF_LAUNCH_CHECK();
}

void launch_group_weights(Ctx& c, Geom& g, int dt, int reg, const void* nu, double eps, double* w2) {
    MMOF_CHECK(reg == MMOF_REG_ISO || reg == MMOF_REG_GS, MMOF_ERR_INVALID, "group weights need IsoTV or GS");
    MMOF_CHECK(g.n_frames <= 65535, MMOF_ERR_SHAPE, "too many frames for one launch (at most 65535)");
    const dim3 grid = frame_grid(g, RB);
    const size_t es = dt == MMOF_F32 ? 4 : 8;
    ScopedTime st(&c, "group_weights", (double)(g.gx_len + g.gy_len) * (es + 8.0), 3.0 * (g.gx_len + g.gy_len));
    dispatch(dt, [&](auto z) {
        using TX = decltype(z);
        const TX* ngx = static_cast<const TX*>(nu);
        const TX* ngy = ngx + g.gx_len;
        if (reg == MMOF_REG_ISO)
            hipLaunchKernelGGL(k_group_weights_iso<TX>, grid, dim3(RB), 0, c.stream, g.dframes(), ngx, ngy, eps * eps,
                               w2, w2 + g.gx_len);
        else
            hipLaunchKernelGGL(k_group_weights_gs<TX>, grid, dim3(RB), 0, c.stream, g.dframes(), ngx, ngy, eps * eps,
                               w2, w2 + g.gx_len);
    });
    MMOF_LAUNCH_CHECK();
}

}  // namespace mmof
