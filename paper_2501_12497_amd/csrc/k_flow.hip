// The optical-flow temporal operator L(v) of the image subproblem, in warp form:
//   direction +1:  r_t = W(v_t) u_{t+1} - u_t      (-M-bar(s), Sec. 3)
//   direction -1:  r_t = W(v_t) u_t - u_{t+1}      (-M-bar'(s'))
// W(v) pulls a bilinear (or nearest, ties to even) sample at p + v(p) with clipped
// coordinates.  The adjoint scatters through the bilinear weights; here it is a
// deterministic gather: every output pixel sums, in a fixed order (per corner of the sample
// cell, sources in raster order), the sources whose sample cell has it as a corner.
// Sources are staged in LDS per output tile and bucketed by cell, so a pixel only visits
// the sources that reach it.
#include <climits>
#include <type_traits>

#include "dev.h"
#include "kernels.h"

namespace mmof {

static constexpr int FTW = 64, FTH = 4;          // dv tiles
static constexpr int RMAX = 8;                   // LDS path of the adjoint handles radius <= RMAX

// Bilinear (INTERP 0) or nearest (INTERP 1) sample of src at (x + vx, y + vy), computed in T
// (source values of type S are rounded to T first).
template <class T, int INTERP, class S = T>
__device__ __forceinline__ T warp_sample(const S* __restrict__ src, int nx, int ny, int x, int y, T vx, T vy) {
    if (INTERP == 1) {
        const int xr = round_clip(x, vx, nx), yr = round_clip(y, vy, ny);
        return (T)src[(int64_t)yr * nx + xr];
    }
    int x0, y0;
    T fx, fy;
    bool cx, cy;
    clip_cell(x, vx, nx, x0, fx, cx);
    clip_cell(y, vy, ny, y0, fy, cy);
    const int y1 = min(y0 + 1, ny - 1);
    const S* r0 = src + (int64_t)y0 * nx;
    const S* r1 = src + (int64_t)y1 * nx;
    // the two pixels of a row as one 2-element load at xa = min(x0, nx - 2) (nx >= 2); a cell
    // clipped to the last column (x0 = nx - 1, fx = 0) takes its value from the second one
    const int xa = min(x0, nx - 2);
    const Pair<S> p0 = ld2(r0 + xa), p1 = ld2(r1 + xa);
    const bool edge = xa != x0;
    const T a0 = (T)(edge ? p0.b : p0.a), a1 = (T)p0.b, b0 = (T)(edge ? p1.b : p1.a), b1 = (T)p1.b;
    return (T(1) - fx) * (T(1) - fy) * a0 + fx * (T(1) - fy) * a1 + (T(1) - fx) * fy * b0 + fx * fy * b1;
}

// A sample position prepared once and used for many source images of the same frame
// geometry: the offsets of the two pixel pairs read (or of the nearest pixel for INTERP 1),
// the edge flag and the fractions, as warp_sample forms them.
template <class T>
struct SampleCell {
    int o0, o1;    // row * nx + xa of the rows y0 and y1 (INTERP 1: the pixel's offset in o0)
    T fx, fy;
    bool edge;
};

template <class T, int INTERP>
__device__ __forceinline__ SampleCell<T> sample_cell(int nx, int ny, int x, int y, T vx, T vy) {
    SampleCell<T> c;
    if (INTERP == 1) {
        c.o0 = round_clip(y, vy, ny) * nx + round_clip(x, vx, nx);
        c.o1 = c.o0;
        c.fx = c.fy = T(0);
        c.edge = false;
        return c;
    }
    int x0, y0;
    bool cx, cy;
    clip_cell(x, vx, nx, x0, c.fx, cx);
    clip_cell(y, vy, ny, y0, c.fy, cy);
    const int y1 = min(y0 + 1, ny - 1);
    const int xa = min(x0, nx - 2);
    c.o0 = y0 * nx + xa;
    c.o1 = y1 * nx + xa;
    c.edge = xa != x0;
    return c;
}

// warp_sample(src, ...) for a prepared cell (the same arithmetic, so the same value).
template <class T, int INTERP, class S>
__device__ __forceinline__ T sample_at(const S* __restrict__ src, const SampleCell<T>& c) {
    if (INTERP == 1) return (T)src[c.o0];
    const Pair<S> p0 = ld2(src + c.o0), p1 = ld2(src + c.o1);
    const T a0 = (T)(c.edge ? p0.b : p0.a), a1 = (T)p0.b, b0 = (T)(c.edge ? p1.b : p1.a), b1 = (T)p1.b;
    const T fx = c.fx, fy = c.fy;
    return (T(1) - fx) * (T(1) - fy) * a0 + fx * (T(1) - fy) * a1 + (T(1) - fx) * fy * b0 + fx * fy * b1;
}

template <class T, int INTERP, int FTW, int FTH>
__global__ __launch_bounds__(256) void k_flow_fwd(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                  const T* __restrict__ u, const T* __restrict__ v,
                                                  T* __restrict__ r, int direction, const T* __restrict__ nuw,
                                                  T* __restrict__ mw, double eps2) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % FTW);
    const int y = tl.y0 + (int)(threadIdx.x / FTW);
    if (x >= f.nx || y >= f.ny) return;
    const int64_t np = (int64_t)f.nx * f.ny;
    const int64_t p = (int64_t)y * f.nx + x;
    const T* ut = u + f.off;
    const T* ut1 = ut + np;
    const T* vx = v + 2 * f.pair_off;
    const T vxx = vx[p], vyy = vx[np + p];
    const T* src = direction > 0 ? ut1 : ut;
    const T* sub = direction > 0 ? ut : ut1;
    const T val = warp_sample<T, INTERP>(src, f.nx, f.ny, x, y, vxx, vyy) - sub[p];
    r[f.pair_off + p] = val;
    if (mw) mw[f.pair_off + p] = mm_weighted(val, nuw[f.pair_off + p], eps2);
}

// Forward and (when vr is not null) reverse flow rows of Theta for K columns at once:
// column j of U (S: FP64, or already T; leading dimension ldu) is rounded to T and mapped to
// out[j*ldo + oF + pair pixel] (forward) and out[j*ldo + oR + pair pixel] (reverse).  The
// values equal those of k_flow_fwd applied to the rounded column.
template <class T, class S, int INTERP, int FTW, int FTH>
__global__ __launch_bounds__(256) void k_flow_fwd_cols(const Tile* __restrict__ tiles,
                                                       const FrameInfo* __restrict__ fr,
                                                       const S* __restrict__ U, int64_t ldu,
                                                       const T* __restrict__ v, const T* __restrict__ vr,
                                                       T* __restrict__ out, int64_t ldo, int64_t oF, int64_t oR) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % FTW);
    const int y = tl.y0 + (int)(threadIdx.x / FTW);
    if (x >= f.nx || y >= f.ny) return;
    const int64_t np = (int64_t)f.nx * f.ny;
    const int64_t p = (int64_t)y * f.nx + x;
    const S* ut = U + (int64_t)blockIdx.y * ldu + f.off;
    const S* ut1 = ut + np;
    T* o = out + (int64_t)blockIdx.y * ldo;
    const T* vf = v + 2 * f.pair_off;
    o[oF + f.pair_off + p] = warp_sample<T, INTERP, S>(ut1, f.nx, f.ny, x, y, vf[p], vf[np + p]) - (T)ut[p];
    if (vr) {
        const T* vb = vr + 2 * f.pair_off;
        o[oR + f.pair_off + p] = warp_sample<T, INTERP, S>(ut, f.nx, f.ny, x, y, vb[p], vb[np + p]) - (T)ut1[p];
    }
}

// Vector forms of the two kernels above: each thread owns 4 consecutive pixels of one row of
// a (4*LW)-pixel-wide tile, so flows, the subtracted frame and the output move as 4-element
// vectors (16 bytes per FP32 access, from element-aligned addresses: frames of any width and
// offset); a row whose width is not a multiple of 4 ends with a thread of 1..3 pixels, whose
// accesses go element by element.  The bilinear samples stay single loads.  Values equal those
// of the scalar kernels.
// mw (may be null; the scalar kernel too): the rows weighted by the MM weights of nuw
// (RowWeighting).
template <class T, int INTERP, int LW>
__global__ __launch_bounds__(256) void k_flow_fwd4(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                   const T* __restrict__ u, const T* __restrict__ v,
                                                   T* __restrict__ r, int direction, const T* __restrict__ nuw,
                                                   T* __restrict__ mw, double eps2) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + 4 * (int)(threadIdx.x % LW);
    const int y = tl.y0 + (int)(threadIdx.x / LW);
    if (x >= f.nx || y >= f.ny) return;
    const int64_t np = (int64_t)f.nx * f.ny;
    const int64_t p = (int64_t)y * f.nx + x;
    const T* ut = u + f.off;
    const T* ut1 = ut + np;
    const int nv = min(4, f.nx - x);   // (fewer than 4 at the end of a row whose width is not a multiple of 4)
    const T* vf = v + 2 * f.pair_off;
    const Quad<T> vx = ld4n(vf + p, nv), vy = ld4n(vf + np + p, nv);
    const T* src = direction > 0 ? ut1 : ut;
    const Quad<T> sub = ld4n((direction > 0 ? ut : ut1) + p, nv);
    Quad<T> o;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        o.v[j] = warp_sample<T, INTERP>(src, f.nx, f.ny, x + j, y, vx.v[j], vy.v[j]) - sub.v[j];
    st4n(r + f.pair_off + p, o, nv);
    if (mw) {
        const Quad<T> nq = ld4n(nuw + f.pair_off + p, nv);
        Quad<T> m;
#pragma unroll
        for (int j = 0; j < 4; ++j) m.v[j] = mm_weighted(o.v[j], nq.v[j], eps2);
        st4n(mw + f.pair_off + p, m, nv);
    }
}

template <class T, class S, int INTERP, int LW>
__global__ __launch_bounds__(256) void k_flow_fwd_cols4(const Tile* __restrict__ tiles,
                                                        const FrameInfo* __restrict__ fr,
                                                        const S* __restrict__ U, int64_t ldu,
                                                        const T* __restrict__ v, const T* __restrict__ vr,
                                                        T* __restrict__ out, int64_t ldo, int64_t oF, int64_t oR) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + 4 * (int)(threadIdx.x % LW);
    const int y = tl.y0 + (int)(threadIdx.x / LW);
    if (x >= f.nx || y >= f.ny) return;
    const int64_t np = (int64_t)f.nx * f.ny;
    const int64_t p = (int64_t)y * f.nx + x;
    const S* ut = U + (int64_t)blockIdx.y * ldu + f.off;
    const S* ut1 = ut + np;
    T* o = out + (int64_t)blockIdx.y * ldo;
    const int nv = min(4, f.nx - x);
    const Quad<S> a = ld4n(ut + p, nv), b = ld4n(ut1 + p, nv);
    {
        const T* vf = v + 2 * f.pair_off;
        const Quad<T> vx = ld4n(vf + p, nv), vy = ld4n(vf + np + p, nv);
        Quad<T> q;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            q.v[j] = warp_sample<T, INTERP, S>(ut1, f.nx, f.ny, x + j, y, vx.v[j], vy.v[j]) - (T)a.v[j];
        st4n(o + oF + f.pair_off + p, q, nv);
    }
    if (vr) {
        const T* vb = vr + 2 * f.pair_off;
        const Quad<T> vx = ld4n(vb + p, nv), vy = ld4n(vb + np + p, nv);
        Quad<T> q;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            q.v[j] = warp_sample<T, INTERP, S>(ut, f.nx, f.ny, x + j, y, vx.v[j], vy.v[j]) - (T)b.v[j];
        st4n(o + oR + f.pair_off + p, q, nv);
    }
}

// k_flow_fwd_cols4 with the sample cells of a lane's four pixels (both directions) formed
// once from the flows and reused for JC consecutive columns (grid.y = column groups): the
// flows are read once per JC columns instead of once per column.
template <class T, class S, int INTERP, int LW, int JC>
__global__ __launch_bounds__(256) void k_flow_fwd_colsJ(const Tile* __restrict__ tiles,
                                                        const FrameInfo* __restrict__ fr,
                                                        const S* __restrict__ U, int64_t ldu, int K,
                                                        const T* __restrict__ v, const T* __restrict__ vr,
                                                        T* __restrict__ out, int64_t ldo, int64_t oF, int64_t oR) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + 4 * (int)(threadIdx.x % LW);
    const int y = tl.y0 + (int)(threadIdx.x / LW);
    if (x >= f.nx || y >= f.ny) return;
    const int64_t np = (int64_t)f.nx * f.ny;
    const int64_t p = (int64_t)y * f.nx + x;
    const int nv = min(4, f.nx - x);
    SampleCell<T> cf[4], cr[4];
    {
        const T* vf = v + 2 * f.pair_off;
        const Quad<T> vx = ld4n(vf + p, nv), vy = ld4n(vf + np + p, nv);
#pragma unroll
        for (int j = 0; j < 4; ++j) cf[j] = sample_cell<T, INTERP>(f.nx, f.ny, x + j, y, vx.v[j], vy.v[j]);
    }
    if (vr) {
        const T* vb = vr + 2 * f.pair_off;
        const Quad<T> vx = ld4n(vb + p, nv), vy = ld4n(vb + np + p, nv);
#pragma unroll
        for (int j = 0; j < 4; ++j) cr[j] = sample_cell<T, INTERP>(f.nx, f.ny, x + j, y, vx.v[j], vy.v[j]);
    }
    const int c0 = blockIdx.y * JC;
    for (int jj = 0; jj < JC; ++jj) {
        const int col = c0 + jj;
        if (col >= K) break;
        const S* ut = U + (int64_t)col * ldu + f.off;
        const S* ut1 = ut + np;
        T* o = out + (int64_t)col * ldo;
        const Quad<S> a = ld4n(ut + p, nv), b = ld4n(ut1 + p, nv);
        Quad<T> q;
#pragma unroll
        for (int j = 0; j < 4; ++j) q.v[j] = sample_at<T, INTERP, S>(ut1, cf[j]) - (T)a.v[j];
        st4n(o + oF + f.pair_off + p, q, nv);
        if (vr) {
#pragma unroll
            for (int j = 0; j < 4; ++j) q.v[j] = sample_at<T, INTERP, S>(ut, cr[j]) - (T)b.v[j];
            st4n(o + oR + f.pair_off + p, q, nv);
        }
    }
}

// Cell of a source pixel: clipped floor coordinates and fractions (0 for INTERP 1).
template <class T, int INTERP>
__device__ __forceinline__ void source_cell(int sx, int sy, T vx, T vy, int nx, int ny, int& x0, int& y0, T& fx,
                                            T& fy) {
    if (INTERP == 1) {
        x0 = round_clip(sx, vx, nx);
        y0 = round_clip(sy, vy, ny);
        fx = T(0);
        fy = T(0);
    } else {
        bool c;
        clip_cell(sx, vx, nx, x0, fx, c);
        clip_cell(sy, vy, ny, y0, fy, c);
    }
}

// Adjoint over an ATX x ATY output tile per workgroup of 256 threads; each thread owns
// RPT = ATX * ATY / 256 consecutive rows of one column.  The sources within the radius of
// the tile are loaded together and dropped into the (ATX+1) x (ATY+1) cells whose corners
// touch the tile: each cell has ADJ_SLOTS slots in LDS (cell fractions, value and the
// source's raster rank in the window), taken in arrival order through an LDS counter.  An
// output is a corner of exactly four cells; for each it sums the cell's sources in raster
// order (the few slots ordered by rank in registers) and adds the four partial sums in a
// fixed corner order, so its value does not depend on the tile shape or on the arrival
// order.  A tile where some cell receives more sources than it has slots (a strongly
// converging flow) forms the same sums by the wide-window path below.
constexpr int ADJ_SLOTS = 4;

template <class T, int INTERP, int ATX, int ATY>
__global__ __launch_bounds__(256) void k_flow_adj(const AdjTile* __restrict__ tiles, const T* __restrict__ r,
                                                  const T* __restrict__ v, T* __restrict__ u, int direction,
                                                  int accumulate, const int32_t* __restrict__ d_radius,
                                                  const T* __restrict__ cx, const double* __restrict__ clam,
                                                  double* __restrict__ cout) {
    constexpr int RPT = ATX * ATY / 256;
    constexpr int SMAX = (ATX + 2 * RMAX) * (ATY + 2 * RMAX);  // source window (raster rank < 2^16)
    constexpr int CW = ATX + 1, NC = (ATX + 1) * (ATY + 1);     // cells touching the tile
    static_assert(SMAX <= 65536, "source ranks are kept in 16 bits");
    __shared__ T s_fx[NC * ADJ_SLOTS], s_fy[NC * ADJ_SLOTS], s_val[NC * ADJ_SLOTS];
    __shared__ unsigned short s_rank[NC * ADJ_SLOTS];
    __shared__ int s_cnt[NC];
    __shared__ int s_over;

    const AdjTile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const int R = *d_radius;  // (independent of the tile: both loads are in flight together)
    const int nx = tl.nx, ny = tl.ny;
    const int64_t np = (int64_t)nx * ny;
    const int qx = tl.x0 + (int)(threadIdx.x % ATX);
    const int qy0 = tl.y0 + (int)(threadIdx.x / ATX) * RPT;
    const bool col_in = qx < nx;

    // direct terms and the pair whose warp gathers into this frame
    const int64_t dp = direction > 0 ? tl.po : tl.pp;  // pair offset of the direct term (-1: none)
    const int64_t gp = direction > 0 ? tl.pp : tl.po;  // pair offset of the gathering pair (-1: none)
    T acc[RPT], direct[RPT], old[RPT];
    // the direct terms and old outputs are loaded first, with the sources (their latency
    // then overlaps the staging instead of following it)
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        acc[k] = direct[k] = old[k] = T(0);
        const int qy = qy0 + k;
        if (col_in && qy < ny) {
            const int64_t q = (int64_t)qy * nx + qx;
            if (dp >= 0) direct[k] = -r[dp + q];
            if (accumulate) old[k] = u[tl.off + q];
        }
    }

    if (gp >= 0) {
        const T* rg = r + gp;
        const T* vxg = v + 2 * gp;
        const T* vyg = vxg + np;
        bool wide = R > RMAX;
        if (!wide) {
            const int sx0 = max(tl.x0 - R, 0), sx1 = min(tl.x0 + ATX - 1 + R, nx - 1);
            const int sy0 = max(tl.y0 - R, 0), sy1 = min(tl.y0 + ATY - 1 + R, ny - 1);
            const int sw = sx1 - sx0 + 1, sh = sy1 - sy0 + 1;
            for (int i = threadIdx.x; i < NC; i += 256) s_cnt[i] = 0;
            if (threadIdx.x == 0) s_over = 0;
            // Staging: a thread first loads all of its sources (independent loads, in flight
            // together), then forms their cells.  Source i of the window (its raster index,
            // pitch sw, which is also its rank) is taken by thread i mod 256; the row is
            // i / sw from an FP32 product (exact: i < 2^16 and the quotient's fraction is
            // at least 1/(2 sw) away from an integer).
            constexpr int NI = (SMAX + 255) / 256;
            const int nsrc = sw * sh;
            const float inv_sw = 1.0f / (float)sw;
            T lvx[NI], lvy[NI], lr[NI];
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int i = (int)threadIdx.x + 256 * k;
                lvx[k] = lvy[k] = lr[k] = T(0);
                if (i < nsrc) {
                    const int ly = (int)(((float)i + 0.5f) * inv_sw), lx = i - ly * sw;
                    const int64_t p = (int64_t)(sy0 + ly) * nx + sx0 + lx;
                    lvx[k] = vxg[p];
                    lvy[k] = vyg[p];
                    lr[k] = rg[p];
                }
            }
            __syncthreads();  // counts cleared
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int i = (int)threadIdx.x + 256 * k;
                if (i < nsrc) {
                    const int ly = (int)(((float)i + 0.5f) * inv_sw), lx = i - ly * sw;
                    int x0, y0;
                    T fx, fy;
                    source_cell<T, INTERP>(sx0 + lx, sy0 + ly, lvx[k], lvy[k], nx, ny, x0, y0, fx, fy);
                    const int cx = x0 - tl.x0 + 1, cy = y0 - tl.y0 + 1;
                    if (cx >= 0 && cx <= ATX && cy >= 0 && cy <= ATY) {
                        const int cell = cy * CW + cx;
                        const int slot = atomicAdd(&s_cnt[cell], 1);
                        if (slot < ADJ_SLOTS) {
                            const int e = cell * ADJ_SLOTS + slot;
                            s_fx[e] = fx;
                            s_fy[e] = fy;
                            s_val[e] = lr[k];
                            s_rank[e] = (unsigned short)i;
                        } else {
                            atomicOr(&s_over, 1);
                        }
                    }
                }
            }
            __syncthreads();
            wide = s_over != 0;  // (the same value on every thread)
            if (!wide && col_in) {
                const int lx = qx - tl.x0;
#pragma unroll
                for (int k = 0; k < RPT; ++k) {
                    const int qy = qy0 + k;
                    if (qy >= ny) break;
                    // the output is corner (1,1), (0,1), (1,0), (0,0) of the cells at
                    // (qx-1, qy-1), (qx, qy-1), (qx-1, qy), (qx, qy): one partial sum per
                    // corner, each over its cell's sources in raster order
                    const int c00 = (qy - tl.y0) * CW + lx;
                    T part[4];
#pragma unroll
                    for (int cr = 0; cr < 4; ++cr) {
                        const int cc = c00 + (cr & 1) + (cr >> 1) * CW;
                        const int n = s_cnt[cc];
                        const int e0 = cc * ADJ_SLOTS;
                        T a = T(0);
                        if (n == 1) {  // the common case: one source
                            const T fx = s_fx[e0], fy = s_fy[e0];
                            const T wx = (cr & 1) ? T(1) - fx : fx;
                            const T wy = (cr >> 1) ? T(1) - fy : fy;
                            a += wx * wy * s_val[e0];
                        } else if (n > 1) {
                            unsigned key[ADJ_SLOTS];
#pragma unroll
                            for (int q = 0; q < ADJ_SLOTS; ++q) key[q] = q < n ? s_rank[e0 + q] : 0xFFFFFu;
                            // visit the slots by increasing rank (selection over at most 4 keys)
                            for (int t = 0; t < n; ++t) {
                                int best = 0;
#pragma unroll
                                for (int q = 1; q < ADJ_SLOTS; ++q)
                                    if (key[q] < key[best]) best = q;
                                key[best] = 0xFFFFFu;
                                const int e = e0 + best;
                                const T fx = s_fx[e], fy = s_fy[e];
                                const T wx = (cr & 1) ? T(1) - fx : fx;
                                const T wy = (cr >> 1) ? T(1) - fy : fy;
                                a += wx * wy * s_val[e];
                            }
                        }
                        part[cr] = a;
                    }
                    acc[k] = ((part[0] + part[1]) + part[2]) + part[3];
                }
            }
        }
        if (wide && col_in) {
            // Large displacements or crowded cells: scan the full window in global memory,
            // with the per-corner partial sums and their combination of the LDS path (same
            // values).
            const int Rw = max(R, 1);
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int qy = qy0 + k;
                if (qy >= ny) break;
                const int py_lo = max(qy - Rw, 0), py_hi = min(qy + Rw, ny - 1);
                const int px_lo = max(qx - Rw, 0), px_hi = min(qx + Rw, nx - 1);
                T part[4] = {T(0), T(0), T(0), T(0)};
                for (int py = py_lo; py <= py_hi; ++py)
                    for (int px = px_lo; px <= px_hi; ++px) {
                        const int64_t p = (int64_t)py * nx + px;
                        int x0, y0;
                        T fx, fy;
                        source_cell<T, INTERP>(px, py, vxg[p], vyg[p], nx, ny, x0, y0, fx, fy);
                        const int ex = qx - x0, ey = qy - y0;  // 1: the output is the cell's far corner
                        if ((unsigned)ex > 1u || (unsigned)ey > 1u) continue;
                        const T wx = ex ? fx : T(1) - fx;
                        const T wy = ey ? fy : T(1) - fy;
                        const T term = wx * wy * rg[p];
                        const int cr = (1 - ex) + 2 * (1 - ey);
                        if (cr == 0) part[0] += term;
                        else if (cr == 1) part[1] += term;
                        else if (cr == 2) part[2] += term;
                        else part[3] += term;
                    }
                acc[k] = ((part[0] + part[1]) + part[2]) + part[3];
            }
        }
    }
    if (!col_in) return;
    // cout (may be null): instead of u, the residual cout = cx + lambda u (ResidualOut)
    const double lam = cout ? clam[0] : 0.0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int qy = qy0 + k;
        if (qy >= ny) break;
        const T val = acc[k] + direct[k];
        const T out = accumulate ? old[k] + val : val;
        const int64_t o = tl.off + (int64_t)qy * nx + qx;
        if (cout)
            cout[o] = (double)cx[o] + lam * (double)out;
        else
            u[o] = out;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_flow_dv(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                 const T* __restrict__ u, const T* __restrict__ v,
                                                 const T* __restrict__ w, T* __restrict__ gv, int direction) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int x = tl.x0 + (int)(threadIdx.x % FTW);
    const int y = tl.y0 + (int)(threadIdx.x / FTW);
    if (x >= f.nx || y >= f.ny) return;
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const int64_t p = (int64_t)y * nx + x;
    const T* src = u + f.off + (direction > 0 ? np : 0);
    const T* vv = v + 2 * f.pair_off;
    int x0, y0;
    T fx, fy;
    bool cx, cy;
    clip_cell(x, vv[p], nx, x0, fx, cx);
    clip_cell(y, vv[np + p], ny, y0, fy, cy);
    const int y1 = min(y0 + 1, ny - 1);
    // row pairs as in warp_sample (a cell clipped to the last column reads the second element)
    const int xa = min(x0, nx - 2);
    const Pair<T> p0 = ld2(src + (int64_t)y0 * nx + xa), p1 = ld2(src + (int64_t)y1 * nx + xa);
    const bool edge = xa != x0;
    const T s00 = edge ? p0.b : p0.a, s01 = p0.b, s10 = edge ? p1.b : p1.a, s11 = p1.b;
    const T ww = w[f.pair_off + p];
    T dx = (T(1) - fy) * (s01 - s00) + fy * (s11 - s10);
    T dy = (T(1) - fx) * (s10 - s00) + fx * (s11 - s01);
    if (cx) dx = T(0);
    if (cy) dy = T(0);
    gv[2 * f.pair_off + p] = ww * dx;
    gv[2 * f.pair_off + np + p] = ww * dy;
}

// out = max(out, floor(max |v|) + 1) over the n values of the flows (a NaN counts as 1e30), the
// radius of the adjoint's source windows; an integer maximum, so it does not depend on the order.
template <class T, int VEC>
__global__ __launch_bounds__(256) void k_flow_radius(const T* __restrict__ v, int64_t n, int32_t* __restrict__ out) {
    // VEC values per load (16 bytes when the flow is 16-byte aligned), four loads in flight per
    // step; the last n % VEC values singly
    typedef T VT __attribute__((ext_vector_type(VEC), aligned(sizeof(T) * VEC)));
    __shared__ T s4[4];
    T m = T(0);
    auto take = [&](T x) {
        x = fabs(x);
        m = (x != x) ? T(1e30) : fmax(m, x);
    };
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = n / VEC;
    const VT* vv = reinterpret_cast<const VT*>(v);
    for (int64_t i0 = tid; i0 < nv; i0 += 4 * stride) {
        VT a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = i0 + u * stride < nv ? vv[i0 + u * stride] : VT{};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < VEC; ++e) take(a[u][e]);
    }
    for (int64_t i = nv * VEC + tid; i < n; i += stride) take(v[i]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) s4[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(s4[0], s4[1]), fmax(s4[2], s4[3]));
        const T c = fmin(floor(m), T(1 << 20));
        atomicMax(out, (int32_t)c + 1);  // integer max: order-independent
    }
}

__global__ void k_set_int(int32_t* p, int32_t val) { *p = val; }

void launch_flow_radius(Ctx& c, Geom& g, int dt, const void* v, int32_t* d_out) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, c.stream, d_out, 1);
    MMOF_LAUNCH_CHECK();
    const int64_t n = 2 * g.pair_px;
    if (n == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        // one atomic per workgroup: 8 workgroups per CU at most (four waves per SIMD with 16-byte
        // loads: 0.36 -> 0.1 ms over the flows of the 1024x1024x64 stack, against 2 per CU and
        // 4-byte loads)
        constexpr int VEC = 16 / (int)sizeof(T);
        if (reinterpret_cast<uintptr_t>(v) % 16 == 0)
            hipLaunchKernelGGL((k_flow_radius<T, VEC>), grid_for(n / VEC, 256 * 4, 8 * c.cu_count), dim3(256), 0,
                               c.stream, (const T*)v, n, d_out);
        else
            hipLaunchKernelGGL((k_flow_radius<T, 1>), grid_for(n, 256 * 4, 8 * c.cu_count), dim3(256), 0, c.stream,
                               (const T*)v, n, d_out);
        MMOF_LAUNCH_CHECK();
    });
}

const TileShape kFlowShapes[] = {{64, 4, 0}, {32, 8, 0}, {128, 2, 0}, {16, 16, 0}};
const int kFlowCandidates = sizeof(kFlowShapes) / sizeof(kFlowShapes[0]);
const TileShape kFlowAdjShapes[] = {{16, 16, 0}, {32, 16, 0}, {64, 8, 0}, {32, 8, 0}};
const int kFlowAdjCandidates = sizeof(kFlowAdjShapes) / sizeof(kFlowAdjShapes[0]);
// vector-form candidates of the forward operator: lanes per tile row (4 pixels each) and
// waves per workgroup
struct Flow4Shape {
    int lw, nw;
    int tw() const { return 4 * lw; }
    int th() const { return 64 * nw / lw; }
};
static const Flow4Shape kFlow4Shapes[] = {{64, 4}, {32, 4}, {64, 2}, {32, 2}};
static_assert(sizeof(kFlow4Shapes) / sizeof(kFlow4Shapes[0]) == sizeof(kFlowShapes) / sizeof(kFlowShapes[0]),
              "both forms offer the same number of tile candidates");

TileShape flow_tile(const Geom& g, int choice) {
    (void)g;   // (the forward runs in its 4-pixel form for every frame width)
    return TileShape{kFlow4Shapes[choice].tw(), kFlow4Shapes[choice].th(), 0};
}

template <class T, int INTERP>
static auto flow_fwd_kernel(int choice) {
    return choice == 0 ? k_flow_fwd<T, INTERP, 64, 4>
           : choice == 1 ? k_flow_fwd<T, INTERP, 32, 8>
           : choice == 2 ? k_flow_fwd<T, INTERP, 128, 2>
                         : k_flow_fwd<T, INTERP, 16, 16>;
}
template <class T, int INTERP>
static auto flow_fwd4_kernel(int choice) {
    return kFlow4Shapes[choice].lw == 64 ? k_flow_fwd4<T, INTERP, 64> : k_flow_fwd4<T, INTERP, 32>;
}
template <class T, int INTERP>
static auto flow_adj_kernel(int choice) {
    return choice == 0 ? k_flow_adj<T, INTERP, 16, 16>
           : choice == 1 ? k_flow_adj<T, INTERP, 32, 16>
           : choice == 2 ? k_flow_adj<T, INTERP, 64, 8>
                         : k_flow_adj<T, INTERP, 32, 8>;
}

void launch_flow_fwd(Ctx& c, Geom& g, int dt, int direction, int interp, const void* u, const void* v, void* r,
                     int choice, const RowWeighting* rw) {
    if (g.n_pairs == 0) return;
    if (choice < 0) choice = g.choice("flow_fwd", dt, 1);
    MMOF_CHECK(choice >= 0 && choice < kFlowCandidates, MMOF_ERR_INVALID, "flow tile candidate out of range");
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        // (with rw also nu read and the weighted rows written)
        ScopedTime st(&c, "flow_fwd", (rw ? 7.0 : 5.0) * sizeof(T) * g.pair_px, 12.0 * g.pair_px);
        const T* nuw = rw ? (const T*)rw->nu_a : nullptr;
        T* mw = rw ? (T*)rw->m_a : nullptr;
        const double eps2 = rw ? rw->eps2 : 0.0;
        if (aligned_to(sizeof(T), {u, v, r, nuw, mw})) {
            const Flow4Shape sh = kFlow4Shapes[choice];
            const TileList& tl = g.tile_list(c.stream, sh.tw(), sh.th(), true);
            auto k = interp == MMOF_INTERP_ROUND ? flow_fwd4_kernel<T, 1>(choice) : flow_fwd4_kernel<T, 0>(choice);
            hipLaunchKernelGGL(k, dim3((unsigned)tl.count), dim3(64 * sh.nw), 0, c.stream, tl.buf.as<Tile>(),
                               g.dframes(), (const T*)u, (const T*)v, (T*)r, direction, nuw, mw, eps2);
        } else {
            const TileShape sh = kFlowShapes[choice];
            const TileList& tl = g.tile_list(c.stream, sh.tw, sh.th, true);
            auto k = interp == MMOF_INTERP_ROUND ? flow_fwd_kernel<T, 1>(choice) : flow_fwd_kernel<T, 0>(choice);
            hipLaunchKernelGGL(k, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(), g.dframes(),
                               (const T*)u, (const T*)v, (T*)r, direction, nuw, mw, eps2);
        }
        MMOF_LAUNCH_CHECK();
    });
}

void launch_flow_fwd_cols(Ctx& c, Geom& g, int dt, int interp, const void* Uv, bool u_op, int64_t ldu, int K,
                          const void* v, const void* vr, void* out, int64_t ldo, int64_t oF, int64_t oR) {
    if (g.n_pairs == 0 || K <= 0) return;
    const int choice = g.choice("flow_fwd", dt, 1);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        auto run = [&](auto s_tag) {
            using S = decltype(s_tag);
            const S* U = static_cast<const S*>(Uv);
            ScopedTime st(&c, "flow_fwd_cols", (vr ? 2.0 : 1.0) * K * (4.0 * sizeof(T) + 2.0 * sizeof(S)) * g.pair_px,
                          (vr ? 2.0 : 1.0) * K * 12.0 * g.pair_px);
            const bool v4 = aligned_to(sizeof(S), {U}) && aligned_to(sizeof(T), {v, vr, out});
            if (v4) {
                const Flow4Shape sh = kFlow4Shapes[choice];
                const TileList& tl = g.tile_list(c.stream, sh.tw(), sh.th(), true);
                if ((int64_t)g.max_ny * g.max_nx < ((int64_t)1 << 31)) {
                    // (prepared cells hold 32-bit offsets within a frame)
                    constexpr int JC = 8;   // columns per thread
                    auto pick = [&](auto interp_tag) {
                        constexpr int I = decltype(interp_tag)::value;
                        return sh.lw == 64 ? k_flow_fwd_colsJ<T, S, I, 64, JC> : k_flow_fwd_colsJ<T, S, I, 32, JC>;
                    };
                    auto k = interp == MMOF_INTERP_ROUND ? pick(std::integral_constant<int, 1>{})
                                                         : pick(std::integral_constant<int, 0>{});
                    hipLaunchKernelGGL(k, dim3((unsigned)tl.count, (unsigned)cdiv(K, JC)), dim3(64 * sh.nw), 0,
                                       c.stream, tl.buf.as<Tile>(), g.dframes(), U, ldu, K, (const T*)v, (const T*)vr,
                                       (T*)out, ldo, oF, oR);
                } else {
                    auto pick = [&](auto interp_tag) {
                        constexpr int I = decltype(interp_tag)::value;
                        return sh.lw == 64 ? k_flow_fwd_cols4<T, S, I, 64> : k_flow_fwd_cols4<T, S, I, 32>;
                    };
                    auto k = interp == MMOF_INTERP_ROUND ? pick(std::integral_constant<int, 1>{})
                                                         : pick(std::integral_constant<int, 0>{});
                    hipLaunchKernelGGL(k, dim3((unsigned)tl.count, (unsigned)K), dim3(64 * sh.nw), 0, c.stream,
                                       tl.buf.as<Tile>(), g.dframes(), U, ldu, (const T*)v, (const T*)vr, (T*)out,
                                       ldo, oF, oR);
                }
            } else {
                const TileShape sh = kFlowShapes[choice];
                const TileList& tl = g.tile_list(c.stream, sh.tw, sh.th, true);
                auto pick = [&](auto interp_tag) {
                    constexpr int I = decltype(interp_tag)::value;
                    return choice == 0 ? k_flow_fwd_cols<T, S, I, 64, 4>
                           : choice == 1 ? k_flow_fwd_cols<T, S, I, 32, 8>
                           : choice == 2 ? k_flow_fwd_cols<T, S, I, 128, 2>
                                         : k_flow_fwd_cols<T, S, I, 16, 16>;
                };
                auto k = interp == MMOF_INTERP_ROUND ? pick(std::integral_constant<int, 1>{})
                                                     : pick(std::integral_constant<int, 0>{});
                hipLaunchKernelGGL(k, dim3((unsigned)tl.count, (unsigned)K), dim3(256), 0, c.stream,
                                   tl.buf.as<Tile>(), g.dframes(), U, ldu, (const T*)v, (const T*)vr, (T*)out, ldo,
                                   oF, oR);
            }
            MMOF_LAUNCH_CHECK();
        };
        if (u_op)
            run(T{});
        else
            run(double{});
    });
}

void launch_flow_adj(Ctx& c, Geom& g, int dt, int direction, int interp, const void* r, const void* v, void* u,
                     bool accumulate, const int32_t* d_radius, int choice, const ResidualOut* res) {
    int32_t* rad = const_cast<int32_t*>(d_radius);
    if (!rad) {
        rad = static_cast<int32_t*>(c.work("flow_radius", 256));
        launch_flow_radius(c, g, dt, v, rad);
    }
    if (choice < 0) choice = g.choice("flow_adj", dt, 3);
    MMOF_CHECK(choice >= 0 && choice < kFlowAdjCandidates, MMOF_ERR_INVALID, "flow adjoint tile candidate out of range");
    const TileShape sh = kFlowAdjShapes[choice];
    const TileList& tl = g.adj_tile_list(c.stream, sh.tw, sh.th);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "flow_adj", 5.0 * sizeof(T) * g.pair_px, 12.0 * g.pair_px);
        auto k = interp == MMOF_INTERP_ROUND ? flow_adj_kernel<T, 1>(choice) : flow_adj_kernel<T, 0>(choice);
        hipLaunchKernelGGL(k, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<AdjTile>(), (const T*)r,
                           (const T*)v, (T*)u, direction, accumulate ? 1 : 0, rad,
                           res ? (const T*)res->x : (const T*)nullptr, res ? res->lam : nullptr,
                           res ? res->out : nullptr);
        MMOF_LAUNCH_CHECK();
    });
}

template <class T>
__global__ void k_zero(T* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

void launch_flow_dv(Ctx& c, Geom& g, int dt, int direction, int interp, const void* u, const void* v,
                    const void* w, void* gv) {
    if (g.n_pairs == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        if (interp == MMOF_INTERP_ROUND) {  // piecewise-constant warp: zero derivative
            hipLaunchKernelGGL(k_zero<T>, grid_for(2 * g.pair_px, 256), dim3(256), 0, c.stream, (T*)gv,
                               2 * g.pair_px);
            MMOF_LAUNCH_CHECK();
            return;
        }
        const TileList& tl = g.tile_list(c.stream, FTW, FTH, true);
        ScopedTime st(&c, "flow_dv");
        hipLaunchKernelGGL(k_flow_dv<T>, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(),
                           g.dframes(), (const T*)u, (const T*)v, (const T*)w, (T*)gv, direction);
        MMOF_LAUNCH_CHECK();
    });
}

}  // namespace mmof
