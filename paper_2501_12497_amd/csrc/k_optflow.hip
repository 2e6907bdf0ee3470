// Optical-flow subproblem kernels: App. C image derivatives, Horn-Schunck block-Jacobi
// sweeps for the p = q = 2 flow energy (eq. of_reg), the reverse-flow estimate of the
// Remark in Sec. 3, and the MM weights of Sec. 4.1.1.
#include <climits>
#include <vector>

#include "dev.h"
#include "kernels.h"
#include "krylov.h"

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

// The same derivatives from an LDS tile: a workgroup of 512 threads owns 64 x 8 outputs of a
// pair and stages both frames over the tile plus a halo of dr <= DTR_MAX (mirrored indices
// resolved while staging), then forms the sums in the order of k_of_derivs, so the values are
// identical.
static constexpr int DTW = 64, DTH = 8, DTR_MAX = 4;

template <class T>
__global__ __launch_bounds__(512) void k_of_derivs_lds(const Tile* __restrict__ tiles,
                                                       const FrameInfo* __restrict__ fr, const T* __restrict__ u,
                                                       T* __restrict__ I, int dr) {
    constexpr int LW = DTW + 2 * DTR_MAX, LH = DTH + 2 * DTR_MAX;
    __shared__ T sa[LH][LW], sb[LH][LW];
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const T* a = u + f.off;  // frame t
    const T* b = a + np;     // frame t+1
    const int hw = DTW + 2 * dr, hh = DTH + 2 * dr;
    for (int i = threadIdx.x; i < hw * hh; i += 512) {
        const int ly = i / hw, lx = i % hw;
        const int yy = tl.y0 - dr + ly, xx = tl.x0 - dr + lx;
        if (yy >= ny + dr || xx >= nx + dr) continue;  // beyond the frame's own halo
        const int64_t o = (int64_t)mirror(yy, ny) * nx + mirror(xx, nx);
        sa[ly][lx] = a[o];
        sb[ly][lx] = b[o];
    }
    __syncthreads();
    const int tx = (int)(threadIdx.x % DTW), ty = (int)(threadIdx.x / DTW);
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    if (x >= nx || y >= ny) return;
    const int cx = tx + dr, cy = ty + dr;  // the output's position in the tile
    T Ix = T(0), Iy = T(0), It = T(0);
    for (int j = -dr; j <= dr; ++j) {
        Ix += sa[cy + j][cx + dr] - sa[cy + j][cx - dr];
        Iy += sa[cy + dr][cx + j] - sa[cy - dr][cx + j];
        for (int k = -dr; k <= dr; ++k) It += sb[cy + j][cx + k] - sa[cy + j][cx + k];
    }
    const T box = T(2 * dr + 1);
    const int64_t p = (int64_t)y * nx + x;
    T* Ip = I + 3 * f.pair_off;
    Ip[p] = Ix / (box * T(2 * dr));
    Ip[np + p] = Iy / (box * T(2 * dr));
    Ip[2 * np + p] = It / (box * box);
}

// Vector form for stacks whose frame widths are multiples of 4 (and dr <= 4): a workgroup of
// DV_LW x DV_TH threads owns a (4*DV_LW) x DV_TH tile; both frames are staged with a halo of
// one 4-pixel vector left and right and DR rows above and below, moved as whole vectors (a
// vector beyond a frame edge is the mirror image of the edge vector, reversed).  Each thread
// forms 4 outputs from register copies of the 4 + 2*DR staged values of each row it needs;
// per output the sums run in the order of k_of_derivs, so the values are identical.
static constexpr int DV_LW = 32, DV_TH = 8;

template <class T, int DR>
__global__ __launch_bounds__(DV_LW * DV_TH) void k_of_derivs4(const Tile* __restrict__ tiles,
                                                              const FrameInfo* __restrict__ fr,
                                                              const T* __restrict__ u, T* __restrict__ I) {
    constexpr int SW = 4 * DV_LW + 8, SH = DV_TH + 2 * DR;  // staged columns start 4 left of the tile
    constexpr int NQ = SW / 4;                              // vectors per staged row
    constexpr int W = 4 + 2 * DR;                           // values a thread needs per row
    __shared__ Quad<T> sa[SH][NQ], sb[SH][NQ];
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const T* a = u + f.off;  // frame t
    const T* b = a + np;     // frame t+1
    for (int i = threadIdx.x; i < SH * NQ; i += DV_LW * DV_TH) {
        const int ly = i / NQ, lq = i % NQ;
        const int yy = tl.y0 - DR + ly, xs = tl.x0 - 4 + 4 * lq;  // first pixel of the vector
        if (yy >= ny + DR || xs >= nx + 4) continue;               // beyond the frame's own halo
        const int64_t row = (int64_t)mirror(yy, ny) * nx;
        if (xs >= 0 && xs < nx) {
            sa[ly][lq] = ld4(a + row + xs);
            sb[ly][lq] = ld4(b + row + xs);
        } else {
            // xs = -4 mirrors the vector at 0, xs = nx the one at nx - 4, both reversed
            const int ms = xs < 0 ? 0 : nx - 4;
            const Quad<T> qa = ld4(a + row + ms), qb = ld4(b + row + ms);
            sa[ly][lq] = Quad<T>{{qa.v[3], qa.v[2], qa.v[1], qa.v[0]}};
            sb[ly][lq] = Quad<T>{{qb.v[3], qb.v[2], qb.v[1], qb.v[0]}};
        }
    }
    __syncthreads();
    const int lx = (int)(threadIdx.x % DV_LW), ty = (int)(threadIdx.x / DV_LW);
    const int x = tl.x0 + 4 * lx, y = tl.y0 + ty;
    if (x >= nx || y >= ny) return;
    // staged values x - DR .. x + 3 + DR of a row (vector lx holds x - 4 .. x - 1)
    auto row_vals = [&](const Quad<T> (*s)[NQ], int ly, T* r) {
        const Quad<T> q0 = s[ly][lx], q1 = s[ly][lx + 1], q2 = s[ly][lx + 2];
        const T all[12] = {q0.v[0], q0.v[1], q0.v[2], q0.v[3], q1.v[0], q1.v[1],
                           q1.v[2], q1.v[3], q2.v[0], q2.v[1], q2.v[2], q2.v[3]};
#pragma unroll
        for (int c = 0; c < W; ++c) r[c] = all[4 - DR + c];
    };
    T Ix[4], Iy[4], It[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) Ix[j] = Iy[j] = It[j] = T(0);
    T ym[W], yp[W];  // rows y - DR and y + DR
    row_vals(sa, ty, ym);
    row_vals(sa, ty + 2 * DR, yp);
#pragma unroll
    for (int i = -DR; i <= DR; ++i) {
        T ra[W], rb[W];
        row_vals(sa, ty + DR + i, ra);
        row_vals(sb, ty + DR + i, rb);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Ix[j] += ra[j + 2 * DR] - ra[j];
            Iy[j] += yp[j + DR + i] - ym[j + DR + i];
#pragma unroll
            for (int k = -DR; k <= DR; ++k) It[j] += rb[j + DR + k] - ra[j + DR + k];
        }
    }
    const T box = T(2 * DR + 1);
    const int64_t p = (int64_t)y * nx + x;
    T* Ip = I + 3 * f.pair_off;
    Quad<T> ox, oy, ot;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        ox.v[j] = Ix[j] / (box * T(2 * DR));
        oy.v[j] = Iy[j] / (box * T(2 * DR));
        ot.v[j] = It[j] / (box * box);
    }
    st4(Ip + p, ox);
    st4(Ip + np + p, oy);
    st4(Ip + 2 * np + p, ot);
}

// Exact 2x2 block-Jacobi sweeps for the p = q = 2 flow energy: per pixel,
// sbar = mean of the in-image 4-neighbours, s = sbar - g (g.sbar + I_t) / (gamma d + |g|^2).
// Up to HS_MAX block-Jacobi sweeps per launch (temporal blocking).  A workgroup owns an
// HTW x HTH tile of a pair and loads the tile with a halo of HS_MAX pixels into LDS; after q
// sweeps the values within q pixels of the halo's outer edge are stale (their outside
// neighbours were not loaded), so the tile itself is exact after up to HS_MAX sweeps.  Each
// thread keeps, for its HPT halo pixels, the derivatives, 1/d and 1/(gamma d + |g|^2) in
// registers, so a sweep is a few LDS reads and multiply-adds per pixel.  (Reciprocals
// replace the divisions of the sweep formula: the values differ from it by rounding only.)
// Every sweep updates the whole region, so the halo costs work as well as traffic: a 52 x 20
// tile with a 6-pixel halo (6 sweeps per launch, 512 threads) measured 0.72 ms per 8 sweeps
// of the 1024 x 1024 x 64 stack, against 1.16 ms for 64 x 16 with 8 (640 threads), 0.97 ms for
// 56 x 24 with 4 and 0.85 ms for 48 x 48 with 8; workgroups of 1024 threads were slower.
static constexpr int HTW = 52, HTH = 20, HS_MAX = 6;
static constexpr int HRW = HTW + 2 * HS_MAX, HRH = HTH + 2 * HS_MAX;  // 64 x 32 halo region
static constexpr int HS_THREADS = 512;
static constexpr int HPT = HRW * HRH / HS_THREADS;                   // pixels per thread (4)
static_assert(HRW * HRH == HS_THREADS * HPT, "halo region must split evenly over the workgroup");
// LDS per buffer and component: the region, then a zero that neighbours outside the image read
// (so every pixel reads its four neighbours unconditionally), padded to 64 elements
static constexpr int HZERO = HRW * HRH, HCS = (HRW * HRH + 64) / 64 * 64;

template <class T>
__global__ __launch_bounds__(HS_THREADS) void k_hs_multi(const Tile* __restrict__ tiles,
                                                         const FrameInfo* __restrict__ fr, const T* __restrict__ I,
                                                         const T* __restrict__ vin, T* __restrict__ vout, T gamma,
                                                         int nsw) {
    __shared__ T sv[2][2][HCS];  // [buffer][component][pixel]
    static_assert(HRH == HPT * (HS_THREADS / HRW) && HS_THREADS % HRW == 0, "strips must tile the halo region");
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const int ox = tl.x0 - HS_MAX, oy = tl.y0 - HS_MAX;  // image coordinates of the region origin
    const T* sx = vin + 2 * f.pair_off;
    const T* Ip = I + 3 * f.pair_off;
    // a thread owns a strip of HPT consecutive rows of one column of the region: the vertical
    // neighbours inside the strip come from its registers (the previous sweep's values), the
    // others from LDS
    const int rx = (int)threadIdx.x % HRW, ry0 = HPT * ((int)threadIdx.x / HRW);
    const int x = ox + rx;
    T av[HPT], bv[HPT], gx[HPT], gy[HPT], gt[HPT], rden[HPT], rd[HPT];
    bool up_in[HPT], dn_in[HPT];  // pixel r's y-1 (y+1) neighbour exists (strip pixels r-1, r+1)
    int lx[HPT][2];                 // LDS index of the x-1, x+1 neighbours, HZERO outside the image
    int l_up = HZERO, l_dn = HZERO;  // LDS index of the y-1 neighbour of pixel 0, y+1 of pixel HPT-1
    bool live[HPT];
#pragma unroll
    for (int r = 0; r < HPT; ++r) {
        const int ry = ry0 + r, idx = ry * HRW + rx;
        const int y = oy + ry;
        const bool in = x >= 0 && x < nx && y >= 0 && y < ny;
        live[r] = in;
        av[r] = bv[r] = T(0);
        gx[r] = gy[r] = gt[r] = T(0);
        rden[r] = rd[r] = T(0);
        // neighbours outside the loaded region read the pixel itself (stale halo only)
        const bool has_u = in && y > 0, has_d = in && y < ny - 1;
        const bool has_l = in && x > 0, has_r = in && x < nx - 1;
        up_in[r] = has_u;
        dn_in[r] = has_d;
        if (r == 0) l_up = has_u ? (ry > 0 ? idx - HRW : idx) : HZERO;
        if (r == HPT - 1) l_dn = has_d ? (ry < HRH - 1 ? idx + HRW : idx) : HZERO;
        lx[r][0] = has_l ? (rx > 0 ? idx - 1 : idx) : HZERO;
        lx[r][1] = has_r ? (rx < HRW - 1 ? idx + 1 : idx) : HZERO;
        if (in) {
            const int64_t p = (int64_t)y * nx + x;
            av[r] = sx[p];
            bv[r] = sx[np + p];
            gx[r] = Ip[p];
            gy[r] = Ip[np + p];
            gt[r] = Ip[2 * np + p];
            const int d = (int)has_u + (int)has_d + (int)has_l + (int)has_r;
            rd[r] = T(1) / T(d);
            rden[r] = T(1) / (gamma * T(d) + gx[r] * gx[r] + gy[r] * gy[r]);
        }
        sv[0][0][idx] = av[r];
        sv[0][1][idx] = bv[r];
    }
    if (threadIdx.x < 4) sv[threadIdx.x >> 1][threadIdx.x & 1][HZERO] = T(0);
    __syncthreads();
    int cur = 0;
    for (int q = 0; q < nsw; ++q) {
        const T* cx = sv[cur][0];
        const T* cy = sv[cur][1];
        // the LDS neighbours first (all in flight together); a pixel outside the image reads
        // zeros and has zero weights, so it stays 0 without a branch
        T la[HPT][2], lb[HPT][2];
#pragma unroll
        for (int r = 0; r < HPT; ++r)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                la[r][e] = cx[lx[r][e]];
                lb[r][e] = cy[lx[r][e]];
            }
        const T ua = cx[l_up], ub = cy[l_up], da = cx[l_dn], db = cy[l_dn];
        T na[HPT], nb[HPT];
#pragma unroll
        for (int r = 0; r < HPT; ++r) {
            // neighbour order: y-1, y+1, x-1, x+1 (a missing one adds 0)
            T ax = T(0), ay = T(0);
            ax += r == 0 ? ua : (up_in[r] ? av[r - 1] : T(0));
            ay += r == 0 ? ub : (up_in[r] ? bv[r - 1] : T(0));
            ax += r == HPT - 1 ? da : (dn_in[r] ? av[r + 1] : T(0));
            ay += r == HPT - 1 ? db : (dn_in[r] ? bv[r + 1] : T(0));
            ax += la[r][0];
            ay += lb[r][0];
            ax += la[r][1];
            ay += lb[r][1];
            ax *= rd[r];
            ay *= rd[r];
            const T k = (gx[r] * ax + gy[r] * ay + gt[r]) * rden[r];
            na[r] = ax - gx[r] * k;
            nb[r] = ay - gy[r] * k;
        }
#pragma unroll
        for (int r = 0; r < HPT; ++r) {
            const int idx = (ry0 + r) * HRW + rx;
            av[r] = na[r];
            bv[r] = nb[r];
            sv[cur ^ 1][0][idx] = na[r];
            sv[cur ^ 1][1][idx] = nb[r];
        }
        cur ^= 1;
        __syncthreads();
    }
    T* o = vout + 2 * f.pair_off;
#pragma unroll
    for (int r = 0; r < HPT; ++r) {
        const int ry = ry0 + r;
        if (rx < HS_MAX || rx >= HS_MAX + HTW || ry < HS_MAX || ry >= HS_MAX + HTH || !live[r]) continue;
        const int64_t p = (int64_t)(oy + ry) * nx + x;
        o[p] = av[r];
        o[np + p] = bv[r];
    }
}

// Reverse flow: target q gathers, in raster order of the sources p, every p with
// rint(p + v(p)) == q; the result is minus the mean of their velocities (0 if none).
// Target boxes of the sources of the pairs: the smallest rectangle (x_min, x_max, y_min,
// y_max) holding the pixels the flows round to, for every 16 x 16 block and for every row
// strip of 16 pixels of a block (empty: x_min > x_max).  Block b's strips are entries
// 16 b .. 16 b + 15 of `strips`.  64 x 64 tiles; wave w takes block row w of the tile, lane l
// column l; 16-lane reductions per row.
__device__ __forceinline__ void box_reduce16(int& x0, int& x1, int& y0, int& y1) {
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) {
        x0 = min(x0, __shfl_xor(x0, o));
        x1 = max(x1, __shfl_xor(x1, o));
        y0 = min(y0, __shfl_xor(y0, o));
        y1 = max(y1, __shfl_xor(y1, o));
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_rev_boxes(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                   const T* __restrict__ v, int4* __restrict__ boxes,
                                                   int4* __restrict__ strips) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int lane = (int)threadIdx.x % 64, w = (int)threadIdx.x / 64;
    const int nx = f.nx, ny = f.ny;
    const int x = tl.x0 + lane, yb = tl.y0 + 16 * w;
    const int64_t np = (int64_t)nx * ny;
    const T* vx = v + 2 * f.pair_off;
    const T* vy = vx + np;
    const int64_t blk = f.blk_off + (int64_t)(yb / 16) * ((nx + 15) / 16) + x / 16;
    const bool writer = lane % 16 == 0 && x < nx && yb < ny;
    int bx0 = INT_MAX, bx1 = INT_MIN, by0 = INT_MAX, by1 = INT_MIN;
    for (int r = 0; r < 16; ++r) {
        const int y = yb + r;
        int x0 = INT_MAX, x1 = INT_MIN, y0 = INT_MAX, y1 = INT_MIN;
        if (x < nx && y < ny) {
            const int64_t p = (int64_t)y * nx + x;
            const T a = vx[p], b = vy[p];
            if (fabs(a) < T(1048576) && fabs(b) < T(1048576)) {
                x0 = x1 = rint_shift(x, a);
                y0 = y1 = rint_shift(y, b);
            }
        }
        box_reduce16(x0, x1, y0, y1);  // the same values on all 16 lanes
        if (writer && y < ny) strips[16 * blk + r] = make_int4(x0, x1, y0, y1);
        bx0 = min(bx0, x0);
        bx1 = max(bx1, x1);
        by0 = min(by0, y0);
        by1 = max(by1, y1);
    }
    if (writer) boxes[blk] = make_int4(bx0, bx1, by0, by1);
}

// s'(rint(p + s(p))) = -s(p), averaged over collisions, 0 at holes: every target pixel q
// gathers the sources within the flow radius R (d_radius) that round to it, in raster order
// of the sources.  Source blocks whose target box does not hold q are skipped (a block is
// tested once per block row; a bit mask keeps up to 64 block columns), and so are the row
// strips of a candidate block whose boxes do not hold q, so large or uneven displacements do
// not make every target scan its (2R + 1)^2 window: a smooth flow leaves a few candidate
// blocks and strips per target whatever its size.
template <class T>
__global__ __launch_bounds__(256) void k_reverse_flow(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                      const T* __restrict__ v, T* __restrict__ vr,
                                                      const int32_t* __restrict__ d_radius,
                                                      const int4* __restrict__ boxes,
                                                      const int4* __restrict__ strips) {
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo f = fr[tl.frame];
    const int qx = tl.x0 + (int)(threadIdx.x % OTW);
    const int qy = tl.y0 + (int)(threadIdx.x / OTW);
    if (qx >= f.nx || qy >= f.ny) return;
    const int nx = f.nx, ny = f.ny;
    const int64_t np = (int64_t)nx * ny;
    const T* vx = v + 2 * f.pair_off;
    const T* vy = vx + np;
    const int4* bb = boxes + f.blk_off;
    const int4* sb = strips + 16 * (int64_t)f.blk_off;
    const int nbx = (nx + 15) / 16;
    const int R = *d_radius;
    T ax = T(0), ay = T(0);
    int cnt = 0;
    const int py_lo = max(qy - R, 0), py_hi = min(qy + R, ny - 1);
    const int px_lo = max(qx - R, 0), px_hi = min(qx + R, nx - 1);
    const int bx_lo = px_lo >> 4, bx_hi = px_hi >> 4;
    const bool wide = bx_hi - bx_lo >= 64;  // columns past the mask are scanned without the test
    for (int by = py_lo >> 4; by <= (py_hi >> 4); ++by) {
        const int y0 = by * 16, y1 = y0 + 15;
        uint64_t mask = 0;
        for (int bx = bx_lo; bx <= bx_hi && bx - bx_lo < 64; ++bx) {
            const int4 t = bb[by * nbx + bx];
            if (qx >= t.x && qx <= t.y && qy >= t.z && qy <= t.w) mask |= 1ull << (bx - bx_lo);
        }
        if (!mask && !wide) continue;
        for (int py = max(py_lo, y0); py <= min(py_hi, y1); ++py)
            for (int bx = bx_lo; bx <= bx_hi; ++bx) {
                const int i = bx - bx_lo;
                if (i < 64 && !((mask >> i) & 1ull)) continue;
                const int4 t = sb[16 * ((int64_t)by * nbx + bx) + (py - y0)];
                if (!(qx >= t.x && qx <= t.y && qy >= t.z && qy <= t.w)) continue;
                const int xa = max(px_lo, bx * 16), xb = min(px_hi, bx * 16 + 15);
                for (int px = xa; px <= xb; ++px) {
                    const int64_t p = (int64_t)py * nx + px;
                    const T a = vx[p], b = vy[p];
                    if (!(fabs(a) < T(1048576)) || !(fabs(b) < T(1048576))) continue;
                    if (rint_shift(px, a) != qx || rint_shift(py, b) != qy) continue;
                    ax -= a;
                    ay -= b;
                    ++cnt;
                }
            }
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
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "of_derivs", 5.0 * sizeof(T) * g.pair_px, (4.0 * (2 * dr + 1) + 2.0 * (2 * dr + 1) * (2 * dr + 1)) * g.pair_px);
        if (dr <= 4 && g.vec4 && aligned_to(4 * sizeof(T), {u, I})) {
            const TileList& tl = g.tile_list(c.stream, 4 * DV_LW, DV_TH, true);
            auto k = dr == 1 ? k_of_derivs4<T, 1> : dr == 2 ? k_of_derivs4<T, 2> : dr == 3 ? k_of_derivs4<T, 3>
                                                                                        : k_of_derivs4<T, 4>;
            hipLaunchKernelGGL(k, dim3((unsigned)tl.count), dim3(DV_LW * DV_TH), 0, c.stream, tl.buf.as<Tile>(),
                               g.dframes(), (const T*)u, (T*)I);
        } else if (dr <= DTR_MAX) {
            const TileList& tl = g.tile_list(c.stream, DTW, DTH, true);
            hipLaunchKernelGGL(k_of_derivs_lds<T>, dim3((unsigned)tl.count), dim3(512), 0, c.stream,
                               tl.buf.as<Tile>(), g.dframes(), (const T*)u, (T*)I, dr);
        } else {
            const TileList& tl = g.tile_list(c.stream, OTW, OTH, true);
            hipLaunchKernelGGL(k_of_derivs<T>, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(),
                               g.dframes(), (const T*)u, (T*)I, dr);
        }
        MMOF_LAUNCH_CHECK();
    });
}

int launch_hs_sweeps(Ctx& c, Geom& g, int dt, const void* I, void* v, void* tmp, double gamma, int n_sweeps) {
    if (g.n_pairs == 0 || n_sweeps <= 0) return 0;
    const TileList& tl = g.tile_list(c.stream, HTW, HTH, true);
    int done = 0, parity = 0;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        T* a = (T*)v;
        T* b = (T*)tmp;
        while (done < n_sweeps) {
            const int q = std::min(HS_MAX, n_sweeps - done);
            ScopedTime st(&c, "hs_multi", 7.0 * sizeof(T) * g.pair_px, 16.0 * q * g.pair_px);
            hipLaunchKernelGGL(k_hs_multi<T>, dim3((unsigned)tl.count), dim3(HS_THREADS), 0, c.stream, tl.buf.as<Tile>(),
                               g.dframes(), (const T*)I, (const T*)a, b, (T)gamma, q);
            MMOF_LAUNCH_CHECK();
            std::swap(a, b);
            parity ^= 1;
            done += q;
        }
    });
    return parity;
}

// Block means over f x f blocks of the frames (mode 0) or of the two flow components of the
// pairs, divided by f (mode 1); a block at the right or bottom edge averages its in-frame
// pixels.  One thread per reduced pixel over the reduced geometry's tiles.
template <class T, int F>
__global__ __launch_bounds__(256) void k_box_down(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ frs,
                                                  const FrameInfo* __restrict__ fr, const T* __restrict__ in,
                                                  T* __restrict__ out, int f_arg, int mode) {
    // F > 0: the factor is F, and a block of full width is read row by row with one F-element
    // load (the same sums in the same order as the element loads of F = 0)
    const int f = F > 0 ? F : f_arg;
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo s = frs[tl.frame], b = fr[tl.frame];  // the reduced frame and its full frame
    const int xs = tl.x0 + (int)(threadIdx.x % OTW), ys = tl.y0 + (int)(threadIdx.x / OTW);
    if (xs >= s.nx || ys >= s.ny) return;
    const int x0 = xs * f, y0 = ys * f;
    const int x1 = min(x0 + f, b.nx), y1 = min(y0 + f, b.ny);
    const T inv = T(1) / T((x1 - x0) * (y1 - y0));
    const int ncomp = mode == 0 ? 1 : 2;
    const int64_t npb = (int64_t)b.nx * b.ny, nps = (int64_t)s.nx * s.ny;
    constexpr int FV = F > 0 ? F : 1;
    typedef T VF __attribute__((ext_vector_type(FV), aligned(sizeof(T))));
    for (int comp = 0; comp < ncomp; ++comp) {
        const T* src = mode == 0 ? in + b.off : in + 2 * b.pair_off + comp * npb;
        T acc = T(0);
        if (F > 0 && x1 - x0 == F && y1 - y0 == F) {
            // a whole block: every row's load in flight before the sum
            VF q[FV];
#pragma unroll
            for (int r = 0; r < FV; ++r) q[r] = *reinterpret_cast<const VF*>(src + (int64_t)(y0 + r) * b.nx + x0);
#pragma unroll
            for (int r = 0; r < FV; ++r)
#pragma unroll
                for (int e = 0; e < FV; ++e) acc += q[r][e];
        } else if (F > 0 && x1 - x0 == F) {
            for (int y = y0; y < y1; ++y) {
                const VF q = *reinterpret_cast<const VF*>(src + (int64_t)y * b.nx + x0);
#pragma unroll
                for (int e = 0; e < FV; ++e) acc += q[e];
            }
        } else {
            for (int y = y0; y < y1; ++y)
                for (int x = x0; x < x1; ++x) acc += src[(int64_t)y * b.nx + x];
        }
        T m = acc * inv;
        if (mode == 1) m = m / T(f);
        T* dst = mode == 0 ? out + s.off : out + 2 * s.pair_off + comp * nps;
        dst[(int64_t)ys * s.nx + xs] = m;
    }
}

// v = f * bilinear sample of the reduced flow at ((x + 1/2)/f - 1/2, (y + 1/2)/f - 1/2),
// positions clamped to the reduced grid.  A lane takes four consecutive pixels of a row
// on each of the UTH rows of a UTW x UTH tile (the workgroup's 256 lanes span its width; few,
// long-lived workgroups): for f >= 2 their samples fall within four consecutive columns of the
// reduced flow, which it reads with one 4-element load per reduced row and component (from
// column c0 = min(first column, reduced width - 4), reduced widths of at least 4) and stores
// its four outputs of a component together.  Its x positions and weights serve every row.
// F = 2, 4, 8 (the factor known at compile time): on a lane whose four samples are unclamped
// and whose window lies inside the reduced row the columns each pixel reads are the same for
// every such lane (F = 4: c0, c0, c0+1, c0+1 and the next ones), so no per-pixel selection is
// needed; other lanes take the general path, which gives the same values.
static constexpr int UTW = 1024, UTH = 8;

template <int F>
__device__ __forceinline__ void up_cols(int i, int& ia, int& ib) {
    // columns (from the lane's first column) of pixel i's two samples on an interior lane
    if (F == 2) {
        ia = (i + 1) >> 1;  // 0, 1, 1, 2
    } else if (F == 4) {
        ia = i >> 1;        // 0, 0, 1, 1
    } else {
        ia = 0;             // F = 8: one cell for all four
    }
    ib = ia + 1;
}

template <class T, int F>
__global__ __launch_bounds__(256) void k_flow_up(const Tile* __restrict__ tiles, const FrameInfo* __restrict__ fr,
                                                 const FrameInfo* __restrict__ frs, const T* __restrict__ vs,
                                                 T* __restrict__ v, int f_arg) {
    const int f = F > 0 ? F : f_arg;
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const FrameInfo b = fr[tl.frame], s = frs[tl.frame];
    const int xq = tl.x0 + 4 * (int)threadIdx.x;  // UTW = 4 x 256: one row of the tile per pass
    if (xq >= b.nx) return;
    const int npx = min(4, b.nx - xq);
    const int64_t npb = (int64_t)b.nx * b.ny, nps = (int64_t)s.nx * s.ny;
    typedef T V4 __attribute__((ext_vector_type(4), aligned(sizeof(T))));
    // the lane's columns: positions, cells and weights in x are the same on every row
    const double invf = 1.0 / f;
    int xa[4], xb[4];
    T fx[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // (x + 1/2) / f as (x + 1/2) (1/f): exact for the power-of-two factors, within an ulp
        // otherwise
        const double X = fmin(fmax(fma(xq + i + 0.5, invf, -0.5), 0.0), (double)(s.nx - 1));
        xa[i] = min((int)floor(X), s.nx - 1);
        xb[i] = min(xa[i] + 1, s.nx - 1);
        fx[i] = (T)(X - xa[i]);
    }
    const bool vec = f >= 2 && s.nx >= 4;
    const int c0 = min(xa[0], s.nx - 4);
    // F > 0: on a lane whose samples are unclamped and whose window lies inside the reduced
    // row, pixel i reads columns c0 + up_cols (the same values as the general path)
    bool fixed = false;
    if constexpr (F > 0) {
        constexpr float iF = 1.0f / F;
        const float X0 = fmaf((float)xq + 0.5f, iF, -0.5f);
        fixed = npx == 4 && X0 >= 0.0f && X0 + 3.0f * iF <= (float)(s.nx - 1) && xa[0] + 3 <= s.nx - 1;
    }
    for (int r = 0; r < UTH; ++r) {
        const int y = tl.y0 + r;
        if (y >= b.ny) break;
        const double Y = fmin(fmax(fma(y + 0.5, invf, -0.5), 0.0), (double)(s.ny - 1));
        const int ya = min((int)floor(Y), s.ny - 1), yb = min(ya + 1, s.ny - 1);
        const T fy = (T)(Y - ya);
        for (int comp = 0; comp < 2; ++comp) {
            const T* q = vs + 2 * s.pair_off + comp * nps;
            T o[4];
            if (fixed) {
                const V4 ra = *reinterpret_cast<const V4*>(q + (int64_t)ya * s.nx + xa[0]);
                const V4 rb = *reinterpret_cast<const V4*>(q + (int64_t)yb * s.nx + xa[0]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int ia = 0, ib = 1;
                    if constexpr (F > 0) up_cols<F>(i, ia, ib);
                    o[i] = T(f) * ((T(1) - fy) * ((T(1) - fx[i]) * ra[ia] + fx[i] * ra[ib]) +
                                   fy * ((T(1) - fx[i]) * rb[ia] + fx[i] * rb[ib]));
                }
            } else if (vec) {
                const V4 ra = *reinterpret_cast<const V4*>(q + (int64_t)ya * s.nx + c0);
                const V4 rb = *reinterpret_cast<const V4*>(q + (int64_t)yb * s.nx + c0);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int ia = xa[i] - c0, ib = xb[i] - c0;  // in [0, 3]
                    const T a00 = ra[ia], a01 = ra[ib], a10 = rb[ia], a11 = rb[ib];
                    o[i] = T(f) * ((T(1) - fy) * ((T(1) - fx[i]) * a00 + fx[i] * a01) +
                                   fy * ((T(1) - fx[i]) * a10 + fx[i] * a11));
                }
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const T a00 = q[(int64_t)ya * s.nx + xa[i]], a01 = q[(int64_t)ya * s.nx + xb[i]];
                    const T a10 = q[(int64_t)yb * s.nx + xa[i]], a11 = q[(int64_t)yb * s.nx + xb[i]];
                    o[i] = T(f) * ((T(1) - fy) * ((T(1) - fx[i]) * a00 + fx[i] * a01) +
                                   fy * ((T(1) - fx[i]) * a10 + fx[i] * a11));
                }
            }
            T* dst = v + 2 * b.pair_off + comp * npb + (int64_t)y * b.nx + xq;
            if (npx == 4) {
                *reinterpret_cast<V4*>(dst) = V4{o[0], o[1], o[2], o[3]};
            } else {
                for (int i = 0; i < npx; ++i) dst[i] = o[i];
            }
        }
    }
}

// The stack with every frame side ceil(n / f), handed to `use`.
template <class F>
static decltype(auto) with_reduced_stack(const Geom& g, int f, F&& use) {
    std::vector<int32_t> ny(g.ny), nx(g.nx);
    for (auto& v : ny) v = (v + f - 1) / f;
    for (auto& v : nx) v = (v + f - 1) / f;
    const mmof_stack s{g.n_seq, g.n_t.data(), ny.data(), nx.data()};
    return use(&s);
}

Geom& reduced_geom(Ctx& c, const Geom& g, int f) {
    return with_reduced_stack(g, f, [&](const mmof_stack* s) -> Geom& { return c.geom(s); });
}

std::unique_ptr<Geom> make_reduced_geom(const Geom& g, int f, hipStream_t st) {
    return with_reduced_stack(g, f, [&](const mmof_stack* s) { return make_geom(s, st); });
}

int resolve_flow_scale(const Geom& g, int f) {
    if (f == 0) return 1;
    if (f != MMOF_FLOW_SCALE_AUTO) return f;
    const int side = std::max(g.max_ny, g.max_nx);
    int s = 1;
    while (s < 64 && (side + s - 1) / s >= 50) s *= 2;
    return s;
}

void check_flow_frames(const Geom& g, int f, int dr) {
    MMOF_CHECK(f >= 1 && f <= 64, MMOF_ERR_INVALID, "flow scale must be in [1, 64]");
    for (int s = 0; s < g.n_seq; ++s) {
        const int ny = (g.ny[s] + f - 1) / f, nx = (g.nx[s] + f - 1) / f;
        MMOF_CHECK(dr >= 1 && dr < nx && dr < ny, MMOF_ERR_INVALID,
                   f == 1 ? "delta_r must be in [1, frame size)" : "delta_r must be in [1, reduced frame size)");
    }
}

void launch_box_down(Ctx& c, Geom& g, Geom& gs, int dt, int mode, int f, const void* in, void* out) {
    if (mode == 1 && gs.n_pairs == 0) return;
    const TileList& tl = gs.tile_list(c.stream, OTW, OTH, mode == 1);
    if (tl.count == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        const double px = mode == 0 ? (double)g.n : 2.0 * g.pair_px, pxs = mode == 0 ? (double)gs.n : 2.0 * gs.pair_px;
        ScopedTime st(&c, "box_down", sizeof(T) * (px + pxs), px);
        auto k = f == 2 ? k_box_down<T, 2> : f == 4 ? k_box_down<T, 4> : f == 8 ? k_box_down<T, 8> : k_box_down<T, 0>;
        hipLaunchKernelGGL(k, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(), gs.dframes(),
                           g.dframes(), (const T*)in, (T*)out, f, mode);
        MMOF_LAUNCH_CHECK();
    });
}

void launch_flow_up(Ctx& c, Geom& g, Geom& gs, int dt, int f, const void* vs, void* v) {
    if (g.n_pairs == 0) return;
    const TileList& tl = g.tile_list(c.stream, UTW, UTH, true);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "flow_up", sizeof(T) * 2.0 * (g.pair_px + gs.pair_px), 2.0 * 8.0 * g.pair_px);
        auto k = f == 2 ? k_flow_up<T, 2> : f == 4 ? k_flow_up<T, 4> : f == 8 ? k_flow_up<T, 8> : k_flow_up<T, 0>;
        hipLaunchKernelGGL(k, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(), g.dframes(),
                           gs.dframes(), (const T*)vs, (T*)v, f);
        MMOF_LAUNCH_CHECK();
    });
}

void flow_update_core(Ctx& c, Geom& g, Geom* gs, int dt, const void* u, void* v, int f, int dr, const FlowMethod& fm,
                      const FlowWork& w) {
    if (g.n_pairs == 0) return;
    MMOF_CHECK(f == 1 || gs, MMOF_ERR_INVALID, "reduced geometry missing");
    Geom& gw = f > 1 ? *gs : g;  // the frames the flow is computed on
    const void* uw = u;
    void* vw = v;
    if (f > 1) {
        launch_box_down(c, g, gw, dt, 0, f, u, w.us);
        if (fm.solver == 0) launch_box_down(c, g, gw, dt, 1, f, v, w.vs);  // the warm start
        uw = w.us;
        vw = w.vs;
    }
    launch_of_derivs(c, gw, dt, uw, w.I, dr);
    if (fm.solver == 1)
        launch_of_gks(c, gw, dt, w.I, vw, fm.ell, fm.n_iter, fm.fixed_lambda, w.gks, fm.of_p == 1, fm.of_eps);
    else if (launch_hs_sweeps(c, gw, dt, w.I, vw, w.tmp, fm.gamma, fm.n_sweeps)) {
        dispatch(dt, [&](auto z) {
            using T = decltype(z);
            convert<T, T>(c, 2 * gw.pair_px, (const T*)w.tmp, (T*)vw);
        });
    }
    if (f > 1) launch_flow_up(c, g, gw, dt, f, w.vs, v);
}

void launch_reverse_flow(Ctx& c, Geom& g, int dt, const void* v, void* vr, const int32_t* d_radius) {
    if (g.n_pairs == 0) return;
    int32_t* rad = const_cast<int32_t*>(d_radius);
    if (!rad) {
        rad = static_cast<int32_t*>(c.work("rev_radius", 256));
        launch_flow_radius(c, g, dt, v, rad);
    }
    const size_t nb = (size_t)std::max<int64_t>(g.pair_blocks, 1);
    int4* boxes = static_cast<int4*>(c.work("rev_boxes", sizeof(int4) * 17 * nb));
    int4* strips = boxes + nb;
    const TileList& tb = g.tile_list(c.stream, 64, 64, true);
    const TileList& tl = g.tile_list(c.stream, OTW, OTH, true);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        hipLaunchKernelGGL(k_rev_boxes<T>, dim3((unsigned)tb.count), dim3(256), 0, c.stream, tb.buf.as<Tile>(),
                           g.dframes(), (const T*)v, boxes, strips);
        MMOF_LAUNCH_CHECK();
        ScopedTime st(&c, "reverse_flow");
        hipLaunchKernelGGL(k_reverse_flow<T>, dim3((unsigned)tl.count), dim3(256), 0, c.stream, tl.buf.as<Tile>(),
                           g.dframes(), (const T*)v, (T*)vr, rad, boxes, strips);
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
