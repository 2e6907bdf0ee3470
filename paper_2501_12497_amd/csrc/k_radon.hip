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

static constexpr int RTW = 16, RTH = 16;  // pixel tiles of the fan-beam transpose

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

// The same transpose with 16-byte accesses, for stacks whose frame sides and offsets are all
// multiples of 4 (Plan::tr_vec): a tile row is 32 / VEC vectors of VEC = 16 / sizeof(T) pixels,
// and each thread reads one (FP32) or two (FP64) of them and writes as many of the transposed
// tile.
template <class T>
__global__ __launch_bounds__(256) void k_transpose_frames4(const Tile* __restrict__ tiles,
                                                           const RadonFrame* __restrict__ rf,
                                                           const T* __restrict__ u, T* __restrict__ ut) {
    constexpr int VEC = 16 / (int)sizeof(T);      // 4 FP32 or 2 FP64 pixels per access
    constexpr int VPR = 32 / VEC;                  // vectors per tile row
    typedef T VT __attribute__((ext_vector_type(VEC)));
    __shared__ T s[32][33];
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[tl.frame];
    for (int i = threadIdx.x; i < 32 * VPR; i += 256) {
        const int r = i / VPR, c = VEC * (i % VPR);
        const int y = tl.y0 + r, x = tl.x0 + c;
        if (y < f.ny && x < f.nx) {   // (x < nx implies x + VEC - 1 < nx: nx is a multiple of 4)
            const VT q = *reinterpret_cast<const VT*>(u + f.u_off + (int64_t)y * f.nx + x);
#pragma unroll
            for (int e = 0; e < VEC; ++e) s[r][c + e] = q[e];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 32 * VPR; i += 256) {
        const int xr = i / VPR, c = VEC * (i % VPR);   // output row (x) and its first y
        const int x = tl.x0 + xr, y = tl.y0 + c;
        if (x < f.nx && y < f.ny) {
            VT q;
#pragma unroll
            for (int e = 0; e < VEC; ++e) q[e] = s[c + e][xr];
            *reinterpret_cast<VT*>(ut + f.u_off + (int64_t)x * f.ny + y) = q;
        }
    }
}

// Sum over the (at most three) pixels of one row (the row starting at offset roff of the
// frame img) with non-zero hat weight for a ray whose centre crosses the row at xs: weights 1 - |a| |x - xs| with |a| >= 1/sqrt(2), so the
// pixels are floor(xs) - 1 .. floor(xs) + 1 when the fraction is below 1/2, else
// floor(xs) .. floor(xs) + 2.
template <class T>
__device__ __forceinline__ T hat_row(const T* __restrict__ img, int roff, int ncol, double xs, T aa) {
    const double fl = floor(xs);
    const int xi = (int)fl;
    const T fr = (T)(xs - fl);
    const int k0 = fr < T(0.5) ? -1 : 0;
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int x = xi + k0 + k;
        const T w = T(1) - aa * fabs(T(k0 + k) - fr);
        if (x >= 0 && x < ncol && w > T(0)) acc += w * img[(uint32_t)(roff + x)];
    }
    return acc;
}

// The same sum for a row where all three candidates lie inside the row (xs in [1, ncol - 2)):
// pixels floor(xs) and floor(xs) + 1 with weights 1 - |a| f and 1 - |a| (1 - f), and the
// outer neighbour on the nearer side with weight max(0, 1 - |a| (1 + min(f, 1 - f))).
template <class T>
__device__ __forceinline__ T hat_row_inner(const T* __restrict__ img, int roff, int ncol, double xs, T aa) {
    // xs >= 1: truncation is the floor; the clamp keeps every access inside the row even if
    // rounding puts xs a hair outside the interior (the weights then still match xs)
    const int xi = min(max((int)xs, 1), ncol - 3);
    const T fr = (T)(xs - (double)xi);
    const bool lo = fr < T(0.5);
    const T w0 = T(1) - aa * fr;
    const T w1 = T(1) - aa * (T(1) - fr);
    const T w2 = fmax(T(1) - aa * (T(1) + (lo ? fr : T(1) - fr)), T(0));
    // the four pixels xi - 1 .. xi + 2 (all inside the row) as one 4-element load
    typedef T V4 __attribute__((ext_vector_type(4), aligned(sizeof(T))));
    const V4 q = *reinterpret_cast<const V4*>(img + (uint32_t)(roff + xi - 1));
    return w0 * q.y + w1 * q.z + w2 * (lo ? q.x : q.w);
}

// Interior rows of an FP32 image in groups of G, three taps centred on the nearest pixel: with
// n = round(xs) and d = xs - n in [-1/2, 1/2], the pixels n - 1, n, n + 1 have the weights
// max(0, 1 - |a| (1 + d)), 1 - |a| |d| and max(0, 1 - |a| (1 - d)), and no other pixel is
// within 1/|a| <= sqrt(2) of xs; the products are added to three running sums s0..s2 (one per
// tap).  The group's first row: xs + 1/2 (xs0h: xs0 + 1/2) in FP64, split into its floor
// and an FP32 fraction fb; row k at t = fb + k step in FP32 (error below 1e-6 px for
// |step| <= 1, k < 8), n = floor(t) + that floor through a floor-convert, f = fract(t) = d + 1/2.
// The three pixels come in one 12-byte load at a 32-bit byte offset (so the frame must hold
// fewer than 2^30 pixels) from a per-row base that is the same for the whole wave; the outer
// weights (1 - |a|/2) - |a| f and (1 - 3|a|/2) + |a| f are single FMAs clamped to [0, 1] by the
// FMA's output clamp.  The caller guarantees 1/2 + INTERIOR_MARGIN <= xs < ncol - 3/2 -
// INTERIOR_MARGIN on every row it passes, so the FP32 position never leaves the row.
static constexpr int RG = 8;
static constexpr double INTERIOR_MARGIN = 1e-3;

template <int G>
__device__ __forceinline__ void hat_rows3_f32(const char* __restrict__ base, int r, int ncol, double xs0h,
                                              double step, float aa, float& s0, float& s1, float& s2) {
    const double xb = fma((double)r, step, xs0h);
    const double flb = floor(xb);
    const float fb = (float)(xb - flb);
    const float stepf = (float)step;
    const float cm = 1.f - 0.5f * aa, cp = 1.f - 1.5f * aa;
    // the group's byte offset, formed once (kept opaque so that each row adds only its own
    // pixel offset to it)
    uint32_t rowb;
    asm("v_mov_b32 %0, %1" : "=v"(rowb) : "v"((uint32_t)(r * ncol + (int)flb - 1) * 4u));
    const uint32_t ncolb = (uint32_t)ncol * 4u;
    typedef float F3 __attribute__((ext_vector_type(3), aligned(4)));
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const float t = fmaf((float)k, stepf, fb);
        int xr;
        asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(xr) : "v"(t));
        const float f = __builtin_amdgcn_fractf(t);
        const char* __restrict__ rowk = base + (size_t)k * ncolb;
        const F3 q = *reinterpret_cast<const F3*>(rowk + (rowb + ((uint32_t)xr << 2)));
        s0 = fmaf(__builtin_amdgcn_fmed3f(fmaf(-aa, f, cm), 0.f, 1.f), q.x, s0);
        s1 = fmaf(fmaf(-aa, fabsf(f - 0.5f), 1.f), q.y, s1);
        s2 = fmaf(__builtin_amdgcn_fmed3f(fmaf(aa, f, cp), 0.f, 1.f), q.z, s2);
    }
}

// One workgroup of 8 waves per (frame, ANG consecutive angles, 64 bins): lane = bin, wave
// w takes angle w / (8/ANG) and the (w % (8/ANG))-th block of rows, walking four rows per
// step (FP32 images: eight, see hat_rows_f32) so that their loads are in flight together.
// The waves of one workgroup read overlapping spans of the same rows, so a wider angle group
// reuses the image through the cache; partial sums are added in a fixed order.
template <class T, int ANG>
__global__ __launch_bounds__(512) void k_radon_fwd(const RayTile* __restrict__ rays, const RadonFrame* __restrict__ rf,
                                                   const double2* __restrict__ trig, const T* __restrict__ u,
                                                   const T* __restrict__ ut, T* __restrict__ b) {
    constexpr int RSL = 8 / ANG;
    __shared__ T part[8][64];
    const RayTile rt = rays[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[rt.frame];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // (uniform: angle, image in SGPRs)
    const int ang = rt.angle + wave / RSL, sl = wave % RSL;
    const int j = rt.bin0 + lane;
    // FP32 interior rows by hat_rows3_f32 (32-bit byte offsets within the frame); FP64 rows by
    // hat_row_inner (a three-tap FP64 form with one 16-byte and one 8-byte load per row measured
    // slower: the row's two load instructions bound either form)
    const bool rows3 = sizeof(T) == 4 && (int64_t)f.ny * f.nx < ((int64_t)1 << 30);
    const double margin = rows3 ? INTERIOR_MARGIN : 0.0;
    T acc = T(0);
    if (ang < f.n_ang && j < f.n_bins) {
        const double2 cs = trig[f.trig_off + ang];
        const double c = cs.x, s = cs.y;
        const double cx = 0.5 * (f.nx - 1), cy = 0.5 * (f.ny - 1);
        const double dj = (double)j - 0.5 * (f.n_bins - 1);
        // row walk over (rows, cols) = (ny, nx) of u, or over (nx, ny) of the transpose
        const bool steep = fabs(s) > fabs(c);
        const double a = steep ? s : c;   // coefficient of the in-row coordinate
        const double bb = steep ? c : s;  // coefficient of the row coordinate
        const int nrow = steep ? f.nx : f.ny, ncol = steep ? f.ny : f.nx;
        const double crow = steep ? cx : cy, ccol = steep ? cy : cx;
        const T* img = (steep ? ut : u) + f.u_off;
        // ray centre in row r: xs(r) = ccol + (dj - (r - crow) bb) / a
        const double xs0 = ccol + (dj + crow * bb) / a;
        const double step = -bb / a;
        const double inv_step = 1.0 / step;  // inf for step 0 (that case is handled apart)
        const T aa = (T)fabs(a);
        const int q = (nrow + RSL - 1) / RSL;
        int r_lo = sl * q, r_hi = min(nrow, r_lo + q);
        // rows where the ray can touch the image (xs in (-1.5, ncol + 0.5)), and among them
        // the rows where every candidate is inside (xs in [1, ncol - 2)), from xs linear in r
        auto row_of = [&](double x) { return (x - xs0) * inv_step; };
        int in_lo = r_lo, in_hi = r_lo;  // [in_lo, in_hi): interior rows
        // the interior of the three-tap rows, or of hat_row_inner
        const double x_in_lo = rows3 ? 0.5 + margin : 1.0;
        const double x_in_hi = rows3 ? (double)ncol - 1.5 - margin : (double)ncol - 2.0;
        // (bounds are clamped to [0, nrow] in double before the conversion, so near-axis
        // angles, whose tiny slope puts the crossings far away, give in-range integers)
        const double dn = (double)nrow;
        auto clamp_row = [&](double x) { return (int)fmin(fmax(x, 0.0), dn); };
        if (r_hi - r_lo < 48) {
            // short row blocks: the bookkeeping below would cost more than it saves
        } else if (step != 0.0) {
            const double ra = row_of(-1.5), rb = row_of((double)ncol + 0.5);
            const double t_lo = fmin(ra, rb), t_hi = fmax(ra, rb);
            r_lo = max(r_lo, clamp_row(floor(t_lo) - 1.0));
            r_hi = min(r_hi, clamp_row(ceil(t_hi) + 2.0));
            const double ia = row_of(x_in_lo), ib = row_of(x_in_hi);
            in_lo = max(r_lo, clamp_row(ceil(fmin(ia, ib)) + 1.0));
            in_hi = min(r_hi, clamp_row(floor(fmax(ia, ib)) - 1.0));
        } else if (xs0 >= x_in_lo && xs0 < x_in_hi) {
            in_lo = r_lo;
            in_hi = r_hi;
        }
        if (in_hi < in_lo || ncol < 4) in_hi = in_lo = r_lo;  // no interior (also for rows shorter than 4)
        int r = r_lo;
        for (; r < min(in_lo, r_hi); ++r) acc += hat_row(img, r * ncol, ncol, fma((double)r, step, xs0), aa);
        if constexpr (sizeof(T) == 4) {
            if (rows3) {
                const char* __restrict__ base = reinterpret_cast<const char*>(img);
                const double xs0h = xs0 + 0.5;
                float s0 = 0.f, s1 = 0.f, s2 = 0.f;
                for (; r < in_hi - (RG - 1); r += RG) hat_rows3_f32<RG>(base, r, ncol, xs0h, step, aa, s0, s1, s2);
                for (; r < in_hi; ++r) hat_rows3_f32<1>(base, r, ncol, xs0h, step, aa, s0, s1, s2);
                acc += (s0 + s2) + s1;
            }
        }
        for (; r < in_hi - 3; r += 4) {
            const T a0 = hat_row_inner(img, r * ncol, ncol, fma((double)r, step, xs0), aa);
            const T a1 = hat_row_inner(img, (r + 1) * ncol, ncol, fma((double)(r + 1), step, xs0), aa);
            const T a2 = hat_row_inner(img, (r + 2) * ncol, ncol, fma((double)(r + 2), step, xs0), aa);
            const T a3 = hat_row_inner(img, (r + 3) * ncol, ncol, fma((double)(r + 3), step, xs0), aa);
            acc += (a0 + a1) + (a2 + a3);
        }
        for (; r < in_hi; ++r) acc += hat_row_inner(img, r * ncol, ncol, fma((double)r, step, xs0), aa);
        for (; r < r_hi - 3; r += 4) {
            const T a0 = hat_row(img, r * ncol, ncol, fma((double)r, step, xs0), aa);
            const T a1 = hat_row(img, (r + 1) * ncol, ncol, fma((double)(r + 1), step, xs0), aa);
            const T a2 = hat_row(img, (r + 2) * ncol, ncol, fma((double)(r + 2), step, xs0), aa);
            const T a3 = hat_row(img, (r + 3) * ncol, ncol, fma((double)(r + 3), step, xs0), aa);
            acc += (a0 + a1) + (a2 + a3);
        }
        for (; r < r_hi; ++r) acc += hat_row(img, r * ncol, ncol, fma((double)r, step, xs0), aa);
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (sl == 0 && ang < f.n_ang && j < f.n_bins) {
        T sum = T(0);
#pragma unroll
        for (int k = 0; k < RSL; ++k) sum += part[wave + k][lane];
        b[f.sino_off + (int64_t)ang * f.n_bins + j] = sum;
    }
}

// Transpose: one workgroup per ATW x ATH = 32 x 16 pixel tile, each lane two pixels 16 apart in
// a row (x and x + 16).  For each angle the tile projects onto fewer than AW - 2 consecutive
// bins (its extent sqrt(31^2 + 15^2) < 35 bins); those sinogram windows are staged in LDS, AC
// angles at a time, as pairs (b_j, b_{j+1} - b_j) with zeros outside the detector, and a pixel
// then gathers b_j0 + f (b_j0+1 - b_j0) per angle with one LDS load.  FP32: per (tile, angle)
// the detector coordinate of the tile centre in FP64, split into its floor J and an FP32
// fraction; the lane's first pixel at (dx, dy) from the centre (|dx| <= 15.5, |dy| <= 7.5) is at
// J + t, t = frac + dx cos + dy sin in FP32, the second at t + 16 cos (error below 5e-6 bins),
// and the weights come from floor(t) and fract(t); the window has one bin of margin on each
// side, so a floor one off at an integer stays inside it (and gives the same value).  FP64:
// each lane's first position in FP64 from its own coordinates, the second 16 cos further.
// The windows cover the whole tile, also where it overhangs the frame, so every lane's
// gathers stay inside them; pixels outside the frame are not written.
static constexpr int ATW = 32, ATH = 16;  // pixel tiles of the transpose (parallel beam)
static constexpr int AW = 48, AC = 32;

struct AdjAngle {
    float frac, c, s;
    uint32_t base;   // LDS byte offset of bin J in the angle's window (from the window array)
};

template <class T>
__global__ __launch_bounds__(256) void k_radon_adj(const Tile* __restrict__ tiles, const RadonFrame* __restrict__ rf,
                                                   const double2* __restrict__ trig, const T* __restrict__ b,
                                                   T* __restrict__ u) {
    typedef T P2 __attribute__((ext_vector_type(2)));  // {b_j, b_{j+1} - b_j}
    __shared__ P2 win[AC][AW];
    __shared__ int jlo[AC];
    __shared__ double2 scs[AC];
    __shared__ AdjAngle aa[AC];
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[tl.frame];
    const int lx = (int)(threadIdx.x % 16), ly = (int)(threadIdx.x / 16);
    const int x = tl.x0 + lx, y = tl.y0 + ly;  // the lane's pixels: (x, y) and (x + 16, y)
    const bool in0 = x < f.nx && y < f.ny, in1 = x + 16 < f.nx && y < f.ny;
    const double hx = 0.5 * (f.nx - 1), hy = 0.5 * (f.ny - 1);
    const double X = x - hx, Y = y - hy;
    const double cd = 0.5 * (f.n_bins - 1);
    // corners of the whole tile for the window bounds
    const double X0 = tl.x0 - hx, X1 = tl.x0 + ATW - 1 - hx;
    const double Y0 = tl.y0 - hy, Y1 = tl.y0 + ATH - 1 - hy;
    const T* sino = b + f.sino_off;
    T acc0 = T(0), acc1 = T(0);
    const double XC = tl.x0 + 0.5 * (ATW - 1) - hx, YC = tl.y0 + 0.5 * (ATH - 1) - hy;
    const float dxc = (float)lx - 0.5f * (ATW - 1);
    const float dyc = (float)ly - 0.5f * (ATH - 1);
    for (int k0 = 0; k0 < f.n_ang; k0 += AC) {
        const int nk = min(AC, f.n_ang - k0);
        __syncthreads();  // the previous chunk's windows are no longer read
        if (threadIdx.x < nk) {
            const double2 cs = trig[f.trig_off + k0 + threadIdx.x];
            const double pmin = cd + fmin(X0 * cs.x, X1 * cs.x) + fmin(Y0 * cs.y, Y1 * cs.y);
            const int lo = (int)floor(pmin) - 1;
            jlo[threadIdx.x] = lo;
            scs[threadIdx.x] = cs;
            if constexpr (sizeof(T) == 4) {
                const double pc = fma(XC, cs.x, fma(YC, cs.y, cd));
                const double J = floor(pc);
                aa[threadIdx.x] = AdjAngle{(float)(pc - J), (float)cs.x, (float)cs.y,
                                           (uint32_t)((int)threadIdx.x * AW + (int)J - lo) * (uint32_t)sizeof(P2)};
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nk * AW; i += 256) {
            const int kk = i / AW, w = i % AW;
            const int j = jlo[kk] + w;
            const T* row = sino + (int64_t)(k0 + kk) * f.n_bins;
            const T v0 = (j >= 0 && j < f.n_bins) ? row[j] : T(0);
            const T v1 = (j + 1 >= 0 && j + 1 < f.n_bins) ? row[j + 1] : T(0);
            win[kk][w] = P2{v0, v1 - v0};
        }
        __syncthreads();
        if (!in0) continue;
        if constexpr (sizeof(T) == 4) {
            const char* wb = reinterpret_cast<const char*>(&win[0][0]);
            float a0 = 0.f, d0 = 0.f, a1 = 0.f, d1 = 0.f;
            auto one = [&](int kk) {
                const AdjAngle g = aa[kk];
                const float t0 = fmaf(dxc, g.c, fmaf(dyc, g.s, g.frac));
                const float t1 = fmaf(16.f, g.c, t0);
                int w0, w1;
                asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(w0) : "v"(t0));
                asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(w1) : "v"(t1));
                const float f0 = __builtin_amdgcn_fractf(t0), f1 = __builtin_amdgcn_fractf(t1);
                const P2 q0 = *reinterpret_cast<const P2*>(wb + (g.base + ((uint32_t)w0 << 3)));
                const P2 q1 = *reinterpret_cast<const P2*>(wb + (g.base + ((uint32_t)w1 << 3)));
                a0 += q0.x;
                d0 = fmaf(f0, q0.y, d0);
                a1 += q1.x;
                d1 = fmaf(f1, q1.y, d1);
            };
            int kk = 0;
            for (; kk + 4 <= nk; kk += 4) {
                one(kk);
                one(kk + 1);
                one(kk + 2);
                one(kk + 3);
            }
            for (; kk < nk; ++kk) one(kk);
            acc0 += a0 + d0;
            acc1 += a1 + d1;
        } else {
#pragma unroll 4
            for (int kk = 0; kk < nk; ++kk) {
                const double2 cs = scs[kk];
                const double p0 = fma(X, cs.x, fma(Y, cs.y, cd));
                const double p1 = fma(16.0, cs.x, p0);
                const double fl0 = floor(p0), fl1 = floor(p1);
                const P2 q0 = win[kk][(int)fl0 - jlo[kk]];
                const P2 q1 = win[kk][(int)fl1 - jlo[kk]];
                acc0 += q0.x + (T)(p0 - fl0) * q0.y;
                acc1 += q1.x + (T)(p1 - fl1) * q1.y;
            }
        }
    }
    if (in0) u[f.u_off + (int64_t)y * f.nx + x] = acc0;
    if (in1) u[f.u_off + (int64_t)y * f.nx + x + 16] = acc1;
}

// ----------------------------------------------------------------------------- host side

void radon_plan_init(Ctx& c, Plan& p, const double* cs) {
    Geom& g = *p.geom;
    std::vector<RadonFrame> rfs;
    std::vector<RayTile> rays[4];  // angle groups of 1, 2, 4, 8
    std::vector<Tile> px, tr;
    int64_t sino = 0, trig = 0;
    p.tr_vec = true;
    for (int64_t fi = 0; fi < g.n_frames; ++fi) {
        const FrameInfo& fr = g.frames[fi];
        // the projectors address pixels by 32-bit offsets within a frame
        MMOF_CHECK((int64_t)fr.ny * fr.nx < ((int64_t)1 << 31), MMOF_ERR_SHAPE, "frames must have fewer than 2^31 pixels");
        if (fr.nx % 4 != 0 || fr.ny % 4 != 0 || fr.off % 4 != 0) p.tr_vec = false;
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
        // a frame's angle groups that walk the rows of u, then those that walk the rows of its
        // transpose (a group is placed by its first angle): consecutive tiles, which run together
        // on one XCD (xcd_remap), then read one image, not both
        for (int gi = 0; gi < 4; ++gi) {
            const int ag = 1 << gi;
            for (int pass = 0; pass < 2; ++pass)
                for (int k = 0; k < r.n_ang; k += ag) {
                    const double c0 = cs[2 * (trig + k)], s0 = cs[2 * (trig + k) + 1];
                    if ((std::fabs(s0) > std::fabs(c0)) != (pass == 1)) continue;
                    for (int j0 = 0; j0 < r.n_bins; j0 += 64) rays[gi].push_back(RayTile{(int32_t)fi, k, j0, 0});
                }
        }
        // pixel tiles of the transpose: 32 x 16 for the parallel beam, 16 x 16 for the fan beam
        const int tw = p.kind == 2 ? RTW : ATW, th = p.kind == 2 ? RTH : ATH;
        for (int y0 = 0; y0 < fr.ny; y0 += th)
            for (int x0 = 0; x0 < fr.nx; x0 += tw) px.push_back(Tile{(int32_t)fi, y0, x0, 0});
        for (int y0 = 0; y0 < fr.ny; y0 += 32)
            for (int x0 = 0; x0 < fr.nx; x0 += 32) tr.push_back(Tile{(int32_t)fi, y0, x0, 0});
        sino += (int64_t)r.n_ang * r.n_bins;
        trig += r.n_ang;
        p.radon_flops += 4.0 * (double)fr.ny * fr.nx * r.n_ang;
    }
    p.m = sino;
    p.d_rinfo.ensure(sizeof(RadonFrame) * rfs.size());
    MMOF_HIP(hipMemcpyAsync(p.d_rinfo.ptr, rfs.data(), sizeof(RadonFrame) * rfs.size(), hipMemcpyHostToDevice, c.stream));
    for (int gi = 0; gi < 4; ++gi) {
        p.n_rays[gi] = (int64_t)rays[gi].size();
        p.d_rays[gi].ensure(sizeof(RayTile) * std::max<size_t>(rays[gi].size(), 1));
        if (!rays[gi].empty())
            MMOF_HIP(hipMemcpyAsync(p.d_rays[gi].ptr, rays[gi].data(), sizeof(RayTile) * rays[gi].size(),
                                    hipMemcpyHostToDevice, c.stream));
    }
    p.n_tiles_a = (int64_t)px.size();
    p.d_tiles_a.ensure(sizeof(Tile) * px.size());
    MMOF_HIP(hipMemcpyAsync(p.d_tiles_a.ptr, px.data(), sizeof(Tile) * px.size(), hipMemcpyHostToDevice, c.stream));
    p.n_tiles_b = (int64_t)tr.size();
    p.d_tiles_b.ensure(sizeof(Tile) * tr.size());
    MMOF_HIP(hipMemcpyAsync(p.d_tiles_b.ptr, tr.data(), sizeof(Tile) * tr.size(), hipMemcpyHostToDevice, c.stream));
    MMOF_HIP(hipStreamSynchronize(c.stream));
}

// ---------------------------------------------------------------- fan beam
//
// Flat-detector fan beam by Joseph's method.  Angle theta: detector axis a = (cos, sin),
// central ray e = (-sin, cos), source S = -dso e, ray j along d_j = dsd e + u_j a with
// u_j = (j - (n_d-1)/2) du.  A ray with |d_y| >= |d_x| is sampled on every pixel row at
// X_c(Y) = S_x + (Y - S_y) d_x / d_y by linear interpolation between the two pixels around
// it (out-of-frame pixels are 0), each sample weighted by the path length per row
// |d| / |d_y|; other rays on the columns.  Forward: one lane per ray (four angles x 64 bins
// per workgroup), column-stepping rays read the transposed frame so that the lanes stay on
// neighbouring addresses.  Transpose: one lane per pixel; per angle, the rays that can
// sample the pixel are those whose detector coordinate lies between the projections of its
// row neighbours (X -+ 1, Y) or of its column neighbours (X, Y -+ 1); each candidate ray's
// weight on the pixel is recomputed exactly as the forward computes it.

struct FanGeo {
    double dso, dsd, du;
};

// Source and direction of ray j (no contraction: the row / column choice is taken on values
// rounded exactly like plain double arithmetic).
__device__ __forceinline__ void fan_ray(double c, double s, int j, int nb, const FanGeo& g, double& sx, double& sy,
                                        double& dx, double& dy) {
#pragma clang fp contract(off)
    const double uj = ((double)j - (nb - 1) / 2.0) * g.du;
    dx = -g.dsd * s + uj * c;
    dy = g.dsd * c + uj * s;
    sx = g.dso * s;
    sy = -g.dso * c;
}

// Per-ray table, built once per plan in the sinogram layout: {A, B, step, dir} with the
// sample position of the ray on row y (dir > 0: |d_y| >= |d_x|) x_c = A + B y, or on column
// x (dir < 0) y_c = A + B x, in pixel-index coordinates, and the path length per step.  Both
// the forward and the transpose evaluate positions as fma(B, index, A) from this table, so
// their weights are the same numbers.
__global__ __launch_bounds__(256) void k_fan_rays(const RayTile* __restrict__ rays, const RadonFrame* __restrict__ rf,
                                                  const double2* __restrict__ trig, FanGeo geo,
                                                  double4* __restrict__ table) {
    const RayTile rt = rays[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[rt.frame];
    const int k = rt.angle + (int)threadIdx.x / 64, j = rt.bin0 + (int)threadIdx.x % 64;
    if (k >= f.n_ang || j >= f.n_bins) return;
    const double2 cs = trig[f.trig_off + k];
    double sx, sy, dx, dy;
    fan_ray(cs.x, cs.y, j, f.n_bins, geo, sx, sy, dx, dy);
    const double cx = (f.nx - 1) / 2.0, cy = (f.ny - 1) / 2.0;
    double4 e;
    if (fabs(dy) >= fabs(dx)) {
        e.y = dx / dy;
        e.x = sx + (-cy - sy) * e.y + cx;
        e.z = sqrt(dx * dx + dy * dy) / fabs(dy);
        e.w = 1.0;
    } else {
        e.y = dy / dx;
        e.x = sy + (-cx - sx) * e.y + cy;
        e.z = sqrt(dx * dx + dy * dy) / fabs(dx);
        e.w = -1.0;
    }
    table[f.sino_off + (int64_t)k * f.n_bins + j] = e;
}

template <class T>
__global__ __launch_bounds__(256) void k_fan_fwd(const RayTile* __restrict__ rays, const RadonFrame* __restrict__ rf,
                                                 const double4* __restrict__ table, const T* __restrict__ u,
                                                 const T* __restrict__ ut, T* __restrict__ b) {
    const RayTile rt = rays[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[rt.frame];
    const int k = rt.angle + (int)threadIdx.x / 64, j = rt.bin0 + (int)threadIdx.x % 64;
    if (k >= f.n_ang || j >= f.n_bins) return;
    const int64_t ri = f.sino_off + (int64_t)k * f.n_bins + j;
    const double4 e = table[ri];
    // rows: samples along x of row y; columns: along y of column x (transposed frame)
    const bool rows = e.w > 0.0;
    const int nsteps = rows ? f.ny : f.nx, nline = rows ? f.nx : f.ny;
    const T* img = rows ? u + f.u_off : ut + f.u_off;
    T acc = T(0);
    for (int q = 0; q < nsteps; ++q) {
        const double pc = fma(e.y, (double)q, e.x);
        const double p0d = floor(pc);
        if (p0d < -1.0 || p0d > (double)nline) continue;
        const T fr = (T)(pc - p0d);
        const int p0 = (int)p0d;
        const T* line = img + (int64_t)q * nline;
        if (p0 >= 0 && p0 + 1 < nline) {  // both pixels inside: one 2-element load
            const Pair<T> pr = ld2(line + p0);
            acc += (T(1) - fr) * pr.a;
            acc += fr * pr.b;
        } else {
            if (p0 >= 0 && p0 < nline) acc += (T(1) - fr) * line[p0];
            if (p0 + 1 >= 0 && p0 + 1 < nline) acc += fr * line[p0 + 1];
        }
    }
    b[ri] = acc * (T)e.z;
}

// Detector position (in bin units) of the ray from the source through the point (X, Y); the
// reciprocal of the depth from the hardware FP32 reciprocal and two Newton steps (relative
// error near FP64 rounding, no FP64 division): it only bounds candidate rays (margin 0.05 bins).
__device__ __forceinline__ double fan_pos_bound(double X, double Y, double c, double s, double dso, double g,
                                                double off) {
    const double t = X * c + Y * s, den = dso - X * s + Y * c;
    double inv = (double)__builtin_amdgcn_rcpf((float)den);
    inv = inv * (2.0 - den * inv);
    inv = inv * (2.0 - den * inv);
    return g * t * inv + off;
}

// Detector position in FP32 (bounds only; the caller's margin covers its rounding, the
// hardware reciprocal's 1 ulp included).
__device__ __forceinline__ float fan_pos_f32(float t, float den, float g, float off) {
    return fmaf(g * t, __builtin_amdgcn_rcpf(den), off);
}

constexpr int FAC = 16;  // angles per staged chunk of the transpose
constexpr int FAW = 64;  // staged bins per angle (wider tile windows read the table directly)

// Transpose: one lane per pixel of a 16 x 16 tile.  Per chunk of FAC angles, the bins whose
// rays can touch the tile (between the projections of the corners of the tile grown by one
// pixel: the projection is monotone along every line that misses the source, so its extremes
// over the box are at the corners) are staged in LDS: the line {A, B}, the path length signed
// by the direction (> 0: rows) and the sinogram value.  Per angle a pixel's candidates lie
// between the projections of its four neighbours, taken in FP32 with the caller's margin
// (bins) when FP32_BOUNDS, else in FP64; a window wider than FAW bins reads the table from
// global memory instead.  Every candidate's weight is the forward's: fma(B, index, A) in FP64.
template <class T, bool FP32_BOUNDS>
__global__ __launch_bounds__(256) void k_fan_adj(const Tile* __restrict__ tiles, const RadonFrame* __restrict__ rf,
                                                 const double2* __restrict__ trig, const double4* __restrict__ table,
                                                 const T* __restrict__ b, T* __restrict__ u, FanGeo geo,
                                                 float margin) {
    __shared__ double2 s_ab[FAC][FAW];
    __shared__ T s_sb[FAC][FAW][2];  // {signed path length, sinogram value}
    __shared__ int s_j0[FAC], s_cnt[FAC];
    const Tile tl = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const RadonFrame f = rf[tl.frame];
    const int x = tl.x0 + (int)threadIdx.x % RTW, y = tl.y0 + (int)threadIdx.x / RTW;
    const bool inside = x < f.nx && y < f.ny;
    const double hx = (f.nx - 1) / 2.0, hy = (f.ny - 1) / 2.0;
    const double X = x - hx, Y = y - hy, xd = x, yd = y;
    const int nb = f.n_bins;
    const double gsc = geo.dsd / geo.du, off = (nb - 1) / 2.0;
    const float Xf = (float)X, Yf = (float)Y, gf = (float)gsc, offf = (float)off, dsof = (float)geo.dso;
    // the tile grown by one pixel (clipped to the frame first)
    const double Xa = tl.x0 - hx - 1.0, Xb = min(tl.x0 + RTW, f.nx) - hx, Ya = tl.y0 - hy - 1.0,
                 Yb = min(tl.y0 + RTH, f.ny) - hy;
    T acc = T(0);
    for (int k0 = 0; k0 < f.n_ang; k0 += FAC) {
        const int nk = min(FAC, f.n_ang - k0);
        __syncthreads();  // the previous chunk is no longer read
        if (threadIdx.x < nk) {
            const double2 cs = trig[f.trig_off + k0 + threadIdx.x];
            const double q0 = fan_pos_bound(Xa, Ya, cs.x, cs.y, geo.dso, gsc, off);
            const double q1 = fan_pos_bound(Xb, Ya, cs.x, cs.y, geo.dso, gsc, off);
            const double q2 = fan_pos_bound(Xa, Yb, cs.x, cs.y, geo.dso, gsc, off);
            const double q3 = fan_pos_bound(Xb, Yb, cs.x, cs.y, geo.dso, gsc, off);
            const double lo = fmin(fmin(q0, q1), fmin(q2, q3)), hi = fmax(fmax(q0, q1), fmax(q2, q3));
            const int j0 = (int)fmin(fmax(ceil(lo - 0.05), 0.0), (double)nb);
            const int j1 = (int)fmax(fmin(floor(hi + 0.05), (double)(nb - 1)), -1.0);
            const int cnt = max(j1 - j0 + 1, 0);
            s_j0[threadIdx.x] = j0;
            s_cnt[threadIdx.x] = cnt <= FAW ? cnt : -1;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nk * FAW; i += 256) {
            const int kk = i / FAW, w = i % FAW;
            if (w < s_cnt[kk]) {
                const int64_t ri = f.sino_off + (int64_t)(k0 + kk) * nb + s_j0[kk] + w;
                const double4 e = table[ri];
                s_ab[kk][w] = make_double2(e.x, e.y);
                s_sb[kk][w][0] = e.w > 0.0 ? (T)e.z : -(T)e.z;
                s_sb[kk][w][1] = b[ri];
            }
        }
        __syncthreads();
        if (!inside) continue;
        for (int kk = 0; kk < nk; ++kk) {
            const int cnt = s_cnt[kk];
            if (cnt == 0) continue;
            const int k = k0 + kk;
            const double2 cs = trig[f.trig_off + k];
            // candidate bins: ray j lies at detector position j, and it can weigh on the
            // pixel only strictly between the neighbours' projections (clamped to the
            // detector, and to the staged window, before the conversion to int)
            int jlo, jhi;
            if (FP32_BOUNDS) {
                const float c = (float)cs.x, sn = (float)cs.y;
                const float t0 = fmaf(Xf, c, Yf * sn), d0 = dsof - Xf * sn + Yf * c;
                const float p0 = fan_pos_f32(t0 - c, d0 + sn, gf, offf), p1 = fan_pos_f32(t0 + c, d0 - sn, gf, offf);
                const float p2 = fan_pos_f32(t0 - sn, d0 - c, gf, offf), p3 = fan_pos_f32(t0 + sn, d0 + c, gf, offf);
                const float lo = fminf(fminf(p0, p1), fminf(p2, p3)) - margin;
                const float hi = fmaxf(fmaxf(p0, p1), fmaxf(p2, p3)) + margin;
                jlo = (int)fminf(fmaxf(ceilf(lo), 0.0f), (float)nb);
                jhi = (int)fmaxf(fminf(floorf(hi), (float)(nb - 1)), -1.0f);
            } else {
                const double p0 = fan_pos_bound(X - 1.0, Y, cs.x, cs.y, geo.dso, gsc, off);
                const double p1 = fan_pos_bound(X + 1.0, Y, cs.x, cs.y, geo.dso, gsc, off);
                const double p2 = fan_pos_bound(X, Y - 1.0, cs.x, cs.y, geo.dso, gsc, off);
                const double p3 = fan_pos_bound(X, Y + 1.0, cs.x, cs.y, geo.dso, gsc, off);
                const double lo = fmin(fmin(p0, p1), fmin(p2, p3)) - 0.05;
                const double hi = fmax(fmax(p0, p1), fmax(p2, p3)) + 0.05;
                jlo = (int)fmin(fmax(ceil(lo), 0.0), (double)nb);
                jhi = (int)fmax(fmin(floor(hi), (double)(nb - 1)), -1.0);
            }
            if (cnt > 0) {
                const int j0 = s_j0[kk];
                jlo = max(jlo, j0);
                jhi = min(jhi, j0 + cnt - 1);
                for (int j = jlo; j <= jhi; ++j) {
                    const double2 ab = s_ab[kk][j - j0];
                    const T sp = s_sb[kk][j - j0][0], bv = s_sb[kk][j - j0][1];
                    const bool rows = sp > T(0);
                    const double pc = fma(ab.y, rows ? yd : xd, ab.x);
                    const double p0d = floor(pc);
                    const T fr = (T)(pc - p0d);
                    // the pixel is the sample's left (dl = 0) or right (dl = 1) neighbour, or
                    // untouched (exact: small integers)
                    const double dl = (rows ? xd : yd) - p0d;
                    const T w = dl == 0.0 ? T(1) - fr : (dl == 1.0 ? fr : T(0));
                    const T term = (w * (rows ? sp : -sp)) * bv;
                    acc = w != T(0) ? acc + term : acc;
                }
            } else {
                const int64_t row = f.sino_off + (int64_t)k * nb;
                for (int j = jlo; j <= jhi; ++j) {
                    const double4 e = table[row + j];
                    const bool rows = e.w > 0.0;
                    const double pc = fma(e.y, rows ? (double)y : (double)x, e.x);
                    const double p0d = floor(pc);
                    const T fr = (T)(pc - p0d);
                    const double own = rows ? (double)x : (double)y;
                    T w = T(0);
                    if (p0d == own) w = T(1) - fr;
                    else if (p0d + 1.0 == own) w = fr;
                    if (w != T(0)) acc += (w * (T)e.z) * b[row + j];
                }
            }
        }
    }
    if (inside) u[f.u_off + (int64_t)y * f.nx + x] = acc;
}

void fan_plan_init(Ctx& c, Plan& p) {
    p.d_fanrays.ensure(sizeof(double4) * (size_t)std::max<int64_t>(p.m, 1));
    if (p.n_rays[2] == 0) return;
    const FanGeo geo{p.fan_dso, p.fan_dsd, p.fan_du};
    hipLaunchKernelGGL(k_fan_rays, dim3((unsigned)p.n_rays[2]), dim3(256), 0, c.stream, p.d_rays[2].as<RayTile>(),
                       p.d_rinfo.as<RadonFrame>(), p.d_trig.as<double2>(), geo, p.d_fanrays.as<double4>());
    MMOF_LAUNCH_CHECK();
    MMOF_HIP(hipStreamSynchronize(c.stream));
}

// ut = the per-frame transpose of u (16-byte accesses when the stack allows them)
template <class T>
static void launch_transpose(Ctx& c, Plan& p, const T* u, T* ut) {
    if (p.tr_vec && aligned_to(16, {u, ut}))
        hipLaunchKernelGGL(k_transpose_frames4<T>, dim3((unsigned)p.n_tiles_b), dim3(256), 0, c.stream,
                           p.d_tiles_b.as<Tile>(), p.d_rinfo.as<RadonFrame>(), u, ut);
    else
        hipLaunchKernelGGL(k_transpose_frames<T>, dim3((unsigned)p.n_tiles_b), dim3(256), 0, c.stream,
                           p.d_tiles_b.as<Tile>(), p.d_rinfo.as<RadonFrame>(), u, ut);
    MMOF_LAUNCH_CHECK();
}

void launch_fan_fwd(Ctx& c, Plan& p, int dt, const void* u, void* b) {
    if (p.n_rays[2] == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        T* ut = static_cast<T*>(c.work("radon_transpose", sizeof(T) * p.n));
        launch_transpose<T>(c, p, (const T*)u, ut);
        ScopedTime st(&c, "fan_fwd", (double)sizeof(T) * (p.n + p.m), 0.0);
        hipLaunchKernelGGL(k_fan_fwd<T>, dim3((unsigned)p.n_rays[2]), dim3(256), 0, c.stream,
                           p.d_rays[2].as<RayTile>(), p.d_rinfo.as<RadonFrame>(), p.d_fanrays.as<double4>(),
                           (const T*)u, (const T*)ut, (T*)b);
        MMOF_LAUNCH_CHECK();
    });
}

// Margin (bins) that covers the rounding of the FP32 candidate bounds: with every point at
// most R from the centre, |t| <= R and den >= dso - R; each of t and den is off by at most a few
// FP32 ulps of dso + R, and the position g t / den + off by the propagated relative errors; a
// factor 4 on top, plus the FP64 path's 0.05.  Geometries where this exceeds 0.5 bins take the
// FP64 bounds.
static float fan_bound_margin(const Plan& p, bool& fp32) {
    const Geom& g = *p.geom;
    double R = 0.0;
    int nbmax = 1;
    for (int s = 0; s < g.n_seq; ++s) {
        R = std::max(R, 0.5 * std::hypot((double)g.nx[s], (double)g.ny[s]) + 1.5);
        nbmax = std::max(nbmax, p.n_bins[s]);
    }
    const double dmin = p.fan_dso - R, gsc = p.fan_dsd / p.fan_du, u = std::ldexp(1.0, -24);
    const double ea = 16.0 * u * (p.fan_dso + R + 2.0);  // absolute error of t and den
    const double pos = gsc * R / dmin;                   // |g t / den|
    const double err = gsc * ea / dmin + pos * (ea / dmin + 8.0 * u) + 4.0 * u * (pos + 0.5 * nbmax);
    const double m = 0.05 + 4.0 * err;
    fp32 = dmin > 0.0 && m <= 0.5;
    return (float)m;
}

void launch_fan_adj(Ctx& c, Plan& p, int dt, const void* b, void* u) {
    const FanGeo geo{p.fan_dso, p.fan_dsd, p.fan_du};
    bool fp32 = false;
    const float margin = fan_bound_margin(p, fp32);
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        ScopedTime st(&c, "fan_adj", (double)sizeof(T) * (p.n + p.m), 0.0);
        auto kern = fp32 ? k_fan_adj<T, true> : k_fan_adj<T, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)p.n_tiles_a), dim3(256), 0, c.stream, p.d_tiles_a.as<Tile>(),
                           p.d_rinfo.as<RadonFrame>(), p.d_trig.as<double2>(), p.d_fanrays.as<double4>(),
                           (const T*)b, (T*)u, geo, margin);
        MMOF_LAUNCH_CHECK();
    });
}

const int kRadonCandidates = 4;  // angle groups of 1, 2, 4, 8 per workgroup

int radon_fwd_choice(Plan& p, int dt) {
    auto it = p.geom->tuned.find(std::string("radon_fwd") + (dt == MMOF_F32 ? "/f32" : "/f64"));
    if (it != p.geom->tuned.end()) return it->second;
    // untuned: one angle per workgroup (more workgroups) on large frames, pairs on small ones
    return p.geom->max_ny >= 512 ? 0 : 1;
}

void launch_radon_fwd(Ctx& c, Plan& p, int dt, const void* u, void* b, int choice) {
    if (choice < 0) choice = radon_fwd_choice(p, dt);
    MMOF_CHECK(choice >= 0 && choice < kRadonCandidates, MMOF_ERR_INVALID, "radon_fwd candidate out of range");
    if (p.n_rays[choice] == 0) return;
    dispatch(dt, [&](auto z) {
        using T = decltype(z);
        T* ut = static_cast<T*>(c.work("radon_transpose", sizeof(T) * p.n));
        launch_transpose<T>(c, p, (const T*)u, ut);
        ScopedTime st(&c, "radon_fwd", (double)sizeof(T) * (p.n + p.m), p.radon_flops);
        auto k = choice == 0 ? k_radon_fwd<T, 1> : choice == 1 ? k_radon_fwd<T, 2> : choice == 2 ? k_radon_fwd<T, 4>
                                                                                                 : k_radon_fwd<T, 8>;
        hipLaunchKernelGGL(k, dim3((unsigned)p.n_rays[choice]), dim3(512), 0, c.stream, p.d_rays[choice].as<RayTile>(),
                           p.d_rinfo.as<RadonFrame>(), p.d_trig.as<double2>(), (const T*)u, (const T*)ut, (T*)b);
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
