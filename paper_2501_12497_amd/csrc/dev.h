// Device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace mmof {

// Block id -> work item such that consecutive work items land on the same XCD.
// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8); this
// gives XCD x the contiguous range of items [x*q + min(x,r), ...) so neighbouring
// tiles of one frame share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n) {
    const int64_t q = n >> 3, r = n & 7;
    const int64_t x = b & 7, s = b >> 3;
    return x * q + (x < r ? x : r) + s;
}

// Clipped floor/fraction of the sample coordinate x + v for an integer pixel x:
// returns x0 in [0, n-1] and f in [0, 1) with x0 + f = clip(x + v, 0, n-1).  The
// fraction is v - floor(v) (exact in the working precision), so no large-number
// cancellation enters the bilinear weights.
template <class T>
__device__ __forceinline__ void clip_cell(int x, T v, int n, int& x0, T& f, bool& clipped) {
    v = fmin(fmax(v, T(-1048576)), T(1048576));  // keeps the int conversion defined (NaN -> low bound)
    T fv = floor(v);
    int xr = x + (int)fv;
    f = v - fv;
    clipped = false;
    if (xr < 0) {
        x0 = 0;
        f = T(0);
        clipped = true;
    } else if (xr >= n - 1) {
        clipped = (xr > n - 1) || (f > T(0));
        x0 = n - 1;
        f = T(0);
    } else {
        x0 = xr;
    }
}

// rint(x + v) (round half to even) for an integer x, computed exactly: the fraction
// v - floor(v) is exact, and a tie is resolved on the parity of x + floor(v).
template <class T>
__device__ __forceinline__ int rint_shift(int x, T v) {
    v = fmin(fmax(v, T(-1048576)), T(1048576));
    const T fv = floor(v);
    const T fr = v - fv;
    int n = x + (int)fv;
    if (fr > T(0.5) || (fr == T(0.5) && (n & 1))) ++n;
    return n;
}

// Nearest pixel (ties to even) of x + v, clipped into [0, n-1].
template <class T>
__device__ __forceinline__ int round_clip(int x, T v, int n) {
    const int r = rint_shift(x, v);
    return r < 0 ? 0 : (r > n - 1 ? n - 1 : r);
}

// Two consecutive values loaded by one instruction from an address aligned to one element
// (global memory accepts element-aligned multi-word loads).
template <class T>
struct Pair {
    T a, b;
};
template <class T>
__device__ __forceinline__ Pair<T> ld2(const T* p) {
    typedef T V2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
    const V2 v = *reinterpret_cast<const V2*>(p);
    return Pair<T>{v.x, v.y};
}

// Four consecutive values moved as one 16-byte (FP32) or two 16-byte (FP64) accesses; the
// address must be aligned to 4 elements.
template <class T>
struct alignas(4 * sizeof(T)) Quad {
    T v[4];
};
template <class T>
__device__ __forceinline__ Quad<T> ld4(const T* p) {
    return *reinterpret_cast<const Quad<T>*>(p);
}
template <class T>
__device__ __forceinline__ void st4(T* p, const Quad<T>& q) {
    *reinterpret_cast<Quad<T>*>(p) = q;
}
// The same four values from an address aligned to one element (global multi-word accesses
// accept it), and the first nv of them (nv < 4: the rest read as zero / are not written).
template <class T>
__device__ __forceinline__ Quad<T> ld4u(const T* p) {
    typedef T V4 __attribute__((ext_vector_type(4), aligned(sizeof(T))));
    const V4 v = *reinterpret_cast<const V4*>(p);
    return Quad<T>{{v.x, v.y, v.z, v.w}};
}
template <class T>
__device__ __forceinline__ void st4u(T* p, const Quad<T>& q) {
    typedef T V4 __attribute__((ext_vector_type(4), aligned(sizeof(T))));
    *reinterpret_cast<V4*>(p) = V4{q.v[0], q.v[1], q.v[2], q.v[3]};
}
template <class T>
__device__ __forceinline__ Quad<T> ld4n(const T* p, int nv) {
    if (nv >= 4) return ld4u(p);
    Quad<T> q;
#pragma unroll
    for (int j = 0; j < 4; ++j) q.v[j] = j < nv ? p[j] : T(0);
    return q;
}
template <class T>
__device__ __forceinline__ void st4n(T* p, const Quad<T>& q, int nv) {
    if (nv >= 4) {
        st4u(p, q);
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (j < nv) p[j] = q.v[j];
}
template <class T>
__device__ __forceinline__ Quad<T> zero4() {
    return Quad<T>{{T(0), T(0), T(0), T(0)}};
}

// Half-sample-symmetric mirror of an index into [0, n): -1 -> 0, n -> n-1.
__device__ __forceinline__ int mirror(int i, int n) {
    if (i < 0) i = -i - 1;
    if (i >= n) i = 2 * n - i - 1;
    return i;
}

// The MM weight 1/sqrt(nu^2 + eps^2) (eps > 0) in FP64, the one formula of every weight path
// (the buffer, the Gram, the residual's weighting and the Theta kernels that fuse it): the
// hardware reciprocal square root (relative error below 2^-22) refined by two Newton steps
// r <- r (3 - x r^2) / 2, each of which squares the relative error, so the result is within a
// few ulp of the rounded value; a sum too large for the refinement takes the division.
__device__ __forceinline__ double mm_weight(double a, double eps2) {
    const double x = fma(a, a, eps2);
    if (!(x < 1.0e300)) return 1.0 / sqrt(x);
    const double h = 0.5 * x;
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(-h * r, r, 1.5);
    r = r * fma(-h * r, r, 1.5);
    return r;
}

// A row value weighted by the MM weight of its nu, rounded to the row type.
template <class T>
__device__ __forceinline__ T mm_weighted(T y, T nu, double eps2) {
    return (T)((double)y * mm_weight((double)nu, eps2));
}

}  // namespace mmof
