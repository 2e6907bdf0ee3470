// Host launchers of the FP64 Krylov kernels and the small projected solve.
#pragma once

#include "common.h"

namespace mmof {

static constexpr int KMAX = 256;        // largest Krylov basis (columns of V)
static constexpr int KLD = 256;         // leading dimension of the projected matrices G_H, G_T
static constexpr int KMAX_SMALL = 64;   // largest basis of the one-wave projected solve (and of
                                        // the allocation-free Gram)

// out[j] = alpha * X_j^T y for j < K (X column-major [K][ld]); one launch.
template <class TX, class TY>
void mdot(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TY* y, double alpha, double* out);
// Row and column j of a Gram matrix and one more inner product, in one launch:
// G[j][k] = G[k][j] = X_k^T X_j (k <= j), dj[0] = X_j^T e.
template <class TX>
void gram_row(Ctx& c, int64_t n, int j, const TX* X, int64_t ld, const double* e, double* G, int ldg, double* dj);
// out = beta*out + alpha * X h
template <class TX>
void gemv_cols(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* h, double alpha, double beta,
               double* out);
// v = alpha * X h + beta * y (y may be null, and may alias out_d), in one launch:
// out_d = v (FP64, may be null), out_t = v rounded to TO (may be null), and, when sq is not
// null, sq[0] = sum_i (v_i - cv_i)^2 (cv may be null: sum of v_i^2).
template <class TX, class TO>
void gemv_fused(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* h, double alpha, const double* y,
                double beta, double* out_d, TO* out_t, const double* cv, double* sq);
// The middle step of classical Gram-Schmidt with reorthogonalisation, in one pass over Q:
// y = x - Q h and hout = Q^T y, FP64 (Q column-major [K][ld], K <= 64; y must not alias x;
// hout may alias h).
void gemv_mdot(Ctx& c, int64_t n, int K, const double* Q, int64_t ld, const double* h, const double* x, double* y,
               double* hout);
// Classical Gram-Schmidt of x against the K orthonormal FP64 columns of Q (column-major
// [K][ld]), x <- x - Q (Q^T x), followed by a second such pass only when the first kept less
// than 1/sqrt(2) of ||x|| (Kahan's test: otherwise one pass already leaves x orthogonal to Q
// to working precision).  The test runs on the device: the second pass's launches return at
// once when it is not needed, so nothing waits for the host.  sq[0] = ||x||^2 afterwards;
// h: device scratch of K + 1 doubles.
void cgs_once(Ctx& c, int64_t n, int K, const double* Q, int64_t ld, double* x, double* sq, double* h);
// Implicit basis: the orthonormal basis is V = Vs T, Vs the stored FP64 columns and T unit upper
// triangular (device, column-major, leading dimension KLD; column j holds the coefficients of
// v_j in Vs).  basis_identity: T's first K0 columns = those of the identity.
void basis_identity(Ctx& c, int K0, double* T);
// Extends the basis by the direction of r: h = Vs^T r and ||r||^2 in one pass over Vs (h:
// device scratch of K + 1 doubles), g = T^T h = V^T r, rho^2 = ||r||^2 - ||g||^2 into sq[0],
// and column K of T = e_K - T g / rho, so that v_K = r / rho - V g / rho; the caller then
// stores r / rho as column K of Vs.  When r keeps less than 1/sqrt(2) of its norm outside the
// basis, r <- r - V g explicitly and h is formed again first (decided on the device; the
// launches of that pass return at once otherwise).  K < KMAX.
void basis_extend(Ctx& c, int64_t n, int K, const double* Vs, int64_t ld, double* r, double* T, double* h,
                  double* sq);
// G = T^T Gs T (K x K, leading dimension KLD, written symmetric) and, when ds is not null,
// d = T^T ds.
void basis_gram(Ctx& c, int K, const double* T, const double* Gs, const double* ds, double* G, double* d);
// zt = T z: the coefficients in Vs of V z.
void basis_coef(Ctx& c, int K, const double* T, const double* z, double* zt);
// s = sqrt(s2[0]) (written to s1 when not null); out_d = x / s and out_t = (TO)(x / s)
// (a zero vector when s = 0).
template <class TO>
void normalize2(Ctx& c, int64_t n, const double* x, const double* s2, double* s1, double* out_d, TO* out_t);
// out = (double)in + sign * s[0] * q
template <class TX>
void axpy_conv(Ctx& c, int64_t n, const TX* in, const double* q, const double* s, double sign, double* out);
// w[i] = 1/sqrt(nu[i]^2 + eps^2) in FP64
template <class TX>
void mm_weights_f64(Ctx& c, int64_t n, const TX* nu, double eps, double* w);
// G (K x K, leading dim ldg) = X^T diag(w) X   (w == null: unweighted), FP64 on the matrix cores
// (v_mfma_f64_4x4x4f64 in 4-column quads for K <= 40, 16-column blocks above)
template <class TX>
void wgram(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* w, double* G, int ldg);
// The same Gram with the weights formed in the kernel from nu, 1/sqrt(nu^2 + eps^2) with the
// arithmetic of mm_weights_f64 (K <= KMAX_SMALL): no weight buffer is written or read.
template <class TX>
void wgram_nu(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TX* nu, double eps, double* G, int ldg);
// The same Gram without device allocation: weights formed in the kernel from nu (null: 1),
// partials in a file-scope device array (noalloc_scratch_bytes() of it) whose address on the
// device was looked up by noalloc_init(device) with that device current.
void noalloc_init(int device);
size_t noalloc_scratch_bytes();
template <class TX>
void wgram_noalloc(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TX* nu, double eps, double* G, int ldg);
template <class TI, class TO>
void convert(Ctx& c, int64_t n, const TI* in, TO* out);
void normalize(Ctx& c, int64_t n, const double* x, const double* nrm, double thr, double* out);
void axpby(Ctx& c, int64_t n, double a, const double* x, double b, const double* y, double* out);
template <class TX>
void residual_combine(Ctx& c, int64_t n, const TX* x, const TX* y, const double* lam, double* out);
template <class TX>
void weight_apply(Ctx& c, int64_t n, const TX* nu, double eps, const double* x, TX* y);
void sub(Ctx& c, int64_t n, const double* x, const double* y, double* d);
template <class T>
void fill_zero(Ctx& c, int64_t n, T* p);
void set_scalar(Ctx& c, double* p, double v);
void copy_scalar(Ctx& c, double* dst, const double* src);
void sqrt_scalar(Ctx& c, const double* in, double* out);
// y += sign * s[0] * x  (s on the device)
void axpy_dev(Ctx& c, int64_t n, const double* x, double* y, const double* s, double sign);
// G[j][0..j] and G[0..j][j] <- h[0..j]
void put_rowcol(Ctx& c, double* G, int ldg, int j, const double* h);
// y = w * x
template <class TX>
void weight_mul(Ctx& c, int64_t n, const double* w, const TX* x, TX* y);
// y = w * x with w = 1/sqrt(nu^2 + eps^2) formed from nu (the arithmetic of mm_weights_f64)
template <class TX>
void weight_mul_nu(Ctx& c, int64_t n, const TX* nu, double eps, const TX* x, TX* y);

// Small projected solve (one wavefront for K <= 64, four above).  Inputs on the device: GA, GT
// (K x K, leading dimension KLD),
// d (K), and the scalars bb = ||b||^2 and target = (eta*delta)^2 in sc[0..1].
// Writes z (K), and res[0] = lambda, res[1] = discrepancy^2, res[2] = status (0 root, 2 clamped,
// 4 factorization failure), res[3] = factorizations done.  fixed_lambda > 0 skips the
// discrepancy principle.  sc[2] is the warm start (previous lambda, 0: none); when
// lam_out is not null the chosen lambda is also written there.
void small_solve(Ctx& c, int K, const double* GA, const double* GT, const double* d, const double* sc,
                 double fixed_lambda, double* z, double* res, double* lam_out = nullptr);

}  // namespace mmof
