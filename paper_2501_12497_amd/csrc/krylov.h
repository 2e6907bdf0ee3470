// Host launchers of the FP64 Krylov kernels and the small projected solve.
#pragma once

#include "common.h"

namespace mmof {

static constexpr int KMAX_SMALL = 64;  // largest Krylov basis handled by the small solve

// out[j] = alpha * X_j^T y for j < K (X column-major [K][ld]).
template <class TX, class TY>
void mdot(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const TY* y, double alpha, double* out);
// out = beta*out + alpha * X h
template <class TX>
void gemv_cols(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* h, double alpha, double beta,
               double* out);
// w[i] = 1/sqrt(nu[i]^2 + eps^2) in FP64
template <class TX>
void mm_weights_f64(Ctx& c, int64_t n, const TX* nu, double eps, double* w);
// G (K x K, leading dim ldg) = X^T diag(w) X   (w == null: unweighted), FP64 on the matrix cores
template <class TX>
void wgram(Ctx& c, int64_t n, int K, const TX* X, int64_t ld, const double* w, double* G, int ldg);
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

// Small projected solve (one wavefront).  Inputs on the device: GA, GT (K x K, ld KMAX_SMALL),
// d (K), and the scalars bb = ||b||^2 and target = (eta*delta)^2 in sc[0..1].
// Writes z (K), and res[0] = lambda, res[1] = discrepancy^2, res[2] = status (0 root, 2 clamped,
// 4 factorization failure).  fixed_lambda > 0 skips the discrepancy principle.
void small_solve(Ctx& c, int K, const double* GA, const double* GT, const double* d, const double* sc,
                 double fixed_lambda, double* z, double* res);

}  // namespace mmof
