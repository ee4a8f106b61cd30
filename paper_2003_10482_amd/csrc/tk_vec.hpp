// Batched FP64 vector kernels of the dual solve.
#pragma once

#include "tk_common.hpp"

namespace tk {

constexpr int kMaxCoefs = 64;   // vectors per launch of a coefficient-carrying kernel

struct Coefs {
    double c[kMaxCoefs];
};

// grad_b = g_b + lam_b alpha_b - y_b, stats_b = [a.g, a.a, y.a, grad.grad]; y_b = y + b * y_stride
hipError_t vec_grad(const double *g, const double *alpha, const double *y, const Coefs &lam,
                    double *grad, double *stats, int64_t B, int64_t n, hipStream_t st, int64_t y_stride = 0);
// logistic loss: grad, Hessian diagonal of the separable term, stats_b = [a.g, a.a, S, grad.grad]
hipError_t vec_grad_logistic(const double *g, const double *alpha, const double *y, int64_t y_stride,
                             const Coefs &lam, double *grad, double *hdiag, double *stats, int64_t B, int64_t n,
                             hipStream_t st);
// largest step keeping lam_b y (alpha_b + t x_b) in [0, 1] (logistic domain)
hipError_t vec_step_cap(const double *alpha, const double *x, const double *y, int64_t y_stride, const Coefs &lam,
                        double *out, int64_t B, int64_t n, hipStream_t st);
// alpha_b = y_b / (2 lam_b)
hipError_t vec_logistic_start(const double *y, int64_t y_stride, const Coefs &lam, double *alpha, int64_t B,
                              int64_t n, hipStream_t st);
// *flag |= 1 when a label is not -1 or +1
hipError_t vec_check_labels(const double *y, int64_t len, int *flag, hipStream_t st);
// count_b = changed entries of mask row b since prev; prev = cur
hipError_t vec_mask_diff(const uint8_t *cur, uint8_t *prev, int64_t B, int64_t d, int *count, hipStream_t st);
hipError_t vec_dot(const double *x, const double *y, int64_t y_stride, double *out, int64_t B,
                   int64_t n, hipStream_t st);
hipError_t vec_lin2(const double *x, const double *y, const Coefs &a, const Coefs &c, double *z,
                    int64_t B, int64_t n, hipStream_t st);
hipError_t vec_shift_dot(const double *d, double *hd, const Coefs &lam, double *out, int64_t B,
                         int64_t n, hipStream_t st, const double *diag = nullptr);
hipError_t vec_cg_update(double *x, double *r, const double *d, const double *hd, const Coefs &a,
                         double *out, int64_t B, int64_t n, hipStream_t st);
hipError_t vec_pow_mul(const double *u, const double *s, int p, double *out, int64_t len,
                       hipStream_t st);
hipError_t vec_sub(const double *a, const double *b, double *out, int64_t len, hipStream_t st);
hipError_t vec_nonfinite(const double *x, int64_t len, int *flag, hipStream_t st);
// Preconditioned CG on (J_b + lam_b I) x_b = -grad_b (J_b + diag(diag_b) when
// diag is given) on the device (one workgroup per problem, n <= 256);
// steps[b] receives the CG steps taken.
hipError_t vec_cg_dense(const double *J, const double *P, const double *grad, const Coefs &lam, const Coefs &eta,
                        const Coefs &act, int64_t B, int64_t n, int max_it, double *x, int *steps, hipStream_t st,
                        const double *diag = nullptr);
// z_b = g_b + t_b a_b + t_b^2 c_b + t_b^3 e_b
hipError_t vec_poly3(const double *g, const double *a, const double *c, const double *e, const Coefs &t, double *z,
                     int64_t B, int64_t n, hipStream_t st);
// Instrumentation: streaming read of `words` 16-byte words by `groups`
// workgroups of 256 threads; sink[0 .. groups) receives one word each.
hipError_t probe_stream_read(const void *src, int64_t words, uint64_t *sink, int groups, hipStream_t st);
// z_b = A_b x_b (A_b symmetric [n][n], row-major)
hipError_t vec_symv(const double *A, const double *x, double *z, int64_t B, int64_t n, hipStream_t st);

// Newton-Schulz inverse of A = J + diag(d) (d_i = lam, or diag[i] when diag
// is given), n x n row-major; the products (with the shift A X = J X + diag(d)
// X and the step 2 X - X (A X) in their epilogues) are launch_gemm_square's:
//   ns_init:     X = I / ||A||_F (every eigenvalue of A X then lies in (0, 1]);
//                part holds kNsResidualDoubles doubles of scratch
//   ns_residual: out[0] = ||I - T||_F, out[1] = ||J||_F (fixed-order sums;
//                out holds kNsResidualDoubles: the norms, then partial sums)
//   ns_symmetrize: Xs = (X + X^T) / 2 (Xs may be X)
hipError_t ns_init(const double *J, double lam, const double *diag, double *X, int64_t n, double *part,
                   hipStream_t st);
constexpr int64_t kNsResidualDoubles = 2 + 2 * 64;
hipError_t ns_residual(const double *T, const double *J, int64_t n, double *out, hipStream_t st);
hipError_t ns_symmetrize(const double *X, double *Xs, int64_t n, hipStream_t st);

}  // namespace tk
