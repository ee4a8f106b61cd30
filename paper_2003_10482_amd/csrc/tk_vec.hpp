// Batched FP64 vector kernels of the dual solve.
#pragma once

#include "tk_common.hpp"

namespace tk {

constexpr int kMaxCoefs = 64;   // vectors per launch of a coefficient-carrying kernel

struct Coefs {
    double c[kMaxCoefs];
};

hipError_t vec_grad(const double *g, const double *alpha, const double *y, const Coefs &lam,
                    double *grad, double *stats, int64_t B, int64_t n, hipStream_t st);
hipError_t vec_dot(const double *x, const double *y, int64_t y_stride, double *out, int64_t B,
                   int64_t n, hipStream_t st);
hipError_t vec_lin2(const double *x, const double *y, const Coefs &a, const Coefs &c, double *z,
                    int64_t B, int64_t n, hipStream_t st);
hipError_t vec_shift_dot(const double *d, double *hd, const Coefs &lam, double *out, int64_t B,
                         int64_t n, hipStream_t st);
hipError_t vec_cg_update(double *x, double *r, const double *d, const double *hd, const Coefs &a,
                         double *out, int64_t B, int64_t n, hipStream_t st);
hipError_t vec_pow_mul(const double *u, const double *s, int p, double *out, int64_t len,
                       hipStream_t st);
hipError_t vec_sub(const double *a, const double *b, double *out, int64_t len, hipStream_t st);
hipError_t vec_nonfinite(const double *x, int64_t len, int *flag, hipStream_t st);
// Preconditioned CG on (J_b + lam_b I) x_b = -grad_b on the device (one
// workgroup per problem, n <= 256); steps[b] receives the CG steps taken.
hipError_t vec_cg_dense(const double *J, const double *P, const double *grad, const Coefs &lam, const Coefs &eta,
                        const Coefs &act, int64_t B, int64_t n, int max_it, double *x, int *steps, hipStream_t st);
// z_b = g_b + t_b a_b + t_b^2 c_b + t_b^3 e_b
hipError_t vec_poly3(const double *g, const double *a, const double *c, const double *e, const Coefs &t, double *z,
                     int64_t B, int64_t n, hipStream_t st);
// z_b = A_b x_b (A_b symmetric [n][n], row-major)
hipError_t vec_symv(const double *A, const double *x, double *z, int64_t B, int64_t n, hipStream_t st);

}  // namespace tk
