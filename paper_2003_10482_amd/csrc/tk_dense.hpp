// Launchers of the dense (MFMA) products and small utility kernels.
#pragma once

#include "tk_common.hpp"

namespace tk {

// C[i][j] = sum_k A[i*lda + k] B[k*bsk + j*bsj], optionally raised to the power epi (> 1).
hipError_t launch_gemm(const double *A, int64_t lda, const double *B, int64_t bsk, int64_t bsj,
                       double *C, int64_t ldc, int64_t M, int64_t N, int64_t K, int epi,
                       hipStream_t st);
// Square products with an epilogue that reads a second n x n matrix Y (not C):
//   kEpiShift:   C = A B + diag(d) Y   (d_i = yd[i], or ys when yd is null)
//   kEpiReflect: C = 2 Y - A B
// Other epi values act as in launch_gemm.
constexpr int kEpiShift = -1;
constexpr int kEpiReflect = -2;
hipError_t launch_gemm_square(const double *A, const double *B, double *C, int64_t n, int epi, const double *Y,
                              const double *yd, double ys, hipStream_t st);
hipError_t launch_support(const double *W, int64_t d, int64_t B, uint8_t *mask, double *tau,
                          hipStream_t st);
hipError_t launch_gather(const double *X, int64_t N, int64_t d, const int64_t *idx, int64_t l,
                         double *out, int *bad, hipStream_t st);
// General-kernel prediction f[b][q] = sum_T c(T) alpha_b^T k(x_T, xq_q) (part:
// predict_groups(n, m, N) * min(B, predict_max_batch()) * N doubles of workspace).
hipError_t launch_predict_kernel(const double *X, int64_t n, int64_t d, int m, int kernel, double kparam,
                                 const double *alpha, int64_t B, const double *Xq, int64_t N, double *f,
                                 double *part, hipStream_t st);
int64_t predict_groups(int64_t n, int m, int64_t N);
int predict_max_batch();
hipError_t launch_build(const double *X, int n, int d, int m, int kernel, double kparam, int dtype,
                        void *K, hipStream_t st);

}  // namespace tk
