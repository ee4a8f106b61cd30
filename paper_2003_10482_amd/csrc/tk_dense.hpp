// Launchers of the dense (MFMA) products and small utility kernels.
#pragma once

#include "tk_common.hpp"

namespace tk {

// C[i][j] = sum_k A[i*lda + k] B[k*bsk + j*bsj], optionally raised to the power epi (> 1).
hipError_t launch_gemm(const double *A, int64_t lda, const double *B, int64_t bsk, int64_t bsj,
                       double *C, int64_t ldc, int64_t M, int64_t N, int64_t K, int epi,
                       hipStream_t st);
hipError_t launch_support(const double *W, int64_t d, int64_t B, uint8_t *mask, double *tau,
                          hipStream_t st);
hipError_t launch_gather(const double *X, int64_t N, int64_t d, const int64_t *idx, int64_t l,
                         double *out, int *bad, hipStream_t st);
hipError_t launch_build(const double *X, int n, int d, int m, int kernel, double kparam, int dtype,
                        void *K, hipStream_t st);

}  // namespace tk
