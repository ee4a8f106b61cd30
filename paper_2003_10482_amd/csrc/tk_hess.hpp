// Hessian of the contraction in a fixed number of passes over the packed tensor.
#pragma once

#include "tk_common.hpp"

namespace tk {

// Workspace bytes of run_hessian for (n, m) (independent of the device).
size_t hessian_ws(int64_t n, int m);

// J = (m-1) K . alpha^{m-2} (n x n, row-major, FP64) for one alpha vector,
// FP64 arithmetic on any storage type.  `passes` (optional) receives the
// number of reads of the packed tensor (2 for m >= 4, 1 for m = 2).
int run_hessian(const void *K, int dtype, int64_t n, int m, const double *alpha, double *J, void *work,
                size_t work_bytes, hipStream_t st, int *passes);

}  // namespace tk
