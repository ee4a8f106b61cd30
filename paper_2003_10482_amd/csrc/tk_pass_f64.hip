// Pass kernels with plain FP64 accumulation.
#include "tk_pass.hpp"

namespace tk {

hipError_t launch_pass_f64(int q, int in_kind, int hv, int bt, const PairParams &pp, int groups, hipStream_t st)
{
    if (in_kind != 0) return hipErrorInvalidValue;
    if (hv == 0) return dispatch_q<double, ACC_PLAIN64, 0>(q, pp, groups, bt, st);
    if (hv == 1) return dispatch_q<double, ACC_PLAIN64, 1>(q, pp, groups, bt, st);
    return dispatch_q<double, ACC_PLAIN64, 2>(q, pp, groups, bt, st);
}

}  // namespace tk
