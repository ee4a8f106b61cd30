// Pass kernels with compensated FP64 accumulation (FP64 tensor, DD intermediate arrays).
#include "tk_pass.hpp"

namespace tk {

hipError_t launch_pass_dd(int q, int in_kind, int hv, int bt, const PairParams &pp, int groups, hipStream_t st)
{
    if (in_kind == 0) {
        if (hv == 0) return dispatch_q<double, ACC_DD, 0>(q, pp, groups, bt, st);
        if (hv == 1) return dispatch_q<double, ACC_DD, 1>(q, pp, groups, bt, st);
        return hipErrorInvalidValue;
    }
    if (in_kind == 3) {
        if (hv == 0) return dispatch_q<DD, ACC_DD, 0>(q, pp, groups, bt, st);
        if (hv == 2) return dispatch_q<DD, ACC_DD, 2>(q, pp, groups, bt, st);
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

}  // namespace tk
