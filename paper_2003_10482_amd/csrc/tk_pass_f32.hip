// Pass kernels with FP32 accumulation (FP32 or BF16 tensor, FP32 intermediate arrays).
#include "tk_pass.hpp"

namespace tk {

hipError_t launch_pass_f32(int q, int in_kind, int hv, int bt, const PairParams &pp, int groups, hipStream_t st)
{
    if (in_kind == 0) {   // FP64 tensor read with FP32 arithmetic (preconditioner Hessians)
        if (hv == 0) return dispatch_q<double, ACC_PLAIN32, 0>(q, pp, groups, bt, st);
        if (hv == 1) return dispatch_q<double, ACC_PLAIN32, 1>(q, pp, groups, bt, st);
        return hipErrorInvalidValue;
    }
    if (in_kind == 1) {
        if (hv == 0) return dispatch_q<float, ACC_PLAIN32, 0>(q, pp, groups, bt, st);
        if (hv == 1) return dispatch_q<float, ACC_PLAIN32, 1>(q, pp, groups, bt, st);
        return dispatch_q<float, ACC_PLAIN32, 2>(q, pp, groups, bt, st);
    }
    if (in_kind == 2) {
        if (hv == 0) return dispatch_q<uint16_t, ACC_PLAIN32, 0>(q, pp, groups, bt, st);
        if (hv == 1) return dispatch_q<uint16_t, ACC_PLAIN32, 1>(q, pp, groups, bt, st);
        return hipErrorInvalidValue;   // BF16 is a storage type of the top array only
    }
    return hipErrorInvalidValue;
}

}  // namespace tk
