"""MI355X-native packed tensor-kernel regression (hot path of arXiv 2003.10482).

The compute path is the HIP library ``libtk.so`` (C ABI in ``include/tk.h``);
this package only marshals torch tensors to it.  Importing the package does not
load the library; the first call does, and raises if it is missing.
"""
from .api import (  # noqa: F401
    ACC_AUTO, ACC_COMPENSATED, ACC_F32, ACC_F64, BF16, EXP, F32, F64, LINEAR, POLY,
    MultiPackedTensor, PackedTensor, TkContract, autotune, build_packed_multi, build_packed_tensor, contract, contract_multi, contract_autograd, contract_dense, contract_noalloc,
    contract_workspace, dmse_dlambda, empty_packed, gather_rows, hessian, hessian_workspace, hvp, max_points,
    packed_bytes,
    packed_count, packed_stride, predict, predict_kernel,
    primal_weights, probe_stream_read, solve_dual, solve_dual_multi, solve_workspace, support, timing_start, timing_stop,
)
