"""Helpers shared by the GPU tests (device selection and bound computations)."""
import numpy as np
import pytest
import torch

from oracle import tensor as T

U64 = 2.0 ** -53
U32 = 2.0 ** -24
UBF16 = 2.0 ** -8


def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device())


def to_np(t):
    return t.detach().to("cpu").numpy()


def abs_terms(K, n, m, alpha):
    """E_i = sum of |terms| of g_i, computed by the oracle on |K| and |alpha|
    (every term becomes nonnegative, so the packed contraction of the absolute
    values is exactly the sum of absolute terms)."""
    return T.contract_packed(np.abs(K), n, m, np.abs(alpha))


def reduction_depth(n, m):
    """Worst-case length of a chain of dependent floating-point additions in the
    GPU contraction for one output, used in the FP32 a-priori bound: per-lane
    accumulation over the rows of one wave's units (at most all rows of the
    array) plus the fixed reduction trees (batch, wave, workgroup, partials).
    We use the number of rows of the largest pass as a conservative bound."""
    from oracle.layout import packed_count
    rows = packed_count(n, m - 1)
    return rows + 64
