"""The allocation-free contraction entry point (tk_contract_noalloc) against
the workspace entry point (tk_contract) through the C ABI: identical kernels
and launch shapes, so identical results; both held to the oracle's bound."""
import numpy as np
import pytest

import paper_2003_10482_amd as tk
from gpu_util import U64, abs_terms, device, to_dev, to_np
from oracle import layout as L
from oracle import tensor as T
from synth import random_alpha, random_symmetric_packed_values

pytestmark = pytest.mark.gpu


def _case(n, m, B, seed):
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=seed)
    A = random_alpha(n, seed=seed + 1, batch=B)
    return K, A, tk.PackedTensor(to_dev(K), n, m, tk.F64)


def test_noalloc_matches_workspace_entry_point_twice():
    """Two calls in a row on one device, the second with a smaller input:
    each equals tk_contract bit for bit and the oracle within depth * u * E."""
    device()
    cap = tk.api._lib.load().tk_contract_noalloc_max_bytes()
    assert cap > 0
    for n, m, B, acc in ((256, 4, 1, tk.ACC_F64), (70, 4, 2, tk.ACC_COMPENSATED), (40, 6, 3, tk.ACC_F64)):
        K, A, Kd = _case(n, m, B, seed=3 * n + m)
        assert tk.contract_workspace(n, m, B, tk.F64) > 0
        g_ws = to_np(tk.contract(Kd, to_dev(A), acc=acc))
        g_na = to_np(tk.contract_noalloc(Kd, to_dev(A), acc=acc))
        np.testing.assert_array_equal(g_na, g_ws)
        depth = L.packed_count(n, m - 1) + 4 * n + 64
        for b in range(B):
            ref = T.contract_packed(K, n, m, A[b])
            E = abs_terms(K, n, m, A[b])
            assert np.all(np.abs(g_na[b] - ref) <= 2 * depth * U64 * E), (n, m, b)


def test_noalloc_rejects_sizes_above_its_scratch():
    """A batch whose workspace exceeds the fixed scratch fails with TK_ENOMEM
    (-3) before any device work, and the next call still works."""
    n, m = 256, 4
    K, A, Kd = _case(n, m, 1, seed=9)
    # 4096 vectors need B * C(n+1, 2) double-double intermediates alone
    # (2.1 GB), far above the fixed scratch
    B = 4096
    assert B * L.packed_count(n, 2) * 16 > tk.api._lib.load().tk_contract_noalloc_max_bytes()
    big = to_dev(np.tile(A, (B, 1)))
    with pytest.raises(tk.api._lib.TkError) as ei:
        tk.contract_noalloc(Kd, big, acc=tk.ACC_COMPENSATED)
    assert ei.value.code == -3
    g = to_np(tk.contract_noalloc(Kd, to_dev(A), acc=tk.ACC_F64))
    np.testing.assert_array_equal(g, to_np(tk.contract(Kd, to_dev(A), acc=tk.ACC_F64)))
