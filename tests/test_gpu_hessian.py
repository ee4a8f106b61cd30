"""GPU parity of the Hessian kernel J = (m-1) K . alpha^{m-2} (the Jacobian of
the contraction, used by the dual solve's preconditioner) through the C ABI,
against the oracle's packed Jacobian, which differentiates every packed entry
term by term (ordered pairs of tuple positions), and at the benchmark size
against the closed form (m-1) X diag(u^{m-2}) X^T.

Bound: the kernel sums in plain FP64; every entry of J is a sum of products
whose longest chain of dependent additions is below the number of units
C(n+m-3, m-2) plus the work items and rows merged after them, so
|J - J_ref| <= L u sum|terms| with sum|terms| = the oracle on |K| and |alpha|.
"""
import numpy as np
import pytest

import paper_2003_10482_amd as tk
from gpu_util import U64, to_dev, to_np
from oracle import tensor as T
from oracle.layout import packed_count
from synth import make_workload, random_alpha, random_symmetric_packed_values
from test_gpu_contract import _packed_dev

pytestmark = pytest.mark.gpu

SHAPES = [(1, 2), (5, 2), (70, 2), (1, 4), (2, 4), (9, 4), (37, 4), (64, 4), (70, 4), (130, 4),
          (5, 6), (13, 6), (30, 6), (9, 8)]


def _chain(n, m):
    return packed_count(n, m - 2) + 2048 + 4 * n


def _check(J, Kv, n, m, a):
    Jr = T.jacobian_packed(Kv, n, m, a)
    Jabs = T.jacobian_packed(np.abs(Kv), n, m, np.abs(a))
    err = np.abs(J - Jr)
    assert np.all(err <= _chain(n, m) * U64 * Jabs + 1e-300), float(np.max(err / (Jabs + 1e-300)))
    # far inside the a-priori bound in practice
    assert float(np.max(err / (Jabs + 1e-300))) < 1e-13


@pytest.mark.parametrize("n,m", SHAPES)
def test_hessian_matches_oracle(n, m):
    Kh = random_symmetric_packed_values(packed_count(n, m), seed=31 * n + m)
    a = random_alpha(n, seed=7 * n + m)
    K, Kv = _packed_dev(Kh, n, m)
    J = to_np(tk.hessian(K, to_dev(a)))
    assert J.shape == (n, n)
    np.testing.assert_array_equal(J, J.T)
    _check(J, Kv, n, m, a)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("n,m", [(70, 4), (13, 6)])
def test_hessian_reduced_storage(n, m, dtype):
    """FP64 arithmetic on FP32/BF16 entries: parity with the oracle on the
    stored (rounded) values to the same FP64 bound."""
    Kh = random_symmetric_packed_values(packed_count(n, m), seed=5 * n + m)
    a = random_alpha(n, seed=3 * n + m)
    K, Kv = _packed_dev(Kh, n, m, dtype)
    J = to_np(tk.hessian(K, to_dev(a)))
    _check(J, Kv, n, m, a)


@pytest.mark.parametrize("n,m", [(70, 4), (30, 6)])
def test_hessian_times_direction_is_hvp(n, m):
    Kh = random_symmetric_packed_values(packed_count(n, m), seed=n + 11 * m)
    a = random_alpha(n, seed=2)
    V = random_alpha(n, seed=3, batch=3)
    K, Kv = _packed_dev(Kh, n, m)
    J = to_np(tk.hessian(K, to_dev(a)))
    A = np.repeat(a[None, :], 3, axis=0)
    H = to_np(tk.hvp(K, to_dev(A), to_dev(V), acc=tk.ACC_COMPENSATED))
    for i in range(3):
        h_abs = T.hvp_packed(np.abs(Kv), n, m, np.abs(a), np.abs(V[i]))
        assert np.all(np.abs(J @ V[i] - H[i]) <= (_chain(n, m) + n) * U64 * h_abs)


def test_hessian_full_size_and_reproducible():
    """The benchmark workload (n=256, m=4, C(259,4) FP64 entries) at a random
    alpha: closed form within storage rounding (gamma_d of each entry) plus
    the kernel's summation bound; two calls agree bitwise."""
    wl = make_workload("c2_n256_m4")
    X = to_dev(wl.X)
    K = tk.build_packed_tensor(X, 4)
    a = random_alpha(256, seed=17)
    J1 = to_np(tk.hessian(K, to_dev(a)))
    J2 = to_np(tk.hessian(K, to_dev(a)))
    np.testing.assert_array_equal(J1, J2)
    Jr = T.jacobian_closed(wl.X, a, 4)
    aX = np.abs(wl.X)
    Jabs = 3.0 * (aX * (aX.T @ np.abs(a)) ** 2) @ aX.T
    bound = (_chain(256, 4) + wl.X.shape[1]) * U64 * Jabs
    assert np.all(np.abs(J1 - Jr) <= bound)


@pytest.mark.parametrize("n,m", [(129, 4), (13, 6), (70, 2)])
def test_hessian_workspace_contents_do_not_matter(n, m):
    import torch
    from gpu_util import device
    Kh = random_symmetric_packed_values(packed_count(n, m), seed=n)
    a = to_dev(random_alpha(n, seed=1))
    K, _ = _packed_dev(Kh, n, m)
    nbytes = tk.hessian_workspace(n, m)
    outs = []
    for fill in (0.0, float("nan")):
        work = torch.full(((nbytes + 7) // 8,), fill, dtype=torch.float64, device=device()).view(torch.uint8)
        outs.append(to_np(tk.hessian(K, a, work=work)))
    assert np.all(np.isfinite(outs[1]))
    np.testing.assert_array_equal(outs[0], outs[1])
