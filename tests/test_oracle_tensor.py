"""Pins for the oracle's tensor routines: brute force over the full n^m tensor,
closed forms of the linear tensor kernel (eq. tensor_1), the multilinear
invariant, symmetry and positivity (Section 4), and finite differences."""
from collections import Counter
from itertools import permutations
from math import factorial

import numpy as np
import pytest

from oracle import layout as L
from oracle import tensor as T
from synth import random_alpha, random_symmetric_packed_values


@pytest.mark.parametrize("n,m", [(1, 2), (3, 2), (6, 2), (5, 3), (6, 4), (4, 5), (5, 6), (3, 6)])
def test_packed_contraction_equals_full_bruteforce_random_tensor(n, m):
    # a random symmetric tensor (not of kernel form) so no structure hides errors
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=100 + 10 * n + m)
    a = random_alpha(n, seed=n * 31 + m)
    F = T.full_tensor(K, n, m)
    # the expansion is symmetric
    for perm in list(permutations(range(m)))[:24]:
        assert np.array_equal(F, np.transpose(F, perm))
    g_full = T.contract_full(F, a)
    g_packed = T.contract_packed(K, n, m, a)
    np.testing.assert_allclose(g_packed, g_full, rtol=1e-12, atol=1e-12 * np.abs(g_full).max())
    # <K, a^{(x)m}> = a^T g, and the full-tensor sum agrees
    ml = T.multilinear_packed(K, n, m, a)
    assert ml == pytest.approx(float(a @ g_full), rel=1e-12)
    letters = "abcdef"[:m]
    full_sum = np.einsum(letters + "," + ",".join(letters) + "->", F, *([a] * m))
    assert ml == pytest.approx(float(full_sum), rel=1e-12)


@pytest.mark.parametrize("n,d,m", [(5, 3, 2), (6, 4, 4), (4, 3, 6), (7, 5, 3)])
def test_build_linear_matches_full_einsum(n, d, m):
    X = np.random.default_rng(n + d + m).standard_normal((n, d))
    K = T.build_packed(X, m)
    F = T.full_tensor_linear(X, m)
    np.testing.assert_allclose(T.full_tensor(K, n, m), F, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n,d,m", [(30, 8, 4), (12, 5, 6), (40, 20, 2), (20, 6, 4)])
def test_packed_equals_closed_form_linear(n, d, m):
    X = np.random.default_rng(3 * n + d).standard_normal((n, d))
    a = random_alpha(n, seed=5 * n + m)
    K = T.build_packed(X, m)
    g_p = T.contract_packed(K, n, m, a)
    g_c = T.contract_closed(X, a, m)
    E = T.abs_bound_closed(X, a, m)
    assert np.all(np.abs(g_p - g_c) <= 64 * 2.0 ** -53 * L.packed_count(n, m) * E)
    np.testing.assert_allclose(g_p, g_c, rtol=1e-11, atol=1e-12 * E.max())
    # invariant <K, a^{(x)m}> = a^T g = ||X^T a||_m^m >= 0 (convexity remark after eq. dual_tensor_kernel)
    u = X.T @ a
    ml = T.multilinear_packed(K, n, m, a)
    assert ml == pytest.approx(float(np.sum(u ** m)), rel=1e-11)
    assert ml == pytest.approx(float(a @ g_p), rel=1e-11)
    assert ml >= 0.0


@pytest.mark.parametrize("kernel,kparam", [("poly", 2), ("poly", 3), ("exp", 0.0)])
def test_poly_exp_kernels_bruteforce_and_psd(kernel, kparam):
    n, d, m = 5, 3, 4
    X = 0.5 * np.random.default_rng(11).standard_normal((n, d))
    K = T.build_packed(X, m, kernel, kparam)
    lin = T.full_tensor_linear(X, m)
    F = lin ** int(kparam) if kernel == "poly" else np.exp(lin)
    np.testing.assert_allclose(T.full_tensor(K, n, m), F, rtol=1e-13, atol=1e-13 * np.abs(F).max())
    for s in range(20):
        a = random_alpha(n, seed=900 + s)
        # positive definiteness of tensor kernels (Section 4)
        assert T.multilinear_packed(K, n, m, a) >= -1e-12
        np.testing.assert_allclose(T.contract_packed(K, n, m, a), T.contract_full(F, a), rtol=1e-11)


def test_kernel_entry_matches_build():
    X = np.random.default_rng(2).standard_normal((6, 4))
    for m in (2, 4):
        K = T.build_packed(X, m, "poly", 2)
        for e, t in enumerate(L.nested_loop_tuples(6, m)):
            assert T.kernel_entry(X, t, "poly", 2) == K[e]


@pytest.mark.parametrize("n,m", [(6, 4), (4, 6), (5, 3), (7, 2)])
def test_hvp_and_jacobian_against_finite_differences(n, m):
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=77 + n)
    a = random_alpha(n, seed=8 + n)
    v = random_alpha(n, seed=9 + n)
    h = T.hvp_packed(K, n, m, a, v)
    eps = 1e-6
    fd = (T.contract_packed(K, n, m, a + eps * v) - T.contract_packed(K, n, m, a - eps * v)) / (2 * eps)
    np.testing.assert_allclose(h, fd, rtol=1e-7, atol=1e-7 * np.abs(fd).max())
    J = T.jacobian_packed(K, n, m, a)
    np.testing.assert_allclose(J @ v, h, rtol=1e-12, atol=1e-12 * np.abs(h).max())
    # the Jacobian of a gradient field is symmetric
    np.testing.assert_allclose(J, J.T, rtol=1e-12, atol=1e-12 * np.abs(J).max())
    # Euler: g is homogeneous of degree m-1, so J a = (m-1) g
    np.testing.assert_allclose(J @ a, (m - 1) * T.contract_packed(K, n, m, a), rtol=1e-11,
                               atol=1e-11 * np.abs(h).max())


def test_hvp_closed_form_linear():
    n, d, m = 9, 4, 6
    X = np.random.default_rng(1).standard_normal((n, d))
    K = T.build_packed(X, m)
    a, v = random_alpha(n, 1), random_alpha(n, 2)
    np.testing.assert_allclose(T.hvp_packed(K, n, m, a, v), T.hvp_closed(X, a, v, m), rtol=1e-11)
    np.testing.assert_allclose(T.jacobian_packed(K, n, m, a), T.jacobian_closed(X, a, m), rtol=1e-10,
                               atol=1e-12)


def _mutant_contract(K, n, m, a, weight):
    g = np.zeros(n)
    for e, t in enumerate(L.nested_loop_tuples(n, m)):
        w = weight(t)
        for p in range(m):
            prod = 1.0
            for q in range(m):
                if q != p:
                    prod *= a[t[q]]
            g[t[p]] += w * K[e] * prod
    return g


def test_bruteforce_pin_catches_plausible_weight_mistakes():
    """The brute-force pin must fail for plausible mistakes in the repeated-index
    weights; this plants them in a throwaway copy on the CPU."""
    n, m = 5, 4
    K = random_symmetric_packed_values(L.packed_count(n, m), seed=3)
    a = random_alpha(n, seed=4)
    ref = T.contract_full(T.full_tensor(K, n, m), a)

    def right(t):
        c = 1
        for v in Counter(t).values():
            c *= factorial(v)
        return factorial(m - 1) / c

    np.testing.assert_allclose(_mutant_contract(K, n, m, a, right), ref, rtol=1e-12)
    mutants = [
        lambda t: factorial(m - 1),                       # no multiplicity correction
        lambda t: factorial(m) / np.prod([factorial(v) for v in Counter(t).values()]),  # m! not (m-1)!
        lambda t: 1.0 / np.prod([factorial(v) for v in Counter(t).values()]),
        lambda t: right(t) * (1.0 if len(set(t)) == m else 0.5),
    ]
    for mut in mutants:
        assert not np.allclose(_mutant_contract(K, n, m, a, mut), ref, rtol=1e-6)
