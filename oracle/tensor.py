"""Tensor kernels, the packed tensor and its contractions (Section 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Three independent routes to g = K . alpha^{m-1}:
  * ``contract_full``   brute force over the full n^m tensor (tiny n);
  * ``contract_packed`` the packed array, one sorted tuple at a time (C);
  * ``contract_closed`` the closed form X (X^T alpha)^{m-1} of the linear
    tensor kernel, read off eq. tensor_1 (linear feature map only).
"""
from __future__ import annotations

import ctypes
from itertools import product

import numpy as np

from . import _clib
from .layout import packed_count, rank_closed_form

KERNELS = {"linear": 0, "poly": 1, "exp": 2}


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def build_packed(X, m: int, kernel: str = "linear", kparam: float = 0.0) -> np.ndarray:
    """Packed tensor kernel values K_t for every sorted tuple t (Section 4:
    linear k = sum(x_1 .. x_m), polynomial (sum)^s, exponential exp(sum))."""
    X = _f64(X)
    n, d = X.shape
    K = np.empty(packed_count(n, m))
    rc = _clib.lib().or_build_packed(_dp(X), n, d, m, KERNELS[kernel], float(kparam), _dp(K))
    if rc != 0:
        raise ValueError("or_build_packed failed")
    return K


def kernel_entry(X, t, kernel: str = "linear", kparam: float = 0.0) -> float:
    """One kernel value k(x_{t_0}, .., x_{t_{m-1}}) computed on its own."""
    X = _f64(X)
    tt = np.ascontiguousarray(np.asarray(t, dtype=np.int64))
    return _clib.lib().or_kernel_entry(_dp(X), X.shape[1], _ip(tt), len(tt), KERNELS[kernel], float(kparam))


def contract_packed(K, n: int, m: int, alpha) -> np.ndarray:
    K = _f64(K)
    a = _f64(alpha)
    g = np.empty(n)
    if K.size != packed_count(n, m) or a.size != n:
        raise ValueError("shape mismatch")
    _clib.lib().or_contract_packed(_dp(K), n, m, _dp(a), _dp(g))
    return g


def hvp_packed(K, n: int, m: int, alpha, v) -> np.ndarray:
    K, a, vv = _f64(K), _f64(alpha), _f64(v)
    h = np.empty(n)
    _clib.lib().or_hvp_packed(_dp(K), n, m, _dp(a), _dp(vv), _dp(h))
    return h


def jacobian_packed(K, n: int, m: int, alpha) -> np.ndarray:
    K, a = _f64(K), _f64(alpha)
    H = np.empty((n, n))
    _clib.lib().or_jacobian_packed(_dp(K), n, m, _dp(a), _dp(H))
    return H


def multilinear_packed(K, n: int, m: int, alpha) -> float:
    """<K, alpha^{(x)m}>: the first dual term of eq. dual_tensor_kernel times m."""
    K, a = _f64(K), _f64(alpha)
    return _clib.lib().or_multilinear_packed(_dp(K), n, m, _dp(a))


def enumerate_tuples(n: int, m: int) -> np.ndarray:
    cnt = packed_count(n, m)
    T = np.empty((cnt, m), dtype=np.int64)
    got = _clib.lib().or_enumerate(n, m, _ip(T), cnt)
    if got != cnt:
        raise RuntimeError("enumeration count mismatch")
    return T


def full_tensor(K, n: int, m: int) -> np.ndarray:
    """Expand a packed tensor to the full n^m array (tiny n only)."""
    K = _f64(K)
    F = np.empty((n,) * m)
    for idx in product(range(n), repeat=m):
        F[idx] = K[rank_closed_form(sorted(idx), n)]
    return F


def full_tensor_linear(X, m: int) -> np.ndarray:
    """Full linear tensor kernel k(x_{i_1}..x_{i_m}) = sum_j prod_p X[i_p, j]
    via einsum (tiny n only)."""
    X = _f64(X)
    letters = "abcdefghijkl"[:m]
    spec = ",".join(f"{c}z" for c in letters) + "->" + letters
    return np.einsum(spec, *([X] * m))


def contract_full(F, alpha) -> np.ndarray:
    """g_a = sum_{i_2..i_m} F[a, i_2, .., i_m] alpha_{i_2} .. alpha_{i_m}."""
    g = np.asarray(F, dtype=np.float64)
    a = _f64(alpha)
    while g.ndim > 1:
        g = g @ a
    return g


def contract_closed(X, alpha, m: int) -> np.ndarray:
    """Linear tensor kernel: g = X (X^T alpha)^{m-1} (eq. tensor_1)."""
    X = _f64(X)
    u = X.T @ _f64(alpha)
    return X @ (u ** (m - 1))


def hvp_closed(X, alpha, v, m: int) -> np.ndarray:
    """(m-1) X diag(u^{m-2}) X^T v with u = X^T alpha (linear kernel)."""
    X = _f64(X)
    u = X.T @ _f64(alpha)
    return (m - 1) * (X @ ((u ** (m - 2)) * (X.T @ _f64(v))))


def jacobian_closed(X, alpha, m: int) -> np.ndarray:
    X = _f64(X)
    u = X.T @ _f64(alpha)
    return (m - 1) * ((X * (u ** (m - 2))) @ X.T)


def abs_bound_closed(X, alpha, m: int) -> np.ndarray:
    """Elementwise bound E_i >= sum of |terms| of g_i for the linear kernel:
    E = |X| (|X|^T |alpha|)^{m-1}."""
    Xa = np.abs(_f64(X))
    return Xa @ ((Xa.T @ np.abs(_f64(alpha))) ** (m - 1))
