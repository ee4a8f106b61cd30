"""Seeded generators for the synthetic workloads.

Data model (Section 5.4): X has i.i.d. N(0, 1) entries; the planted weight
vector w* is zero except at ``s`` indices drawn uniformly without replacement;
each planted value is sgn(h)(1 - 0.3 u) with h ~ N(0, 1), u ~ U(0, 1); the
response is y = X w* + sigma * eps with eps ~ N(0, 1) of length n (the text
writes eps in R^d, which cannot be added to X w* in R^n; we read it as R^n).

The small parity workload uses planted values U[-1, 1] instead, as its
description states.  Seeds are 1000 + workload number (2002 for the order-6
variant of workload 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    m: int                      # tensor order (even)
    lam: float                  # regularisation lambda (= 1/gamma of the text)
    X: np.ndarray               # training points [n, d], float64, C-contiguous
    y: np.ndarray               # responses [n]
    w_true: np.ndarray          # planted weights [d]
    support: np.ndarray         # sorted indices of the planted nonzeros
    X_val: Optional[np.ndarray] = None
    y_val: Optional[np.ndarray] = None
    X_test: Optional[np.ndarray] = None
    y_test: Optional[np.ndarray] = None
    landmarks: Optional[np.ndarray] = None   # int64 indices into X (Nystrom)
    lambdas: Optional[np.ndarray] = None     # lambda path
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]


def planted_regression(rng: np.random.Generator, n: int, d: int, s: int, sigma: float,
                       values: str = "paper", n_extra: int = 0):
    """Draw (X, y, w*, support) following the synthetic data model.

    ``n_extra`` additional points are drawn from the same law with the same w*
    (held-out validation / test points) and returned stacked under X.
    """
    if s > d:
        raise ValueError("support larger than dimension")
    X = rng.standard_normal((n + n_extra, d))
    support = np.sort(rng.choice(d, size=s, replace=False))
    w = np.zeros(d)
    if values == "paper":
        h = rng.standard_normal(s)
        u = rng.random(s)
        w[support] = np.sign(h) * (1.0 - 0.3 * u)
    elif values == "uniform":
        w[support] = rng.uniform(-1.0, 1.0, size=s)
    else:
        raise ValueError(values)
    eps = rng.standard_normal(n + n_extra)
    y = X @ w + sigma * eps
    return np.ascontiguousarray(X), y, w, support


def lambda_grid(count: int = 64, lo_exp: float = -4.0, hi_exp: float = 0.0) -> np.ndarray:
    """Log-spaced lambda path 10^(lo + (hi-lo) k/(count-1)), k = 0..count-1."""
    k = np.arange(count, dtype=np.float64)
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * k / (count - 1))


CONFIGS = {
    # name: (n, d, s, sigma, m, lam, values, seed)
    "c1_n64_m4": (64, 20, 4, 0.01, 4, 1e-2, "uniform", 1001),
    "c2_n256_m4": (256, 200, 10, 0.05, 4, 1e-2, "paper", 1002),
    "c2b_n64_m6": (64, 50, 5, 0.05, 6, 1e-2, "paper", 2002),
    "c3_nystrom": (20000, 1000, 20, 0.1, 4, 1e-2, "paper", 1003),
    "c4_lampath": (256, 200, 10, 0.05, 4, 1e-2, "paper", 1002),
    "c5_n128_m6": (128, 100, 8, 0.05, 6, 1e-2, "paper", 1005),
}


def make_workload(name: str, *, n: Optional[int] = None, d: Optional[int] = None,
                  seed: Optional[int] = None) -> Workload:
    """Build one named workload; ``n``/``d``/``seed`` override for reduced cases."""
    n0, d0, s, sigma, m, lam, values, seed0 = CONFIGS[name]
    n = n0 if n is None else n
    d = d0 if d is None else d
    s = min(s, d)
    rng = np.random.default_rng(seed0 if seed is None else seed)
    if name == "c3_nystrom":
        X, y, w, sup = planted_regression(rng, n, d, s, sigma, values)
        n_land = min(200, n)
        land = np.sort(rng.choice(n, size=n_land, replace=False)).astype(np.int64)
        rest = np.setdiff1d(np.arange(n), land)
        return Workload(name, m, lam, X, y, w, sup, landmarks=land,
                        X_test=np.ascontiguousarray(X[rest]), y_test=y[rest])
    if name == "c5_n128_m6":
        n_val = 2000
        Xa, ya, w, sup = planted_regression(rng, n, d, s, sigma, values, n_extra=n_val)
        return Workload(name, m, lam, np.ascontiguousarray(Xa[:n]), ya[:n], w, sup,
                        X_val=np.ascontiguousarray(Xa[n:]), y_val=ya[n:])
    X, y, w, sup = planted_regression(rng, n, d, s, sigma, values)
    wl = Workload(name, m, lam, X, y, w, sup)
    if name == "c4_lampath":
        wl.lambdas = lambda_grid(64)
    return wl


def landmark_draws(n_total: int, ell: int, draws: int, seed: int) -> np.ndarray:
    """``draws`` independent uniform draws of ``ell`` distinct indices out of
    ``n_total`` (sorted within a draw), int64 [draws, ell]: the random
    subsamples of Section 6.1, drawn here and handed to both sides."""
    rng = np.random.default_rng(seed)
    return np.stack([np.sort(rng.choice(n_total, size=ell, replace=False)) for _ in range(draws)]).astype(np.int64)


def planted_classification(rng: np.random.Generator, n: int, d: int, s: int, flip: float = 0.0):
    """Labels y = sign(X w*) in {-1, +1} for the planted-weight model above,
    with a fraction ``flip`` of them flipped at random."""
    X = rng.standard_normal((n, d))
    support = np.sort(rng.choice(d, size=s, replace=False))
    w = np.zeros(d)
    h = rng.standard_normal(s)
    u = rng.random(s)
    w[support] = np.sign(h) * (1.0 - 0.3 * u)
    y = np.sign(X @ w)
    y[y == 0] = 1.0
    flips = rng.random(n) < flip
    y[flips] = -y[flips]
    return np.ascontiguousarray(X), y, w, support


def random_alpha(n: int, seed: int, batch: Optional[int] = None, scale: float = 1.0) -> np.ndarray:
    """Seeded N(0, scale^2) dual vectors, shape [n] or [batch, n]."""
    rng = np.random.default_rng(seed)
    shape = (n,) if batch is None else (batch, n)
    return scale * rng.standard_normal(shape)


def random_symmetric_packed_values(count: int, seed: int) -> np.ndarray:
    """``count`` seeded N(0,1) values, used as the unique entries of a random
    symmetric tensor (one value per sorted index tuple)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(count)
