"""Round-to-nearest-even rounding of FP64 values to the storage formats.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

BF16 keeps 8 significant bits (1 implicit + 7 stored) with FP32's exponent
range.  The rounding below works on the exact binary value of each float64:
x = f * 2^e with f in [0.5, 1); the nearest multiple of 2^(e-8) is found with
Python's round(), which breaks exact ties to the even neighbour.
"""
from __future__ import annotations

import math

import numpy as np

_BF16_MIN_NORMAL_EXP = -126
_BF16_SUBNORMAL_QUANTUM = 2.0 ** -133
_BF16_OVERFLOW = 2.0 ** 128


def round_bf16_scalar(x: float) -> float:
    if math.isnan(x) or math.isinf(x) or x == 0.0:
        return x
    ax = abs(x)
    if ax < 2.0 ** _BF16_MIN_NORMAL_EXP:
        q = round(ax / _BF16_SUBNORMAL_QUANTUM) * _BF16_SUBNORMAL_QUANTUM
    else:
        f, e = math.frexp(ax)            # ax = f * 2^e, f in [0.5, 1)
        q = math.ldexp(round(math.ldexp(f, 8)), e - 8)
    if q >= _BF16_OVERFLOW:
        q = math.inf
    return math.copysign(q, x)


def round_bf16(a) -> np.ndarray:
    """Vectorised form of round_bf16_scalar: the same steps on whole arrays
    (np.round also breaks exact ties to the even neighbour)."""
    a = np.asarray(a, dtype=np.float64)
    out = a.copy()
    fin = np.isfinite(a) & (a != 0.0)
    ax = np.abs(a[fin])
    q = np.empty_like(ax)
    small = ax < 2.0 ** _BF16_MIN_NORMAL_EXP
    q[small] = np.round(ax[small] / _BF16_SUBNORMAL_QUANTUM) * _BF16_SUBNORMAL_QUANTUM
    f, e = np.frexp(ax[~small])
    q[~small] = np.ldexp(np.round(np.ldexp(f, 8)), e - 8)
    q[q >= _BF16_OVERFLOW] = np.inf
    out[fin] = np.copysign(q, a[fin])
    return out


def round_fp32(a) -> np.ndarray:
    """IEEE round-to-nearest-even float64 -> float32, returned as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8}
