"""Build and load the plain-C part of the oracle (``packed_oracle.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "packed_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "liboracle.so")
_lock = threading.Lock()
_handle = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _handle
    with _lock:
        if _handle is None:
            build(force=False)
            h = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int64)
            i64 = ctypes.c_int64
            h.or_build_packed.argtypes = [dp, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
            h.or_contract_packed.argtypes = [dp, i64, ctypes.c_int, dp, dp]
            h.or_hvp_packed.argtypes = [dp, i64, ctypes.c_int, dp, dp, dp]
            h.or_jacobian_packed.argtypes = [dp, i64, ctypes.c_int, dp, dp]
            h.or_multilinear_packed.argtypes = [dp, i64, ctypes.c_int, dp]
            h.or_multilinear_packed.restype = ctypes.c_double
            h.or_enumerate.argtypes = [i64, ctypes.c_int, ip, i64]
            h.or_enumerate.restype = i64
            h.or_orderings.argtypes = [ip, ctypes.c_int]
            h.or_orderings.restype = ctypes.c_double
            h.or_kernel_entry.argtypes = [dp, i64, ip, ctypes.c_int, ctypes.c_int, ctypes.c_double]
            h.or_kernel_entry.restype = ctypes.c_double
            for f in ("or_build_packed", "or_contract_packed", "or_hvp_packed", "or_jacobian_packed"):
                getattr(h, f).restype = ctypes.c_int
            _handle = h
    return _handle
