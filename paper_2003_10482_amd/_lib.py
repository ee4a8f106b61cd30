"""ctypes loader of the in-tree HIP library ``libtk.so`` (argument marshalling only).

There is no fallback: if the library is missing or cannot be loaded, every
call raises.  Build it with ``python -m paper_2003_10482_amd.build`` (or
``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtk.so")

_lock = threading.Lock()
_lib = None

c_i64 = ctypes.c_int64
c_int = ctypes.c_int
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("max_newton", c_int),
        ("max_cg", c_int),
        ("tol", c_dbl),
        ("fixed_iters", c_int),
        ("warm_start", c_int),
        ("polish_K", c_vp),
        ("polish_dtype", c_int),
        ("verbose", c_int),
        ("precond", c_int),
        ("precond_refresh", c_int),
        ("continuation", c_int),
        ("loss", c_int),
        ("support_stop", c_int),
        ("support_X", c_vp),
        ("support_d", c_i64),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("newton_iters", c_int),
        ("cg_iters", c_int),
        ("passes", c_int),
        ("grad_norm", c_dbl),
        ("objective", c_dbl),
        ("alpha_norm", c_dbl),
        ("status", c_int),
        ("hess_passes", c_int),
        ("precond_updates", c_int),
        ("stop_reason", c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes)
_SIGNATURES = {
    "tk_last_error": (ctypes.c_char_p, []),
    "tk_max_points": (c_i64, []),
    "tk_packed_count": (c_int, [c_i64, c_int, ctypes.POINTER(c_i64)]),
    "tk_packed_bytes": (c_int, [c_i64, c_int, c_int, ctypes.POINTER(c_i64)]),
    "tk_build_packed_tensor": (c_int, [c_vp, c_i64, c_i64, c_int, c_int, c_dbl, c_int, c_vp, c_vp]),
    "tk_contract_workspace": (c_int, [c_i64, c_int, c_i64, c_int, ctypes.POINTER(c_sz)]),
    "tk_contract": (c_int, [c_vp, c_int, c_i64, c_int, c_vp, c_i64, c_vp, c_int, c_vp, c_sz, c_vp]),
    "tk_contract_noalloc": (c_int, [c_vp, c_int, c_i64, c_int, c_vp, c_i64, c_vp, c_int, c_vp]),
    "tk_contract_noalloc_max_bytes": (c_sz, []),
    "tk_hvp": (c_int, [c_vp, c_int, c_i64, c_int, c_vp, c_vp, c_i64, c_vp, c_vp, c_int, c_vp, c_sz, c_vp]),
    "tk_hessian_workspace": (c_int, [c_i64, c_int, ctypes.POINTER(c_sz)]),
    "tk_hessian": (c_int, [c_vp, c_int, c_i64, c_int, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "tk_autotune": (c_int, [c_vp, c_int, c_i64, c_int, c_vp, c_vp, c_i64, c_int, c_vp, c_vp, c_sz, c_vp,
                            ctypes.POINTER(c_int), ctypes.POINTER(c_dbl)]),
    "tk_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "tk_solve_workspace": (c_int, [c_i64, c_int, c_i64, c_int, ctypes.POINTER(c_sz)]),
    "tk_solve_workspace_ex": (c_int, [c_i64, c_int, c_i64, c_int, c_i64, ctypes.POINTER(c_sz)]),
    "tk_packed_stride": (c_int, [c_i64, c_int, c_int, ctypes.POINTER(c_i64)]),
    "tk_build_packed_multi": (c_int, [c_vp, c_i64, c_i64, c_i64, c_int, c_int, c_dbl, c_int, c_vp, c_i64, c_vp]),
    "tk_contract_multi": (c_int, [c_vp, c_int, c_i64, c_int, c_i64, c_i64, c_vp, c_vp, c_int, c_vp, c_sz, c_vp]),
    "tk_solve_dual_multi": (c_int, [c_vp, c_int, c_i64, c_int, c_i64, c_i64, c_vp, ctypes.POINTER(c_dbl), c_i64,
                                    ctypes.POINTER(SolveOpts), c_vp, ctypes.POINTER(SolveInfo), c_vp, c_sz, c_vp]),
    "tk_solve_dual": (c_int, [c_vp, c_int, c_i64, c_int, c_vp, ctypes.POINTER(c_dbl), c_i64,
                              ctypes.POINTER(SolveOpts), c_vp, ctypes.POINTER(SolveInfo), c_vp, c_sz, c_vp]),
    "tk_primal_weights": (c_int, [c_vp, c_i64, c_i64, c_int, c_vp, c_i64, c_vp, c_vp]),
    "tk_predict": (c_int, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "tk_predict_kernel_workspace": (c_int, [c_i64, c_int, c_i64, c_i64, ctypes.POINTER(c_sz)]),
    "tk_predict_kernel": (c_int, [c_vp, c_i64, c_i64, c_int, c_int, c_dbl, c_vp, c_i64, c_vp, c_i64, c_vp,
                                  c_vp, c_sz, c_vp]),
    "tk_contract_dense": (c_int, [c_vp, c_i64, c_i64, c_int, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "tk_support": (c_int, [c_vp, c_i64, c_i64, c_vp, c_vp, c_vp]),
    "tk_gather_rows": (c_int, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "tk_dmse_workspace": (c_int, [c_i64, c_int, c_i64, c_i64, c_int, ctypes.POINTER(c_sz)]),
    "tk_dmse_dlambda": (c_int, [c_vp, c_int, c_i64, c_int, c_vp, c_i64, c_vp, c_dbl, c_vp, c_vp, c_i64,
                                c_dbl, c_int, ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl), c_vp, c_vp,
                                c_sz, c_vp]),
    "tk_probe_stream_read": (c_int, [c_vp, c_i64, c_vp, c_int, c_vp]),
    "tk_timing_start": (c_int, []),
    "tk_timing_stop": (c_int, [ctypes.POINTER(c_i64), ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl)]),
}


class TkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tk error {code}: {msg}")
        self.code = code


def load():
    """Load libtk.so (once).  Raises if it is missing: there is no CPU fallback."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                                   "`python -m paper_2003_10482_amd.build`")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(rc: int) -> int:
    if rc != 0:
        msg = load().tk_last_error().decode(errors="replace")
        raise TkError(rc, msg)
    return rc


def exported_symbols():
    return list(_SIGNATURES)
