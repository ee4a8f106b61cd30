"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects bad arguments on the host (no device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tk.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tk_[a-z0-9_]+)\s*\(", src)))


def _lib():
    from paper_2003_10482_amd import _lib
    return _lib.load()


def test_header_symbols_exported():
    lib = _lib()
    names = _declared()
    assert "tk_contract" in names and "tk_solve_dual" in names and "tk_build_packed_tensor" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_2003_10482_amd import _lib
    assert sorted(_lib.exported_symbols()) == _declared()


def test_packed_count_and_errors():
    from paper_2003_10482_amd import _lib
    lib = _lib.load()
    out = ctypes.c_int64()
    assert lib.tk_packed_count(256, 4, ctypes.byref(out)) == 0 and out.value == 183181376
    assert lib.tk_packed_count(128, 6, ctypes.byref(out)) == 0 and out.value == 6856577728
    assert lib.tk_packed_count(10 ** 6, 16, ctypes.byref(out)) == -2          # overflow
    assert lib.tk_packed_count(0, 4, ctypes.byref(out)) == -1
    assert b"n and m" in lib.tk_last_error()
    nb = ctypes.c_int64()
    assert lib.tk_packed_bytes(256, 4, 2, ctypes.byref(nb)) == 0 and nb.value == 2 * 183181376
    ws = ctypes.c_size_t()
    assert lib.tk_contract_workspace(256, 3, 1, 0, ctypes.byref(ws)) == -1     # odd order
    assert lib.tk_contract_workspace(257, 4, 1, 0, ctypes.byref(ws)) == -7     # above the tile limit
    assert lib.tk_contract_workspace(256, 4, 1, 9, ctypes.byref(ws)) == -1     # bad dtype
    assert lib.tk_contract_workspace(256, 4, 1, 0, ctypes.byref(ws)) == 0 and ws.value > 0


def test_invalid_calls_fail_before_device_work():
    from paper_2003_10482_amd import _lib
    lib = _lib.load()
    # null pointers and bad sizes are rejected on the host
    assert lib.tk_contract(None, 0, 64, 4, None, 1, None, 0, None, 0, None) == -1
    assert lib.tk_build_packed_tensor(None, 64, 20, 4, 0, 0.0, 0, None, None) == -1
    assert lib.tk_build_packed_tensor(None, 64, 20, 5, 0, 0.0, 0, None, None) == -1
    lams = (ctypes.c_double * 1)(-1.0)
    info = (_lib.SolveInfo * 1)()
    assert lib.tk_solve_dual(ctypes.c_void_p(8), 0, 64, 4, ctypes.c_void_p(8), lams, 1, None,
                             ctypes.c_void_p(8), info, ctypes.c_void_p(8), 1 << 30, None) == -1
    assert b"lambda" in lib.tk_last_error()


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(ROOT, "paper_2003_10482_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"#.*|//.*", "", txt).replace("Oracle", ""), f


def test_hessian_entry_points_on_host():
    """tk_hessian_workspace is host arithmetic that grows with the order and
    covers the unit vectors of m >= 4; tk_hessian rejects bad arguments
    before any device work, and the binding rejects host tensors."""
    import torch

    import paper_2003_10482_amd as tk
    from paper_2003_10482_amd import _lib
    lib = _lib.load()
    ws = ctypes.c_size_t()
    assert lib.tk_hessian_workspace(256, 4, ctypes.byref(ws)) == 0
    w4 = ws.value
    # at least the order-3 array of unit vectors, C(258, 3) doubles
    assert w4 >= 8 * 2829056
    assert lib.tk_hessian_workspace(64, 2, ctypes.byref(ws)) == 0 and 0 < ws.value < w4
    assert lib.tk_hessian_workspace(64, 3, ctypes.byref(ws)) == -1        # odd order
    assert lib.tk_hessian_workspace(300, 4, ctypes.byref(ws)) == -7       # above the tile limit
    assert lib.tk_hessian(None, 0, 64, 4, None, None, None, 0, None) == -1
    assert lib.tk_hessian(ctypes.c_void_p(8), 7, 64, 4, ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), 1, None) == -1                # bad dtype
    K = tk.PackedTensor(torch.zeros(tk.packed_count(5, 4), dtype=torch.float64), 5, 4, tk.F64)
    with pytest.raises(ValueError):
        tk.hessian(K, torch.zeros(5, dtype=torch.float64))
