"""Thin torch-facing binding of the C ABI (``include/tk.h``).

Every function only checks shapes, allocates outputs and workspaces with torch
on the current HIP device and forwards raw pointers plus the current stream to
``libtk.so``.  All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib

F64, F32, BF16 = 0, 1, 2
LINEAR, POLY, EXP = 0, 1, 2
ACC_AUTO, ACC_COMPENSATED, ACC_F64, ACC_F32 = 0, 1, 2, 3

_DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}
_TORCH_STORAGE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}
_KERNELS = {"linear": LINEAR, "poly": POLY, "exp": EXP, LINEAR: LINEAR, POLY: POLY, EXP: EXP}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    return t.contiguous()


def packed_count(n: int, m: int) -> int:
    out = ctypes.c_int64()
    _lib.check(_lib.load().tk_packed_count(n, m, ctypes.byref(out)))
    return out.value


def max_points() -> int:
    return int(_lib.load().tk_max_points())


class PackedTensor:
    """Device buffer of a packed symmetric tensor plus its shape metadata."""

    def __init__(self, data: torch.Tensor, n: int, m: int, dtype: int):
        self.data, self.n, self.m, self.dtype = data, n, m, dtype

    @property
    def count(self) -> int:
        return packed_count(self.n, self.m)

    @property
    def nbytes(self) -> int:
        return self.data.numel() * self.data.element_size()


def build_packed_tensor(X: torch.Tensor, m: int, kernel="linear", kparam: float = 0.0,
                        dtype="f64") -> PackedTensor:
    X = _dev_f64(X, "X")
    n, d = X.shape
    dt = _DTYPES[dtype]
    K = empty_packed(n, m, dt, X.device)
    _lib.check(_lib.load().tk_build_packed_tensor(_ptr(X), n, d, m, _KERNELS[kernel], float(kparam),
                                                  dt, _ptr(K), _stream()))
    return PackedTensor(K, n, m, dt)


def packed_bytes(n: int, m: int, dtype) -> int:
    out = ctypes.c_int64()
    _lib.check(_lib.load().tk_packed_bytes(n, m, _DTYPES[dtype], ctypes.byref(out)))
    return out.value


def empty_packed(n: int, m: int, dtype, device) -> torch.Tensor:
    """A device buffer for a packed tensor: C(n+m-1, m) elements of the storage
    type, padded to tk_packed_bytes (BF16 buffers are read a dword at a time)."""
    dt = _DTYPES[dtype]
    count = packed_count(n, m)
    esz = {F64: 8, F32: 4, BF16: 2}[dt]
    total = (packed_bytes(n, m, dt) + esz - 1) // esz
    buf = torch.empty(total, dtype=_TORCH_STORAGE[dt], device=device)
    buf[count:].zero_()   # padding read together with the last entries
    return buf[:count]


def contract_workspace(n: int, m: int, B: int, dtype) -> int:
    out = ctypes.c_size_t()
    _lib.check(_lib.load().tk_contract_workspace(n, m, B, _DTYPES[dtype], ctypes.byref(out)))
    return out.value


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def contract(K: PackedTensor, alpha: torch.Tensor, acc: int = ACC_AUTO,
             work: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g = K . alpha^{m-1}; alpha [n] or [B, n] float64 -> same shape."""
    alpha = _dev_f64(alpha, "alpha")
    a2 = alpha.reshape(-1, K.n)
    B = a2.shape[0]
    g = torch.empty_like(a2) if out is None else out
    if B == 0:   # an empty batch: nothing to compute
        return g.reshape(alpha.shape)
    if work is None:
        work = _workspace(contract_workspace(K.n, K.m, B, K.dtype), alpha.device)
    _lib.check(_lib.load().tk_contract(_ptr(K.data), K.dtype, K.n, K.m, _ptr(a2), B, _ptr(g), acc,
                                       _ptr(work), work.numel(), _stream()))
    return g.reshape(alpha.shape)


def contract_noalloc(K: PackedTensor, alpha: torch.Tensor, acc: int = ACC_AUTO,
                     out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g = K . alpha^{m-1} through the allocation-free entry point (its
    workspace is the library's fixed device scratch).  `out` may be given so
    the call itself allocates nothing."""
    alpha = _dev_f64(alpha, "alpha")
    a2 = alpha.reshape(-1, K.n)
    B = a2.shape[0]
    g = torch.empty_like(a2) if out is None else out
    if B == 0:
        return g.reshape(alpha.shape)
    _lib.check(_lib.load().tk_contract_noalloc(_ptr(K.data), K.dtype, K.n, K.m, _ptr(a2), B, _ptr(g), acc,
                                               _stream()))
    return g.reshape(alpha.shape)


def hvp(K: PackedTensor, alpha: torch.Tensor, v: torch.Tensor, with_g: bool = False,
        work: Optional[torch.Tensor] = None, acc: int = ACC_AUTO):
    """h = (m-1) K x_2 v x_3 alpha .. x_m alpha (and g when with_g)."""
    alpha = _dev_f64(alpha, "alpha")
    v = _dev_f64(v, "v")
    a2 = alpha.reshape(-1, K.n)
    v2 = v.reshape(-1, K.n)
    if a2.shape != v2.shape:
        raise ValueError("alpha and v shapes differ")
    B = a2.shape[0]
    h = torch.empty_like(a2)
    g = torch.empty_like(a2) if with_g else None
    if B == 0:   # an empty batch: nothing to compute
        return (h.reshape(alpha.shape), g.reshape(alpha.shape)) if with_g else h.reshape(alpha.shape)
    if work is None:
        work = _workspace(contract_workspace(K.n, K.m, B, K.dtype), alpha.device)
    _lib.check(_lib.load().tk_hvp(_ptr(K.data), K.dtype, K.n, K.m, _ptr(a2), _ptr(v2), B, _ptr(h), _ptr(g),
                                  acc, _ptr(work), work.numel(), _stream()))
    if with_g:
        return h.reshape(alpha.shape), g.reshape(alpha.shape)
    return h.reshape(alpha.shape)


def hessian_workspace(n: int, m: int) -> int:
    out = ctypes.c_size_t()
    _lib.check(_lib.load().tk_hessian_workspace(n, m, ctypes.byref(out)))
    return out.value


def hessian(K: PackedTensor, alpha: torch.Tensor, work: Optional[torch.Tensor] = None) -> torch.Tensor:
    """J = (m-1) K . alpha^{m-2}, the n x n Jacobian of the contraction (J v
    equals hvp(K, alpha, v)), in two reads of the packed tensor."""
    a = _dev_f64(alpha, "alpha").reshape(K.n)
    J = torch.empty(K.n, K.n, dtype=torch.float64, device=a.device)
    if work is None:
        work = _workspace(hessian_workspace(K.n, K.m), a.device)
    _lib.check(_lib.load().tk_hessian(_ptr(K.data), K.dtype, K.n, K.m, _ptr(a), _ptr(J), _ptr(work), work.numel(),
                                      _stream()))
    return J


def solve_workspace(n: int, m: int, B: int, dtype) -> int:
    out = ctypes.c_size_t()
    _lib.check(_lib.load().tk_solve_workspace(n, m, B, _DTYPES[dtype], ctypes.byref(out)))
    return out.value


def autotune(K: PackedTensor, alpha: torch.Tensor, v: Optional[torch.Tensor] = None, acc: int = ACC_AUTO):
    """Pick (and remember for this device and shape) the vector tile of
    contract (v None) or hvp with these B vectors.  Returns (tile, {tile: ms},
    out) where out holds the results of the last tile timed (the largest)."""
    a2 = _dev_f64(alpha, "alpha").reshape(-1, K.n)
    B = a2.shape[0]
    v2 = None if v is None else _dev_f64(v, "v").reshape(B, K.n)
    out = torch.empty(B, K.n, dtype=torch.float64, device=a2.device)
    work = _workspace(contract_workspace(K.n, K.m, B, K.dtype), a2.device)
    tile = ctypes.c_int()
    ms = (ctypes.c_double * 4)()
    _lib.check(_lib.load().tk_autotune(_ptr(K.data), K.dtype, K.n, K.m, _ptr(a2), _ptr(v2), B, acc, _ptr(out),
                                       _ptr(work), work.numel(), _stream(), ctypes.byref(tile), ms))
    return tile.value, {t: ms[i] for i, t in enumerate((1, 2, 4, 16)) if ms[i] >= 0}, out


LOSSES = {"square": 0, "logistic": 1}


def _opts(tol, max_newton, max_cg, fixed_iters, verbose, precond, precond_refresh, continuation, loss):
    opts = _lib.SolveOpts()
    _lib.load().tk_solve_opts_default(ctypes.byref(opts))
    opts.tol = tol
    opts.max_newton = max_newton
    opts.max_cg = max_cg
    opts.fixed_iters = fixed_iters
    opts.verbose = int(verbose)
    opts.precond = int(precond)
    opts.precond_refresh = int(precond_refresh)
    opts.continuation = int(continuation)
    opts.loss = LOSSES[loss] if isinstance(loss, str) else int(loss)
    return opts


def solve_dual(K: PackedTensor, y: torch.Tensor, lambdas: Sequence[float], tol: float = 1e-11,
               max_newton: int = 100, max_cg: int = 2000, fixed_iters: int = 0,
               alpha0: Optional[torch.Tensor] = None, polish: Optional[PackedTensor] = None,
               verbose: bool = False, raise_on_noconv: bool = False, precond: bool = True,
               precond_refresh: int = 25, continuation: bool = True, loss="square",
               support_stop: int = 0, support_X: Optional[torch.Tensor] = None):
    """Dual solve for every lambda.  Returns (alpha [B, n], list of info dicts).
    precond: Newton systems on the assembled Hessian with an inverse
    preconditioner (else unpreconditioned CG on tensor passes); continuation: lambdas solved from the
    largest down, each from the previous solution (else in lock step).  loss: "square" or
    "logistic" (labels in {-1, +1}).  support_stop > 0 (linear kernel, support_X = the points):
    also stop once the 2-std support of w has not changed for that many Newton steps."""
    y = _dev_f64(y, "y")
    if y.numel() != K.n:
        raise ValueError(f"y has {y.numel()} entries but the tensor has n = {K.n}")
    lams = [float(x) for x in lambdas]
    B = len(lams)
    opts = _opts(tol, max_newton, max_cg, fixed_iters, verbose, precond, precond_refresh, continuation, loss)
    sd = 0
    if support_stop > 0:
        if support_X is None:
            raise ValueError("support_stop needs support_X (the points the tensor was built from)")
        support_X = _dev_f64(support_X, "support_X")
        if support_X.shape[0] != K.n:
            raise ValueError("support_X must have n rows")
        sd = support_X.shape[1]
        opts.support_stop = int(support_stop)
        opts.support_X = support_X.data_ptr()
        opts.support_d = sd
    if polish is not None:
        if polish.n != K.n or polish.m != K.m or polish.dtype != F64:
            raise ValueError("the polish tensor must be an FP64 tensor of the same n and m")
        opts.polish_K = polish.data.data_ptr()
        opts.polish_dtype = polish.dtype
    alpha = torch.zeros(B, K.n, dtype=torch.float64, device=y.device)
    if alpha0 is not None:
        alpha.copy_(alpha0.reshape(B, K.n))
        opts.warm_start = 1
    infos = (_lib.SolveInfo * B)()
    h_l = (ctypes.c_double * B)(*lams)
    ws = ctypes.c_size_t()
    _lib.check(_lib.load().tk_solve_workspace_ex(K.n, K.m, B, K.dtype, sd, ctypes.byref(ws)))
    work = _workspace(ws.value, y.device)
    rc = _lib.load().tk_solve_dual(_ptr(K.data), K.dtype, K.n, K.m, _ptr(y), h_l, B, ctypes.byref(opts),
                                   _ptr(alpha), infos, _ptr(work), work.numel(), _stream())
    if rc != 0 and (raise_on_noconv or rc not in (-5, -6)):
        _lib.check(rc)
    return alpha, [infos[i].as_dict() for i in range(B)]


class MultiPackedTensor:
    """T packed tensors of the same (n, m, dtype), tensor t at t * stride entries."""

    def __init__(self, data: torch.Tensor, T: int, n: int, m: int, dtype: int, stride: int):
        self.data, self.T, self.n, self.m, self.dtype, self.stride = data, T, n, m, dtype, stride

    def tensor(self, t: int) -> PackedTensor:
        return PackedTensor(self.data[t * self.stride: t * self.stride + packed_count(self.n, self.m)],
                            self.n, self.m, self.dtype)


def packed_stride(n: int, m: int, dtype) -> int:
    out = ctypes.c_int64()
    _lib.check(_lib.load().tk_packed_stride(n, m, _DTYPES[dtype], ctypes.byref(out)))
    return out.value


def build_packed_multi(Xs: torch.Tensor, m: int, kernel="linear", kparam: float = 0.0,
                       dtype="f64") -> MultiPackedTensor:
    """Xs [T, n, d]: one packed tensor per draw, side by side."""
    Xs = _dev_f64(Xs, "Xs")
    T, n, d = Xs.shape
    dt = _DTYPES[dtype]
    stride = packed_stride(n, m, dt)
    data = torch.zeros(T * stride, dtype=_TORCH_STORAGE[dt], device=Xs.device)
    _lib.check(_lib.load().tk_build_packed_multi(_ptr(Xs), T, n, d, m, _KERNELS[kernel], float(kparam), dt,
                                                 _ptr(data), stride, _stream()))
    return MultiPackedTensor(data, T, n, m, dt, stride)


def contract_multi(Km: MultiPackedTensor, alpha: torch.Tensor, acc: int = ACC_AUTO) -> torch.Tensor:
    """g_t = K_t . alpha_t^{m-1}, alpha [T, n] -> [T, n], one launch per pass."""
    alpha = _dev_f64(alpha, "alpha").reshape(Km.T, Km.n)
    g = torch.empty_like(alpha)
    work = _workspace(contract_workspace(Km.n, Km.m, Km.T, Km.dtype), alpha.device)
    _lib.check(_lib.load().tk_contract_multi(_ptr(Km.data), Km.dtype, Km.n, Km.m, Km.T, Km.stride, _ptr(alpha),
                                             _ptr(g), acc, _ptr(work), work.numel(), _stream()))
    return g


def solve_dual_multi(Km: MultiPackedTensor, Y: torch.Tensor, lambdas: Sequence[float], tol: float = 1e-11,
                     max_newton: int = 100, max_cg: int = 2000, loss="square", verbose: bool = False):
    """Every (draw, lambda) dual: Y [T, n] responses; returns (alpha [L, T, n],
    infos [L][T]).  Draws in lock step, lambdas by continuation."""
    Y = _dev_f64(Y, "Y").reshape(Km.T, Km.n)
    lams = [float(x) for x in lambdas]
    L = len(lams)
    opts = _opts(tol, max_newton, max_cg, 0, verbose, True, 25, True, loss)
    alpha = torch.zeros(L, Km.T, Km.n, dtype=torch.float64, device=Y.device)
    infos = (_lib.SolveInfo * (L * Km.T))()
    h_l = (ctypes.c_double * L)(*lams)
    work = _workspace(solve_workspace(Km.n, Km.m, min(Km.T, 64), Km.dtype), Y.device)
    rc = _lib.load().tk_solve_dual_multi(_ptr(Km.data), Km.dtype, Km.n, Km.m, Km.T, Km.stride, _ptr(Y), h_l, L,
                                         ctypes.byref(opts), _ptr(alpha), infos, _ptr(work), work.numel(),
                                         _stream())
    if rc != 0 and rc not in (-5, -6):
        _lib.check(rc)
    return alpha, [[infos[l * Km.T + t].as_dict() for t in range(Km.T)] for l in range(L)]


def primal_weights(X: torch.Tensor, alpha: torch.Tensor, m: int) -> torch.Tensor:
    X = _dev_f64(X, "X")
    alpha = _dev_f64(alpha, "alpha")
    n, d = X.shape
    a2 = alpha.reshape(-1, n)
    W = torch.empty(a2.shape[0], d, dtype=torch.float64, device=X.device)
    _lib.check(_lib.load().tk_primal_weights(_ptr(X), n, d, m, _ptr(a2), a2.shape[0], _ptr(W), _stream()))
    return W if alpha.dim() == 2 else W[0]


def predict(W: torch.Tensor, Xq: torch.Tensor) -> torch.Tensor:
    W = _dev_f64(W, "W")
    Xq = _dev_f64(Xq, "Xq")
    W2 = W.reshape(-1, W.shape[-1])
    N, d = Xq.shape
    f = torch.empty(W2.shape[0], N, dtype=torch.float64, device=W.device)
    _lib.check(_lib.load().tk_predict(_ptr(W2), d, W2.shape[0], _ptr(Xq), N, _ptr(f), _stream()))
    return f if W.dim() == 2 else f[0]


def predict_kernel(X: torch.Tensor, alpha: torch.Tensor, Xq: torch.Tensor, m: int, kernel="linear",
                   kparam: float = 0.0) -> torch.Tensor:
    """General tensor-kernel prediction: f_b(x) = sum over sorted (m-1)-tuples T
    of c(T) alpha_b^T k(x_T, x).  alpha [n] or [B, n] -> f [N] or [B, N]."""
    X, alpha, Xq = _dev_f64(X, "X"), _dev_f64(alpha, "alpha"), _dev_f64(Xq, "Xq")
    n, d = X.shape
    N, dq = Xq.shape
    if dq != d:
        raise ValueError("X and Xq have different feature counts")
    a2 = alpha.reshape(-1, n)
    B = a2.shape[0]
    f = torch.empty(B, N, dtype=torch.float64, device=X.device)
    ws = ctypes.c_size_t()
    _lib.check(_lib.load().tk_predict_kernel_workspace(n, m, B, N, ctypes.byref(ws)))
    work = _workspace(ws.value, X.device)
    _lib.check(_lib.load().tk_predict_kernel(_ptr(X), n, d, m, _KERNELS[kernel], float(kparam), _ptr(a2), B,
                                             _ptr(Xq), N, _ptr(f), _ptr(work), work.numel(), _stream()))
    return f if alpha.dim() == 2 else f[0]


def contract_dense(X: torch.Tensor, alpha: torch.Tensor, m: int) -> torch.Tensor:
    X = _dev_f64(X, "X")
    alpha = _dev_f64(alpha, "alpha")
    n, d = X.shape
    a2 = alpha.reshape(-1, n)
    g = torch.empty_like(a2)
    work = torch.empty(a2.shape[0] * d, dtype=torch.float64, device=X.device)
    _lib.check(_lib.load().tk_contract_dense(_ptr(X), n, d, m, _ptr(a2), a2.shape[0], _ptr(g), _ptr(work),
                                             _stream()))
    return g.reshape(alpha.shape)


def support(W: torch.Tensor):
    W = _dev_f64(W, "W")
    W2 = W.reshape(-1, W.shape[-1])
    mask = torch.empty(W2.shape, dtype=torch.uint8, device=W.device)
    tau = torch.empty(W2.shape[0], dtype=torch.float64, device=W.device)
    _lib.check(_lib.load().tk_support(_ptr(W2), W2.shape[1], W2.shape[0], _ptr(mask), _ptr(tau), _stream()))
    if W.dim() == 1:
        return mask[0].bool(), tau[0]
    return mask.bool(), tau


def gather_rows(X: torch.Tensor, idx: torch.Tensor) -> torch.Tensor:
    X = _dev_f64(X, "X")
    if idx.dtype != torch.int64 or not idx.is_cuda:
        raise ValueError("idx must be an int64 device tensor")
    idx = idx.contiguous()
    N, d = X.shape
    out = torch.empty(idx.numel(), d, dtype=torch.float64, device=X.device)
    _lib.check(_lib.load().tk_gather_rows(_ptr(X), N, d, _ptr(idx), idx.numel(), _ptr(out), _stream()))
    return out


def dmse_dlambda(K: PackedTensor, X: torch.Tensor, alpha: torch.Tensor, lam: float, X_val: torch.Tensor,
                 y_val: torch.Tensor, cg_tol: float = 1e-12, max_cg: int = 5000):
    """(MSE_val, dMSE_val/dlambda, z) at a dual optimum alpha (implicit differentiation)."""
    X, alpha = _dev_f64(X, "X"), _dev_f64(alpha, "alpha")
    X_val, y_val = _dev_f64(X_val, "X_val"), _dev_f64(y_val, "y_val")
    n, d = X.shape
    if n != K.n:
        raise ValueError(f"X has {n} rows but the tensor has n = {K.n}")
    if alpha.numel() != n or X_val.shape[1] != d or y_val.numel() != X_val.shape[0]:
        raise ValueError("alpha, X_val or y_val shape does not match X")
    nval = X_val.shape[0]
    ws = ctypes.c_size_t()
    _lib.check(_lib.load().tk_dmse_workspace(n, K.m, d, nval, K.dtype, ctypes.byref(ws)))
    work = _workspace(ws.value, X.device)
    z = torch.empty(n, dtype=torch.float64, device=X.device)
    mse = ctypes.c_double()
    dmse = ctypes.c_double()
    _lib.check(_lib.load().tk_dmse_dlambda(_ptr(K.data), K.dtype, n, K.m, _ptr(X), d, _ptr(alpha.reshape(-1)),
                                           float(lam), _ptr(X_val), _ptr(y_val), nval, cg_tol, max_cg,
                                           ctypes.byref(mse), ctypes.byref(dmse), _ptr(z), _ptr(work),
                                           work.numel(), _stream()))
    return mse.value, dmse.value, z


class TkContract(torch.autograd.Function):
    """g = K . alpha^{m-1} with its adjoint: the Jacobian (m-1) K x_3 alpha .. is
    symmetric, so the backward product is the directional derivative kernel."""

    @staticmethod
    def forward(ctx, alpha: torch.Tensor, K: PackedTensor):
        ctx.K = K
        ctx.save_for_backward(alpha)
        return contract(K, alpha.detach())

    @staticmethod
    def backward(ctx, grad_g: torch.Tensor):
        (alpha,) = ctx.saved_tensors
        return hvp(ctx.K, alpha.detach(), grad_g.contiguous()), None


def contract_autograd(K: PackedTensor, alpha: torch.Tensor) -> torch.Tensor:
    return TkContract.apply(alpha, K)


def timing_start() -> None:
    """Start bracketing every packed-tensor pass with HIP events (instrumentation)."""
    _lib.check(_lib.load().tk_timing_start())


TIMING_KINDS = ("contract", "hvp", "contract_plain", "hessian_tiles", "hessian_units")


def timing_stop() -> dict:
    """Stop and return {kind: (launches, total_ms, bytes)} for every kind in
    TIMING_KINDS (compensated contraction, directional derivative, plain
    contraction, the two streaming kernels of the Hessian)."""
    k = len(TIMING_KINDS)
    n = (ctypes.c_int64 * k)()
    ms = (ctypes.c_double * k)()
    by = (ctypes.c_double * k)()
    _lib.check(_lib.load().tk_timing_stop(n, ms, by))
    return {name: (n[i], ms[i], by[i]) for i, name in enumerate(TIMING_KINDS)}


def probe_stream_read(buf: torch.Tensor, groups: int = 2048,
                      sink: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Instrumentation: stream the bytes of a device buffer (its size rounded
    down to 16 bytes) through a plain read kernel; returns the per-workgroup
    checksums.  Timed with events, it gives the device's achievable HBM read
    rate."""
    if not buf.is_cuda:
        raise ValueError("buf must be a device tensor")
    nbytes = (buf.numel() * buf.element_size()) // 16 * 16
    if sink is None:
        sink = torch.empty(groups, dtype=torch.int64, device=buf.device)
    _lib.check(_lib.load().tk_probe_stream_read(_ptr(buf), nbytes, _ptr(sink), groups, _stream()))
    return sink
