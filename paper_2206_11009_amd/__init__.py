"""otip: interior-point-inspired column generation for the Kantorovich OT LP
on AMD MI355X (Zanetti & Gondzio, arXiv 2206.11009).

Thin Python binding of the C-ABI library ``libotip.so`` (``include/otip.h``).
The functions carry the C names; they only marshal arguments -- torch tensors
hold device memory, torch's current stream is the stream -- and every step of
the method runs in the library's HIP kernels.  There is no CPU fallback: the
calls raise if the library is not built or no GPU is present.
"""
from __future__ import annotations

import ctypes
import os as _os
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import (OTIP_OK, OTIP_EINVAL, OTIP_ENOMEM, OTIP_EHIP, OTIP_ENUMERIC, OTIP_EUNSUPPORTED,  # noqa: F401
                   OTIP_EMAXITER, OTIP_FP64, OTIP_MIXED, OTIP_LS_AUTO, OTIP_LS_PCG,  # noqa: F401
                   OTIP_LS_DIRECT, OTIP_COST_SQEUCLID, OTIP_COST_L1, OTIP_COST_L2,  # noqa: F401
                   OTIP_COST_LINF, otip_params, otip_problem, otip_info)

__all__ = ["otip_version", "otip_params_default", "Context", "OtipError", "SolveResult",
           "otip_solve", "otip_solve_batch", "otip_price", "otip_price_subset", "otip_rmin", "otip_kron_apply",
           "otip_kron_apply_t", "otip_kron_apply_noalloc", "otip_schur", "otip_ldl_solve", "otip_pcg", "PCGResult", "otip_state_save",
           "otip_state_load", "params", "otip_ws_param_count", "otip_ws_forward",
           "otip_ws_grad", "otip_ws_adam", "otip_ws_predict", "load_ws_weights"]


class OtipError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"otip error {code}: {msg}")
        self.code = code


def otip_version() -> int:
    return _abi.load().otip_version()


def otip_params_default() -> otip_params:
    p = otip_params()
    _abi.load().otip_params_default(ctypes.byref(p))
    return p


def params(**kw) -> otip_params:
    """Defaults with some fields overridden, e.g. params(tol=1e-8, verbose=1)."""
    p = otip_params_default()
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise OtipError(_abi.OTIP_EINVAL, "no GPU: the otip library runs on an AMD GPU only")
    return torch


class Context:
    """An otip context bound to a device and torch's current stream on it."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = device
        with torch.cuda.device(device):
            stream = torch.cuda.current_stream(device).cuda_stream
        self._lib = _abi.load()
        h = ctypes.c_void_p()
        rc = self._lib.otip_create(ctypes.byref(h), device, ctypes.c_void_p(stream))
        if rc != OTIP_OK:
            raise OtipError(rc, "otip_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self._lib.otip_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc, allow=(OTIP_OK,)):
        if rc not in allow:
            raise OtipError(rc, self._lib.otip_last_error(self.handle).decode())
        return rc


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev(x, dtype, device):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        return x.to(device=f"cuda:{device}", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=f"cuda:{device}")


@dataclass
class SolveResult:
    status: int
    info: dict
    rows: np.ndarray
    cols: np.ndarray
    flows: np.ndarray
    y: np.ndarray
    z: np.ndarray

    def __getattr__(self, k):
        info = self.__dict__.get("info", {})
        if k in info:
            return info[k]
        raise AttributeError(k)


def _problem(ctx, a, b, xs, xt, y0=None, z0=None, cost_kind=0):
    torch = _torch()
    A = _dev(a, torch.float64, ctx.device)
    B = _dev(b, torch.float64, ctx.device)
    XS = _dev(xs, torch.int32, ctx.device)
    XT = _dev(xt, torch.int32, ctx.device)
    Y0 = _dev(y0, torch.float64, ctx.device) if y0 is not None else None
    Z0 = _dev(z0, torch.float64, ctx.device) if z0 is not None else None
    pr = otip_problem(int(A.shape[0]), int(B.shape[0]), A.data_ptr(), B.data_ptr(),
                      XS.data_ptr(), XT.data_ptr(),
                      Y0.data_ptr() if Y0 is not None else None,
                      Z0.data_ptr() if Z0 is not None else None, int(cost_kind))
    return pr, (A, B, XS, XT, Y0, Z0)


def _collect(ctx, res_handle, rc):
    lib = ctx._lib
    info = otip_info()
    ctx.check(lib.otip_result_info(res_handle, ctypes.byref(info)))
    d = info.as_dict()
    nnz = int(info.nnz)
    rows = np.empty(nnz, np.int32)
    cols = np.empty(nnz, np.int32)
    vals = np.empty(nnz, np.float64)
    return d, rows, cols, vals


def otip_solve(ctx: Context, a, b, xs, xt, prm: otip_params | None = None, y0=None,
               z0=None, cost_kind: int = OTIP_COST_SQEUCLID) -> SolveResult:
    """Solve one problem; a, b, xs, xt (and the optional warm-start duals y0,
    z0) may be numpy arrays or torch tensors; cost_kind is an OTIP_COST_*."""
    pr, keep = _problem(ctx, a, b, xs, xt, y0, z0, cost_kind)
    h = ctypes.c_void_p()
    rc = ctx._lib.otip_solve(ctx.handle, ctypes.byref(pr),
                             ctypes.byref(prm) if prm is not None else None, ctypes.byref(h))
    ctx.check(rc, (OTIP_OK, OTIP_EMAXITER, OTIP_ENUMERIC))
    try:
        d, rows, cols, vals = _collect(ctx, h, rc)
        y = np.empty(pr.m, np.float64)
        z = np.empty(pr.n, np.float64)
        ctx.check(ctx._lib.otip_result_copy(h, rows.ctypes.data, cols.ctypes.data,
                                            vals.ctypes.data, y.ctypes.data, z.ctypes.data))
    finally:
        ctx._lib.otip_result_free(h)
    del keep
    return SolveResult(rc, d, rows, cols, vals, y, z)


def otip_solve_batch(ctx: Context, problems, prm: otip_params | None = None,
                     cost_kind: int = OTIP_COST_SQEUCLID):
    """Solve a list of (a, b, xs, xt) or (a, b, xs, xt, y0, z0) problems, all
    with the cost cost_kind; returns a list of SolveResult in the same order."""
    prs = (otip_problem * len(problems))()
    keep = []
    for k, prob in enumerate(problems):
        prob = tuple(prob) + (None,) * (6 - len(prob))
        pr, kk = _problem(ctx, *prob, cost_kind=cost_kind)
        prs[k] = pr
        keep.append(kk)
    outs = (ctypes.c_void_p * len(problems))()
    rc = ctx._lib.otip_solve_batch(ctx.handle, prs, len(problems),
                                   ctypes.byref(prm) if prm is not None else None, outs)
    ctx.check(rc, (OTIP_OK, OTIP_EMAXITER, OTIP_ENUMERIC))
    results = []
    for k in range(len(problems)):
        h = ctypes.c_void_p(outs[k])
        d, rows, cols, vals = _collect(ctx, h, rc)
        y = np.empty(prs[k].m, np.float64)
        z = np.empty(prs[k].n, np.float64)
        ctx.check(ctx._lib.otip_result_copy(h, rows.ctypes.data, cols.ctypes.data,
                                            vals.ctypes.data, y.ctypes.data, z.ctypes.data))
        ctx._lib.otip_result_free(h)
        results.append(SolveResult(d["status"], d, rows, cols, vals, y, z))
    return results


def otip_price(ctx: Context, xs, xt, y, z, bitmap, kmax: int, precision: int = OTIP_FP64,
               tile: int = 0, cost_kind: int = OTIP_COST_SQEUCLID):
    """Pricing scan; returns (i, j, r) device tensors of the selected columns and
    the count of negative reduced costs outside the support."""
    torch = _torch()
    XS, XT = _dev(xs, torch.int32, ctx.device), _dev(xt, torch.int32, ctx.device)
    Y, Z = _dev(y, torch.float64, ctx.device), _dev(z, torch.float64, ctx.device)
    BM = _dev(bitmap, torch.int32, ctx.device) if bitmap is not None else None
    m, n = int(XS.shape[0]), int(XT.shape[0])
    k = max(int(kmax), 1)
    oi = torch.empty(k, dtype=torch.int32, device=Y.device)
    oj = torch.empty(k, dtype=torch.int32, device=Y.device)
    orr = torch.empty(k, dtype=torch.float64, device=Y.device)
    cnt, nneg = ctypes.c_int64(), ctypes.c_int64()
    ctx.check(ctx._lib.otip_price(ctx.handle, m, n, _ptr(XS), _ptr(XT), _ptr(Y), _ptr(Z),
                                  _ptr(BM) if BM is not None else None, int(kmax), precision,
                                  int(tile), int(cost_kind), _ptr(oi), _ptr(oj), _ptr(orr),
                                  ctypes.byref(cnt),
                                  ctypes.byref(nneg)))
    c = int(cnt.value)
    return oi[:c], oj[:c], orr[:c], int(nneg.value)


def otip_price_subset(ctx: Context, xs, xt, y, z, bitmap, kmax: int, key_limit: int,
                      cost_kind: int = OTIP_COST_SQEUCLID):
    """Heuristic pricing over J = {cost key < key_limit} (Section 3.4); returns
    (i, j, r) device tensors, the count of negative reduced costs in J outside
    the support, and |J|."""
    torch = _torch()
    XS, XT = _dev(xs, torch.int32, ctx.device), _dev(xt, torch.int32, ctx.device)
    Y, Z = _dev(y, torch.float64, ctx.device), _dev(z, torch.float64, ctx.device)
    BM = _dev(bitmap, torch.int32, ctx.device) if bitmap is not None else None
    m, n = int(XS.shape[0]), int(XT.shape[0])
    k = max(int(kmax), 1)
    oi = torch.empty(k, dtype=torch.int32, device=Y.device)
    oj = torch.empty(k, dtype=torch.int32, device=Y.device)
    orr = torch.empty(k, dtype=torch.float64, device=Y.device)
    cnt, nneg, size = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    ctx.check(ctx._lib.otip_price_subset(ctx.handle, m, n, _ptr(XS), _ptr(XT), _ptr(Y), _ptr(Z),
                                         _ptr(BM) if BM is not None else None, int(kmax),
                                         int(cost_kind), int(key_limit), _ptr(oi), _ptr(oj),
                                         _ptr(orr), ctypes.byref(cnt), ctypes.byref(nneg),
                                         ctypes.byref(size)))
    c = int(cnt.value)
    return oi[:c], oj[:c], orr[:c], int(nneg.value), int(size.value)


def otip_rmin(ctx: Context, xs, xt, y, z, cost_kind: int = OTIP_COST_SQEUCLID):
    torch = _torch()
    XS, XT = _dev(xs, torch.int32, ctx.device), _dev(xt, torch.int32, ctx.device)
    Y, Z = _dev(y, torch.float64, ctx.device), _dev(z, torch.float64, ctx.device)
    v, arg = ctypes.c_double(), ctypes.c_int64()
    ctx.check(ctx._lib.otip_rmin(ctx.handle, int(XS.shape[0]), int(XT.shape[0]), _ptr(XS),
                                 _ptr(XT), _ptr(Y), _ptr(Z), int(cost_kind), ctypes.byref(v),
                                 ctypes.byref(arg)))
    return float(v.value), int(arg.value)


def otip_kron_apply(ctx: Context, X, rowsum, colsum):
    """rowsum = X e_n, colsum = X^T e_m for a column-major m x n float64 tensor
    (pass X as an (n, m) row-major tensor, i.e. vec(X) contiguous)."""
    n, m = X.shape
    ctx.check(ctx._lib.otip_kron_apply(ctx.handle, m, n, _ptr(X), _ptr(rowsum), _ptr(colsum)))


def otip_kron_apply_noalloc(ctx: Context, X, rowsum, colsum):
    """otip_kron_apply with its partial sums in the library's static per-GPU
    scratch (no device allocation); raises OtipError for sizes beyond it."""
    n, m = X.shape
    ctx.check(ctx._lib.otip_kron_apply_noalloc(ctx.handle, m, n, _ptr(X), _ptr(rowsum),
                                               _ptr(colsum)))


def otip_kron_apply_t(ctx: Context, y, z, X):
    n, m = X.shape
    ctx.check(ctx._lib.otip_kron_apply_t(ctx.handle, m, n, _ptr(y), _ptr(z), _ptr(X)))


def otip_schur(ctx: Context, m: int, n: int, idx, theta):
    """S_M of the support idx (sorted variable indices) with weights theta;
    returns (rowptr, colidx, vals, M, N) as device tensors."""
    torch = _torch()
    I = _dev(idx, torch.int64, ctx.device)
    T = _dev(theta, torch.float64, ctx.device)
    nnz = ctypes.c_int64()
    ctx.check(ctx._lib.otip_schur(ctx.handle, m, n, int(I.shape[0]), _ptr(I), _ptr(T),
                                  ctypes.byref(nnz), None, None, None, None, None))
    dev = I.device
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
    va = torch.empty(max(nnz.value, 1), dtype=torch.float64, device=dev)
    M = torch.empty(m, dtype=torch.float64, device=dev)
    N = torch.empty(n, dtype=torch.float64, device=dev)
    ctx.check(ctx._lib.otip_schur(ctx.handle, m, n, int(I.shape[0]), _ptr(I), _ptr(T),
                                  ctypes.byref(nnz), _ptr(rp), _ptr(ci), _ptr(va), _ptr(M),
                                  _ptr(N)))
    return rp, ci[:nnz.value], va[:nnz.value], M, N


def otip_ldl_solve(ctx: Context, rowptr, colidx, vals, b, pivot_tol: float = 1e-12,
                   substitution: bool = False):
    """Dense FP64 L D L^T with the infinite-pivot rule of a CSR matrix, then one
    solve; returns (x as a device tensor, infinite pivots, nnz(L))."""
    torch = _torch()
    RP = _dev(rowptr, torch.int32, ctx.device)
    CI = _dev(colidx, torch.int32, ctx.device)
    VA = _dev(vals, torch.float64, ctx.device)
    B = _dev(b, torch.float64, ctx.device)
    n = int(RP.shape[0]) - 1
    x = torch.empty(n, dtype=torch.float64, device=B.device)
    ninf, nnzl = ctypes.c_int32(), ctypes.c_int64()
    ctx.check(ctx._lib.otip_ldl_solve(ctx.handle, n, int(CI.shape[0]), _ptr(RP), _ptr(CI),
                                      _ptr(VA), float(pivot_tol), 1 if substitution else 0,
                                      _ptr(B), _ptr(x), ctypes.byref(ninf), ctypes.byref(nnzl)))
    return x, int(ninf.value), int(nnzl.value)


def otip_state_save(ctx: Context) -> bytes:
    """The record of where the context's latest otip_solve stopped iterating."""
    size = ctypes.c_int64()
    ctx.check(ctx._lib.otip_state_save(ctx.handle, None, 0, ctypes.byref(size)))
    buf = ctypes.create_string_buffer(size.value)
    ctx.check(ctx._lib.otip_state_save(ctx.handle, buf, size.value, ctypes.byref(size)))
    return buf.raw[:size.value]


def otip_state_load(ctx: Context, data: bytes) -> None:
    """Make the context's next otip_solve (of the same problem) continue from
    a record written by otip_state_save."""
    data = bytes(data)
    ctx.check(ctx._lib.otip_state_load(ctx.handle, ctypes.c_char_p(data), len(data)))


class PCGResult:
    """Outcome of otip_pcg: status (OTIP_OK, OTIP_EMAXITER or OTIP_ENUMERIC),
    iterations, final residual norm, and the timed iteration launches that did
    work (one per iteration; the SpMV launch for a matrix beyond 96 MB) with
    their mean duration (s) and algorithmic bytes per launch."""

    def __init__(self, status, iterations, res_norm, stats):
        self.status = status
        self.iterations = iterations
        self.res_norm = res_norm
        self.spmv_launches = int(stats[0])
        self.spmv_seconds = stats[1]
        self.spmv_bytes = stats[2]


def otip_pcg(ctx: Context, rowptr, colidx, vals, b, x=None, rtol=1e-6, maxit=1000,
             precision=0):
    """Jacobi-PCG on the CSR matrix (device tensors); x (device, n) is
    written.  Returns (x, PCGResult); errors other than the iteration limit
    and a breakdown raise."""
    torch = _torch()
    n = int(rowptr.shape[0]) - 1
    nnz = int(vals.shape[0])
    rp = _dev(rowptr, torch.int32, ctx.device)
    ci = _dev(colidx, torch.int32, ctx.device)
    va = _dev(vals, torch.float64, ctx.device)
    bb = _dev(b, torch.float64, ctx.device)
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=bb.device)
    elif not (x.dtype == torch.float64 and x.is_contiguous() and x.numel() == n
              and x.device == bb.device):
        raise OtipError(_abi.OTIP_EINVAL, "x must be a contiguous float64 device tensor of n")
    its = ctypes.c_int32()
    rn = ctypes.c_double()
    st = (ctypes.c_double * 3)()
    rc = ctx._lib.otip_pcg(ctx.handle, n, nnz, _ptr(rp), _ptr(ci), _ptr(va), _ptr(bb), _ptr(x),
                           float(rtol), int(maxit), int(precision), ctypes.byref(its),
                           ctypes.byref(rn), st)
    ctx.check(rc, allow=(_abi.OTIP_OK, _abi.OTIP_EMAXITER, _abi.OTIP_ENUMERIC))
    return x, PCGResult(rc, its.value, rn.value, list(st))


# ------------------------------------------------------------ learned warm start
def otip_ws_param_count() -> int:
    return int(_abi.load().otip_ws_param_count())


def otip_ws_forward(ctx: Context, weights, x):
    """net(x) for an (N, 2, H, W) float32 device tensor; returns a new tensor."""
    torch = _torch()
    x = x.contiguous()
    out = torch.empty_like(x)
    N, C, H, W = x.shape
    if C != 2:
        raise OtipError(_abi.OTIP_EINVAL, "input must have 2 channels")
    ctx.check(ctx._lib.otip_ws_forward(ctx.handle, _ptr(weights), N, H, W, _ptr(x), _ptr(out)))
    return out


def otip_ws_grad(ctx: Context, weights, x, target, grad=None):
    """(loss, grad) of the mean-squared error of net(x) against target."""
    torch = _torch()
    x, target = x.contiguous(), target.contiguous()
    if grad is None:
        grad = torch.empty_like(weights)
    N, _, H, W = x.shape
    loss = ctypes.c_double()
    ctx.check(ctx._lib.otip_ws_grad(ctx.handle, _ptr(weights), N, H, W, _ptr(x), _ptr(target),
                                    _ptr(grad), ctypes.byref(loss)))
    return float(loss.value), grad


def otip_ws_adam(ctx: Context, weights, m, v, grad, step: int, lr: float, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8):
    ctx.check(ctx._lib.otip_ws_adam(ctx.handle, _ptr(weights), _ptr(m), _ptr(v), _ptr(grad),
                                    int(step), float(lr), float(beta1), float(beta2), float(eps)))


def otip_ws_predict(ctx: Context, weights, side: int, a, b):
    """Predicted duals (y0, z0) of a side x side grid pair, as device tensors."""
    torch = _torch()
    A = _dev(a, torch.float64, ctx.device)
    B = _dev(b, torch.float64, ctx.device)
    y0 = torch.empty(side * side, dtype=torch.float64, device=A.device)
    z0 = torch.empty(side * side, dtype=torch.float64, device=A.device)
    ctx.check(ctx._lib.otip_ws_predict(ctx.handle, _ptr(weights), int(side), _ptr(A), _ptr(B),
                                       _ptr(y0), _ptr(z0)))
    return y0, z0


WS_WEIGHTS = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "ws_weights.bin")


def load_ws_weights(ctx: Context, path: str = WS_WEIGHTS):
    """The trained warm-start parameters (FP32 file written by ws_train) as a
    device tensor."""
    torch = _torch()
    w = np.fromfile(path, dtype="<f4")
    if w.size != otip_ws_param_count():
        raise OtipError(_abi.OTIP_EINVAL, f"{path}: {w.size} values, expected "
                        f"{otip_ws_param_count()}")
    return torch.as_tensor(w, device=f"cuda:{ctx.device}")
