"""Python face of the C ABI: a handle wrapper and the stencil builders.

PyTorch supplies device memory and the current HIP stream; every step of the
solve runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _capi
from ._capi import BCGError, check


def _stream_ptr(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require(t: torch.Tensor, name: str, dtype: torch.dtype, shape=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise BCGError(_capi.BCG_EINVAL, f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise BCGError(_capi.BCG_EINVAL, f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise BCGError(_capi.BCG_EINVAL, f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise BCGError(_capi.BCG_EINVAL, f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class BCG:
    """Block CG solver for one sparse SPD matrix and k right-hand sides.

    subalgebra: "block" (p = k), "global" (p | k, default 1), "parallel"
    (p = 1) or "hybrid" (p | k) -- the *-subalgebras of Section 2.
    """

    def __init__(self, rowptr: torch.Tensor, colind: torch.Tensor, values: torch.Tensor, k: int,
                 subalgebra: str = "block", p: int = 0):
        n = rowptr.numel() - 1
        nnz = colind.numel()
        _require(rowptr, "rowptr", torch.int32, (n + 1,))
        _require(colind, "colind", torch.int32, (nnz,))
        _require(values, "values", torch.float64, (nnz,))
        if subalgebra not in _capi.SUBALGEBRA:
            raise BCGError(_capi.BCG_EINVAL, f"unknown subalgebra {subalgebra!r}")
        self.n, self.nnz, self.k = n, nnz, k
        self.subalgebra = subalgebra
        self.device = values.device
        self._lib = _capi.lib()
        csr = _capi.Csr(n, nnz, rowptr.data_ptr(), colind.data_ptr(), values.data_ptr())
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            torch.cuda.current_stream(self.device).synchronize()
            check(self._lib.bcg_create(ctypes.byref(csr), k, _capi.SUBALGEBRA[subalgebra], p, ctypes.byref(h)))
        self._h = h
        self.rowptr, self.colind = rowptr, colind
        self.precision = "fp64"
        self.precond = "none"

    # -- configuration --------------------------------------------------
    def set_precision(self, mode: str = "fp64", inner_tol: float = 0.0, inner_maxit: int = 1000,
                      max_outer: int = 50) -> None:
        if mode not in _capi.PRECISION:
            raise BCGError(_capi.BCG_EINVAL, f"unknown precision {mode!r}")
        check(self._lib.bcg_set_precision(self._h, _capi.PRECISION[mode], inner_tol, inner_maxit, max_outer))
        self.precision = mode

    def set_preconditioner(self, kind: str = "none") -> None:
        """M of Algorithm 1: "none" (M = I) or "jacobi" (M = diag(A)); the stop
        rule then uses M^{-1}-norms of the residual columns."""
        if kind not in _capi.PRECOND:
            raise BCGError(_capi.BCG_EINVAL, f"unknown preconditioner {kind!r}")
        with torch.cuda.device(self.device):
            self._bind_stream()
            check(self._lib.bcg_set_preconditioner(self._h, _capi.PRECOND[kind]))
        self.precond = kind

    def _bind_stream(self):
        check(self._lib.bcg_set_stream(self._h, _stream_ptr(self.device)))

    # -- solve ------------------------------------------------------------
    def solve(self, B: torch.Tensor, X: torch.Tensor | None = None, tol: float = 1e-8, maxit: int = 10000):
        """Solve A X = B in place of X (zeros if None); returns (X, info)."""
        _require(B, "B", torch.float64, (self.n, self.k))
        if X is None:
            X = torch.zeros_like(B)
        _require(X, "X", torch.float64, (self.n, self.k))
        with torch.cuda.device(self.device):
            self._bind_stream()
            status = check(self._lib.bcg_solve(self._h, B.data_ptr(), X.data_ptr(), float(tol), int(maxit)))
        return X, self.info(status)

    def info(self, status: int | None = None) -> dict:
        inf = _capi.Info()
        check(self._lib.bcg_get_info(self._h, ctypes.byref(inf)))
        d = inf.as_dict()
        d["status_name"] = _capi.STATUS_NAME.get(d["status"], str(d["status"]))
        ratios = (ctypes.c_double * self.k)()
        check(self._lib.bcg_get_column_ratios(self._h, ratios, self.k))
        d["ratios"] = list(ratios)
        return d

    def update_values(self, values: torch.Tensor) -> None:
        _require(values, "values", torch.float64, (self.nnz,))
        with torch.cuda.device(self.device):
            self._bind_stream()
            check(self._lib.bcg_update_values(self._h, values.data_ptr()))

    def csr_outer(self, Y: torch.Tensor, X: torch.Tensor, alpha: float = -1.0) -> torch.Tensor:
        """out[e] = alpha * <Y[row(e)], X[col(e)]> on A's pattern."""
        _require(Y, "Y", torch.float64, (self.n, self.k))
        _require(X, "X", torch.float64, (self.n, self.k))
        out = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self._bind_stream()
            check(self._lib.bcg_csr_outer(self._h, Y.data_ptr(), X.data_ptr(), float(alpha), out.data_ptr()))
        return out

    def set_row_schedule(self, order: torch.Tensor | None) -> None:
        """Processing order of the sparse-product rows (a permutation), or None."""
        if order is not None:
            _require(order, "order", torch.int32, (self.n,))
        with torch.cuda.device(self.device):
            self._bind_stream()
            check(self._lib.bcg_set_row_schedule(self._h, None if order is None else order.data_ptr()))
        self._sched = order

    def set_sell(self, enable: bool = True, sigma: int = 1) -> None:
        """Run the matrix-core sparse product on a SELL-16-sigma copy of A.

        sigma: 1 (rows keep their positions) or a multiple of 16 (rows sorted
        by decreasing length within windows of sigma positions).
        """
        with torch.cuda.device(self.device):
            self._bind_stream()
            check(self._lib.bcg_set_sell(self._h, int(bool(enable)), int(sigma)))

    def set_profiling(self, on: bool = True, classes=None) -> None:
        """Record HIP events around the launches of later solves.

        classes: names from KERNEL_CLASSES to record (default: all).
        """
        mask = 0
        if on:
            names = _capi.KERNEL_CLASSES if classes is None else classes
            for c in names:
                mask |= 1 << _capi.KERNEL_CLASSES.index(c)
        with torch.cuda.device(self.device):
            self._bind_stream()
            check(self._lib.bcg_set_profiling(self._h, mask))

    def kernel_times(self) -> dict:
        """{class: (launches, total_ms)} accumulated since profiling was enabled."""
        n = len(_capi.KERNEL_CLASSES)
        arr = (_capi.KernelTime * n)()
        check(self._lib.bcg_get_kernel_times(self._h, arr, n))
        return {name: (int(arr[i].launches), float(arr[i].total_ms)) for i, name in enumerate(_capi.KERNEL_CLASSES)}

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.bcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_noalloc(rowptr: torch.Tensor, colind: torch.Tensor, values: torch.Tensor, B: torch.Tensor,
                  X: torch.Tensor, subalgebra: str = "block", p: int = 0, tol: float = 1e-8,
                  maxit: int = 10000) -> dict:
    """FP64 solve of A X = B in place of X (X holds the initial guess) that
    allocates no device memory: its workspace is the library's fixed per-GPU
    array (bcg_solve_noalloc). Returns the info dict of the solve."""
    n, nnz = rowptr.numel() - 1, colind.numel()
    _require(rowptr, "rowptr", torch.int32, (n + 1,))
    _require(colind, "colind", torch.int32, (nnz,))
    _require(values, "values", torch.float64, (nnz,))
    if B.dim() != 2:
        raise BCGError(_capi.BCG_EINVAL, "B must be n x k")
    k = B.shape[1]
    _require(B, "B", torch.float64, (n, k))
    _require(X, "X", torch.float64, (n, k))
    if subalgebra not in _capi.SUBALGEBRA:
        raise BCGError(_capi.BCG_EINVAL, f"unknown subalgebra {subalgebra!r}")
    csr = _capi.Csr(n, nnz, rowptr.data_ptr(), colind.data_ptr(), values.data_ptr())
    inf = _capi.Info()
    with torch.cuda.device(B.device):
        status = check(_capi.lib().bcg_solve_noalloc(ctypes.byref(csr), k, _capi.SUBALGEBRA[subalgebra], p,
                                                     B.data_ptr(), X.data_ptr(), float(tol), int(maxit),
                                                     _stream_ptr(B.device), ctypes.byref(inf)))
    d = inf.as_dict()
    d["status"] = status
    d["status_name"] = _capi.STATUS_NAME.get(status, str(status))
    return d


def stencil_nnz(dim: int, N: int) -> int:
    nnz = _capi.lib().bcg_stencil_nnz(dim, N)
    if nnz < 0:
        raise BCGError(_capi.BCG_EINVAL, f"invalid stencil dim={dim} N={N}")
    return int(nnz)


def stencil(dim: int, N: int, kappa: torch.Tensor | None = None, device="cuda"):
    """(rowptr, colind, values) of the 5-/7-point stencil on the GPU."""
    device = torch.device(device)
    n = N ** dim
    nnz = stencil_nnz(dim, N)
    if kappa is not None:
        _require(kappa, "kappa", torch.float64, (n,))
        device = kappa.device
    rowptr = torch.empty(n + 1, dtype=torch.int32, device=device)
    colind = torch.empty(nnz, dtype=torch.int32, device=device)
    values = torch.empty(nnz, dtype=torch.float64, device=device)
    with torch.cuda.device(device):
        check(_capi.lib().bcg_stencil_build(dim, N, kappa.data_ptr() if kappa is not None else None,
                                            rowptr.data_ptr(), colind.data_ptr(), values.data_ptr(),
                                            _stream_ptr(device)))
    return rowptr, colind, values


def stencil_schedule(dim: int, N: int, tile: int = 32, device="cuda") -> torch.Tensor:
    """Tiled row order (x-y tiles swept through z) for the 3D stencil."""
    device = torch.device(device)
    order = torch.empty(N ** dim, dtype=torch.int32, device=device)
    with torch.cuda.device(device):
        check(_capi.lib().bcg_stencil_schedule(dim, N, tile, order.data_ptr(), _stream_ptr(device)))
    return order


def stencil_brick_schedule(N: int, tile=(16, 32, 2), brick=(4, 2, 2), device="cuda") -> torch.Tensor:
    """Brick row order of the 3D stencil on an N^3 grid (bcg_stencil_brick_schedule)."""
    device = torch.device(device)
    order = torch.empty(N ** 3, dtype=torch.int32, device=device)
    t = (ctypes.c_int * 3)(*tile)
    b = (ctypes.c_int * 3)(*brick)
    with torch.cuda.device(device):
        check(_capi.lib().bcg_stencil_brick_schedule(N, t, b, order.data_ptr(), _stream_ptr(device)))
    return order


def stencil_kappa_vjp(dim: int, N: int, kappa: torch.Tensor, dvalues: torch.Tensor) -> torch.Tensor:
    """dL/dkappa from dL/dvalues through the stencil assembly."""
    n = N ** dim
    _require(kappa, "kappa", torch.float64, (n,))
    _require(dvalues, "dvalues", torch.float64, (stencil_nnz(dim, N),))
    out = torch.empty_like(kappa)
    with torch.cuda.device(kappa.device):
        check(_capi.lib().bcg_stencil_kappa_vjp(dim, N, kappa.data_ptr(), dvalues.data_ptr(), out.data_ptr(),
                                                _stream_ptr(kappa.device)))
    return out
