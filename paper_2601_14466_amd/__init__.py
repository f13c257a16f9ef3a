"""MI355X-native dense SPD solver (Cholesky potrf + potrs) -- Python binding.

Thin torch-facing wrappers over the C ABI of ``libmg.so`` (declared in
``include/mg.h``).  PyTorch provides device memory and the current HIP stream;
all arithmetic runs in the library's HIP kernels.  There is no CPU fallback:
importing works without a GPU, but every call needs the built library and a
ROCm device.

Layout: the C ABI is column-major.  A torch tensor ``M`` of shape (r, c) is
handed over as the contiguous buffer ``M.T.contiguous()`` (column-major M);
results come back as ``buf.T`` views, so every returned tensor has ordinary
(row, column) semantics.  Only the lower triangle of ``A`` is read.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import MgError, call, load, raw  # noqa: F401

__all__ = [
    "Handle", "handle", "potrf", "potrs", "posv", "logdet", "colmajor",
    "MgError", "load", "call", "raw",
]


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return _lib.MG_F64
    if t.dtype == torch.float32:
        return _lib.MG_F32
    raise TypeError(f"unsupported dtype {t.dtype}; use float64 or float32")


def _check_cuda(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("mg: tensors must live on a ROCm device (no CPU path)")


class Handle:
    """Owns an mg_handle_t bound to one device; the stream is refreshed to
    torch's current stream before every call."""

    def __init__(self, device=None):
        torch = _torch()
        load()
        self.device = torch.cuda.current_device() if device is None else device
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            call("mg_create", ctypes.byref(h), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        self.h = h

    def sync_stream(self):
        torch = _torch()
        call("mg_set_stream", self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        return self.h

    def set_block_size(self, nb: int):
        call("mg_set_block_size", self.h, int(nb))

    def block_size(self, n: int, dtype_code: int = _lib.MG_F64) -> int:
        out = ctypes.c_int64()
        call("mg_get_block_size", self.h, dtype_code, int(n), ctypes.byref(out))
        return out.value

    def set_profiling(self, on: bool):
        call("mg_set_profiling", self.h, 1 if on else 0)

    def profile(self, kind: int, reset: bool = True):
        ms, cnt, fl, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        call("mg_profile_query", self.h, int(kind), ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(fl),
             ctypes.byref(by), 1 if reset else 0)
        return dict(ms=ms.value, launches=cnt.value, flops=fl.value, bytes=by.value)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                raw("mg_destroy", self.h)
                self.h = None
        except Exception:
            pass


_handles = {}


def handle(device=None) -> Handle:
    """Per-device cached handle with its stream set to the current stream."""
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else device
    h = _handles.get(dev)
    if h is None:
        h = _handles[dev] = Handle(dev)
    h.sync_stream()
    return h


def colmajor(M):
    """Contiguous column-major buffer for M's values (no copy when M is
    already the transpose of a contiguous tensor)."""
    Mt = M.T if M.dim() == 2 else M.reshape(-1, 1).T
    return Mt if Mt.is_contiguous() else Mt.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def potrf(A, nb: int | None = None):
    """Cholesky factor of SPD A: returns (L, info).  L is lower triangular
    (strict upper part holds whatever A's buffer held there); info is a
    0-dim int32 device tensor (0, or k for a non-PD leading minor)."""
    torch = _torch()
    _check_cuda(A)
    n = A.shape[0]
    h = handle()
    if nb is not None:
        h.set_block_size(nb)
    buf = A.T.clone(memory_format=torch.contiguous_format)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    try:
        call("mg_potrf", h.h, _dtype_code(A), n, _ptr(buf), max(1, n), _ptr(info))
    finally:
        if nb is not None:
            h.set_block_size(0)
    return buf.T, info


def _work(h, dt, n, nrhs, device):
    torch = _torch()
    nbytes = ctypes.c_size_t()
    call("mg_potrs_buffer_size", h.h, dt, n, nrhs, ctypes.byref(nbytes))
    return torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=device), nbytes.value


def potrs(L, B, info=None):
    """X = (L L^T)^{-1} B from a factor returned by potrf."""
    torch = _torch()
    _check_cuda(L, B)
    flat = B.dim() == 1
    n = L.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    Lc = colmajor(L)
    Xc = (B.reshape(n, 1) if flat else B).T.clone(memory_format=torch.contiguous_format)
    dt = _dtype_code(L)
    work, wb = _work(h, dt, n, nrhs, L.device)
    call("mg_potrs", h.h, dt, n, nrhs, _ptr(Lc), max(1, n), _ptr(Xc), max(1, n), _ptr(work), wb,
         _ptr(info) if info is not None else None)
    X = Xc.T
    return X.reshape(n) if flat else X


def posv(A, B, nb: int | None = None):
    """Solve A X = B (A SPD, lower triangle read).  Returns (X, info); on
    info != 0, X holds B unchanged."""
    torch = _torch()
    _check_cuda(A, B)
    flat = B.dim() == 1
    n = A.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    if nb is not None:
        h.set_block_size(nb)
    Ac = A.T.clone(memory_format=torch.contiguous_format)
    Xc = (B.reshape(n, 1) if flat else B).T.clone(memory_format=torch.contiguous_format)
    dt = _dtype_code(A)
    work, wb = _work(h, dt, n, nrhs, A.device)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    try:
        call("mg_posv", h.h, dt, n, nrhs, _ptr(Ac), max(1, n), _ptr(Xc), max(1, n), _ptr(work), wb, _ptr(info))
    finally:
        if nb is not None:
            h.set_block_size(0)
    X = Xc.T
    return (X.reshape(n) if flat else X), info


def logdet(L, info=None):
    """log det A = 2 sum log L_jj from a factor; returns a 0-dim float64 tensor."""
    torch = _torch()
    _check_cuda(L)
    n = L.shape[0]
    h = handle()
    Lc = colmajor(L)
    out = torch.empty((), dtype=torch.float64, device=L.device)
    call("mg_logdet", h.h, _dtype_code(L), n, _ptr(Lc), max(1, n), _ptr(out),
         _ptr(info) if info is not None else None)
    return out
