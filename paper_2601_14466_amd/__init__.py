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
    "Handle", "handle", "potrf", "potrs", "posv", "posv_noalloc", "posv_mixed", "posv_backward", "potrf_backward", "PosvFunction", "CholeskyFunction", "BatchPlan",
    "getrf", "getrs", "gesv", "lu_solve", "zpotrf", "zpotrs", "zposv",
    "posv_batched", "logdet", "gp_loglik", "gp_loglik_grad", "GPLogLik", "colmajor",
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

    def set_sweep_spin_limit(self, limit: int = -1):
        """Polls before a triangular-sweep wait gives up (-1: built-in limit;
        0: give up at once, which drives the failure path for tests)."""
        call("mg_set_sweep_spin_limit", self.h, int(limit))

    def set_solve_mode(self, mode: str = "inverse"):
        """How the triangular sweeps apply a diagonal block: "inverse"
        (default; an MFMA product with the block's inverse) or
        "substitution" (exact on exactly representable data)."""
        code = {"inverse": _lib.MG_SOLVE_INVERSE, "substitution": _lib.MG_SOLVE_SUBSTITUTION}[mode]
        call("mg_set_solve_mode", self.h, code)

    def block_size(self, n: int, dtype_code: int = _lib.MG_F64) -> int:
        out = ctypes.c_int64()
        call("mg_get_block_size", self.h, dtype_code, int(n), ctypes.byref(out))
        return out.value

    def set_profiling(self, on: bool, kinds=None):
        """Bracket launches with events: every kind (on=True), none, or the
        kinds listed in `kinds` (MG_PROF_* values)."""
        if kinds is None:
            call("mg_set_profiling", self.h, 1 if on else 0)
        else:
            call("mg_set_profiling_kinds", self.h, sum(1 << int(k) for k in kinds) if on else 0)

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
    """X = (L L^T)^{-1} B from a factor returned by potrf.  ``info`` (the
    factor's 0-dim int32 device tensor, optional) is read and, if a sweep
    gives up, set to MG_INFO_SOLVE_ABORTED (X is then NaN)."""
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
    info > 0 (A not positive definite) X holds B unchanged; on
    info == MG_INFO_SOLVE_ABORTED X is NaN."""
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


def posv_noalloc(A, B):
    """posv through mg_posv_noalloc: the solve's scratch is the library's own
    per-GPU array, so the call allocates no device memory in the library
    (this wrapper still allocates the column-major copies it hands over).
    Returns (X, info) as posv; raises MgError (MG_ERR_SCRATCH_LIMIT) when
    n * nrhs is too large for the array.  Calls that overlap in time on one
    GPU share the array and must be serialised."""
    torch = _torch()
    _check_cuda(A, B)
    flat = B.dim() == 1
    n = A.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    Ac = A.T.clone(memory_format=torch.contiguous_format)
    Xc = (B.reshape(n, 1) if flat else B).T.clone(memory_format=torch.contiguous_format)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    call("mg_posv_noalloc", h.h, _dtype_code(A), n, nrhs, _ptr(Ac), max(1, n), _ptr(Xc), max(1, n), _ptr(info))
    X = Xc.T
    return (X.reshape(n) if flat else X), info


def gp_loglik(A, Y, M=None):
    """Gaussian-process marginal log likelihood of each column of Y (or of
    the vector Y) under covariance A (FP64, SPD, lower triangle read) and
    mean M (same shape as Y, or None for zero mean):
    -1/2 (y-m)^T A^{-1} (y-m) - 1/2 log det A - n/2 log(2 pi).
    Returns (loglik, alpha, L, info): loglik has one entry per column (a
    0-d tensor for vector Y), alpha = A^{-1}(y - m), L the Cholesky factor
    (lower triangle significant).  A, Y and M are not modified."""
    torch = _torch()
    _check_cuda(A, Y)
    if A.dtype != torch.float64 or Y.dtype != torch.float64 or (M is not None and M.dtype != torch.float64):
        raise TypeError("gp_loglik takes FP64 A, Y and M")
    flat = Y.dim() == 1
    n = A.shape[0]
    nrhs = 1 if flat else Y.shape[1]
    if M is not None and tuple(M.shape) != tuple(Y.shape):
        raise ValueError("M must have the shape of Y")
    h = handle()
    Lc = A.T.clone(memory_format=torch.contiguous_format)
    Yc = (Y.reshape(n, 1) if flat else Y).T.contiguous()
    Mc = None if M is None else (M.reshape(n, 1) if flat else M).T.contiguous()
    Al = torch.empty((nrhs, n), dtype=torch.float64, device=A.device)
    ll = torch.empty(nrhs, dtype=torch.float64, device=A.device)
    wb = ctypes.c_size_t()
    call("mg_gp_loglik_buffer_size", h.h, n, nrhs, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=A.device)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    call("mg_gp_loglik", h.h, n, nrhs, _ptr(Lc), max(1, n), _ptr(Yc), max(1, n),
         None if Mc is None else _ptr(Mc), max(1, n), _ptr(Al), max(1, n), _ptr(ll),
         _ptr(work), wb.value, _ptr(info))
    alpha = Al.T
    if flat:
        return ll[0], alpha.reshape(n), Lc.T, info
    return ll, alpha, Lc.T, info


def gp_loglik_grad(L, alpha, g, info, with_mean: bool = True):
    """Gradients of sum_j g_j loglik_j (see gp_loglik) from its factor L
    and alpha: returns (gA, gY, gM) with gA the full symmetric n x n
    gradient (alpha alpha^T - A^{-1}) / 2 weighted by g, gY = -g alpha and
    gM = g alpha (None unless with_mean)."""
    torch = _torch()
    flat = alpha.dim() == 1
    n = L.shape[0]
    nrhs = 1 if flat else alpha.shape[1]
    h = handle()
    Lc = L.T.contiguous()
    Ac = (alpha.reshape(n, 1) if flat else alpha).T.contiguous()
    gv = torch.as_tensor(g, dtype=torch.float64, device=L.device).reshape(nrhs).contiguous()
    gA = torch.empty((n, n), dtype=torch.float64, device=L.device)
    gY = torch.empty((nrhs, n), dtype=torch.float64, device=L.device)
    gM = torch.empty((nrhs, n), dtype=torch.float64, device=L.device) if with_mean else None
    wb = ctypes.c_size_t()
    call("mg_gp_loglik_grad_buffer_size", h.h, n, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=L.device)
    call("mg_gp_loglik_grad", h.h, n, nrhs, _ptr(Lc), max(1, n), _ptr(Ac), max(1, n), _ptr(gv), _ptr(gA),
         max(1, n), _ptr(gY), max(1, n), None if gM is None else _ptr(gM), max(1, n), _ptr(work), wb.value,
         _ptr(info))
    gY = gY.T.reshape(n) if flat else gY.T
    if gM is not None:
        gM = gM.T.reshape(n) if flat else gM.T
    return gA, gY, gM   # gA is symmetric, so its row-major buffer is also the column-major one


def posv_mixed(A, B, precision: str = "fp32", tol: float = 1e-12, max_iter: int = 30, fallback: bool = True):
    """Solve A X = B (FP64 A, B) with a binary32 (``precision="fp32"``) or
    bfloat16-update (``"bf16"``) factor and FP64 iterative refinement.
    Returns (X, stats) with stats = dict(iters, fell_back, lo_info, eta, info).
    A and B are not modified."""
    torch = _torch()
    _check_cuda(A, B)
    if A.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("posv_mixed takes FP64 A and B")
    lo = {"fp32": _lib.MG_PREC_F32, "bf16": _lib.MG_PREC_BF16}[precision]
    flat = B.dim() == 1
    n = A.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    Ac = colmajor(A) if A.T.is_contiguous() else A.T.contiguous()
    Bc = (B.reshape(n, 1) if flat else B).T.contiguous()
    Xc = torch.empty_like(Bc)
    nbytes = ctypes.c_size_t()
    call("mg_posv_mixed_buffer_size", h.h, lo, n, nrhs, 1 if fallback else 0, ctypes.byref(nbytes))
    work = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=A.device)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    opts = _lib.IrOpts(tol, max_iter, 1 if fallback else 0)
    res = _lib.IrResult()
    call("mg_posv_mixed", h.h, lo, n, nrhs, _ptr(Ac), max(1, n), _ptr(Bc), max(1, n), _ptr(Xc), max(1, n),
         ctypes.byref(opts), _ptr(work), nbytes.value, ctypes.byref(res), _ptr(info))
    X = Xc.T
    stats = dict(iters=res.iters, fell_back=bool(res.fell_back), lo_info=res.lo_info, eta=res.eta, info=int(info))
    return (X.reshape(n) if flat else X), stats


def posv_backward(L, X, gX, mode: str = "sym", info=None):
    """Adjoint of X = A^{-1} B for A = L L^T: returns (gB, gA).

    mode="sym"  : gA = -1/2 (gB X^T + X gB^T), symmetric;
    mode="lower": gradient with respect to the lower triangle the solver
                  reads (off-diagonal entries doubled, strict upper part 0)."""
    torch = _torch()
    _check_cuda(L, X, gX)
    flat = X.dim() == 1
    n = L.shape[0]
    nrhs = 1 if flat else X.shape[1]
    h = handle()
    Lc = colmajor(L)
    Xc = colmajor(X.reshape(n, nrhs))
    Gc = colmajor(gX.reshape(n, nrhs).to(torch.float64))
    gB = torch.empty((nrhs, n), dtype=torch.float64, device=L.device)
    gA = torch.zeros((n, n), dtype=torch.float64, device=L.device)
    work, wb = _work(h, _lib.MG_F64, n, nrhs, L.device)
    m = {"sym": _lib.MG_GRAD_SYM, "lower": _lib.MG_GRAD_LOWER}[mode]
    call("mg_posv_backward", h.h, n, nrhs, _ptr(Lc), max(1, n), _ptr(Xc), max(1, n), _ptr(Gc), max(1, n),
         _ptr(gB), max(1, n), _ptr(gA), max(1, n), m, _ptr(work), wb, _ptr(info) if info is not None else None)
    gBv = gB.T
    return (gBv.reshape(n) if flat else gBv), gA.T


def potrf_backward(L, gL, info=None, mode: str = "sym"):
    """Gradient with respect to A of f(L), L = chol(A), from gL = df/dL (only
    its lower triangle is read): mode "sym" returns the full symmetric
    gradient (S + S^T)/2, S = L^{-T} Phi(L^T gL) L^{-1}; "lower" the gradient
    with respect to the lower-triangle entries (strict upper part 0).  NaN
    when ``info`` (the factor's) is non-zero."""
    torch = _torch()
    _check_cuda(L, gL)
    if L.dtype != torch.float64 or gL.dtype != torch.float64:
        raise TypeError("potrf_backward takes FP64 L and gL")
    n = L.shape[0]
    h = handle()
    Lc = colmajor(L)
    Gc = colmajor(gL)
    gA = torch.zeros((n, n), dtype=torch.float64, device=L.device)   # column-major buffer
    wb = ctypes.c_size_t()
    call("mg_potrf_backward_buffer_size", h.h, n, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=L.device)
    m = {"sym": _lib.MG_GRAD_SYM, "lower": _lib.MG_GRAD_LOWER}[mode]
    call("mg_potrf_backward", h.h, n, _ptr(Lc), max(1, n), _ptr(Gc), max(1, n), _ptr(gA), max(1, n), m,
         _ptr(work), wb.value, _ptr(info) if info is not None else None)
    return gA.T


def _bytes_work(name, h, device, *dims):
    torch = _torch()
    nbytes = ctypes.c_size_t()
    call(name, h.h, *dims, ctypes.byref(nbytes))
    return torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=device), nbytes.value


def _check_f64(*ts):
    torch = _torch()
    if any(t.dtype != torch.float64 for t in ts):
        raise TypeError("the general solve takes FP64 tensors")


def getrf(A):
    """LU factorisation with partial pivoting, P A = L U (FP64): returns
    (LU, ipiv, info).  LU holds L's strict lower triangle (unit diagonal
    implied) and U; ipiv is an int32 device tensor of 1-based interchanges
    (row k swapped with row ipiv[k] - 1, in order); info is a 0-dim int32
    device tensor (0, or k when U[k-1, k-1] is exactly zero; the
    factorisation still completes)."""
    torch = _torch()
    _check_cuda(A)
    _check_f64(A)
    n = A.shape[0]
    h = handle()
    buf = A.T.clone(memory_format=torch.contiguous_format)
    ipiv = torch.zeros(max(1, n), dtype=torch.int32, device=A.device)[:n]
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    work, wb = _bytes_work("mg_getrf_buffer_size", h, A.device, n)
    call("mg_getrf", h.h, n, _ptr(buf), max(1, n), _ptr(ipiv), _ptr(work), wb, _ptr(info))
    return buf.T, ipiv, info


def getrs(LU, ipiv, B, info=None):
    """X = A^{-1} B from getrf's (LU, ipiv).  ``info`` (getrf's, optional):
    when non-zero, X is B unchanged; a sweep that gives up sets it to
    MG_INFO_SOLVE_ABORTED (X NaN), an ipiv entry outside 1..n to
    MG_INFO_BAD_PIVOT (X NaN)."""
    torch = _torch()
    _check_cuda(LU, B)
    _check_f64(LU, B)
    flat = B.dim() == 1
    n = LU.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    LUc = colmajor(LU)
    Xc = (B.reshape(n, 1) if flat else B).T.clone(memory_format=torch.contiguous_format)
    ip = ipiv.to(torch.int32).contiguous()
    work, wb = _bytes_work("mg_getrs_buffer_size", h, LU.device, n, nrhs)
    call("mg_getrs", h.h, n, nrhs, _ptr(LUc), max(1, n), _ptr(ip), _ptr(Xc), max(1, n), _ptr(work), wb,
         _ptr(info) if info is not None else None)
    X = Xc.T
    return X.reshape(n) if flat else X


def gesv(A, B):
    """Solve A X = B for a general A (FP64) by getrf + getrs in one call
    (mg_gesv).  Returns (X, LU, ipiv, info); on info > 0 X is B unchanged."""
    torch = _torch()
    _check_cuda(A, B)
    _check_f64(A, B)
    flat = B.dim() == 1
    n = A.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    Ac = A.T.clone(memory_format=torch.contiguous_format)
    Xc = (B.reshape(n, 1) if flat else B).T.clone(memory_format=torch.contiguous_format)
    ipiv = torch.zeros(max(1, n), dtype=torch.int32, device=A.device)[:n]
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    work, wb = _bytes_work("mg_gesv_buffer_size", h, A.device, n, nrhs)
    call("mg_gesv", h.h, n, nrhs, _ptr(Ac), max(1, n), _ptr(ipiv), _ptr(Xc), max(1, n), _ptr(work), wb,
         _ptr(info))
    X = Xc.T
    return (X.reshape(n) if flat else X), Ac.T, ipiv, info


def _zdtype(t):
    torch = _torch()
    if t.dtype == torch.complex128:
        return _lib.MG_F64
    if t.dtype == torch.complex64:
        return _lib.MG_F32
    raise TypeError("the complex solve takes complex128 or complex64 tensors")


def _zwork(h, dt, n, nrhs, device):
    return _bytes_work("mg_zposv_buffer_size", h, device, dt, n, nrhs)


def zpotrf(A):
    """Complex Hermitian positive-definite factor A = L L^H (complex128 or
    complex64; lower triangle read, the diagonal's imaginary part ignored):
    returns (L, info), L lower with a real positive diagonal (the strict upper
    part holds A's), info a 0-dim int32 device tensor."""
    torch = _torch()
    _check_cuda(A)
    dt = _zdtype(A)
    n = A.shape[0]
    h = handle()
    buf = A.T.clone(memory_format=torch.contiguous_format)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    work, wb = _zwork(h, dt, n, 0, A.device)
    call("mg_zpotrf", h.h, dt, n, _ptr(buf), max(1, n), _ptr(work), wb, _ptr(info))
    return buf.T, info


def zpotrs(L, B, info=None):
    """X = (L L^H)^{-1} B from zpotrf's factor (same dtype as L)."""
    torch = _torch()
    _check_cuda(L, B)
    dt = _zdtype(L)
    flat = B.dim() == 1
    n = L.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    Lc = colmajor(L)
    Xc = (B.reshape(n, 1) if flat else B).T.clone(memory_format=torch.contiguous_format)
    work, wb = _zwork(h, dt, n, nrhs, L.device)
    call("mg_zpotrs", h.h, dt, n, nrhs, _ptr(Lc), max(1, n), _ptr(Xc), max(1, n), _ptr(work), wb,
         _ptr(info) if info is not None else None)
    X = Xc.T
    return X.reshape(n) if flat else X


def zposv(A, B):
    """Solve A X = B for a complex Hermitian positive-definite A (complex128 or
    complex64).  Returns (X, info); on info > 0 X is B unchanged."""
    torch = _torch()
    _check_cuda(A, B)
    dt = _zdtype(A)
    flat = B.dim() == 1
    n = A.shape[0]
    nrhs = 1 if flat else B.shape[1]
    h = handle()
    Ac = A.T.clone(memory_format=torch.contiguous_format)
    Xc = (B.reshape(n, 1) if flat else B).T.clone(memory_format=torch.contiguous_format)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    work, wb = _zwork(h, dt, n, nrhs, A.device)
    call("mg_zposv", h.h, dt, n, nrhs, _ptr(Ac), max(1, n), _ptr(Xc), max(1, n), _ptr(work), wb, _ptr(info))
    X = Xc.T
    return (X.reshape(n) if flat else X), info


def lu_solve(A, B):
    """The paper's lu_solve: X with A X = B for a general A (FP64).
    Returns (X, info)."""
    X, _, _, info = gesv(A, B)
    return X, info


def _make_cholesky_function():
    torch = _torch()

    class CholeskyFunction(torch.autograd.Function):
        """L = chol(A) (lower, zeros above) with the hand-written adjoint of
        mg_potrf_backward.  ``CholeskyFunction.apply(A, mode)``: mode "sym"
        (default) gives the symmetric gradient; "lower" the derivative with
        respect to the entries the factorisation reads (for gradcheck of a
        function of A's lower triangle).  NaN gradients when A is not
        positive definite."""

        @staticmethod
        def forward(ctx, A, mode="sym"):
            L, info = potrf(A)
            L = torch.tril(L)
            L.masked_fill_(info != 0, float("nan"))
            ctx.save_for_backward(L, info)
            ctx.mode = mode
            return L

        @staticmethod
        def backward(ctx, gL):
            L, info = ctx.saved_tensors
            return potrf_backward(L, gL.contiguous(), info=info.clone(), mode=ctx.mode), None

    return CholeskyFunction


def _make_posv_function():
    torch = _torch()

    class PosvFunction(torch.autograd.Function):
        """X = A^{-1} B with a hand-written adjoint that reuses the stored
        Cholesky factor (no refactorisation in backward).

        ``PosvFunction.apply(A, B, mode)``: mode "sym" (default) returns the
        symmetric gradient -1/2 (gB X^T + X gB^T) for A; "lower" returns the
        exact derivative of the solver as a function of all entries of A
        (only the lower triangle is read, so the strict upper part is 0).
        When A is not positive definite (or a sweep gave up) X is all NaN,
        and so are the gradients; nothing synchronises to find out."""

        @staticmethod
        def forward(ctx, A, B, mode="sym"):
            L, info = potrf(A)
            X = potrs(L, B, info)
            X.masked_fill_(info != 0, float("nan"))   # device-side: a failed factor leaves B in X
            ctx.save_for_backward(L, X, info)
            ctx.mode = mode
            return X

        @staticmethod
        def backward(ctx, gX):
            L, X, info = ctx.saved_tensors
            gB, gA = posv_backward(L, X, gX, mode=ctx.mode, info=info)
            return gA, gB, None

    return PosvFunction


def _make_gp_function():
    import torch

    class GPLogLik(torch.autograd.Function):
        """log L = gp_loglik(A, Y, M) (one value per column of Y) with a
        hand-written adjoint from the stored factor: dA = (alpha alpha^T -
        A^{-1}) / 2 (symmetric), dY = -alpha, dM = alpha.  ``M`` may be
        None (zero mean)."""

        @staticmethod
        def forward(ctx, A, Y, M=None):
            ll, alpha, L, info = gp_loglik(A, Y, M)
            ctx.save_for_backward(L, alpha, info)
            ctx.with_mean = M is not None
            return ll

        @staticmethod
        def backward(ctx, g):
            L, alpha, info = ctx.saved_tensors
            gA, gY, gM = gp_loglik_grad(L, alpha, g, info, with_mean=ctx.with_mean)
            return gA, gY, gM

    return GPLogLik


class _LazyFunction:
    def __init__(self, make):
        self._make = make
        self._cls = None

    def __getattr__(self, name):
        if name.startswith("_"):
            raise AttributeError(name)
        if self._cls is None:
            self._cls = self._make()
        return getattr(self._cls, name)


PosvFunction = _LazyFunction(_make_posv_function)
GPLogLik = _LazyFunction(_make_gp_function)
CholeskyFunction = _LazyFunction(_make_cholesky_function)


class BatchPlan:
    """A batched-posv plan (mg_batch_plan_create): fixed orders, nrhs and
    dtype, launch shape picked by the library's autotuner, persistent kernel
    replayed from a HIP graph on every solve."""

    def __init__(self, sizes, nrhs: int = 1, dtype=None, autotune: bool = True, grid_per_cu: int = 0,
                 order: int = -1, cache_path: str | None = None, variant: int = -1):
        torch = _torch()
        import numpy as np
        self.dtype = dtype or torch.float64
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.nrhs = int(nrhs)
        self.h = handle()
        self._cache = cache_path.encode() if cache_path else None
        opts = _lib.TuneOpts(1 if autotune else 0, int(grid_per_cu), int(order), self._cache, int(variant))
        p = ctypes.c_void_p()
        call("mg_batch_plan_create", self.h.h, _dtype_code(torch.empty(0, dtype=self.dtype)), len(self.sizes),
             self.sizes.ctypes.data_as(ctypes.c_void_p), self.nrhs, ctypes.byref(opts), ctypes.byref(p))
        self.p = p

    def info(self):
        g, o, t, v = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
        call("mg_batch_plan_info", self.p, ctypes.byref(g), ctypes.byref(o), ctypes.byref(t), ctypes.byref(v))
        return dict(variant=v.value, grid_per_cu=g.value, order=o.value, tuned_ms=t.value)

    def solve_raw(self, A_ptrs, lda, B_ptrs, ldb, info):
        """Device int64 tensors of pointers / leading dimensions, int32 info."""
        call("mg_posv_batched", handle().h, self.p, _ptr(A_ptrs), _ptr(lda), _ptr(B_ptrs), _ptr(ldb), _ptr(info))

    def solve(self, As, Bs, return_factors: bool = False):
        """Solve every A_k X_k = B_k; returns (list of X_k, int32 info tensor),
        and with ``return_factors`` also the list of factors L_k (lower
        triangle significant) that ``backward`` takes."""
        torch = _torch()
        dev = As[0].device if len(As) else torch.device("cuda")
        Ab = [a.T.clone(memory_format=torch.contiguous_format) for a in As]
        Xb = [b.reshape(b.shape[0], -1).T.clone(memory_format=torch.contiguous_format) for b in Bs]
        ap = torch.tensor([t.data_ptr() for t in Ab], dtype=torch.int64, device=dev)
        bp = torch.tensor([t.data_ptr() for t in Xb], dtype=torch.int64, device=dev)
        ld = torch.tensor([max(1, int(a.shape[0])) for a in As], dtype=torch.int64, device=dev)
        info = torch.zeros(len(As), dtype=torch.int32, device=dev)
        self.solve_raw(ap, ld, bp, ld, info)
        torch.cuda.current_stream().synchronize()
        if return_factors:
            return [x.T for x in Xb], info, [a.T for a in Ab]
        return [x.T for x in Xb], info

    def backward(self, Ls, Xs, GXs, info, mode: str = "sym"):
        """Adjoint of the batched solve (mg_posv_batched_backward): from the
        factors L_k and solutions X_k of ``solve`` and upstream gradients
        gX_k, returns (list of gB_k = A_k^{-1} gX_k, list of gA_k), gA_k the
        symmetric -1/2 (gB X^T + X gB^T) ("sym") or the lower-triangle
        gradient ("lower"; strict upper part 0).  NaN for systems whose
        info is non-zero."""
        torch = _torch()
        dev = Ls[0].device if len(Ls) else torch.device("cuda")
        Lc = [colmajor(t) for t in Ls]
        Xc = [colmajor(x.reshape(x.shape[0], -1)) for x in Xs]
        Gc = [colmajor(gx.reshape(gx.shape[0], -1)) for gx in GXs]
        GB = [torch.empty_like(x) for x in Xc]
        GA = [torch.zeros((int(t.shape[0]), int(t.shape[0])), dtype=t.dtype, device=dev) for t in Ls]
        P = lambda ts: torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=dev)
        ld = torch.tensor([max(1, int(t.shape[0])) for t in Ls], dtype=torch.int64, device=dev)
        m = {"sym": _lib.MG_GRAD_SYM, "lower": _lib.MG_GRAD_LOWER}[mode]
        ptrs = [P(Lc), P(Xc), P(Gc), P(GB), P(GA)]
        call("mg_posv_batched_backward", handle().h, self.p, _ptr(ptrs[0]), _ptr(ld), _ptr(ptrs[1]), _ptr(ld),
             _ptr(ptrs[2]), _ptr(ld), _ptr(ptrs[3]), _ptr(ld), _ptr(ptrs[4]), _ptr(ld), m, _ptr(info))
        torch.cuda.current_stream().synchronize()
        return [g.T for g in GB], [g.T for g in GA]

    def __del__(self):
        try:
            if getattr(self, "p", None):
                raw("mg_batch_plan_destroy", self.p)
                self.p = None
        except Exception:
            pass


def posv_batched(As, Bs, autotune: bool = True, cache_path: str | None = None):
    """One-shot batched solve (builds a plan, solves, releases it)."""
    sizes = [int(a.shape[0]) for a in As]
    nrhs = 1 if Bs[0].dim() == 1 else int(Bs[0].shape[1])
    plan = BatchPlan(sizes, nrhs=nrhs, dtype=As[0].dtype, autotune=autotune, cache_path=cache_path)
    return plan.solve(As, Bs)


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
