"""CPU oracle for the Cholesky solver -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It wraps ``oracle.c`` (plain FP64 C, built by
``oracle/build.sh`` / ``__graft_entry__.build()``) through ctypes and shares
nothing with the GPU library.

Every function takes numpy arrays with (row, column) semantics and converts
them to column-major (Fortran) order before the C call; results come back in
Fortran order with the same semantics.  Only the lower triangle of ``A`` is
read, so a full symmetric array or one whose upper triangle holds garbage give
the same answer.

What each routine computes (definitions, paper: JAXMg "Software design",
potrs bullet -- a Cholesky solve of a symmetric positive-definite system,
optionally with log det):

* ``potrf``     -- lower L with positive diagonal, A = L L^T; info = first
                   1-based column whose pivot is not > 0 (0 on success).
* ``potrs``     -- X = A^{-1} B by forward then back substitution.
* ``residual``  -- R = B - A X in extended precision and the per-column
                   normwise backward error eta_j = |r_j|inf / (|A|inf |x_j|inf
                   + |b_j|inf).
* ``logdet``    -- 2 sum log L_jj.
* ``potrf_lo``  -- low-precision factor: the column algorithm in binary32,
                   or the blocked reading (FP64 diagonal blocks, binary32
                   panel solve, operands of the trailing products rounded to
                   binary32 or bfloat16, binary32 sums).
* ``round_bf16``-- nearest-even rounding of binary32 values to bfloat16.
* ``posv_ir``   -- low-precision factor plus FP64 iterative refinement;
                   falls back to FP64 when it stalls.
* ``posv_backward`` -- gB = A^{-1} gX, gA = -1/2 (gB X^T + X gB^T).
* ``getrf`` / ``getrs`` / ``lu_solve`` -- the paper's general solve: P A = L U
                   by partial pivoting (LAPACK ipiv convention), then the
                   swaps, L y = P b and U x = y.
* ``zpotrf`` / ``zpotrs`` / ``zposv`` / ``backward_error_z`` -- the complex
                   Hermitian case (the paper lists complex64 and complex128):
                   A = L L^H, L lower with a real positive diagonal, then
                   L y = b, L^H x = y; backward error with the complex
                   modulus.
* ``potrf_backward`` -- gradient with respect to A of f(chol(A)) from
                   gL = df/dL: sym(L^{-T} Phi(L^T gL) L^{-1}), Phi the lower
                   triangle with the diagonal halved (Murray 2016; the paper
                   is silent).
* ``gp_loglik`` -- Gaussian-process marginal log likelihood (paper: Research
                   Impact Statement, "Scientific applications", Cholesky
                   solve): -1/2 r^T A^{-1} r - 1/2 log det A - N/2 log(2 pi),
                   r = y - m, per column.
* ``gp_loglik_grad`` -- its gradient weighted by g: dA = sum_j g_j
                   (alpha_j alpha_j^T - A^{-1}) / 2 (symmetric), dY = -g alpha,
                   dM = g alpha.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int)


def build() -> str:
    """Compile oracle.c with gcc into liboracle.so (always recompiles)."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _LIB_PATH, src, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.or_potrf.argtypes = [_i64, _dp, _i64]
    lib.or_potrf.restype = _i64
    lib.or_potrs.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
    lib.or_potrs.restype = None
    lib.or_posv.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
    lib.or_posv.restype = _i64
    lib.or_logdet.argtypes = [_i64, _dp, _i64]
    lib.or_logdet.restype = ctypes.c_double
    lib.or_sym_norm_inf.argtypes = [_i64, _dp, _i64]
    lib.or_sym_norm_inf.restype = ctypes.c_double
    lib.or_residual.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64, _dp, _i64, _dp]
    lib.or_residual.restype = ctypes.c_double
    lib.or_potrf_lo.argtypes = [_i64, _fp, _i64, ctypes.c_int]
    lib.or_potrf_lo.restype = _i64
    lib.or_potrs_lo.argtypes = [_i64, _i64, _fp, _i64, _fp, _i64]
    lib.or_potrs_lo.restype = None
    lib.or_potrf_lo_blocked.argtypes = [_i64, _fp, _i64, ctypes.c_int, _i64]
    lib.or_potrf_lo_blocked.restype = _i64
    lib.or_round_bf16_array.argtypes = [_i64, _fp, _fp]
    lib.or_round_bf16_array.restype = None
    lib.or_posv_ir.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64,
                               ctypes.c_int, ctypes.c_double, ctypes.c_int, _i64, _ip, _ip, _dp, _dp, _ip]
    lib.or_posv_ir.restype = _i64
    lib.or_posv_backward.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64,
                                     _dp, _i64, _dp, _i64, ctypes.c_int]
    lib.or_posv_backward.restype = None
    lib.or_potrf_backward.argtypes = [_i64, _dp, _i64, _dp, _i64, _dp, _i64, ctypes.c_int]
    lib.or_potrf_backward.restype = None
    lib.or_getrf.argtypes = [_i64, _dp, _i64, ctypes.POINTER(ctypes.c_int32)]
    lib.or_getrf.restype = _i64
    lib.or_getrs.argtypes = [_i64, _i64, _dp, _i64, ctypes.POINTER(ctypes.c_int32), _dp, _i64]
    lib.or_getrs.restype = None
    lib.or_residual_gen.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64, _dp]
    lib.or_residual_gen.restype = ctypes.c_double
    lib.or_zpotrf.argtypes = [_i64, _dp, _i64]
    lib.or_zpotrf.restype = _i64
    lib.or_zpotrs.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
    lib.or_zpotrs.restype = None
    lib.or_residual_z.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64, _dp]
    lib.or_residual_z.restype = ctypes.c_double
    lib.or_num_threads.argtypes = []
    lib.or_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


def _ld(a: np.ndarray) -> int:
    return max(1, a.shape[0])


def _c128(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.complex128))


def _as2d(b):
    b = np.asarray(b)
    return (b.reshape(-1, 1), True) if b.ndim == 1 else (b, False)


def num_threads() -> int:
    return int(_load().or_num_threads())


def potrf(A):
    """Return (L, info).  L is lower triangular (strict upper set to 0)."""
    lib = _load()
    W = _f64(A).copy(order="F")
    n = W.shape[0]
    info = lib.or_potrf(n, _ptr(W), _ld(W))
    return np.tril(W), int(info)


def potrs(L, B):
    """X with L L^T X = B (L lower; only its lower triangle is read)."""
    lib = _load()
    Lf = _f64(L)
    B2, flat = _as2d(B)
    X = _f64(B2).copy(order="F")
    n, nrhs = X.shape
    lib.or_potrs(n, nrhs, _ptr(Lf), _ld(Lf), _ptr(X), _ld(X))
    return X.ravel() if flat else X


def posv(A, B):
    """Return (X, info) for A X = B."""
    lib = _load()
    W = _f64(A).copy(order="F")
    B2, flat = _as2d(B)
    X = _f64(B2).copy(order="F")
    n, nrhs = X.shape
    info = lib.or_posv(n, nrhs, _ptr(W), _ld(W), _ptr(X), _ld(X))
    return (X.ravel() if flat else X), int(info)


def logdet(L) -> float:
    Lf = _f64(L)
    return float(_load().or_logdet(Lf.shape[0], _ptr(Lf), _ld(Lf)))


def sym_norm_inf(A) -> float:
    Af = _f64(A)
    return float(_load().or_sym_norm_inf(Af.shape[0], _ptr(Af), _ld(Af)))


def residual(A, X, B):
    """Return (R, eta, anorm): R = B - A X in extended precision (rounded to
    FP64 on output), eta per column, |A|inf of the symmetric matrix."""
    lib = _load()
    Af = _f64(A)
    X2, flat = _as2d(X)
    B2, _ = _as2d(B)
    Xf, Bf = _f64(X2), _f64(B2)
    n, nrhs = Xf.shape
    R = np.zeros((n, nrhs), dtype=np.float64, order="F")
    eta = np.zeros(nrhs, dtype=np.float64)
    anorm = lib.or_residual(n, nrhs, _ptr(Af), _ld(Af), _ptr(Xf), _ld(Xf),
                            _ptr(Bf), _ld(Bf), _ptr(R), _ld(R), _ptr(eta))
    return (R.ravel() if flat else R), eta, float(anorm)


def backward_error(A, X, B) -> np.ndarray:
    """Per-column normwise backward error eta_j (extended-precision residual)."""
    return residual(A, X, B)[1]


def potrf_lo(A, lo: int = 1, nb: int = 0):
    """Low-precision factor of fl32(A): lo=1 binary32, lo=2 bfloat16
    operands in the trailing products.  nb = 0: the column algorithm with
    every operation in binary32; nb > 0: the blocked reading (FP64 diagonal
    blocks of nb columns stored rounded, binary32 panel solve, trailing
    update with operands rounded to the working precision)."""
    lib = _load()
    W = np.asfortranarray(np.asarray(A, dtype=np.float64).astype(np.float32))
    n = W.shape[0]
    if nb > 0:
        info = lib.or_potrf_lo_blocked(n, _ptr(W, _fp), _ld(W), int(lo), int(nb))
    else:
        info = lib.or_potrf_lo(n, _ptr(W, _fp), _ld(W), int(lo))
    return np.tril(W), int(info)


def round_bf16(x) -> np.ndarray:
    """bfloat16 rounding (nearest-even) of binary32 values, widened back to
    binary32 (bit patterns pass through unconverted, NaN payloads included)."""
    lib = _load()
    v = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).ravel()
    out = np.empty_like(v)
    lib.or_round_bf16_array(v.size, _ptr(v, _fp), _ptr(out, _fp))
    return out.reshape(np.shape(x))


def posv_ir(A, B, lo: int = 1, tol: float = 1e-12, max_iter: int = 30, nb: int = 128):
    """Mixed-precision solve with FP64 iterative refinement; the
    low-precision factor is the blocked one with block nb (0: the column
    algorithm).

    Returns (X, dict(iters, fell_back, eta, info, hist)); hist lists the
    largest eta of every residual the refinement loop evaluated."""
    lib = _load()
    Af = _f64(A)
    B2, flat = _as2d(B)
    Bf = _f64(B2)
    n, nrhs = Bf.shape
    X = np.zeros((n, nrhs), dtype=np.float64, order="F")
    iters, fb = ctypes.c_int(0), ctypes.c_int(0)
    eta = ctypes.c_double(0.0)
    hist = np.zeros(max(1, int(max_iter) + 1), dtype=np.float64)
    nh = ctypes.c_int(0)
    info = lib.or_posv_ir(n, nrhs, _ptr(Af), _ld(Af), _ptr(Bf), _ld(Bf), _ptr(X), _ld(X),
                          int(lo), float(tol), int(max_iter), int(nb),
                          ctypes.byref(iters), ctypes.byref(fb), ctypes.byref(eta), _ptr(hist), ctypes.byref(nh))
    stats = dict(iters=iters.value, fell_back=bool(fb.value), eta=eta.value, info=int(info),
                 hist=hist[:nh.value].tolist())
    return (X.ravel() if flat else X), stats


def posv_backward(L, X, GX, mode: int = 0):
    """Return (gB, gA) for X = A^{-1} B, A = L L^T, upstream gradient gX."""
    lib = _load()
    Lf = _f64(L)
    X2, flat = _as2d(X)
    G2, _ = _as2d(GX)
    Xf, Gf = _f64(X2), _f64(G2)
    n, nrhs = Xf.shape
    GB = np.zeros((n, nrhs), dtype=np.float64, order="F")
    GA = np.zeros((n, n), dtype=np.float64, order="F")
    lib.or_posv_backward(n, nrhs, _ptr(Lf), _ld(Lf), _ptr(Xf), _ld(Xf), _ptr(Gf), _ld(Gf),
                         _ptr(GB), _ld(GB), _ptr(GA), _ld(GA), int(mode))
    return (GB.ravel() if flat else GB), GA


def getrf(A):
    """Return (LU, ipiv, info): P A = L U by partial pivoting; LU holds the
    unit lower L below the diagonal and U on and above it; ipiv[k] is the
    1-based row swapped with row k (LAPACK convention)."""
    lib = _load()
    W = _f64(A).copy(order="F")
    n = W.shape[0]
    ipiv = np.zeros(max(1, n), dtype=np.int32)
    info = lib.or_getrf(n, _ptr(W), _ld(W), ipiv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return W, ipiv[:n], int(info)


def getrs(LU, ipiv, B):
    """X with A X = B from getrf's LU and ipiv."""
    lib = _load()
    LUf = _f64(LU)
    B2, flat = _as2d(B)
    X = _f64(B2).copy(order="F")
    n, nrhs = X.shape
    piv = np.ascontiguousarray(np.asarray(ipiv, dtype=np.int32))
    lib.or_getrs(n, nrhs, _ptr(LUf), _ld(LUf), piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(X), _ld(X))
    return X.ravel() if flat else X


def lu_solve(A, B):
    """Return (X, info) for a general A X = B (getrf then getrs)."""
    LU, ipiv, info = getrf(A)
    return getrs(LU, ipiv, B), info


def backward_error_gen(A, X, B) -> np.ndarray:
    """Per-column normwise backward error of a general system (extended
    precision residual, |A|inf the largest row sum)."""
    lib = _load()
    Af = _f64(A)
    X2, _ = _as2d(X)
    B2, _ = _as2d(B)
    Xf, Bf = _f64(X2), _f64(B2)
    n, nrhs = Xf.shape
    eta = np.zeros(nrhs, dtype=np.float64)
    lib.or_residual_gen(n, nrhs, _ptr(Af), _ld(Af), _ptr(Xf), _ld(Xf), _ptr(Bf), _ld(Bf), _ptr(eta))
    return eta


def potrf_backward(L, GL, mode: int = 0):
    """Gradient with respect to A of a scalar f(L), L = chol(A), given
    GL = df/dL (only its lower triangle is used): the symmetric matrix
    (S + S^T)/2 with S = L^{-T} Phi(L^T GL) L^{-1} (mode 0), or the gradient
    with respect to the lower-triangle entries of A (mode 1; the strict
    upper triangle of the result is 0)."""
    lib = _load()
    Lf = _f64(L)
    Gf = _f64(np.tril(np.asarray(GL, dtype=np.float64)))
    n = Lf.shape[0]
    GA = np.zeros((n, n), dtype=np.float64, order="F")
    lib.or_potrf_backward(n, _ptr(Lf), _ld(Lf), _ptr(Gf), _ld(Gf), _ptr(GA), _ld(GA), int(mode))
    return GA


def posv_batched(As, Bs):
    """Loop of independent posv calls; returns (list of X, list of info)."""
    xs, infos = [], []
    for A, B in zip(As, Bs):
        x, info = posv(A, B)
        xs.append(x)
        infos.append(info)
    return xs, infos


def gp_loglik(A, Y, M=None):
    """Marginal log likelihood of each column y of Y under covariance A and
    mean m (column of M, or 0), in the paper's order: factor A, solve
    alpha = A^{-1} (y - m), log det A from the factor, then
    -1/2 (y - m)^T alpha - 1/2 log det A - N/2 log(2 pi) with the dot product
    summed exactly (math.fsum).  Returns (loglik, alpha, info); loglik is NaN
    and alpha = y - m when the factorisation fails."""
    L, info = potrf(A)
    Y2, flat = _as2d(Y)
    R = _f64(Y2).copy(order="F")
    if M is not None:
        R = R - _f64(_as2d(M)[0])
    n, k = R.shape
    if info != 0:
        ll = np.full(k, np.nan)
        return (ll[0] if flat else ll), (R.ravel() if flat else R), info
    alpha = potrs(L, R)
    ld = logdet(L) if n > 0 else 0.0
    ll = np.array([-0.5 * math.fsum(R[:, j] * alpha[:, j]) - 0.5 * ld - 0.5 * n * math.log(2.0 * math.pi)
                   for j in range(k)])
    return (ll[0] if flat else ll), (alpha.ravel() if flat else alpha), 0


def gp_loglik_grad(A, Y, M=None, g=None):
    """Gradient of sum_j g_j log L_j (gp_loglik) with respect to the
    symmetric A, to Y and to M, from the definitions: alpha_j = A^{-1} r_j,
    A^{-1} from the factor by solving against the identity (its lower
    triangle mirrored, so the result is exactly symmetric), then
    dA = sum_j g_j alpha_j alpha_j^T / 2 - (sum_j g_j) A^{-1} / 2,
    dY = -g alpha, dM = g alpha.  Returns (dA, dY, dM, info)."""
    L, info = potrf(A)
    Y2, flat = _as2d(Y)
    R = _f64(Y2).copy(order="F")
    if M is not None:
        R = R - _f64(_as2d(M)[0])
    n, k = R.shape
    gv = np.ones(k) if g is None else np.asarray(g, dtype=np.float64).reshape(k)
    if info != 0:
        nanv = np.full(R.shape, np.nan)
        return np.full((n, n), np.nan), (nanv.ravel() if flat else nanv), (nanv.ravel() if flat else nanv), info
    alpha = potrs(L, R)
    Ainv = potrs(L, np.eye(n))
    Ainv = np.tril(Ainv) + np.tril(Ainv, -1).T
    dA = 0.5 * (alpha * gv) @ alpha.T - 0.5 * gv.sum() * Ainv
    dY = -alpha * gv
    return dA, (dY.ravel() if flat else dY), (-dY.ravel() if flat else -dY), 0


# ------------------------------------------------------------ complex Hermitian


def zpotrf(A):
    """Return (L, info): complex Hermitian A = L L^H, L lower with a real
    positive diagonal (only the lower triangle of A is read; the imaginary
    part of its diagonal is ignored).  Entries above the diagonal of the
    returned array are those of A."""
    lib = _load()
    W = _c128(A).copy(order="F")
    info = lib.or_zpotrf(W.shape[0], W.ctypes.data_as(_dp), _ld(W))
    return W, int(info)


def zpotrs(L, B):
    """X with L L^H X = B from zpotrf's L."""
    lib = _load()
    Lf = _c128(L)
    B2, flat = _as2d(B)
    X = _c128(B2).copy(order="F")
    n, nrhs = X.shape
    lib.or_zpotrs(n, nrhs, Lf.ctypes.data_as(_dp), _ld(Lf), X.ctypes.data_as(_dp), _ld(X))
    return X.ravel() if flat else X


def zposv(A, B):
    """Return (X, info) for a complex Hermitian positive-definite A X = B."""
    L, info = zpotrf(A)
    if info:
        return np.array(B, dtype=np.complex128, copy=True), info
    return zpotrs(L, B), 0


def backward_error_z(A, X, B) -> np.ndarray:
    """Per-column normwise backward error of A X = B, A Hermitian from its
    lower triangle (extended precision, complex modulus)."""
    lib = _load()
    Af = _c128(A)
    X2, _ = _as2d(X)
    B2, _ = _as2d(B)
    Xf, Bf = _c128(X2), _c128(B2)
    n, nrhs = Xf.shape
    eta = np.zeros(nrhs, dtype=np.float64)
    lib.or_residual_z(n, nrhs, Af.ctypes.data_as(_dp), _ld(Af), Xf.ctypes.data_as(_dp), _ld(Xf),
                      Bf.ctypes.data_as(_dp), _ld(Bf), _ptr(eta))
    return eta
