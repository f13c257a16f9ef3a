"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only *constructs* inputs; it contains none of the solver's
arithmetic (no factorisation, no triangular solve, no residual).  Both the GPU
path and the CPU oracle receive the same arrays from here.

The paper benchmarks on synthetic matrices only (JAXMg, "Performance and
scaling": A = diag(1..N) with b = ones for the solves).  The workload recipes
below follow the solver's published test configurations:

* ``gram_spd``   : G with i.i.d. N(0,1) entries, A = G G^T / n + shift * I.
* ``cond_shift`` : the shift that puts cond(G G^T/n + shift I) near a target,
                   from a seeded power-iteration estimate of lambda_max.
* ``haar_spd``   : A = Q diag(lam) Q^T, Q Haar-distributed (Householder QR of
                   a Gaussian matrix with the sign of R's diagonal fixed),
                   lam log-spaced on [1/cond, 1] so cond(A) is exact.  On the
                   device, for n^2 >= 2^31 the same construction runs panel by
                   panel so that no library call sees 2^31 or more elements
                   (library kernels index with 32-bit integers).
* ``batch_sizes``: n_i uniform on [16, 512].
* closed-form families used as pins: ``lehmer``, ``laplacian_1d``,
  ``diag_1_to_n`` (the paper's own benchmark matrix), ``integer_exact``.

Every generated matrix is exactly symmetric: the lower triangle is mirrored
into the upper one.  numpy generators use ``Generator(PCG64(seed))``; the torch
generators use a seeded device generator and are meant for sizes where a CPU
Gram product would take minutes.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------- numpy


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def symmetrize_lower(A: np.ndarray) -> np.ndarray:
    """Copy the lower triangle onto the upper one (exact symmetry)."""
    L = np.tril(A)
    return L + np.tril(A, -1).T


def gram_spd(n: int, seed: int, shift: float = 1.0) -> np.ndarray:
    """A = G G^T / n + shift I with G ~ N(0,1), seeded."""
    g = rng(seed)
    G = g.standard_normal((n, n))
    A = (G @ G.T) / n
    A[np.diag_indices(n)] += shift
    return symmetrize_lower(A)


def power_lambda_max(M: np.ndarray, iters: int = 100, seed: int = 12345) -> float:
    """Seeded power-iteration estimate of the largest eigenvalue of SPD M."""
    v = rng(seed).standard_normal(M.shape[0])
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = M @ v
        lam = float(v @ w)
        v = w / np.linalg.norm(w)
    return lam


def cond_shift(lam_max: float, target_cond: float) -> float:
    """delta such that (lam_max + delta) / delta = target_cond (lambda_min ~ 0)."""
    return lam_max / (target_cond - 1.0)


def gram_spd_cond(n: int, seed: int, target_cond: float = 1e4) -> np.ndarray:
    g = rng(seed)
    G = g.standard_normal((n, n))
    M = (G @ G.T) / n
    delta = cond_shift(power_lambda_max(M, 100, seed + 1), target_cond)
    M[np.diag_indices(n)] += delta
    return symmetrize_lower(M)


def haar_q(n: int, seed: int) -> np.ndarray:
    """Haar-distributed orthogonal Q from a seeded Gaussian (Mezzadri 2007)."""
    Z = rng(seed).standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def logspaced_spectrum(n: int, cond: float) -> np.ndarray:
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    return cond ** (-i / (n - 1))


def haar_spd(n: int, cond: float, seed: int) -> np.ndarray:
    Q = haar_q(n, seed)
    lam = logspaced_spectrum(n, cond)
    return symmetrize_lower((Q * lam) @ Q.T)


def normal(shape, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(shape)


def batch_sizes(batch: int, seed: int, nmin: int = 16, nmax: int = 512) -> np.ndarray:
    return rng(seed).integers(nmin, nmax + 1, size=batch).astype(np.int64)


def batch_systems(sizes, seed: int, nrhs: int = 1):
    """Per-system A_i = G_i G_i^T / n_i + I, x_i ~ N(0,1), b_i = A_i x_i."""
    As, xs, bs = [], [], []
    for k, n in enumerate(np.asarray(sizes).tolist()):
        A = gram_spd(int(n), seed * 100003 + k)
        x = normal((int(n), nrhs), seed * 100003 + k + 7919)
        As.append(A)
        xs.append(x)
        bs.append(A @ x)
    return As, xs, bs


# ------------------------------------------------------ closed-form families


def lehmer(n: int) -> np.ndarray:
    """A_ij = min(i,j) / max(i,j), 1-based indices."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.minimum.outer(i, i) / np.maximum.outer(i, i)


def laplacian_1d(n: int) -> np.ndarray:
    """tridiag(-1, 2, -1)."""
    A = 2.0 * np.eye(n)
    if n > 1:
        A[np.arange(1, n), np.arange(n - 1)] = -1.0
        A[np.arange(n - 1), np.arange(1, n)] = -1.0
    return A


def diag_1_to_n(n: int) -> np.ndarray:
    """The paper's benchmark matrix diag(1, ..., N)."""
    return np.diag(np.arange(1, n + 1, dtype=np.float64))


def integer_exact(n: int, seed: int, diag_choices=(1, 2, 4), offmax: int = 3):
    """(L0, A) with L0 lower, integer off-diagonal entries in [-offmax, offmax],
    diagonal drawn from ``diag_choices`` (powers of two), A = L0 L0^T computed
    in exact integer arithmetic.  Every intermediate of a substitution-based
    Cholesky of A is an integer far below 2^24, and every division is by a
    power of two, so such a factorisation reproduces L0 exactly."""
    g = rng(seed)
    L0 = np.tril(g.integers(-offmax, offmax + 1, size=(n, n)), -1).astype(np.int64)
    L0[np.diag_indices(n)] = g.choice(np.asarray(diag_choices, dtype=np.int64), size=n)
    A = L0 @ L0.T
    return L0.astype(np.float64), A.astype(np.float64)


def lu_exact(n: int, seed: int):
    """(perm, L0, U0, A) with A = P0^T L0 U0 for a general-solve pin: L0 unit
    lower with entries in {-1/2, -1/4, 0, 1/4, 1/2}, U0 upper with integer
    entries in [-3, 3] and a diagonal in {+-2, +-4, +-8}, P0 a random row
    permutation (row i of L0 U0 is row perm[i] of A).  Every partial sum of
    the elimination is a multiple of 1/4 far below 2^53 and every pivot a
    power of two, and |L0| < 1 below the diagonal makes each pivot a strict
    column maximum, so partial pivoting reproduces P0, L0 and U0 exactly."""
    g = rng(seed)
    L0 = np.tril(g.choice(np.array([-0.5, -0.25, 0.0, 0.25, 0.5]), size=(n, n)), -1) + np.eye(n)
    U0 = np.triu(g.integers(-3, 4, size=(n, n)).astype(np.float64), 1)
    U0[np.diag_indices(n)] = g.choice(np.array([-8.0, -4.0, -2.0, 2.0, 4.0, 8.0]), size=n)
    perm = g.permutation(n)
    M = L0 @ U0                       # exact: dyadic values of small magnitude
    A = np.empty_like(M)
    A[perm] = M
    return perm, L0, U0, A


def general_matrix(n: int, seed: int) -> np.ndarray:
    """Dense general test matrix: i.i.d. N(0, 1) entries (well conditioned
    with high probability at the sizes used), seeded."""
    return rng(seed).standard_normal((n, n))


def hermitian_pd(n: int, seed: int, shift: float = 1.0) -> np.ndarray:
    """Complex Hermitian positive definite A = G G^H / n + shift I, G with
    i.i.d. standard complex normal entries (real and imaginary parts
    N(0, 1/2)), seeded; the full matrix is returned."""
    g = rng(seed)
    G = (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))) / np.sqrt(2.0)
    A = G @ G.conj().T / n + shift * np.eye(n)
    A = (A + A.conj().T) / 2
    A[np.diag_indices(n)] = A.diagonal().real
    return A


def gaussian_integer_hpd(n: int, seed: int, diag_choices=(1, 2, 4), offmax: int = 2):
    """(L0, A) with A = L0 L0^H exact: L0 lower, Gaussian-integer entries
    (real and imaginary parts in [-offmax, offmax]) below a real
    power-of-two diagonal, so every product and partial sum of the complex
    Cholesky factorisation is an exact small dyadic number and the factor
    is L0 itself."""
    g = rng(seed)
    L0 = np.tril(g.integers(-offmax, offmax + 1, size=(n, n)) + 1j * g.integers(-offmax, offmax + 1, size=(n, n)), -1)
    L0 = L0 + np.diag(g.choice(np.array(diag_choices, dtype=np.float64), size=n))
    return L0, L0 @ L0.conj().T


def integer_vector(shape, seed: int, vmax: int = 3) -> np.ndarray:
    return rng(seed).integers(-vmax, vmax + 1, size=shape).astype(np.float64)


# --------------------------------------------------------------------- torch


def torch_gram_spd(n: int, seed: int, shift: float = 1.0, device="cuda", dtype=None):
    """Device version of ``gram_spd`` (torch generator, FP64)."""
    import torch

    dtype = dtype or torch.float64
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    G = torch.randn((n, n), generator=gen, device=device, dtype=dtype)
    A = torch.matmul(G, G.T.contiguous()) / n
    del G
    A.diagonal().add_(shift)
    return torch_symmetrize_lower_(A)


def torch_symmetrize_lower_(A):
    """Mirror the lower triangle onto the upper one, in place, in column slabs."""
    import torch

    n = A.shape[0]
    step = 4096
    for c0 in range(0, n, step):
        c1 = min(n, c0 + step)
        # rows c0..c1 of the upper part come from columns c0..c1 of the lower part
        blk = A[c0:, c0:c1].T.contiguous()      # (c1-c0) x (n-c0), lower part transposed
        mask = torch.triu(torch.ones(c1 - c0, n - c0, dtype=torch.bool, device=A.device), 1)
        rows = A[c0:c1, c0:]
        rows.copy_(torch.where(mask, blk, rows))
    return A


def torch_power_lambda_max(M, iters: int = 100, seed: int = 12345) -> float:
    import torch

    gen = torch.Generator(device=M.device)
    gen.manual_seed(seed)
    v = torch.randn(M.shape[0], generator=gen, device=M.device, dtype=M.dtype)
    v /= torch.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = M @ v
        lam = float(torch.dot(v, w))
        v = w / torch.linalg.norm(w)
    return lam


def torch_gram_spd_cond(n: int, seed: int, target_cond: float = 1e4, device="cuda"):
    A = torch_gram_spd(n, seed, shift=0.0, device=device)
    delta = cond_shift(torch_power_lambda_max(A, 100, seed + 1), target_cond)
    A.diagonal().add_(delta)
    return A


# Largest number of elements any single vendor-library call (QR, GEMM) made
# by these generators may see: library kernels index with 32-bit integers.
VENDOR_CALL_MAX = 2 ** 31 - 1


def _rows_per_call(n: int) -> int:
    """Rows of an n-wide row-major block such that the block stays below
    VENDOR_CALL_MAX elements (a multiple of 1024 when n is large)."""
    r = VENDOR_CALL_MAX // max(1, n)
    return max(1, r // 1024 * 1024 if r >= 1024 else r)


def torch_matmul_rows(A, X):
    """A @ X with A split into row blocks of fewer than 2^31 elements each."""
    import torch

    n = A.shape[0]
    step = _rows_per_call(A.shape[1])
    if n * A.shape[1] <= VENDOR_CALL_MAX:
        return A @ X
    out = torch.empty((n, X.shape[1]), dtype=A.dtype, device=A.device)
    for r0 in range(0, n, step):
        out[r0:r0 + step] = A[r0:r0 + step] @ X
    return out


def _torch_haar_q_panels(n: int, gen, device, b: int = 4096, log=None):
    """Haar Q for n^2 >= 2^31, built so that no library call sees 2^31 or
    more elements.  Q is the orthogonal factor, with positive R diagonal,
    of the QR factorisation of a seeded Gaussian matrix Z (Mezzadri 2007),
    formed panel by panel: panel k of Z (b columns, drawn from the seeded
    generator in panel order) is made orthogonal to the finished columns by
    block Gram-Schmidt applied twice (Giraud et al. 2005: twice is enough),
    then factored by a Householder QR of the n x b panel; R's diagonal signs
    fix the column signs.  Columns of Q are kept as rows of Qt (row-major)
    so every operand is a contiguous block of rows.  Returns Q row-major."""
    import torch

    Qt = torch.empty((n, n), dtype=torch.float64, device=device)
    chunk = _rows_per_call(n)
    for k0 in range(0, n, b):
        k1 = min(n, k0 + b)
        W = torch.randn((k1 - k0, n), generator=gen, device=device, dtype=torch.float64)  # columns of Z as rows
        for _ in range(2):
            for c0 in range(0, k0, chunk):
                c1 = min(k0, c0 + chunk)
                C = Qt[c0:c1] @ W.T                  # (c1-c0) x b: projections on finished columns
                W -= C.T @ Qt[c0:c1]
        Qk, Rk = torch.linalg.qr(W.T)               # n x b panel
        s = torch.sign(torch.diagonal(Rk))
        s[s == 0] = 1.0
        Qt[k0:k1] = (Qk * s).T
        del W, Qk, Rk
        if log:
            log(f"Q panel {k0 // b + 1}/{(n + b - 1) // b}")
    Q = Qt.T.contiguous()
    del Qt
    return Q


def torch_haar_spd(n: int, cond: float, seed: int, device="cuda", log=None):
    """A = Q diag(lambda) Q^T, Haar Q, lambda log-spaced with exact cond;
    `log` (optional) receives progress messages for the large-order path."""
    import torch

    if n * n > VENDOR_CALL_MAX:
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        Q = _torch_haar_q_panels(n, gen, device, log=log)
        lam = torch.as_tensor(logspaced_spectrum(n, cond), device=device)
        A = torch.empty((n, n), dtype=torch.float64, device=device)
        step = min(_rows_per_call(n), 8192)
        for i0 in range(0, n, step):                 # lower block triangle, row blocks of Q
            i1 = min(n, i0 + step)
            Qi = Q[i0:i1] * lam
            for j0 in range(0, i1, step):
                j1 = min(n, j0 + step)
                A[i0:i1, j0:j1] = Qi @ Q[j0:j1].T
            del Qi
            if log:
                log(f"A row block {i0 // step + 1}/{(n + step - 1) // step}")
        del Q
        return torch_symmetrize_lower_(A)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    Z = torch.randn((n, n), generator=gen, device=device, dtype=torch.float64)
    Q, R = torch.linalg.qr(Z)
    del Z
    s = torch.sign(torch.diagonal(R))
    s[s == 0] = 1.0
    del R
    Q.mul_(s)
    lam = torch.as_tensor(logspaced_spectrum(n, cond), device=device)
    A = torch.matmul(Q * lam, Q.T.contiguous())
    del Q
    return torch_symmetrize_lower_(A)


def torch_normal(shape, seed: int, device="cuda", dtype=None):
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return torch.randn(shape, generator=gen, device=device, dtype=dtype or torch.float64)
