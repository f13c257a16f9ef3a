"""Pins for the CPU oracle: every check here is fixed by mathematics or by the
paper's own benchmark recipe, never by re-running the oracle's formula.

Paper: JAXMg, "Software design" (potrs: Cholesky solve of an SPD system,
optionally log det) and "Performance and scaling" (A = diag(1..N), b = ones).
"""
import ctypes
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from golden_io import as_float, worked_examples

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------- worked examples
@pytest.mark.parametrize("name", ["2x2", "3x3", "diag_1_to_8"])
def test_worked_examples_exact(orc, name):
    case = worked_examples()[name]
    A = as_float(case["A"])
    L, info = orc.potrf(A)
    assert info == 0
    if "L" in case:
        assert np.array_equal(L, as_float(case["L"]))
    else:  # diag(1..N): L = diag(sqrt(i))
        assert np.allclose(L, np.diag(np.sqrt(np.diag(A))), rtol=0, atol=0)
    x = orc.potrs(L, as_float(case["b"]))
    xt = as_float(case["x"])
    assert np.allclose(x, xt, rtol=4 * EPS, atol=0)
    assert math.isclose(orc.logdet(L), case["logdet"], rel_tol=1e-14)


# ---------------------------------------------------- integer-exact family
@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (64, 2), (200, 3), (333, 4)])
def test_integer_family_bitwise(orc, n, seed):
    L0, A = synth.integer_exact(n, seed)
    L, info = orc.potrf(A)
    assert info == 0
    assert np.array_equal(L, L0)
    xt = synth.integer_vector((n, 3), seed + 10)
    B = A @ xt  # exact: integers well below 2^53
    X = orc.potrs(L, B)
    assert np.array_equal(X, xt)
    assert orc.logdet(L) == pytest.approx(2 * np.sum(np.log(np.diag(L0))), rel=1e-14, abs=1e-14)


# ----------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 2, 5, 64, 300])
def test_lehmer_closed_form(orc, n):
    A = synth.lehmer(n)
    L, info = orc.potrf(A)
    assert info == 0
    i = np.arange(1, n + 1, dtype=np.float64)
    # L_ij = sqrt(2j-1)/i for i >= j (1-based)
    Lx = np.tril(np.sqrt(2 * i - 1)[None, :] / i[:, None])
    assert np.allclose(L, Lx, rtol=8 * EPS * n, atol=0)
    ld = np.sum(np.log((2 * i - 1) / i ** 2))
    assert orc.logdet(L) == pytest.approx(ld, rel=1e-12, abs=1e-12)
    # inverse is tridiagonal with a closed form
    Ainv = orc.potrs(L, np.eye(n))
    T = np.zeros((n, n))
    for k in range(1, n + 1):
        T[k - 1, k - 1] = 4 * k ** 3 / (4 * k ** 2 - 1) if k < n else n ** 2 / (2 * n - 1)
        if k < n:
            T[k - 1, k] = T[k, k - 1] = -k * (k + 1) / (2 * k + 1)
    if n == 1:
        T[0, 0] = 1.0
    assert np.allclose(Ainv, T, rtol=0, atol=1e-9 * max(1.0, np.abs(T).max()))


@pytest.mark.parametrize("n", [1, 3, 50, 400])
def test_laplacian_closed_form(orc, n):
    A = synth.laplacian_1d(n)
    L, info = orc.potrf(A)
    assert info == 0
    j = np.arange(1, n + 1, dtype=np.float64)
    # the pivots follow a length-n recurrence, one rounding per step
    assert np.allclose(np.diag(L), np.sqrt((j + 1) / j), rtol=4 * n * EPS, atol=0)
    if n > 1:
        jj = j[:-1]
        assert np.allclose(np.diag(L, -1), -np.sqrt(jj / (jj + 1)), rtol=4 * n * EPS, atol=0)
        assert np.count_nonzero(np.tril(L, -2)) == 0
    assert orc.logdet(L) == pytest.approx(math.log(n + 1), rel=1e-12)
    Ainv = orc.potrs(L, np.eye(n))
    I, J = np.meshgrid(j, j, indexing="ij")
    Tinv = np.minimum(I, J) * (n + 1 - np.maximum(I, J)) / (n + 1)
    cond = (2 + 2 * np.cos(np.pi / (n + 1))) / (2 - 2 * np.cos(np.pi / (n + 1)))
    assert np.allclose(Ainv, Tinv, rtol=0, atol=16 * cond * EPS * np.abs(Tinv).max())


@pytest.mark.parametrize("n", [1, 10, 1000])
def test_paper_benchmark_matrix(orc, n):
    """A = diag(1..N), b = ones (paper, 'Performance and scaling')."""
    A = synth.diag_1_to_n(n)
    x, info = orc.posv(A, np.ones(n))
    assert info == 0
    assert np.allclose(x, 1.0 / np.arange(1, n + 1), rtol=4 * EPS, atol=0)
    L, _ = orc.potrf(A)
    assert orc.logdet(L) == pytest.approx(math.lgamma(n + 1), rel=1e-13)


# --------------------------------------------------- library cross-checks
@pytest.mark.parametrize("n,seed", [(17, 0), (256, 1), (700, 2)])
def test_scipy_cross_check(orc, n, seed):
    A = synth.gram_spd(n, seed)
    L, info = orc.potrf(A)
    assert info == 0
    Ls = sla.cholesky(A, lower=True)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(L - Ls) / np.linalg.norm(Ls) <= 10 * kappa * n * EPS
    B = synth.normal((n, 4), seed + 1)
    X = orc.potrs(L, B)
    Xs = sla.cho_solve((Ls, True), B)
    assert np.linalg.norm(X - Xs) / np.linalg.norm(Xs) <= 10 * kappa * n * EPS
    # reconstruction
    assert np.linalg.norm(A - L @ L.T) / np.linalg.norm(A) <= 4 * n * EPS


def test_metamorphic_power_of_two_scaling(orc):
    n = 150
    A = synth.gram_spd(n, 5)
    d = 2.0 ** synth.rng(6).integers(-6, 7, size=n)
    L, _ = orc.potrf(A)
    LD, _ = orc.potrf(d[:, None] * A * d[None, :])
    assert np.array_equal(LD, d[:, None] * L)


def test_only_lower_triangle_read_and_written(orc):
    n = 40
    A = synth.gram_spd(n, 7)
    W = np.asfortranarray(A.copy())
    W[np.triu_indices(n, 1)] = np.nan  # poison the strict upper triangle
    lib = orc._load()
    info = lib.or_potrf(n, W.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)
    assert info == 0
    assert np.all(np.isnan(W[np.triu_indices(n, 1)]))
    L, _ = orc.potrf(A)
    assert np.array_equal(np.tril(W), L)
    # lda > n: guard rows never touched
    lda = n + 5
    G = np.full((lda, n), -7.0, order="F")
    G[:n, :] = A
    info = lib.or_potrf(n, G.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lda)
    assert info == 0 and np.all(G[n:, :] == -7.0)
    assert np.array_equal(np.tril(G[:n]), L)


# --------------------------------------------------------- failure / edges
@pytest.mark.parametrize("k", [1, 5, 64])
def test_not_spd_info(orc, k):
    n = 64
    d = np.ones(n)
    d[k - 1] = -1.0
    _, info = orc.potrf(np.diag(d))
    assert info == k


def test_nan_info(orc):
    n = 30
    A = synth.gram_spd(n, 3)
    A[9, 9] = np.nan
    assert orc.potrf(A)[1] == 10
    A = synth.gram_spd(n, 3)
    A[20, 4] = A[4, 20] = np.nan     # poisons L[20,4]; pivot 21 is the first NaN pivot
    assert orc.potrf(A)[1] == 21


def test_edge_sizes(orc):
    L, info = orc.potrf(np.zeros((0, 0)))
    assert info == 0 and L.shape == (0, 0)
    L, info = orc.potrf(np.array([[9.0]]))
    assert info == 0 and L[0, 0] == 3.0
    X = orc.potrs(np.array([[3.0]]), np.zeros((1, 0)))
    assert X.shape == (1, 0)


# ----------------------------------------------------------- residual / eta
def test_residual_against_exact_rationals(orc):
    n, nrhs = 6, 2
    g = synth.rng(11)
    A = synth.symmetrize_lower(g.standard_normal((n, n)))
    X = g.standard_normal((n, nrhs))
    B = g.standard_normal((n, nrhs))
    R, eta, anorm = orc.residual(A, X, B)
    Af = [[Fraction(A[i, j]) for j in range(n)] for i in range(n)]
    for r in range(nrhs):
        rex = [Fraction(B[i, r]) - sum(Af[i][j] * Fraction(X[j, r]) for j in range(n))
               for i in range(n)]
        for i in range(n):
            assert R[i, r] == float(rex[i])     # correctly rounded within 1 rounding
        an = max(sum(abs(Af[i][j]) for j in range(n)) for i in range(n))
        assert anorm == float(an)
        den = an * max(abs(Fraction(X[i, r])) for i in range(n)) + max(abs(Fraction(B[i, r])) for i in range(n))
        assert eta[r] == pytest.approx(float(max(abs(v) for v in rex) / den), rel=1e-15)


def test_eta_zero_for_exact_solution_and_scale_invariant(orc):
    L0, A = synth.integer_exact(50, 9)
    xt = synth.integer_vector((50, 2), 1)
    B = A @ xt
    _, eta, _ = orc.residual(A, xt, B)
    assert np.all(eta == 0.0)
    x = xt + 1e-3
    _, e1, _ = orc.residual(A, x, B)
    _, e2, _ = orc.residual(8.0 * A, x, 8.0 * B)
    assert np.array_equal(e1, e2) and np.all(e1 > 0)


def test_posv_backward_error_random(orc):
    n = 500
    A = synth.gram_spd_cond(n, 21, 1e4)
    xt = synth.normal((n, 5), 22)
    B = A @ xt
    X, info = orc.posv(A, B)
    assert info == 0
    eta = orc.backward_error(A, X, B)
    assert np.all(eta <= 1e-15)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(X - xt) / np.linalg.norm(xt) <= kappa * 1e-13


# ------------------------------------------------------------ generators
def test_generators_shape_symmetry_cond():
    A = synth.gram_spd_cond(512, 3, 1e4)
    assert np.array_equal(A, A.T)
    w = np.linalg.eigvalsh(A)
    assert 0.9e4 <= w[-1] / w[0] <= 1.1e4
    H = synth.haar_spd(256, 1e6, 4)
    assert np.array_equal(H, H.T)
    w = np.linalg.eigvalsh(H)
    assert w[-1] / w[0] == pytest.approx(1e6, rel=1e-6)
    assert np.array_equal(synth.gram_spd(64, 1), synth.gram_spd(64, 1))
    s = synth.batch_sizes(4096, 0)
    assert s.min() >= 16 and s.max() <= 512 and len(s) == 4096


# ------------------------------------------------------ mixed precision IR
@pytest.mark.parametrize("lo", [1, 2])
def test_ir_integer_family_is_exact(orc, lo):
    L0, A = synth.integer_exact(120, 3)
    Lw, info = orc.potrf_lo(A, lo)
    assert info == 0 and np.array_equal(Lw.astype(np.float64), L0)
    xt = synth.integer_vector((120, 2), 4)
    X, st = orc.posv_ir(A, A @ xt, lo=lo)
    assert st["iters"] == 0 and not st["fell_back"]
    assert np.array_equal(X, xt)


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_ir_fp32_converges(orc, cond):
    n = 256
    A = synth.haar_spd(n, cond, 5)
    xt = synth.normal((n, 3), 6)
    B = A @ xt
    X, st = orc.posv_ir(A, B, lo=1)
    assert not st["fell_back"]
    assert 1 <= st["iters"] <= 6
    assert np.all(orc.backward_error(A, X, B) <= 1e-12)
    # forward error <= ~2 kappa eta (Higham, Thm 7.2) with eta <= tol at exit
    assert np.linalg.norm(X - xt) / np.linalg.norm(xt) <= 4 * cond * 1e-12


def test_ir_bf16_low_cond_and_fallback(orc):
    n = 128
    A = synth.haar_spd(n, 1e2, 7)
    xt = synth.normal((n, 2), 8)
    B = A @ xt
    X, st = orc.posv_ir(A, B, lo=2)
    assert np.all(orc.backward_error(A, X, B) <= 1e-12)
    # max_iter = 0 forces the FP64 fallback on an inexact first solve
    X, st = orc.posv_ir(A, B, lo=1, max_iter=0)
    assert st["fell_back"] and st["info"] == 0
    assert np.all(orc.backward_error(A, X, B) <= 1e-12)
    # an indefinite matrix fails in both precisions
    D = np.diag(np.r_[np.ones(10), -1.0, np.ones(5)])
    X, st = orc.posv_ir(D, np.ones(16), lo=1)
    assert st["fell_back"] and st["info"] == 11


# ----------------------------------------------------------------- adjoint
def _loss_and_grad(orc, A, B, W):
    X, info = orc.posv(A, B)
    assert info == 0
    L, _ = orc.potrf(A)
    gB, gA = orc.posv_backward(L, X, W, mode=0)
    return float(np.sum(W * X)), gB, gA


def test_adjoint_central_differences(orc):
    n, nrhs = 9, 3
    A = synth.gram_spd(n, 13)
    B = synth.normal((n, nrhs), 14)
    W = synth.normal((n, nrhs), 15)
    _, gB, gA = _loss_and_grad(orc, A, B, W)
    h = 1e-6
    for i in range(n):
        for j in range(i + 1):
            E = np.zeros((n, n))
            E[i, j] = E[j, i] = 1.0
            fp = np.sum(W * orc.posv(A + h * E, B)[0])
            fm = np.sum(W * orc.posv(A - h * E, B)[0])
            fd = (fp - fm) / (2 * h)
            an = np.sum(gA * E)
            assert an == pytest.approx(fd, rel=1e-6, abs=1e-8)
    for i in range(n):
        for r in range(nrhs):
            E = np.zeros((n, nrhs))
            E[i, r] = 1.0
            fd = (np.sum(W * orc.posv(A, B + h * E)[0]) - np.sum(W * orc.posv(A, B - h * E)[0])) / (2 * h)
            assert gB[i, r] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_adjoint_special_cases(orc):
    n, nrhs = 12, 2
    B = synth.normal((n, nrhs), 1)
    W = synth.normal((n, nrhs), 2)
    _, gB, gA = _loss_and_grad(orc, np.eye(n), B, W)
    assert np.array_equal(gB, W)
    assert np.allclose(gA, -0.5 * (W @ B.T + B @ W.T), rtol=0, atol=1e-15)
    d = 4.0 ** np.arange(n)  # perfect squares: L = diag(2^i) exactly
    _, gB, _ = _loss_and_grad(orc, np.diag(d), B, W)
    assert np.array_equal(gB, W / d[:, None])
    # lower-parameter mode: off-diagonal entries are twice the symmetric ones
    A = synth.gram_spd(n, 3)
    X, _ = orc.posv(A, B)
    L, _ = orc.potrf(A)
    _, g0 = orc.posv_backward(L, X, W, mode=0)
    _, g1 = orc.posv_backward(L, X, W, mode=1)
    il = np.tril_indices(n, -1)
    assert np.allclose(g1[il], 2 * g0[il], rtol=1e-15, atol=0)
    assert np.allclose(np.diag(g1), np.diag(g0), rtol=1e-15, atol=1e-300)
    assert np.all(g1[np.triu_indices(n, 1)] == 0)


def test_planted_mistakes_are_caught():
    """A plausible slip in a Cholesky routine (a transposed operand, a dropped
    term, a sign) breaks at least one of the pins above.  Implemented on a
    throw-away Python copy of the column algorithm, never the oracle itself."""
    def chol(A, variant):
        n = A.shape[0]
        L = np.tril(A).astype(np.float64)
        for j in range(n):
            for k in range(j if variant != "drop_last" else max(j - 1, 0)):
                if variant == "transpose":
                    L[j:, j] -= L[j:, k] * L[k, j]
                elif variant == "sign":
                    L[j:, j] += L[j:, k] * L[j, k]
                else:
                    L[j:, j] -= L[j:, k] * L[j, k]
            L[j:, j] /= np.sqrt(L[j, j]) if L[j, j] > 0 else np.nan
        return L
    L0, A = synth.integer_exact(20, 1)
    assert np.array_equal(chol(A, "ok"), L0)
    for v in ("transpose", "sign", "drop_last"):
        with np.errstate(all="ignore"):
            assert not np.array_equal(chol(A, v), L0)


# ------------------------------------------------------ general solve (lu_solve)
# The paper's general solve: P A = L U by partial pivoting, then the two
# triangular solves ("Software design", lu_solve bullet).
def _perm_from_ipiv(ipiv):
    p = np.arange(len(ipiv))
    for k, r in enumerate(ipiv):
        p[[k, r - 1]] = p[[r - 1, k]]
    return p


def test_getrf_hand_worked_2x2(orc):
    """A = [[1, 2], [4, 4]]: |4| > |1| so the rows swap (ipiv = [2, 2]);
    l = 1/4, U = [[4, 4], [0, 2 - 4/4]] = [[4, 4], [0, 1]]."""
    LU, ipiv, info = orc.getrf(np.array([[1.0, 2.0], [4.0, 4.0]]))
    assert info == 0 and list(ipiv) == [2, 2]
    assert np.array_equal(LU, np.array([[4.0, 4.0], [0.25, 1.0]]))
    # x1 + 2 x2 = 5, 4 x1 + 4 x2 = 12  =>  x = (1, 2)
    assert np.array_equal(orc.getrs(LU, ipiv, np.array([5.0, 12.0])), np.array([1.0, 2.0]))


@pytest.mark.parametrize("n,seed", [(1, 1), (3, 2), (17, 3), (64, 4), (150, 5)])
def test_getrf_dyadic_family_exact(orc, n, seed):
    perm, L0, U0, A = synth.lu_exact(n, seed)
    LU, ipiv, info = orc.getrf(A)
    assert info == 0
    assert np.array_equal(np.tril(LU, -1) + np.eye(n), L0)
    assert np.array_equal(np.triu(LU), U0)
    assert np.array_equal(_perm_from_ipiv(ipiv), perm)       # row k of P A is row perm[k] of A
    xt = synth.integer_vector((n, 3), seed)
    assert np.array_equal(orc.getrs(LU, ipiv, A @ xt), xt)


def test_getrf_reconstruction_and_backward_error(orc):
    n = 120
    A = synth.general_matrix(n, 7)
    LU, ipiv, info = orc.getrf(A)
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    p = _perm_from_ipiv(ipiv)
    assert np.linalg.norm(A[p] - L @ U) / np.linalg.norm(A) <= 8 * n * EPS
    assert np.all(np.abs(np.tril(LU, -1)) <= 1.0)               # partial pivoting: |l| <= 1
    xt = synth.normal((n, 4), 8)
    B = A @ xt
    X = orc.getrs(LU, ipiv, B)
    assert np.all(orc.backward_error_gen(A, X, B) <= 4 * n * EPS)


def test_getrf_matches_lapack_pivots(orc):
    """Library cross-check: LAPACK dgetrf (scipy) picks the same pivots."""
    from scipy.linalg import lu_factor
    n = 80
    A = synth.general_matrix(n, 9)
    LU, ipiv, info = orc.getrf(A)
    lu, piv = lu_factor(A)
    assert np.array_equal(ipiv, piv + 1)
    assert np.allclose(LU, lu, rtol=0, atol=1e-12 * np.abs(lu).max())


def test_getrf_singular_info(orc):
    """A zero pivot (here an all-zero column 3) is reported as info = 3 and
    elimination continues (LAPACK semantics)."""
    A = synth.general_matrix(6, 10)
    A[:, 2] = 0.0
    LU, ipiv, info = orc.getrf(A)
    assert info == 3
    assert np.all(np.isfinite(LU))


def test_getrf_planted_mistakes_are_caught(orc):
    """No pivoting, pivoting on the signed maximum, or an update that skips
    the first column's multiplier each break a pin above (on a throw-away
    numpy copy, never the oracle)."""
    def lu(A, variant):
        A = A.copy()
        n = A.shape[0]
        perm = np.arange(n)
        for k in range(n):
            col = A[k:, k]
            p = k if variant == "no_pivot" else k + int(np.argmax(col if variant == "signed" else np.abs(col)))
            A[[k, p]] = A[[p, k]]
            perm[[k, p]] = perm[[p, k]]
            A[k + 1:, k] /= A[k, k]
            if not (variant == "skip" and k == 0):
                A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
        return A, perm
    perm, L0, U0, A = synth.lu_exact(30, 11)
    ok, p_ok = lu(A, "ok")
    assert np.array_equal(np.triu(ok), U0) and np.array_equal(p_ok, perm)
    for v in ("no_pivot", "signed", "skip"):
        with np.errstate(all="ignore"):
            bad, p_bad = lu(A, v)
        assert not (np.array_equal(np.triu(bad), U0) and np.array_equal(p_bad, perm)), v


# ------------------------------------------------------ complex Hermitian
# The paper lists complex64 and complex128 for its routines.  Pins: a
# factor worked by hand, the real special case (bit-identical to the real
# column algorithm), the Gaussian-integer family (every operation exact),
# scipy's LAPACK ZPOTRF/ZPOTRS, info, and the parts of A that are never read.
def test_zpotrf_hand_worked_2x2(orc):
    """A = [[4, 2-2i], [2+2i, 6]]: L11 = 2, l21 = (2+2i)/2 = 1+i,
    L22 = sqrt(6 - |1+i|^2) = 2; b = A [1, i]^T = [4+2+2i, 2+2i+6i]."""
    A = np.array([[4, 2 - 2j], [2 + 2j, 6]])
    L, info = orc.zpotrf(A)
    assert info == 0
    assert np.array_equal(np.tril(L), np.array([[2, 0], [1 + 1j, 2]]))
    x = orc.zpotrs(L, np.array([6 + 2j, 2 + 8j]))
    assert np.array_equal(x, np.array([1, 1j]))


@pytest.mark.parametrize("n", [1, 5, 40])
def test_zpotrf_real_case_is_real_cholesky(orc, n):
    A = synth.gram_spd(n, 70 + n)
    L, info = orc.zpotrf(A.astype(np.complex128))
    Lr, info_r = orc.potrf(A)
    assert info == info_r == 0
    assert np.array_equal(np.tril(L).real, np.tril(Lr)) and not np.any(np.tril(L).imag)


@pytest.mark.parametrize("n,seed", [(6, 1), (33, 2), (80, 3)])
def test_zpotrf_gaussian_integer_family_exact(orc, n, seed):
    L0, A = synth.gaussian_integer_hpd(n, seed)
    L, info = orc.zpotrf(A)
    assert info == 0 and np.array_equal(np.tril(L), L0)
    xt = synth.integer_vector((n, 2), seed) + 1j * synth.integer_vector((n, 2), seed + 1)
    X, info = orc.zposv(A, A @ xt)
    assert info == 0 and np.array_equal(X, xt)
    assert np.all(orc.backward_error_z(A, X, A @ xt) == 0.0)


def test_zpotrf_matches_lapack(orc):
    scipy_linalg = pytest.importorskip("scipy.linalg")
    n = 60
    A = synth.hermitian_pd(n, 5)
    L, info = orc.zpotrf(A)
    Ls = scipy_linalg.cholesky(A, lower=True)
    assert info == 0 and np.allclose(np.tril(L), Ls, rtol=1e-13, atol=1e-14)
    B = synth.normal((n, 3), 6) + 1j * synth.normal((n, 3), 7)
    X = orc.zpotrs(L, B)
    Xs = scipy_linalg.cho_solve((Ls, True), B)
    assert np.allclose(X, Xs, rtol=1e-12, atol=1e-13)
    assert np.all(orc.backward_error_z(A, X, B) <= 1e-15)


def test_zpotrf_info_and_unread_parts(orc):
    n = 12
    A = synth.hermitian_pd(n, 8)
    G = A.copy()
    G[np.triu_indices(n, 1)] = np.nan + 1j * np.nan       # strict upper never read
    G[np.diag_indices(n)] += 1j * 7.0                      # imaginary diagonal ignored
    L, info = orc.zpotrf(G)
    L2, _ = orc.zpotrf(A)
    assert info == 0 and np.array_equal(np.tril(L), np.tril(L2))
    B = A.copy()
    B[5, 5] = -1.0
    _, info = orc.zpotrf(B)
    assert info == 6


def test_zpotrf_planted_mistakes_are_caught(orc):
    """A factor that drops the conjugate (A = L L^T) or a solve that uses L^T
    instead of L^H each break the Gaussian-integer pin (throw-away numpy
    code, never the oracle)."""
    L0, A = synth.gaussian_integer_hpd(20, 4)
    def chol(A, conj):
        A = A.copy()
        n = A.shape[0]
        for j in range(n):
            for k in range(j):
                A[j:, j] -= A[j:, k] * (np.conj(A[j, k]) if conj else A[j, k])
            A[j, j] = np.sqrt(A[j, j].real)
            A[j + 1:, j] /= A[j, j]
        return np.tril(A)
    assert np.array_equal(chol(A, True), L0)
    with np.errstate(all="ignore"):
        assert not np.array_equal(chol(A, False), L0)
    xt = synth.integer_vector(20, 9) + 1j * synth.integer_vector(20, 10)
    b = A @ xt
    y = np.linalg.solve(L0, b)
    assert np.allclose(np.linalg.solve(L0.conj().T, y), xt)
    assert not np.allclose(np.linalg.solve(L0.T, y), xt)


# ------------------------------------------------------ Cholesky adjoint
# Gradient with respect to A of f(L), L = chol(A), given gL = df/dL (Murray
# 2016; the paper is silent).  Pins: central differences of the oracle's own
# (independently pinned) factor over every symmetric direction, the diagonal
# closed form derived by hand below, exact power-of-two scaling, symmetry and
# the relation between the two modes.
def _chol_loss(orc, A, W):
    L, info = orc.potrf(A)
    assert info == 0
    return float(np.sum(np.tril(W) * L))


@pytest.mark.parametrize("n", [1, 2, 7, 12])
def test_potrf_backward_central_differences(orc, n):
    A = synth.gram_spd(n, 40 + n)
    W = synth.normal((n, n), 41 + n)
    L, _ = orc.potrf(A)
    g0 = orc.potrf_backward(L, W, mode=0)
    g1 = orc.potrf_backward(L, W, mode=1)
    assert np.array_equal(g0, g0.T)
    h = 1e-6
    for i in range(n):
        for j in range(i + 1):
            E = np.zeros((n, n))
            E[i, j] = E[j, i] = 1.0
            fd = (_chol_loss(orc, A + h * E, W) - _chol_loss(orc, A - h * E, W)) / (2 * h)
            assert np.sum(g0 * E) == pytest.approx(fd, rel=1e-6, abs=1e-8), (i, j)
            # mode 1: derivative with respect to the lower entry (i, j), which
            # the symmetric input carries at (i, j) and (j, i)
            assert g1[i, j] == pytest.approx(fd, rel=1e-6, abs=1e-8), (i, j)
    assert np.all(g1[np.triu_indices(n, 1)] == 0)


def test_potrf_backward_diagonal_closed_form(orc):
    """A = diag(d): to first order chol(A + dA) = diag(sqrt d) + dL with
    dL_jj = dA_jj / (2 sqrt d_j) and dL_ij = dA_ij / sqrt d_j (i > j), so
    df = sum_j gL_jj dA_jj / (2 sqrt d_j) + sum_{i>j} gL_ij dA_ij / sqrt d_j
    and the symmetric gradient is gA_jj = gL_jj / (2 sqrt d_j),
    gA_ij = gA_ji = gL_ij / (2 sqrt d_j)."""
    n = 9
    d = 4.0 ** np.arange(-3, n - 3)                   # exact square roots
    W = np.tril(synth.normal((n, n), 7))
    L, _ = orc.potrf(np.diag(d))
    g = orc.potrf_backward(L, W, mode=0)
    sq = np.sqrt(d)
    want = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            want[i, j] = want[j, i] = W[i, j] / (2 * sq[j])
    assert np.allclose(g, want, rtol=4e-16, atol=0)
    # 1 x 1: d sqrt(a) / da = 1 / (2 sqrt(a))
    g1 = orc.potrf_backward(np.array([[3.0]]), np.array([[5.0]]))
    assert g1[0, 0] == pytest.approx(5.0 / 6.0, rel=1e-15)


def test_potrf_backward_power_of_two_scaling(orc):
    """chol(4 A) = 2 chol(A), so f(4 A) = 2 f(A) and the gradient at 4 A is
    the gradient at A halved, bit for bit (every intermediate scales by a
    power of two)."""
    n = 10
    A = synth.gram_spd(n, 8)
    W = synth.normal((n, n), 9)
    L, _ = orc.potrf(A)
    L4, _ = orc.potrf(4.0 * A)
    assert np.array_equal(L4, 2.0 * L)
    assert np.array_equal(orc.potrf_backward(L4, W), orc.potrf_backward(L, W) / 2.0)


def test_potrf_backward_planted_mistakes_are_caught(orc):
    """Plausible slips in the adjoint (no halving of the diagonal in Phi,
    gL^T L instead of L^T gL, a missing symmetrisation) each break one of the
    pins above.  Implemented on a throw-away numpy copy, never the oracle."""
    def adj(L, W, variant):
        W = np.tril(W)
        M = W.T @ L if variant == "transpose" else L.T @ W
        P = np.tril(M)
        if variant != "no_half":
            P[np.diag_indices_from(P)] *= 0.5
        Li = np.linalg.inv(L)
        S = Li.T @ P @ Li
        return S if variant == "no_sym" else 0.5 * (S + S.T)
    n = 8
    A = synth.gram_spd(n, 21)
    W = synth.normal((n, n), 22)
    L, _ = orc.potrf(A)
    ref = orc.potrf_backward(L, W)
    assert np.allclose(adj(L, W, "ok"), ref, rtol=1e-12, atol=1e-12)
    assert not np.allclose(adj(L, W, "no_half"), ref, rtol=1e-6)
    assert not np.allclose(adj(L, W, "transpose"), ref, rtol=1e-6)
    g = adj(L, W, "no_sym")
    assert not np.array_equal(g, g.T)


# ---------------------------------------------------------------- GP likelihood
# The paper (Research Impact Statement, "Scientific applications", Cholesky
# solve) defines log L = -1/2 r^T A^{-1} r - 1/2 log det A - N/2 log(2 pi),
# r = y - m.  The pins below evaluate that formula in closed form, without
# the oracle's factor or solve.
def _lehmer_inverse_quadform(r):
    """r^T A^{-1} r for the Lehmer matrix, from its tridiagonal inverse:
    (A^{-1})_ii = 4 i^3 / (4 i^2 - 1) for i < n, (A^{-1})_nn = n^2 / (2n - 1),
    (A^{-1})_{i,i+1} = -i (i + 1) / (2 i + 1) (1-based)."""
    n = len(r)
    terms = []
    for i in range(1, n + 1):
        d = 4.0 * i ** 3 / (4.0 * i * i - 1.0) if i < n else n * n / (2.0 * n - 1.0)
        terms.append(d * r[i - 1] * r[i - 1])
        if i < n:
            terms.append(2.0 * (-i * (i + 1.0) / (2.0 * i + 1.0)) * r[i - 1] * r[i])
    return math.fsum(terms)


def test_gp_loglik_diagonal_closed_form(orc):
    n = 300
    d = 0.5 + synth.rng(31).random(n) * 3.0
    y = synth.normal((n, 3), 32)
    m = synth.normal((n, 3), 33)
    ll, alpha, info = orc.gp_loglik(np.diag(d), y, m)
    assert info == 0
    for j in range(3):
        r = y[:, j] - m[:, j]
        want = (-0.5 * math.fsum(r * r / d) - 0.5 * math.fsum(np.log(d)) - 0.5 * n * math.log(2 * math.pi))
        assert ll[j] == pytest.approx(want, rel=1e-13)
        assert np.allclose(alpha[:, j], r / d, rtol=1e-14, atol=0)


def test_gp_loglik_lehmer_closed_form(orc):
    n = 200
    A = synth.lehmer(n)
    y = synth.normal(n, 34)
    ll, alpha, info = orc.gp_loglik(A, y)
    ld = math.fsum(math.log((2.0 * j - 1.0) / (j * j)) for j in range(1, n + 1))
    want = -0.5 * _lehmer_inverse_quadform(y) - 0.5 * ld - 0.5 * n * math.log(2 * math.pi)
    assert info == 0
    assert ll == pytest.approx(want, rel=1e-11)


def test_gp_loglik_special_cases(orc):
    n = 50
    # A = I, y = m: only the normalisation remains
    y = synth.normal(n, 35)
    ll, _, info = orc.gp_loglik(np.eye(n), y, y.copy())
    assert info == 0 and ll == -0.5 * n * math.log(2 * math.pi)
    # n = 1 by hand
    ll1, a1, _ = orc.gp_loglik(np.array([[4.0]]), np.array([3.0]))
    assert ll1 == pytest.approx(-0.5 * 9.0 / 4.0 - 0.5 * math.log(4.0) - 0.5 * math.log(2 * math.pi), rel=1e-15)
    assert a1[0] == 0.75
    # a mean is the same as subtracting it from the observations
    A = synth.gram_spd(n, 36)
    m = synth.normal(n, 37)
    assert orc.gp_loglik(A, y, m)[0] == pytest.approx(orc.gp_loglik(A, y - m)[0], rel=1e-14)
    # not positive definite: NaN and the centred observations
    B = np.eye(n)
    B[7, 7] = -1.0
    llb, ab, infob = orc.gp_loglik(B, y, m)
    assert infob == 8 and math.isnan(llb) and np.array_equal(ab, y - m)


def test_gp_loglik_grad_closed_forms_and_finite_differences(orc):
    # diagonal A: alpha = r / d, dA = g (alpha alpha^T - diag(1 / d)) / 2, dY = -g r / d
    n = 40
    d = 0.5 + synth.rng(60).random(n) * 3.0
    y = synth.normal(n, 61)
    dA, dY, dM, info = orc.gp_loglik_grad(np.diag(d), y, None, g=[2.0])
    assert info == 0
    assert np.allclose(dA, np.outer(y / d, y / d) - np.diag(1.0 / d), rtol=1e-13, atol=1e-15)
    assert np.allclose(dY, -2.0 * y / d, rtol=1e-14) and np.allclose(dM, 2.0 * y / d, rtol=1e-14)
    # A = I: dA = (r r^T - I) / 2
    dA, _, _, _ = orc.gp_loglik_grad(np.eye(n), y)
    assert np.allclose(dA, 0.5 * (np.outer(y, y) - np.eye(n)), rtol=1e-14, atol=1e-15)
    # central differences of the oracle's own log L along symmetric directions
    n = 10
    A = synth.gram_spd(n, 62)
    Y = synth.normal((n, 2), 63)
    M = synth.normal((n, 2), 64)
    g = np.array([0.7, -1.3])
    dA, dY, dM, _ = orc.gp_loglik_grad(A, Y, M, g)
    f = lambda A_, Y_, M_: float(np.dot(g, orc.gp_loglik(A_, Y_, M_)[0]))
    h = 1e-6
    for i in range(n):
        for j in range(i + 1):
            E = np.zeros((n, n))
            E[i, j] = E[j, i] = 1.0
            fd = (f(A + h * E, Y, M) - f(A - h * E, Y, M)) / (2 * h)
            want = dA[i, j] if i == j else dA[i, j] + dA[j, i]
            assert fd == pytest.approx(want, rel=1e-6, abs=1e-8)
    for i in range(n):
        E = np.zeros((n, 2))
        E[i, 1] = 1.0
        assert (f(A, Y + h * E, M) - f(A, Y - h * E, M)) / (2 * h) == pytest.approx(dY[i, 1], rel=1e-6, abs=1e-8)
        assert (f(A, Y, M + h * E) - f(A, Y, M - h * E)) / (2 * h) == pytest.approx(dM[i, 1], rel=1e-6, abs=1e-8)


# ------------------------------------------------ bfloat16 rounding (by hand)
# Round-to-nearest-even from binary32 (23 fraction bits) to bfloat16 (7): the
# upper 16 bits are kept and the lower 16 decide, 0x8000 being the tie.  Each
# row was worked out by hand; the last column names the slip it catches.
BF16_TABLE = [
    (0x3F800000, 0x3F800000, "1.0 is exact (any rounding)"),
    (0x3F807FFF, 0x3F800000, "just below half an ulp rounds down (round-half-up on a wrong bit)"),
    (0x3F808000, 0x3F800000, "tie with an even kept part rounds down (ties away from zero)"),
    (0x3F818000, 0x3F820000, "tie with an odd kept part rounds up (truncation)"),
    (0x3F80C000, 0x3F810000, "three quarters of an ulp rounds up (truncation)"),
    (0x3FFF8000, 0x40000000, "tie, odd, significand carry into the exponent (masking the carry)"),
    (0xBF818000, 0xBF820000, "negative tie: the magnitude rounds, the sign stays (sign handling)"),
    (0x00018000, 0x00020000, "subnormal tie with an odd kept part rounds up"),
    (0x7F7FFFFF, 0x7F800000, "largest binary32 is past the last bfloat16 midpoint: infinity"),
    (0x7F800000, 0x7F800000, "+infinity passes through"),
    (0xFF800000, 0xFF800000, "-infinity passes through"),
    (0x7F800001, 0x7F800001, "NaN with a low payload stays that NaN (rounding would make it infinity)"),
    (0x7FC12345, 0x7FC12345, "quiet NaN passes through unchanged"),
]


def _bits_to_f32(b):
    return np.array(b, dtype=np.uint32).view(np.float32)


def test_round_bf16_hand_worked_bit_patterns(orc):
    ins = _bits_to_f32([r[0] for r in BF16_TABLE])
    out = orc.round_bf16(ins).view(np.uint32)
    for (a, want, why), got in zip(BF16_TABLE, out.tolist()):
        assert got == want, f"{a:#010x} -> {got:#010x}, want {want:#010x}: {why}"


def test_round_bf16_table_catches_wrong_roundings():
    """Plausible wrong roundings (truncation, ties away from zero, no
    special-value guard) each disagree with at least one hand-worked row.
    Implemented on throw-away Python copies, never on the oracle."""
    def ok(u):
        if (u & 0x7F800000) == 0x7F800000:
            return u
        return (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000

    def trunc(u):
        return u & 0xFFFF0000

    def away(u):
        if (u & 0x7F800000) == 0x7F800000:
            return u
        return (u + 0x8000) & 0xFFFF0000

    def unguarded(u):
        return (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000

    assert all(ok(a) == w for a, w, _ in BF16_TABLE)
    for bad in (trunc, away, unguarded):
        assert any(bad(a) != w for a, w, _ in BF16_TABLE), bad.__name__


# --------------------------------------- blocked low-precision factor reading
def test_blocked_lo_factor_one_block_is_fp64_factor_rounded(orc):
    """nb >= n: the whole matrix is one diagonal block, so the blocked
    factor is the FP64 Cholesky factor of fl32(A), rounded to binary32
    (catches a diagonal block factored in binary32, or left unrounded)."""
    n = 90
    A = synth.haar_spd(n, 1e3, 41)
    A32 = A.astype(np.float32).astype(np.float64)
    L64, info = orc.potrf(A32)
    assert info == 0
    for lo in (1, 2):
        Lb, info = orc.potrf_lo(A, lo, nb=n)
        assert info == 0
        assert np.array_equal(Lb, L64.astype(np.float32))
        Lb, info = orc.potrf_lo(A, lo, nb=4 * n)
        assert np.array_equal(Lb, L64.astype(np.float32))


@pytest.mark.parametrize("lo", [1, 2])
@pytest.mark.parametrize("nb", [1, 16, 64, 128])
def test_blocked_lo_factor_integer_family_bitwise(orc, lo, nb):
    """Every intermediate of the integer family is an integer below 2^24 and
    every division is by a power of two; |L0| <= 3 is exact in bfloat16, so
    the blocked factor reproduces L0 in both precisions whatever nb."""
    L0, A = synth.integer_exact(150, 60 + nb)
    Lb, info = orc.potrf_lo(A, lo, nb=nb)
    assert info == 0
    assert np.array_equal(Lb.astype(np.float64), L0)


@pytest.mark.parametrize("b_bits,b_bf16", [
    (0x3F802000, 1.0),               # 1 + 2^-10: below half a bfloat16 ulp -> 1
    (0x3F80C000, 1.0 + 2.0 ** -7),   # 1 + 3 2^-9: above half -> 1 + 2^-7 (truncation would give 1)
])
def test_blocked_lo_factor_2x2_by_hand(orc, b_bits, b_bf16):
    """A = [[1, b], [b, 4]], nb = 1.  Block 0: L11 = 1.  Panel: L21 = b / 1 =
    b.  Trailing: binary32 mode W22 = 4 - fl32(b^2); bfloat16 mode
    W22 = 4 - r(b)^2 with r(b) worked out by hand.  Then L22 =
    fl32(sqrt(W22)) taken in FP64.  The two modes must differ (a no-op
    bfloat16 rounding fails here)."""
    b = float(_bits_to_f32([b_bits])[0])
    A = np.array([[1.0, b], [b, 4.0]])
    f32 = np.float32
    w1 = f32(f32(4.0) - f32(f32(b) * f32(b)))
    want1 = f32(np.sqrt(np.float64(w1)))
    w2 = f32(f32(4.0) - f32(f32(b_bf16) * f32(b_bf16)))
    want2 = f32(np.sqrt(np.float64(w2)))
    assert want1 != want2
    for lo, want in ((1, want1), (2, want2)):
        Lb, info = orc.potrf_lo(A, lo, nb=1)
        assert info == 0
        assert Lb[0, 0] == 1.0 and Lb[1, 0] == f32(b) and Lb[1, 1] == want, (lo, Lb)


def test_blocked_lo_factor_error_scales_with_working_precision(orc):
    """Random SPD: the binary32 and bfloat16 factors differ, and each is
    within its unit roundoff times kappa of the FP64 factor (Higham, Thm
    10.5, normwise form); bfloat16 is the looser of the two."""
    n = 200
    A = synth.haar_spd(n, 1e2, 43)
    L64, _ = orc.potrf(A)
    L1, i1 = orc.potrf_lo(A, 1, nb=64)
    L2, i2 = orc.potrf_lo(A, 2, nb=64)
    assert i1 == 0 and i2 == 0
    e1 = np.linalg.norm(L1 - L64) / np.linalg.norm(L64)
    e2 = np.linalg.norm(L2 - L64) / np.linalg.norm(L64)
    assert not np.array_equal(L1, L2)
    assert e1 <= 1e2 * n * 2.0 ** -24
    assert e2 <= 1e2 * n * 2.0 ** -8
    assert e2 > 8 * e1


@pytest.mark.parametrize("lo", [1, 2])
def test_blocked_lo_factor_reports_first_bad_pivot(orc, lo):
    d = np.ones(40)
    d[25] = -1.0
    for nb in (1, 8, 64):
        _, info = orc.potrf_lo(np.diag(d), lo, nb=nb)
        assert info == 26, (nb, info)


# ------------------------------------------------------ refinement exits
def test_ir_stagnation_exit(orc):
    """tol = 0 cannot be met by an inexact solution, so refinement runs until
    the largest eta fails to halve on two consecutive corrections, then falls
    back to FP64.  The recorded eta history fixes where that must happen
    (catches a stagnation rule that never fires, fires after one slow step,
    or forgets to reset after a good one)."""
    n = 60
    A = synth.haar_spd(n, 1e2, 44)
    xt = synth.normal((n, 2), 45)
    B = A @ xt
    X, st = orc.posv_ir(A, B, lo=1, tol=0.0, max_iter=30)
    h = st["hist"]
    k = st["iters"]
    assert st["fell_back"] and st["info"] == 0
    assert len(h) == k + 1 and 2 <= k < 30
    assert all(e > 0.0 for e in h)
    slow = [i >= 1 and not (h[i] <= 0.5 * h[i - 1]) for i in range(len(h))]
    assert slow[k] and slow[k - 1]
    assert not any(slow[i] and slow[i - 1] for i in range(1, k))
    assert np.all(orc.backward_error(A, X, B) <= 1e-12)


def test_ir_history_and_cap(orc):
    """max_iter caps the corrections: with tol = 0 and max_iter = 1 the loop
    evaluates two residuals and stops at the cap."""
    n = 50
    A = synth.haar_spd(n, 1e4, 46)
    B = A @ synth.normal((n, 1), 47)
    _, st = orc.posv_ir(A, B, lo=1, tol=0.0, max_iter=1)
    assert st["iters"] == 1 and len(st["hist"]) == 2 and st["fell_back"]
    assert st["hist"][1] < st["hist"][0]
