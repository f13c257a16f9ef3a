"""GPU parity of the complex Hermitian solve (mg_zpotrf / mg_zpotrs /
mg_zposv; the paper's routines take complex64 and complex128) against the
oracle's complex column Cholesky.

Bars: the Gaussian-integer family (every operation exact) gives L and X bit
for bit (X with substitution sweeps); random Hermitian positive-definite A:
complex128 L within 1e-12 relative (Frobenius) of the oracle's and X within a
backward error of 1e-12 (the FP64 bar), complex64 within 2e-5 / 1e-5 (binary32
arithmetic: a small multiple of n u_32 at these orders); info equal to the
oracle's; the strict upper triangle and the diagonal's imaginary part never
read."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_2601_14466_amd as m
    m.load()
    return m


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev(a, dtype=np.complex128):
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).cuda()


def _crand(shape, seed):
    return synth.normal(shape, seed) + 1j * synth.normal(shape, seed + 1)


@pytest.mark.parametrize("n", [1, 2, 33, 64, 65, 300, 700])
def test_gaussian_integer_family_bitwise(mg, orc, substitution, n):
    L0, A = synth.gaussian_integer_hpd(n, 600 + n)
    xt = synth.integer_vector((n, 3), 601 + n) + 1j * synth.integer_vector((n, 3), 602 + n)
    print(f"[z] gaussian-integer n={n}", flush=True)
    L, info = mg.zpotrf(_dev(A))
    assert int(info) == 0
    assert np.array_equal(np.tril(L.cpu().numpy()), L0)
    X = mg.zpotrs(L, _dev(A @ xt), info=info).cpu().numpy()
    assert np.array_equal(X, xt)
    X2, info2 = mg.zposv(_dev(A), _dev(A @ xt))
    assert int(info2) == 0 and np.array_equal(X2.cpu().numpy(), xt)


@pytest.mark.parametrize("n,nrhs", [(1, 1), (65, 2), (300, 16), (1100, 5)])
def test_complex128_matches_oracle(mg, orc, n, nrhs):
    A = synth.hermitian_pd(n, 610 + n)
    B = _crand((n, nrhs), 611 + n)
    print(f"[z] c128 n={n} nrhs={nrhs}", flush=True)
    L, info = mg.zpotrf(_dev(A))
    Lo, info_o = orc.zpotrf(A)
    assert int(info) == info_o == 0
    assert _rel(np.tril(L.cpu().numpy()), np.tril(Lo)) <= 1e-12
    X, info2 = mg.zposv(_dev(A), _dev(B))
    assert int(info2) == 0
    assert np.all(orc.backward_error_z(A, X.cpu().numpy(), B) <= 1e-12)
    assert _rel(X.cpu().numpy(), orc.zpotrs(Lo, B)) <= 1e-10


@pytest.mark.parametrize("n", [65, 700])
def test_complex64_matches_oracle(mg, orc, n):
    A = synth.hermitian_pd(n, 620 + n)
    B = _crand((n, 4), 621 + n)
    L, info = mg.zpotrf(_dev(A, np.complex64))
    Lo, _ = orc.zpotrf(A.astype(np.complex64).astype(np.complex128))
    assert int(info) == 0
    assert _rel(np.tril(L.cpu().numpy().astype(np.complex128)), np.tril(Lo)) <= 2e-5
    X, info2 = mg.zposv(_dev(A, np.complex64), _dev(B, np.complex64))
    assert int(info2) == 0
    assert np.all(orc.backward_error_z(A, X.cpu().numpy().astype(np.complex128), B) <= 1e-5)


def test_info_and_unread_parts(mg, orc):
    n = 150
    A = synth.hermitian_pd(n, 9)
    P = A.copy()
    P[np.triu_indices(n, 1)] = np.nan + 1j * np.nan
    P[np.diag_indices(n)] += 5j
    L, info = mg.zpotrf(_dev(P))
    Lo, _ = orc.zpotrf(A)
    assert int(info) == 0 and _rel(np.tril(L.cpu().numpy()), np.tril(Lo)) <= 1e-12
    assert np.all(np.isnan(np.triu(L.cpu().numpy(), 1)[np.triu_indices(n, 1)]))   # never written
    Bad = A.copy()
    Bad[100, 100] = -3.0
    _, info_o = orc.zpotrf(Bad)
    Bd = _crand((n, 2), 10)
    X, info2 = mg.zposv(_dev(Bad), _dev(Bd))
    assert int(info2) == info_o == 101
    assert np.array_equal(X.cpu().numpy(), Bd)


def test_large_n4096(mg, orc):
    n, nrhs = 4096, 4
    A = synth.hermitian_pd(n, 4096)
    B = _crand((n, nrhs), 4097)
    print(f"[z] n={n}", flush=True)
    X, info = mg.zposv(_dev(A), _dev(B))
    assert int(info) == 0
    assert np.all(orc.backward_error_z(A, X.cpu().numpy(), B) <= 1e-12)
