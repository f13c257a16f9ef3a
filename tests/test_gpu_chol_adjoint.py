"""GPU parity of the Cholesky adjoint (mg_potrf_backward): the gradient with
respect to A of f(L), L = chol(A), given gL = df/dL.

Bars: against the oracle's or_potrf_backward (pinned by central differences
and closed forms) on the same L and gL, relative Frobenius error <= 1e-11 in
both modes and both solve modes; exact symmetry in the symmetric mode; the
diagonal closed form; torch.autograd.gradcheck through CholeskyFunction;
NaN after a failed factorisation."""
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


@pytest.mark.parametrize("n", [1, 2, 17, 64, 65, 128, 200, 512, 513, 1024])
def test_matches_oracle(mg, orc, n):
    """Orders that are multiples of 64 take the blocked right solves, the
    others the sweeps."""
    A = synth.gram_spd(n, 300 + n)
    W = synth.normal((n, n), 301 + n)
    L, info = mg.potrf(torch.from_numpy(A).cuda())
    Lt = torch.tril(L)
    gL = torch.from_numpy(W).cuda()
    for mode, om in (("sym", 0), ("lower", 1)):
        g = mg.potrf_backward(Lt, gL, info=info, mode=mode).cpu().numpy()
        want = orc.potrf_backward(Lt.cpu().numpy(), W, mode=om)
        if mode == "lower":
            g = np.tril(g)
        assert _rel(g, want) <= 1e-11, (mode, _rel(g, want))
        if mode == "sym":
            assert np.array_equal(g, g.T)


@pytest.mark.parametrize("n", [150, 256])
def test_substitution_mode_and_strict_upper_never_read(mg, orc, substitution, n):
    """Substitution sweeps (n = 150) or the blocked right solves (n = 256);
    NaN poison in the strict upper triangles of L and gL changes nothing."""
    A = synth.gram_spd(n, 17)
    W = synth.normal((n, n), 18)
    L, info = mg.potrf(torch.from_numpy(A).cuda())
    Ln = torch.tril(L) + torch.triu(torch.full_like(L, float("nan")), 1)
    Wn = torch.from_numpy(np.tril(W) + np.triu(np.full((n, n), np.nan), 1)).cuda()
    g = mg.potrf_backward(Ln, Wn, info=info).cpu().numpy()
    want = orc.potrf_backward(np.tril(L.cpu().numpy()), W)
    assert np.all(np.isfinite(g))
    assert _rel(g, want) <= 1e-11


def test_diagonal_closed_form(mg):
    n = 40
    d = 4.0 ** (np.arange(n) % 9 - 4)
    W = np.tril(synth.normal((n, n), 5))
    L, info = mg.potrf(torch.from_numpy(np.diag(d)).cuda())
    g = mg.potrf_backward(torch.tril(L), torch.from_numpy(W).cuda(), info=info).cpu().numpy()
    sq = np.sqrt(d)
    want = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            want[i, j] = want[j, i] = W[i, j] / (2 * sq[j])
    assert np.allclose(g, want, rtol=1e-14, atol=0)


def test_gradcheck(mg):
    n = 8
    A0 = synth.gram_spd(n, 3)
    A = torch.from_numpy(A0).cuda().requires_grad_(True)
    f = lambda M: mg.CholeskyFunction.apply(0.5 * (M + M.T))
    assert torch.autograd.gradcheck(f, (A,), eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("n", [70, 128])
def test_failed_factor_gives_nan(mg, n):
    A = synth.gram_spd(n, 9)
    A[30, 30] = -5.0
    L, info = mg.potrf(torch.from_numpy(A).cuda())
    assert int(info) == 31
    g = mg.potrf_backward(torch.tril(L), torch.ones((n, n), dtype=torch.float64, device="cuda"), info=info)
    assert torch.isnan(g).all()


def test_full_size_n2048(mg, orc):
    n = 2048
    A = synth.gram_spd(n, 2048)
    W = synth.normal((n, n), 2049)
    L, info = mg.potrf(torch.from_numpy(A).cuda())
    Lt = torch.tril(L)
    g = mg.potrf_backward(Lt, torch.from_numpy(W).cuda(), info=info).cpu().numpy()
    want = orc.potrf_backward(Lt.cpu().numpy(), W)
    assert _rel(g, want) <= 1e-11, _rel(g, want)
