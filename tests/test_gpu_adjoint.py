"""GPU parity of the hand-written adjoint of X = A^{-1} B (mg_posv_backward and
PosvFunction): central finite differences over every symmetric direction at
n = 64, torch.autograd.gradcheck on the lower-parameter form, closed-form
special cases, and the oracle's gradient at n = 8192, nrhs = 64."""
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


def test_central_differences_n64(mg):
    n, nrhs = 64, 3
    A = torch.from_numpy(synth.gram_spd(n, 31)).cuda()
    B = torch.from_numpy(synth.normal((n, nrhs), 32)).cuda()
    W = torch.from_numpy(synth.normal((n, nrhs), 33)).cuda()
    L, info = mg.potrf(A)
    X = mg.potrs(L, B, info)
    gB, gA = mg.posv_backward(L, X, W, mode="sym")
    h = 1e-6
    f = lambda M: float((W * mg.posv(M, B)[0]).sum())
    iu = [(i, j) for i in range(n) for j in range(i + 1)]
    worst = 0.0
    for (i, j) in iu:
        E = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        E[i, j] = 1.0
        E[j, i] = 1.0
        fd = (f(A + h * E) - f(A - h * E)) / (2 * h)
        an = float((gA * E).sum())
        worst = max(worst, abs(fd - an) / max(1e-8, abs(fd)))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-8), (i, j)
    for i in range(n):
        for r in range(nrhs):
            E = torch.zeros((n, nrhs), dtype=torch.float64, device="cuda")
            E[i, r] = 1.0
            fd = (float((W * mg.posv(A, B + h * E)[0]).sum()) - float((W * mg.posv(A, B - h * E)[0]).sum())) / (2 * h)
            assert float(gB[i, r]) == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_gradcheck_lower_mode(mg):
    n, nrhs = 10, 2
    A = torch.from_numpy(synth.gram_spd(n, 41)).cuda().requires_grad_(True)
    B = torch.from_numpy(synth.normal((n, nrhs), 42)).cuda().requires_grad_(True)
    fn = lambda a, b: mg.PosvFunction.apply(a, b, "lower")
    assert torch.autograd.gradcheck(fn, (A, B), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_symmetric_mode_matches_symmetrised_gradcheck(mg):
    n, nrhs = 8, 2
    A0 = torch.from_numpy(synth.gram_spd(n, 43)).cuda()
    B = torch.from_numpy(synth.normal((n, nrhs), 44)).cuda()
    W = torch.from_numpy(synth.normal((n, nrhs), 45)).cuda()
    A = A0.clone().requires_grad_(True)
    X = mg.PosvFunction.apply(A, B, "sym")
    (W * X).sum().backward()
    gsym = A.grad.clone()
    # gradient of f(S) = posv(1/2 (S + S^T)) by autograd through the lower mode
    S = A0.clone().requires_grad_(True)
    Xs = mg.PosvFunction.apply(0.5 * (S + S.T), B, "lower")
    (W * Xs).sum().backward()
    assert torch.allclose(gsym, S.grad, rtol=1e-12, atol=1e-14)
    assert torch.allclose(gsym, gsym.T, rtol=0, atol=0)


def test_special_cases(mg):
    n, nrhs = 50, 3
    B = torch.from_numpy(synth.normal((n, nrhs), 1)).cuda()
    W = torch.from_numpy(synth.normal((n, nrhs), 2)).cuda()
    I = torch.eye(n, dtype=torch.float64, device="cuda")
    L, info = mg.potrf(I)
    X = mg.potrs(L, B, info)
    gB, gA = mg.posv_backward(L, X, W)
    assert torch.equal(gB, W)
    assert torch.allclose(gA, -0.5 * (W @ B.T + B @ W.T), rtol=0, atol=1e-15)
    d = 4.0 ** torch.arange(8, dtype=torch.float64, device="cuda").repeat(7)[:n]
    L, info = mg.potrf(torch.diag(d))
    X = mg.potrs(L, B, info)
    gB, _ = mg.posv_backward(L, X, W)
    assert torch.equal(gB, W / d[:, None])


@pytest.mark.parametrize("n,nrhs", [(300, 5), (8192, 64)])
def test_oracle_gradient(mg, orc, n, nrhs):
    """Configuration: A = G G^T/n + I, B and W ~ N(0,1); loss = sum(W * X)."""
    if n > 1000:
        A = synth.torch_gram_spd(n, 800 + n, 1.0)
        B = synth.torch_normal((n, nrhs), 801 + n)
        W = synth.torch_normal((n, nrhs), 802 + n)
    else:
        A = torch.from_numpy(synth.gram_spd(n, 800 + n)).cuda()
        B = torch.from_numpy(synth.normal((n, nrhs), 801 + n)).cuda()
        W = torch.from_numpy(synth.normal((n, nrhs), 802 + n)).cuda()
    L, info = mg.potrf(A)
    X = mg.potrs(L, B, info)
    gB, gA = mg.posv_backward(L, X, W, mode="sym", info=info)
    torch.cuda.synchronize()
    Ah, Bh, Wh = A.cpu().numpy(), B.cpu().numpy(), W.cpu().numpy()
    Lo, oinfo = orc.potrf(Ah.T)
    assert oinfo == 0
    Xo = orc.potrs(Lo, Bh)
    gBo, gAo = orc.posv_backward(Lo, Xo, Wh, mode=0)
    eB = np.linalg.norm(gB.cpu().numpy() - gBo) / np.linalg.norm(gBo)
    eA = np.linalg.norm(gA.cpu().numpy() - gAo) / np.linalg.norm(gAo)
    assert eB <= 1e-12 and eA <= 1e-12, (eB, eA)
