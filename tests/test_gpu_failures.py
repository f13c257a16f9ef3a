"""Failure reporting through the C ABI: a triangular sweep whose bounded wait
gives up (driven from the host with a spin limit of 0, so every kernel still
exits normally), a mixed-precision breakdown with the FP64 fallback turned
off, and gradients after a failed factorisation.  In every case the failure
must be visible to the caller (info, status, NaN results), never a plausible
number."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import Raw, dev_colmajor, host_colmajor, ptr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_2601_14466_amd as m
    m.load()
    return m


@pytest.fixture
def giveup(mg):
    """Every sweep block that depends on another gives up at once."""
    h = mg.handle()
    h.set_sweep_spin_limit(0)
    try:
        yield h
    finally:
        h.set_sweep_spin_limit(-1)


def test_sweep_giveup_sets_info_and_nan(mg, orc, giveup):
    n = 300
    A = synth.gram_spd(n, 61)
    B = synth.normal((n, 3), 62)
    X, info = mg.posv(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), nb=64)
    torch.cuda.synchronize()
    assert int(info) == mg._lib.MG_INFO_SOLVE_ABORTED
    assert torch.isnan(X).all()


def test_sweep_giveup_potrs_without_info(mg, orc, giveup):
    n = 200
    A = synth.gram_spd(n, 63)
    L, info = mg.potrf(torch.from_numpy(A).cuda(), nb=64)
    Xn = mg.potrs(L, torch.from_numpy(synth.normal((n, 2), 64)).cuda())   # info NULL
    torch.cuda.synchronize()
    assert int(info) == 0 and torch.isnan(Xn).all()


def test_sweep_giveup_mixed_returns_status(mg, giveup):
    n = 200
    A = torch.from_numpy(synth.haar_spd(n, 1e2, 65)).cuda()
    B = torch.from_numpy(synth.normal((n, 2), 66)).cuda()
    with pytest.raises(mg.MgError) as e:
        mg.posv_mixed(A, B, precision="fp32")
    assert e.value.code == mg._lib.MG_ERR_ABORTED


def test_sweep_giveup_backward_nan(mg, giveup):
    n, nrhs = 150, 2
    A = synth.gram_spd(n, 67)
    L, info = mg.potrf(torch.from_numpy(A).cuda())
    X = torch.from_numpy(synth.normal((n, nrhs), 68)).cuda()
    gX = torch.from_numpy(synth.normal((n, nrhs), 69)).cuda()
    gB, gA = mg.posv_backward(L, X, gX, info=info)
    torch.cuda.synchronize()
    assert int(info) == mg._lib.MG_INFO_SOLVE_ABORTED
    assert torch.isnan(gB).all() and torch.isnan(gA).all()


def test_solves_recover_after_giveup(mg, orc):
    """The spin limit is per handle and restorable; the next solve is exact
    again (sweep words are reset by every solve)."""
    n = 300
    A = synth.gram_spd(n, 70)
    xt = synth.normal((n, 2), 71)
    h = mg.handle()
    h.set_sweep_spin_limit(0)
    mg.posv(torch.from_numpy(A).cuda(), torch.from_numpy(A @ xt).cuda(), nb=64)
    h.set_sweep_spin_limit(-1)
    X, info = mg.posv(torch.from_numpy(A).cuda(), torch.from_numpy(A @ xt).cuda(), nb=64)
    torch.cuda.synchronize()
    assert int(info) == 0
    assert np.all(orc.backward_error(A, X.cpu().numpy(), A @ xt) <= 1e-12)
    assert mg.raw("mg_set_sweep_spin_limit", h.h, -2) == -2


def test_mixed_breakdown_without_fallback_is_visible(mg):
    """lo factor breaks down, fallback off: no solution exists, so X is NaN
    and eta is NaN (not 0 with garbage in X)."""
    n = 200
    d = np.ones(n)
    d[120] = -2.0
    A = torch.from_numpy(np.diag(d)).cuda()
    B = torch.ones((n, 2), dtype=torch.float64, device="cuda")
    X, st = mg.posv_mixed(A, B, precision="fp32", fallback=False)
    torch.cuda.synchronize()
    assert st["lo_info"] == 121 and not st["fell_back"] and st["info"] == 0
    assert np.isnan(st["eta"])
    assert torch.isnan(X).all()


def test_posv_function_on_indefinite_is_nan(mg):
    n = 40
    d = np.ones(n)
    d[7] = -1.0
    A = torch.from_numpy(np.diag(d)).cuda().requires_grad_(True)
    B = torch.from_numpy(synth.normal((n, 2), 72)).cuda().requires_grad_(True)
    X = mg.PosvFunction.apply(A, B)
    X.sum().backward()
    torch.cuda.synchronize()
    assert torch.isnan(X).all()
    assert torch.isnan(B.grad).all() and torch.isnan(A.grad).all()


def test_backward_after_failed_factor_is_nan(mg):
    n = 64
    d = np.ones(n)
    d[30] = -1.0
    L, info = mg.potrf(torch.from_numpy(np.diag(d)).cuda())
    X = torch.ones((n, 1), dtype=torch.float64, device="cuda")
    gB, gA = mg.posv_backward(L, X, X, info=info)
    gB2, gA2 = mg.posv_backward(L, X, X, mode="lower", info=info)
    torch.cuda.synchronize()
    assert int(info) == 31
    assert torch.isnan(gB).all() and torch.isnan(gA).all()
    assert torch.isnan(gB2).all()
    assert torch.isnan(torch.tril(gA2)[torch.tril(torch.ones(n, n, dtype=torch.bool, device="cuda"))]).all()
