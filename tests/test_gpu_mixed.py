"""GPU parity of the mixed-precision solve with FP64 iterative refinement
(binary32 factor, or bfloat16 trailing-update operands), through the C ABI.

Bar: every returned column has normwise backward error eta <= 1e-12, computed
by the CPU oracle in extended precision on the original FP64 A and B; the
iteration count, the fallback flag and the device-side eta are reported and
checked for consistency.  The paper is silent on precision; the scheme is
Langou et al. (SC'06) for SPD systems.
"""
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


def _solve(mg, A, B, **kw):
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    A0, B0 = Ad.clone(), Bd.clone()
    X, st = mg.posv_mixed(Ad, Bd, **kw)
    torch.cuda.synchronize()
    assert torch.equal(Ad, A0) and torch.equal(Bd, B0), "inputs must not be modified"
    return X.cpu().numpy(), st


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [65, 300, 700])
def test_integer_family_needs_no_refinement(mg, orc, substitution, n, prec):
    """The low-precision factor and solve (by substitution) are exact on the
    integer family (all values below 2^24, power-of-two pivots, entries
    representable in bfloat16), so x0 = x_true and no correction is taken."""
    L0, A = synth.integer_exact(n, 500 + n)
    xt = synth.integer_vector((n, 2), n)
    X, st = _solve(mg, A, A @ xt, precision=prec)
    assert st["iters"] == 0 and not st["fell_back"] and st["lo_info"] == 0
    assert np.array_equal(X, xt)


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
@pytest.mark.parametrize("n", [300, 1500])
def test_fp32_refinement_converges(mg, orc, n, cond):
    A = synth.haar_spd(n, cond, 7 + n)
    xt = synth.normal((n, 8), 8 + n)
    B = A @ xt
    X, st = _solve(mg, A, B, precision="fp32")
    assert not st["fell_back"], st
    assert 1 <= st["iters"] <= 8, st
    eta = orc.backward_error(A, X, B)
    assert np.all(eta <= 1e-12), eta.max()
    assert st["eta"] == pytest.approx(eta.max(), rel=0.5, abs=1e-15)


@pytest.mark.parametrize("cond", [1e2, 1e6])
def test_bf16_converges_or_falls_back(mg, orc, cond):
    n = 700
    A = synth.haar_spd(n, cond, 3)
    xt = synth.normal((n, 4), 4)
    B = A @ xt
    X, st = _solve(mg, A, B, precision="bf16")
    eta = orc.backward_error(A, X, B)
    assert np.all(eta <= 1e-12), (st, eta.max())
    if cond >= 1e6:
        assert st["fell_back"], st   # bfloat16 updates cannot resolve cond 1e6


def test_forced_fallback_and_no_fallback(mg, orc):
    n = 500
    A = synth.haar_spd(n, 1e3, 11)
    xt = synth.normal((n, 3), 12)
    B = A @ xt
    X, st = _solve(mg, A, B, precision="fp32", max_iter=0)
    assert st["fell_back"] and st["iters"] == 0
    assert np.all(orc.backward_error(A, X, B) <= 1e-12)
    X, st = _solve(mg, A, B, precision="fp32", max_iter=0, fallback=False)
    assert not st["fell_back"] and st["eta"] > 1e-12
    eta = orc.backward_error(A, X, B)
    assert eta.max() == pytest.approx(st["eta"], rel=0.5)


def test_not_spd_reports_info(mg, orc):
    n = 200
    d = np.ones(n)
    d[120] = -2.0
    X, st = _solve(mg, np.diag(d), np.ones((n, 2)), precision="fp32")
    assert st["lo_info"] == 121 and st["fell_back"] and st["info"] == 121


def test_rhs_one_and_many(mg, orc):
    n = 400
    A = synth.haar_spd(n, 1e4, 21)
    for nrhs in (1, 3, 40):
        xt = synth.normal((n, nrhs), nrhs)
        B = A @ xt
        X, st = _solve(mg, A, B, precision="fp32")
        assert np.all(orc.backward_error(A, X, B) <= 1e-12), (nrhs, st)


# ------------------------------------------ large-rank variants at small n
@pytest.fixture
def block_size(mg):
    h = mg.handle()

    def set_nb(nb):
        h.set_block_size(nb)
    yield set_nb
    h.set_block_size(0)
    assert mg.raw("mg_set_lookahead", h.h, 1) == 0


@pytest.mark.parametrize("nb", [256, 512])
@pytest.mark.parametrize("n", [1100, 2600, 4100])
def test_large_rank_integer_family_bitwise(mg, orc, block_size, substitution, n, nb):
    """Block columns of 256 / 512 drive the rank-256/512 binary32 update (the
    8-deep operand ring at 512), and in bfloat16 mode the packed row-major
    panel copies (three buffers rotating over the look-ahead streams) and the
    16x16x32 bfloat16 matrix instruction.  On the integer family every one of
    them is exact, so the factor is L0 and x0 = x_true with no correction,
    in every look-ahead mode."""
    block_size(nb)
    L0, A = synth.integer_exact(n, 1300 + n)
    xt = synth.integer_vector((n, 2), 1301 + n)
    h = mg.handle()
    for la in (0, 1, 2):
        assert mg.raw("mg_set_lookahead", h.h, la) == 0
        for prec in ("fp32", "bf16"):
            X, st = _solve(mg, A, A @ xt, precision=prec)
            assert st["iters"] == 0 and not st["fell_back"] and st["lo_info"] == 0, (la, prec, st)
            assert np.array_equal(X, xt), (la, prec)
        L, info = mg.potrf(torch.from_numpy(A).to("cuda", torch.float32))
        Xf, info2 = mg.posv(torch.from_numpy(A).to("cuda", torch.float32),
                            torch.from_numpy(A @ xt).to("cuda", torch.float32))
        torch.cuda.synchronize()
        assert int(info) == 0 and int(info2) == 0
        assert np.array_equal(np.tril(L.double().cpu().numpy()), L0), la
        assert np.array_equal(Xf.double().cpu().numpy(), xt), la


@pytest.mark.parametrize("nb", [256, 512])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_large_rank_random_same_in_every_lookahead_mode(mg, orc, block_size, prec, nb):
    """Haar input, cond 1e2, n = 2600 with a ragged last block: the refined
    solution meets eta <= 1e-12, and the three schedules give bitwise the
    same X and iteration count (a race in the panel-copy rotation would not)."""
    block_size(nb)
    n = 2600
    A = synth.haar_spd(n, 1e2, 1400 + nb)
    xt = synth.normal((n, 4), 1401)
    B = A @ xt
    h = mg.handle()
    outs = []
    for la in (1, 0, 2):
        assert mg.raw("mg_set_lookahead", h.h, la) == 0
        X, st = _solve(mg, A, B, precision=prec)
        assert not st["fell_back"], st
        outs.append((X, st["iters"]))
    assert np.all(orc.backward_error(A, outs[0][0], B) <= 1e-12)
    for X, it in outs[1:]:
        assert it == outs[0][1] and np.array_equal(X, outs[0][0])


# ------------------------------------- refinement decisions vs the oracle
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
@pytest.mark.parametrize("n", [300, 700])
def test_refinement_decisions_match_oracle(mg, orc, n, cond, prec):
    """Same input, same block size (64 at these orders; the oracle's blocked
    reading with the same diagonal-block width): the GPU and the oracle agree
    on whether the low-precision factor breaks down and whether refinement
    falls back, and converged iteration counts differ by at most one (the
    two sum in different orders, so their factors differ in the last bits)."""
    nb = mg.handle().block_size(n, mg._lib.MG_F32)
    assert nb == 64
    A = synth.haar_spd(n, cond, 1500 + n)
    xt = synth.normal((n, 3), 1501 + n)
    B = A @ xt
    X, st = _solve(mg, A, B, precision=prec)
    lo = 1 if prec == "fp32" else 2
    Xo, so = orc.posv_ir(A, B, lo=lo, nb=nb)
    o_broke = so["fell_back"] and len(so["hist"]) == 0
    assert (st["lo_info"] > 0) == o_broke, (st, so)
    assert st["fell_back"] == so["fell_back"], (st, so)
    if not st["fell_back"]:
        assert abs(st["iters"] - so["iters"]) <= 1, (st, so)
    assert np.all(orc.backward_error(A, X, B) <= 1e-12)


def test_stagnation_exit_matches_oracle(mg, orc):
    """tol = 0: both leave through the stagnation rule and fall back."""
    n = 300
    A = synth.haar_spd(n, 1e2, 1600)
    B = A @ synth.normal((n, 2), 1601)
    X, st = _solve(mg, A, B, precision="fp32", tol=0.0)
    _, so = orc.posv_ir(A, B, lo=1, tol=0.0, nb=64)
    assert st["fell_back"] and so["fell_back"]
    assert st["lo_info"] == 0 and st["iters"] < 30 and so["iters"] < 30
    assert abs(st["iters"] - so["iters"]) <= 1, (st, so)
    assert np.all(orc.backward_error(A, X, B) <= 1e-12)


@pytest.mark.parametrize("n,precision,cond", [
    (16384, "fp32", 1e2), (16384, "fp32", 1e4), (16384, "fp32", 1e6),
    (16384, "bf16", 1e2), (16384, "bf16", 1e4), (16384, "bf16", 1e6),
    (32768, "fp32", 1e4), (32768, "bf16", 1e2),
])
def test_full_size_config2(mg, orc, n, precision, cond):
    """A = Q diag(lambda) Q^T with Haar Q, nrhs = 8 (the mixed configuration;
    n = 32768 is the size the benchmark times), with the library's default
    block size, checked by the oracle's extended-precision residual on every
    column.  Binary32 converges at every conditioning; bfloat16 updates
    cannot resolve cond >= 1e4 (kappa u_bf16 >> 1), so those cases must fall
    back to FP64 and say so."""
    A = synth.torch_haar_spd(n, cond, 700 + n)
    Xt = synth.torch_normal((n, 8), 701 + n)
    B = A @ Xt
    X, st = mg.posv_mixed(A, B, precision=precision)
    torch.cuda.synchronize()
    assert st["info"] == 0, st
    if precision == "fp32":
        assert not st["fell_back"] and st["lo_info"] == 0 and st["iters"] <= 3, st
    else:
        assert st["fell_back"] == (cond >= 1e4), st
        if cond < 1e4:
            assert st["iters"] <= 8, st
    Ah = A.cpu().numpy()
    eta = orc.backward_error(Ah.T, X.cpu().numpy(), B.cpu().numpy())
    assert np.all(eta <= 1e-12), eta.max()


@pytest.mark.timeout(900)
def test_full_size_config2_n65536(mg, orc):
    """The mixed configuration's largest order, n = 65536 (A is 34 GB in
    FP64), binary32 factor, cond 1e4, nrhs = 8.  The input is built so that
    no library call sees 2^31 or more elements; the generation, the solve and
    the check are logged separately."""
    n, cond = 65536, 1e4
    print(f"[n65536] generating Haar input n={n} cond={cond:g}", flush=True)
    A = synth.torch_haar_spd(n, cond, 700 + n, log=lambda m: print(f"[n65536] {m}", flush=True))
    Xt = synth.torch_normal((n, 8), 701 + n)
    B = synth.torch_matmul_rows(A, Xt)
    del Xt
    torch.cuda.synchronize()
    print("[n65536] input ready; solving (fp32 factor + FP64 refinement)", flush=True)
    X, st = mg.posv_mixed(A, B, precision="fp32")
    torch.cuda.synchronize()
    print(f"[n65536] solved: {st}", flush=True)
    assert not st["fell_back"] and st["info"] == 0 and st["lo_info"] == 0 and st["iters"] <= 3, st
    Ah = A.cpu().numpy()
    del A
    torch.cuda.empty_cache()
    print("[n65536] A copied to the host; oracle residual", flush=True)
    eta = orc.backward_error(Ah.T, X.cpu().numpy(), B.cpu().numpy())
    print(f"[n65536] oracle eta max {eta.max():.3e}", flush=True)
    assert np.all(eta <= 1e-12), eta.max()
