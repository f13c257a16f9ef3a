"""mg_posv_noalloc (scratch in the library's per-GPU device array) against
mg_posv (caller workspace) through the C ABI: the two run the same kernels
on the same inputs, so X, L and info must agree bitwise, on two calls in a
row (the second smaller, so stale scratch from the first is present), in
FP64 and FP32, with a ragged order; the scratch limit is refused before
anything is enqueued."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import Raw, dev_colmajor, host_colmajor, ptr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def raw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a ROCm GPU")
    r = Raw()
    yield r
    r.close()


def _bits_equal(a, b):
    """Bitwise equality of two device buffers (guard rows hold NaN, which
    compares unequal to itself as a value)."""
    import torch
    it = torch.int64 if a.element_size() == 8 else torch.int32
    return torch.equal(a.view(it), b.view(it))


def _both(raw, dt, A, B):
    import torch
    from paper_2601_14466_amd import _lib
    n, nrhs = B.shape
    npdt = np.float64 if dt == _lib.MG_F64 else np.float32
    lda, ldb = n + 3, n + 1          # padded leading dimensions (guard rows)
    A1, B1 = dev_colmajor(A, npdt, lda), dev_colmajor(B, npdt, ldb)
    A2, B2 = A1.clone(), B1.clone()
    i1 = torch.zeros((), dtype=torch.int32, device="cuda")
    i2 = torch.full((), 7, dtype=torch.int32, device="cuda")
    work, wb = raw.potrs_work(dt, n, nrhs)
    assert raw.lib.mg_posv(raw.h, dt, n, nrhs, ptr(A1), lda, ptr(B1), ldb, ptr(work), wb, ptr(i1)) == 0
    assert raw.lib.mg_posv_noalloc(raw.h, dt, n, nrhs, ptr(A2), lda, ptr(B2), ldb, ptr(i2)) == 0
    torch.cuda.synchronize()
    return (A1, B1, i1), (A2, B2, i2), lda, ldb


@pytest.mark.parametrize("dt_name", ["f64", "f32"])
def test_noalloc_matches_posv_twice(raw, orc, dt_name):
    import torch
    from paper_2601_14466_amd import _lib
    dt = _lib.MG_F64 if dt_name == "f64" else _lib.MG_F32
    for call_no, (n, nrhs, seed) in enumerate([(1100, 37, 4100), (300, 5, 4200)]):
        print(f"[noalloc] {dt_name} call {call_no}: n={n} nrhs={nrhs} seed={seed}", flush=True)
        A = synth.gram_spd(n, seed)
        B = A @ synth.normal((n, nrhs), seed + 1)
        if dt == _lib.MG_F32:
            A = A.astype(np.float32).astype(np.float64)
            B = B.astype(np.float32).astype(np.float64)
        (A1, B1, i1), (A2, B2, i2), lda, ldb = _both(raw, dt, A, B)
        assert int(i1) == 0 and int(i2) == 0
        assert _bits_equal(B1, B2), "X differs from mg_posv"
        assert _bits_equal(A1, A2), "L differs from mg_posv"
        X = host_colmajor(B2, n, nrhs, ldb)
        eta = orc.backward_error(A, X, B)
        bound = 1e-12 if dt == _lib.MG_F64 else n * 2.0 ** -24
        assert np.all(eta <= bound), eta.max()


def test_noalloc_failure_and_limit(raw):
    import torch
    from paper_2601_14466_amd import _lib
    n, nrhs = 200, 3
    A = synth.gram_spd(n, 4300)
    A[150, 150] = -1.0                       # leading minor of order 151 not positive definite
    B = synth.normal((n, nrhs), 4301)
    (A1, B1, i1), (A2, B2, i2), _, ldb = _both(raw, _lib.MG_F64, A, B)
    assert int(i1) == 151 and int(i2) == 151
    assert _bits_equal(B1, B2)
    assert np.array_equal(host_colmajor(B2, n, nrhs, ldb), B)      # B untouched on failure
    # more than MG_NOALLOC_SCRATCH_BYTES of Y: refused on the host, nothing enqueued
    big_n, big_r = 65536, 65
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    info = torch.zeros((), dtype=torch.int32, device="cuda")
    rc = raw.lib.mg_posv_noalloc(raw.h, _lib.MG_F64, big_n, big_r, ptr(d), big_n, ptr(d), big_n, ptr(info))
    assert rc == _lib.MG_ERR_SCRATCH_LIMIT
    assert raw.lib.mg_posv_noalloc(raw.h, _lib.MG_F64, 0, 0, None, 1, None, 1, ptr(info)) == 0
    assert raw.lib.mg_posv_noalloc(raw.h, _lib.MG_F64, n, nrhs, ptr(d), n, ptr(d), n, None) == -9
