"""32-bit offsets of the library's kernels at the largest configured order.

The trailing-update kernels address memory through buffer resources with
32-bit byte offsets (a per-lane offset plus a per-step offset, both from a
64-bit base), and the host refuses a launch whose offsets could reach 2^31.
This test evaluates each of those expressions, as the kernels form them, at
their extremes for the mixed-precision configuration's largest order
(n = 65536: the binary32 working copy and the FP64 fallback copy, both with
leading dimension n, block columns of 512 and their rank-128 steps), checks
that every one stays below 2^31 and that the host guard admits these sizes
while refusing the first sizes at which an offset would overflow; the same
for the LDS-staged bfloat16 update.  Kernels that index with 64-bit element
offsets (the bfloat16 panel copy the panel solve writes, the residual, the
sweeps, the lower-triangle copies) are checked for that by reading their source."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_14466_amd", "csrc")
LIM = 2 ** 31


def host_guard_ok(m, kdim, lda, es):
    """The launch guard of the binary32/binary64 and bfloat16 trailing updates."""
    return (m + (kdim + 64) * lda) * es < LIM - 65536 and kdim % 16 == 0


def syrk_offsets(m, kdim, lda, es):
    """Largest values of the 32-bit byte offsets k_syrk_lower forms: the C
    quarter's offsets from its corner (rows and columns clamped to 63), the
    operand lane offsets (row clamped to m - 1, lane group g <= 3), the
    per-step offset (k-step kn < kdim / 4) and their sum at a load."""
    c_off = (63 + 63 * lda) * es
    xo = ((m - 1) + 3 * lda) * es
    soff = (kdim // 4 - 1) * 4 * lda * es
    return dict(c_off=c_off, xo=xo, zo=xo, soff=soff, load=xo + soff + es)


def syrk_bf16_offsets(m, kdim, lda, ldp=512):
    """k_syrk_lower_bf16: C in binary32 as above; the row-major bfloat16
    panel (row stride ldp: the block column's copy is 512 wide) read 16 bytes
    at a time: lane offset ((row) ldp + 8 g) 2 bytes, step offset kn 64
    bytes, kn < kdim / 32."""
    c_off = (63 + 63 * lda) * 4
    xo = ((m - 1) * ldp + 8 * 3) * 2
    soff = (kdim // 32 - 1) * 64
    return dict(c_off=c_off, xo=xo, zo=xo, soff=soff, load=xo + soff + 16)


def bf16_ring_guard_ok(m, ldp=512):
    """The copy's own guard for the register-ring bfloat16 update."""
    return (m + 1) * ldp * 2 < LIM


def test_bf16_ring_guard_is_tight():
    """Where the copy's guard admits the register-ring kernel its last
    operand load stays below 2^31 bytes; one row more and it refuses."""
    ldp = 512
    m = LIM // (2 * ldp) - 2
    assert bf16_ring_guard_ok(m, ldp) and not bf16_ring_guard_ok(m + 1, ldp)
    assert syrk_bf16_offsets(m, 512, 1, ldp)["load"] < LIM
    src = open(os.path.join(CSRC, "potrf.hip")).read()
    assert "(m + 1) * ldp * 2 < ((int64_t)1 << 31)" in src


def bf16l_guard_ok(m, kdim, ldp=512):
    """The launch guard of the LDS-staged bfloat16 update (64-k chunks)."""
    return kdim % 64 == 0 and (m + 128) * ldp * 2 < LIM


def syrk_bf16l_offsets(m, kdim, lda, ldp=512):
    """k_syrk_lower_bf16l: the row-major bfloat16 panel (row stride ldp)
    moved in 64-k chunks of 16-byte pieces (8 per row): lane offset
    ((tid / 8) ldp + 8 (tid % 8)) 2 bytes, tid < 256; per-tile offset
    I 128 ldp 2 bytes, I < ceil(m / 128); per-piece offset
    (32 u ldp + 64 c) 2 bytes, u < 4, c < kdim / 64; C as
    in k_syrk_lower (interior quarters: the same entries, split into a lane
    part (i + 4 g lda) 4 and uniform parts 16 bi 4 and (16 bj + r) lda 4)."""
    pvo = (31 * ldp + 8 * 7) * 2
    xso = (-(-m // 128) - 1) * 128 * ldp * 2
    so = (32 * 3 * ldp + (kdim // 64 - 1) * 64) * 2
    c_lane = (15 + 4 * 3 * lda) * 4
    c_uni = 16 * 3 * 4 + (16 * 3 + 3) * lda * 4
    return dict(pvo=pvo, xso=xso, so=so, load=pvo + xso + so + 16, c_lane=c_lane, c_uni=c_uni,
                c_sum=c_lane + c_uni)


@pytest.mark.parametrize("kdim", [128, 256, 512])
def test_bf16_lds_update_offsets_at_n65536(kdim):
    """At the largest order the bfloat16 mode runs (block columns 256 or 512
    wide, their rank-128 steps; the copy's rows are 512 wide), every offset
    of the LDS-staged update fits and the guard admits the launch."""
    n = 65536
    for m in (n - kdim, n // 2, 129, 1):
        assert bf16l_guard_ok(m, kdim)
        for k, v in syrk_bf16l_offsets(m, kdim, n).items():
            assert 0 <= v < LIM, (kdim, m, k, v)


def test_bf16_lds_guard_is_tight():
    """Wherever the guard admits the launch the last operand load stays
    below 2^31 bytes; just past its edge it refuses."""
    for kdim in (64, 128, 256, 512):
        ldp = 512
        m = LIM // (2 * ldp) - 128 - 1
        assert bf16l_guard_ok(m, kdim, ldp) and syrk_bf16l_offsets(m, kdim, 1, ldp)["load"] < LIM
        assert not bf16l_guard_ok(m + 1, kdim, ldp)
    src = open(os.path.join(CSRC, "potrf.hip")).read()
    assert "kdim % BFL_KC == 0 && (m + 128) * ldp * 2 < ((int64_t)1 << 31)" in src
    assert "constexpr int BFL_KC = 64;" in src
    assert "constexpr int BF_LDP = 512;" in src


@pytest.mark.parametrize("es,label", [(4, "binary32 working copy"), (8, "FP64 fallback copy")])
@pytest.mark.parametrize("kdim", [128, 512])
def test_trailing_update_offsets_at_n65536(es, label, kdim):
    n = 65536
    for m in (n - kdim, n - 128 - kdim, n // 2, 1):          # first and later steps
        off = syrk_offsets(m, kdim, n, es)
        for k, v in off.items():
            assert 0 <= v < LIM, (label, kdim, m, k, v)
        assert host_guard_ok(m, kdim, n, es), (label, kdim, m)
    if es == 4:
        for m in (n - kdim, 1):
            off = syrk_bf16_offsets(m, kdim, n)
            for k, v in off.items():
                assert 0 <= v < LIM, ("bf16", kdim, m, k, v)


@pytest.mark.parametrize("es", [4, 8])
@pytest.mark.parametrize("kdim", [128, 256, 512, 1024])
def test_host_guard_implies_every_offset_fits(es, kdim):
    """Wherever the guard admits a launch (scanning square trailing matrices
    with lda = m up to the guard's edge), every offset fits in 31 bits, the
    bfloat16 panel's included; just past the edge the guard refuses."""
    m = 1
    last_ok = None
    while m < 1 << 22:
        if host_guard_ok(m, kdim, m, es):
            last_ok = m
            for v in syrk_offsets(m, kdim, m, es).values():
                assert v < LIM
            if es == 4 and bf16_ring_guard_ok(m):
                for v in syrk_bf16_offsets(m, kdim, m).values():
                    assert v < LIM
        m = m * 2 if m < 4096 else m + 4096
    assert last_ok is not None and not host_guard_ok(last_ok + 4096, kdim, last_ok + 4096, es)


def _kernel_text(fname, kname):
    src = open(os.path.join(CSRC, fname)).read()
    k = src.find(kname + "(")
    assert k >= 0, kname
    end = src.find("\n}\n", k)
    return src[k:end]


def test_library_guard_matches_the_formula():
    """The launch guard in the source is the formula this test evaluates."""
    src = open(os.path.join(CSRC, "potrf.hip")).read()
    assert "(m + (kdim + 64) * lda) * (int64_t)sizeof(S) >= ((int64_t)1 << 31) - 65536" in src
    assert "(m + (kdim + 64) * lda) * 4 >= ((int64_t)1 << 31) - 65536" in src


@pytest.mark.parametrize("fname,kname,pattern", [
    ("potrf.hip", "k_trsm_panel", r"const int64_t row = R \+ 16 \* h2 \+ i;"),
    ("potrf.hip", "k_trsm_panel", r"\(Pq \+ row \* ldq \+ 16 \* t \+ tcol<S>\(g, 0\)\)"),
    ("mixed.hip", "k_sym_rowprod", r"\(size_t\)blockIdx\.y \* n \+ gi"),
    ("mixed.hip", "k_sym_finish", r"\(\(size_t\)sp \* n \+ gi\)"),
    ("potrs.hip", "k_sweep", r"L\[idx\(rwc, c0 \+ c, lda\)\]"),
    ("mixed.hip", "k_copy_lower", r"W\[idx\(i, b, ldw\)\] = \(D\)A\[idx\(i, b, lda\)\]"),
    ("mixed.hip", "k_copy_lower", r"W\[idx\(i, j2, ldw\)\] = \(D\)A\[idx\(i, j2, lda\)\]"),
])
def test_other_kernels_use_64_bit_offsets(fname, kname, pattern):
    assert re.search(pattern, _kernel_text(fname, kname)), (fname, kname)


def test_idx_is_64_bit():
    src = open(os.path.join(CSRC, "tile16.h")).read()
    assert "return (size_t)i + (size_t)j * (size_t)ld;" in src


def test_lower_triangle_kernels_grid_capped():
    """The cast and copy kernel of the mixed path strides pairs of columns
    over a one-dimensional grid capped at 65535 workgroups (one workgroup per
    column would sit on the grid-y limit at n = 65536)."""
    src = open(os.path.join(CSRC, "mixed.hip")).read()
    assert "for (int64_t b = blockIdx.x; b < (n + 1) / 2; b += gridDim.x)" in src
    assert "dim3((unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + 1) / 2), 65535))" in src
