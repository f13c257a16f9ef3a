"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/mg.h declares, the binding's table matches the header,
and argument validation answers before anything touches a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mg.h")
PKG = os.path.join(ROOT, "paper_2601_14466_amd")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_2601_14466_amd as mg
    return mg.load()


def test_header_declares_core_entry_points():
    fns = header_functions()
    for name in ("mg_create", "mg_destroy", "mg_potrf", "mg_potrs", "mg_posv", "mg_logdet"):
        assert name in fns


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), f"libmg.so does not export {name}"
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(PKG, "libmg.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mg_[a-z0-9_]+)$", out, flags=re.M))
    assert set(header_functions()) <= exported


def test_binding_table_matches_header():
    from paper_2601_14466_amd import _lib
    assert sorted(_lib.SIGNATURES) == header_functions()


def test_version(lib):
    assert lib.mg_version() == 10000


def test_null_handle_is_argument_one(lib):
    from paper_2601_14466_amd import _lib as L
    vp = ctypes.c_void_p
    n = 4
    assert L.raw("mg_create", None, None) == -1
    assert L.raw("mg_destroy", None) == 0
    assert L.raw("mg_set_stream", None, None) == -1
    assert L.raw("mg_set_block_size", None, 64) == -1
    assert L.raw("mg_get_block_size", None, 0, n, None) == -1
    assert L.raw("mg_potrf", None, 0, n, vp(8), n, vp(8)) == -1
    sz = ctypes.c_size_t()
    assert L.raw("mg_potrs_buffer_size", None, 0, n, 1, ctypes.byref(sz)) == -1
    assert L.raw("mg_potrs", None, 0, n, 1, vp(8), n, vp(8), n, vp(8), 64, None) == -1
    assert L.raw("mg_posv", None, 0, n, 1, vp(8), n, vp(8), n, vp(8), 64, vp(8)) == -1
    assert L.raw("mg_logdet", None, 0, n, vp(8), n, vp(8), None) == -1
    assert L.raw("mg_set_profiling", None, 1) == -1
    assert L.raw("mg_set_profiling_kinds", None, 1) == -1
    assert L.raw("mg_gp_loglik_buffer_size", None, n, 1, ctypes.byref(sz)) == -1
    assert L.raw("mg_gp_loglik", None, n, 1, vp(8), n, vp(8), n, None, n, vp(8), n, vp(8), vp(8), 64,
                 vp(8)) == -1
    assert L.raw("mg_zposv_buffer_size", None, 0, n, 1, ctypes.byref(sz)) == -1
    assert L.raw("mg_zpotrf", None, 0, n, vp(8), n, vp(8), 64, vp(8)) == -1
    assert L.raw("mg_zpotrs", None, 0, n, 1, vp(8), n, vp(8), n, vp(8), 64, None) == -1
    assert L.raw("mg_zposv", None, 0, n, 1, vp(8), n, vp(8), n, vp(8), 64, vp(8)) == -1
    assert L.raw("mg_getrf_buffer_size", None, n, ctypes.byref(sz)) == -1
    assert L.raw("mg_getrf", None, n, vp(8), n, vp(8), vp(8), 64, vp(8)) == -1
    assert L.raw("mg_getrs_buffer_size", None, n, 1, ctypes.byref(sz)) == -1
    assert L.raw("mg_getrs", None, n, 1, vp(8), n, vp(8), vp(8), n, vp(8), 64, None) == -1
    assert L.raw("mg_gesv_buffer_size", None, n, 1, ctypes.byref(sz)) == -1
    assert L.raw("mg_gesv", None, n, 1, vp(8), n, vp(8), vp(8), n, vp(8), 64, vp(8)) == -1
    d, i = ctypes.c_double(), ctypes.c_int64()
    assert L.raw("mg_profile_query", None, 0, ctypes.byref(d), ctypes.byref(i), ctypes.byref(d),
                 ctypes.byref(d), 0) == -1


def test_product_never_imports_the_oracle():
    """The product path must not route through the CPU oracle."""
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, flags=re.M), f
                assert "liboracle" not in txt, f
                assert "or_potrf" not in txt, f


def test_cpu_tensors_are_rejected():
    import torch
    import paper_2601_14466_amd as mg
    with pytest.raises(ValueError):
        mg.potrf(torch.eye(4, dtype=torch.float64))
