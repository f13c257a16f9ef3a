"""ctypes view of libmg.so: one Python callable per C entry point, same names.

Argument marshalling only; every step of the computation runs in the HIP
kernels of libmg.so.  Loading fails loudly when the library is missing: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmg.so")

MG_OK = 0
MG_ERR_HIP = 1
MG_ERR_UNSUPPORTED = 2
MG_ERR_INTERNAL = 3
MG_ERR_ABORTED = 4
MG_ERR_SCRATCH_LIMIT = 5
MG_NOALLOC_SCRATCH_BYTES = 32 << 20
MG_INFO_SOLVE_ABORTED = -1
MG_INFO_BAD_PIVOT = -2
MG_F64 = 0
MG_F32 = 1
MG_PREC_F32 = 1
MG_PREC_BF16 = 2
MG_PROF_TRAILING = 0
MG_PROF_DIAG = 1
MG_PROF_TRSM = 2
MG_PROF_SOLVE = 3
MG_PROF_ADJOINT = 4
MG_PROF_BATCHED = 5
MG_PROF_TRAILING_NARROW = 6
MG_PROF_LU_PANEL = 7
MG_PROF_LU_UPDATE = 8
MG_GRAD_SYM = 0
MG_GRAD_LOWER = 1
MG_SOLVE_INVERSE = 0
MG_SOLVE_SUBSTITUTION = 1

i32 = ctypes.c_int32
i64 = ctypes.c_int64
vp = ctypes.c_void_p
sz = ctypes.c_size_t
dbl = ctypes.c_double

# name -> (restype, argtypes); the order follows include/mg.h
SIGNATURES = {
    "mg_version": (i32, []),
    "mg_create": (i32, [ctypes.POINTER(vp), vp]),
    "mg_destroy": (i32, [vp]),
    "mg_set_stream": (i32, [vp, vp]),
    "mg_set_block_size": (i32, [vp, i64]),
    "mg_set_lookahead": (i32, [vp, i32]),
    "mg_set_sweep_spin_limit": (i32, [vp, i64]),
    "mg_set_solve_mode": (i32, [vp, i32]),
    "mg_get_block_size": (i32, [vp, i32, i64, ctypes.POINTER(i64)]),
    "mg_potrf": (i32, [vp, i32, i64, vp, i64, vp]),
    "mg_potrs_buffer_size": (i32, [vp, i32, i64, i64, ctypes.POINTER(sz)]),
    "mg_potrs": (i32, [vp, i32, i64, i64, vp, i64, vp, i64, vp, sz, vp]),
    "mg_posv": (i32, [vp, i32, i64, i64, vp, i64, vp, i64, vp, sz, vp]),
    "mg_posv_noalloc": (i32, [vp, i32, i64, i64, vp, i64, vp, i64, vp]),
    "mg_posv_mixed_buffer_size": (i32, [vp, i32, i64, i64, i32, ctypes.POINTER(sz)]),
    "mg_posv_mixed": (i32, [vp, i32, i64, i64, vp, i64, vp, i64, vp, i64, vp, vp, sz, vp, vp]),
    "mg_posv_backward": (i32, [vp, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64, i32, vp, sz, vp]),
    "mg_potrf_backward_buffer_size": (i32, [vp, i64, ctypes.POINTER(sz)]),
    "mg_potrf_backward": (i32, [vp, i64, vp, i64, vp, i64, vp, i64, i32, vp, sz, vp]),
    "mg_zposv_buffer_size": (i32, [vp, i32, i64, i64, ctypes.POINTER(sz)]),
    "mg_zpotrf": (i32, [vp, i32, i64, vp, i64, vp, sz, vp]),
    "mg_zpotrs": (i32, [vp, i32, i64, i64, vp, i64, vp, i64, vp, sz, vp]),
    "mg_zposv": (i32, [vp, i32, i64, i64, vp, i64, vp, i64, vp, sz, vp]),
    "mg_getrf_buffer_size": (i32, [vp, i64, ctypes.POINTER(sz)]),
    "mg_getrf": (i32, [vp, i64, vp, i64, vp, vp, sz, vp]),
    "mg_getrs_buffer_size": (i32, [vp, i64, i64, ctypes.POINTER(sz)]),
    "mg_getrs": (i32, [vp, i64, i64, vp, i64, vp, vp, i64, vp, sz, vp]),
    "mg_gesv_buffer_size": (i32, [vp, i64, i64, ctypes.POINTER(sz)]),
    "mg_gesv": (i32, [vp, i64, i64, vp, i64, vp, vp, i64, vp, sz, vp]),
    "mg_batch_plan_create": (i32, [vp, i32, i32, vp, i32, vp, ctypes.POINTER(vp)]),
    "mg_batch_plan_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(dbl),
                                 ctypes.POINTER(i32)]),
    "mg_posv_batched": (i32, [vp, vp, vp, vp, vp, vp, vp]),
    "mg_posv_batched_backward": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp]),
    "mg_batch_plan_destroy": (i32, [vp]),
    "mg_logdet": (i32, [vp, i32, i64, vp, i64, vp, vp]),
    "mg_gp_loglik_buffer_size": (i32, [vp, i64, i64, ctypes.POINTER(sz)]),
    "mg_gp_loglik": (i32, [vp, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, vp, sz, vp]),
    "mg_gp_loglik_grad_buffer_size": (i32, [vp, i64, ctypes.POINTER(sz)]),
    "mg_gp_loglik_grad": (i32, [vp, i64, i64, vp, i64, vp, i64, vp, vp, i64, vp, i64, vp, i64, vp, sz, vp]),
    "mg_set_profiling": (i32, [vp, i32]),
    "mg_set_profiling_kinds": (i32, [vp, ctypes.c_uint32]),
    "mg_profile_query": (i32, [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl),
                               ctypes.POINTER(dbl), i32]),
}



class IrOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("fallback", ctypes.c_int32)]


class IrResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("fell_back", ctypes.c_int32), ("lo_info", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("eta", ctypes.c_double)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("grid_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("cache_path", ctypes.c_char_p), ("variant", ctypes.c_int32)]


_lib = None


class MgError(RuntimeError):
    def __init__(self, fn: str, code: int):
        kind = ("invalid argument %d" % -code) if code < 0 else {
            MG_ERR_HIP: "HIP runtime error", MG_ERR_UNSUPPORTED: "unsupported",
            MG_ERR_INTERNAL: "internal error",
            MG_ERR_ABORTED: "a triangular sweep gave up waiting (bounded wait); the result is NaN",
            MG_ERR_SCRATCH_LIMIT: "the solve needs more than the %d-byte no-allocation scratch array"
                                  % MG_NOALLOC_SCRATCH_BYTES}.get(
                code, "error %d" % code)
        super().__init__(f"{fn}: {kind} (status {code})")
        self.code = code


def load():
    """Load libmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2601_14466_amd.build.build() "
                          "(hipcc, gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def call(name: str, *args) -> int:
    """Call an entry point; raise MgError on a non-zero status."""
    rc = getattr(load(), name)(*args)
    if rc != MG_OK:
        raise MgError(name, rc)
    return rc


def raw(name: str, *args) -> int:
    """Call an entry point and return its status unchanged."""
    return getattr(load(), name)(*args)
