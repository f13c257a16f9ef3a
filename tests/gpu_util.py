"""Helpers shared by the GPU tests: column-major device buffers and raw C-ABI calls."""
from __future__ import annotations

import ctypes

import numpy as np


def dev_colmajor(M: np.ndarray, dtype=None, lda: int | None = None, fill=np.nan):
    """Device buffer holding M column-major with leading dimension lda
    (rows n..lda-1 filled with `fill`); returns the flat torch tensor."""
    import torch
    M = np.asarray(M)
    if M.ndim == 1:
        M = M.reshape(-1, 1)
    r, c = M.shape
    lda = lda or max(1, r)
    buf = np.full((max(c, 1), lda), fill, dtype=np.float64)   # row j of buf = column j of M
    buf[:c, :r] = M.T
    t = torch.from_numpy(buf.astype(dtype or np.float64)).cuda()
    return t


def host_colmajor(t, rows: int, cols: int, lda: int | None = None) -> np.ndarray:
    """Read a column-major device buffer back as an (rows, cols) float64 array."""
    lda = lda or max(1, rows)
    a = t.detach().cpu().numpy().astype(np.float64).reshape(-1, lda)
    return a[:cols, :rows].T.copy()


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Raw:
    """Direct C-ABI calls with a private handle on the current stream."""

    def __init__(self):
        import torch
        import paper_2601_14466_amd as mg
        self.mg = mg
        self.lib = mg.load()
        self.h = ctypes.c_void_p()
        assert self.lib.mg_create(ctypes.byref(self.h), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0

    def close(self):
        self.lib.mg_destroy(self.h)

    def potrs_work(self, dt, n, nrhs):
        import torch
        b = ctypes.c_size_t()
        assert self.lib.mg_potrs_buffer_size(self.h, dt, n, nrhs, ctypes.byref(b)) == 0
        return torch.empty(max(1, b.value), dtype=torch.uint8, device="cuda"), b.value
