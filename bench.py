#!/usr/bin/env python3
"""Benchmark: potrf+potrs TFLOP/s on one MI355X.

Headline workload (FP64): A = G G^T / n + delta I with cond(A) ~ 1e4,
n = 32768, nrhs = 16, B = A X_true; one step = mg_posv (blocked Cholesky with
look-ahead, then the two triangular sweeps) on an input that is already
resident in HBM.  Each timed step factors its own pre-staged copy of A, so no
restore copy runs inside the timed region.  TFLOP/s uses the nominal LAWN-41
count n^3/3 + n^2/2 + n/6 + 2 n^2 nrhs.

The JSON line also carries
  roofline     : the trailing-update kernel (dominant), algorithmic flops per
                 launch over its average launch duration from HIP events on
                 the streams it runs on, against the FP64 matrix peak;
  cpu_baseline : the CPU oracle on a bounded sample of the same workload
                 (n = 8192, nrhs = 16), timed on this host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--nrhs R]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "potrf+potrs TFLOP/s: FP64 vs mixed-precision+IR at 1e-12 backward error, 1 GPU"
FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 matrix peak (public specification)
FP32_PEAK_TFLOPS = 157.3     # dense FP32 matrix peak
BF16_PEAK_TFLOPS = 2500.0    # dense bfloat16 matrix peak
HBM_PEAK_GBS = 8000.0

# HBM traffic of the rank-512 trailing-update kernel, k_syrk_lower<double, true, 4, false>,
# from two rocprofv3 --pmc runs of this benchmark (profiles/k_syrk_lower_n32768_hbm_traffic.md):
# average FETCH_SIZE and WRITE_SIZE per dispatch in KiB, each scaled by what the
# same counter reads for an 8 GiB device-to-device copy (FETCH_SIZE reads half
# the bytes moved, WRITE_SIZE all of them).  Valid only for the kernel source
# it was measured on: reported as null once that source changes.
SYRK_TRAFFIC = dict(fetch_kib=650335.8, write_kib=469937.5, fetch_scale=2.0, write_scale=1.0,
                    kernel_sha1="58b5967db306b75585bd919d2d57994bd68a0289")


def syrk_traffic_bytes():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2601_14466_amd", "csrc", "potrf.hip")).read()
    # the kernel's text with the tile-order and buffer helpers above it:
    # from the tile size through the kernel's closing brace
    a = src.find("constexpr int SY_BM")
    k = src.find("template <typename S, bool FOLD", a) if a >= 0 else -1
    b = src.find("\n}\n", k) + 3 if k >= 0 else -1
    if a < 0 or b < 3 or hashlib.sha1(src[a:b].encode()).hexdigest() != SYRK_TRAFFIC["kernel_sha1"]:
        return None
    t = SYRK_TRAFFIC
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def roofline_obj(kernel: str, flops: float, nbytes: float, ms: float, launches: int, peak_tflops: float,
                 traffic=None) -> dict:
    """Roofline entry for one kernel: algorithmic flops and bytes per launch
    over the average launch time; the bound is whichever of the matrix peak
    and HBM bandwidth needs more time for that work."""
    t = ms / launches / 1e3
    f, b = flops / launches, nbytes / launches
    hbm = b / (HBM_PEAK_GBS * 1e9) > f / (peak_tflops * 1e12)
    if hbm:
        ach, peak, unit = b / t / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        ach, peak, unit = f / t / 1e12, peak_tflops, "TFLOP/s"
    return dict(bound="hbm" if hbm else "mfma", achieved=round(ach, 3), peak=peak, unit=unit,
                frac=round(ach / peak, 4), traffic=traffic, kernel=kernel, launches=launches,
                flops_per_launch=f, algorithmic_bytes_per_launch=b, avg_launch_ms=ms / launches)


def nominal_flops(n: int, nrhs: int) -> float:
    return n ** 3 / 3 + n ** 2 / 2 + n / 6 + 2.0 * n * n * nrhs


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def bench_fp64(torch, mg, synth, n: int, nrhs: int, steps: int, warmup: int, nb: int = 0, seed: int = 9000):
    from paper_2601_14466_amd import _lib
    dev = torch.device("cuda", 0)
    log(f"[bench] generating n={n} nrhs={nrhs} (cond 1e4)")
    A0 = synth.torch_gram_spd_cond(n, seed + n, 1e4)
    Xt = synth.torch_normal((n, nrhs), seed + 100 + n)
    B0 = A0 @ Xt
    B0c = B0.T.contiguous()                    # column-major B
    free, _ = torch.cuda.mem_get_info()
    per_copy = A0.numel() * 8 + B0c.numel() * 8
    ncopy = max(1, min(steps, int(0.8 * free // per_copy)))
    restore_in_timed = ncopy < steps
    As = [A0.clone() for _ in range(ncopy)]    # symmetric: row-major bytes == column-major
    Bs = [B0c.clone() for _ in range(ncopy)]
    infos = torch.zeros(ncopy, dtype=torch.int32, device=dev)
    h = mg.handle()
    h.set_block_size(nb)
    wbytes = ctypes.c_size_t()
    _lib.call("mg_potrs_buffer_size", h.h, _lib.MG_F64, n, nrhs, ctypes.byref(wbytes))
    work = torch.empty(max(1, wbytes.value), dtype=torch.uint8, device=dev)
    nb = h.block_size(n)

    def step(i):
        j = i % ncopy
        if restore_in_timed and i >= ncopy:
            As[j].copy_(A0)
            Bs[j].copy_(B0c)
        _lib.call("mg_posv", h.sync_stream(), _lib.MG_F64, n, nrhs, ctypes.c_void_p(As[j].data_ptr()), n,
                  ctypes.c_void_p(Bs[j].data_ptr()), n, ctypes.c_void_p(work.data_ptr()), wbytes.value,
                  ctypes.c_void_p(infos[j:j + 1].data_ptr()))

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    for j in range(ncopy):                     # fresh inputs for the timed steps
        As[j].copy_(A0)
        Bs[j].copy_(B0c)
    torch.cuda.synchronize()
    # only the dominant kernel is bracketed by events inside the timed region
    # (events on the look-ahead chain would lengthen its critical path)
    h.set_profiling(True, kinds=[_lib.MG_PROF_TRAILING])
    for kind in range(_lib.MG_PROF_TRAILING_NARROW + 1):
        h.profile(kind, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        step(i)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    tr = h.profile(_lib.MG_PROF_TRAILING, reset=True)
    h.set_profiling(False)
    info_max = int(infos.max())
    # sanity residual of the last step's solution, FP64 on the device (harness, not the method)
    X = Bs[(steps - 1) % ncopy].T
    R = B0 - A0 @ X
    anorm = float(A0.abs().sum(1).max())
    eta = (R.abs().amax(0) / (anorm * X.abs().amax(0) + B0.abs().amax(0))).max().item()
    # per-kind breakdown from one more step, untimed, with every kind bracketed
    As[0].copy_(A0)
    Bs[0].copy_(B0c)
    torch.cuda.synchronize()
    h.set_profiling(True)
    for kind in range(_lib.MG_PROF_TRAILING_NARROW + 1):
        h.profile(kind, reset=True)
    step(0)
    torch.cuda.synchronize()
    prof = {k: h.profile(v, reset=True) for k, v in
            (("trailing", _lib.MG_PROF_TRAILING), ("trailing_narrow", _lib.MG_PROF_TRAILING_NARROW),
             ("diag", _lib.MG_PROF_DIAG), ("trsm", _lib.MG_PROF_TRSM), ("solve", _lib.MG_PROF_SOLVE))}
    h.set_profiling(False)
    info_max = max(info_max, int(infos.max()))
    # potrs alone on the factor that step left in As[0] (both sweeps, median of 5)
    Bw = B0c.clone()
    st_ms = []
    for r in range(6):
        Bw.copy_(B0c)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.call("mg_potrs", h.sync_stream(), _lib.MG_F64, n, nrhs, ctypes.c_void_p(As[0].data_ptr()), n,
                  ctypes.c_void_p(Bw.data_ptr()), n, ctypes.c_void_p(work.data_ptr()), wbytes.value,
                  ctypes.c_void_p(infos[0:1].data_ptr()))
        e1.record()
        torch.cuda.synchronize()
        if r:
            st_ms.append(e0.elapsed_time(e1))
    solve_ms = _median(st_ms)
    # both sweeps read the lower triangle of L once; B, Y and X move 4 n nrhs elements
    solve_bytes = (n * (n + 1) + 4.0 * n * nrhs) * 8
    solve = dict(n=n, nrhs=nrhs, ms=round(solve_ms, 4),
                 roofline=roofline_obj("k_sweep<double, 1, fwd/bwd, inverse> (two launches)",
                                       2.0 * n * n * nrhs, solve_bytes, solve_ms, 1, FP64_PEAK_TFLOPS))
    del Bw
    ms_step = ms / steps
    tflops = nominal_flops(n, nrhs) / (ms_step / 1e3) / 1e12
    achieved = (tr["flops"] / tr["launches"]) / (tr["ms"] / tr["launches"] / 1e3) / 1e12 if tr["launches"] else None
    out = dict(ms_step=ms_step, tflops=tflops, wall_s=wall, info=info_max, eta_fp64_device=eta, nb=nb,
               restore_in_timed=restore_in_timed, copies=ncopy, prof=prof, trailing=tr, trailing_tflops=achieved,
               solve=solve)
    del As, Bs, A0, B0, B0c, Xt, R
    torch.cuda.empty_cache()
    return out


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def bench_mixed(torch, mg, synth, n: int, nrhs: int, cond: float, precision: str, reps: int, seed: int = 9500,
                gram: bool = False):
    """Mixed precision + FP64 refinement to eta <= 1e-12 on A = Q diag(lambda) Q^T
    (Haar Q, log-spaced spectrum with exact cond).  Time covers the cast, the
    low-precision factor, every refinement step and any fallback; TFLOP/s uses
    the same nominal FP64 count as the FP64 path.  gram: A = G G^T/n + delta I
    with the same cond instead (no QR in the generator; for counter runs,
    whose profiler does not survive the vendor QR)."""
    from paper_2601_14466_amd import _lib
    log(f"[bench] mixed {precision}: generating n={n} nrhs={nrhs} cond={cond:g} ({'Gram' if gram else 'Haar'})")
    if gram:
        A = synth.torch_gram_spd_cond(n, seed + n, cond)
    else:
        A = synth.torch_haar_spd(n, cond, seed + n, log=lambda m: log(f"[bench] mixed {precision}: {m}"))
    Xt = synth.torch_normal((n, nrhs), seed + 1 + n)   # A symmetric: row-major bytes == column-major
    Bc = synth.torch_matmul_rows(A, Xt).T.contiguous()
    Xc = torch.empty_like(Bc)
    h = mg.handle()
    h.set_block_size(0)
    lo = {"fp32": _lib.MG_PREC_F32, "bf16": _lib.MG_PREC_BF16}[precision]
    nbytes = ctypes.c_size_t()
    _lib.call("mg_posv_mixed_buffer_size", h.h, lo, n, nrhs, 1, ctypes.byref(nbytes))
    work = torch.empty(nbytes.value, dtype=torch.uint8, device=A.device)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    opts = _lib.IrOpts(1e-12, 30, 1)
    res = _lib.IrResult()

    def run():
        _lib.call("mg_posv_mixed", h.sync_stream(), lo, n, nrhs, _p(A), n, _p(Bc), n, _p(Xc), n, ctypes.byref(opts),
                  _p(work), nbytes.value, ctypes.byref(res), _p(info))

    run()
    torch.cuda.synchronize()
    # the rank-512 trailing update (binary32 or bfloat16 kernel) is bracketed
    # by events inside the timed region, as on the FP64 leg
    h.set_profiling(True, kinds=[_lib.MG_PROF_TRAILING])
    h.profile(_lib.MG_PROF_TRAILING, reset=True)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    tr = h.profile(_lib.MG_PROF_TRAILING, reset=True)
    h.set_profiling(False)
    ms = _median(times)
    roof = None
    if tr["launches"]:
        if precision == "fp32":
            roof = roofline_obj("k_syrk_lower<float, true, 8, false>", tr["flops"], tr["bytes"], tr["ms"],
                                tr["launches"], FP32_PEAK_TFLOPS)
        else:
            # binary32 C read and written once, the packed bfloat16 panel read once
            roof = roofline_obj("k_syrk_lower_bf16l", tr["flops"], tr["bytes"], tr["ms"], tr["launches"],
                                BF16_PEAK_TFLOPS)
    X = Xc.T
    B = Bc.T
    R = B - synth.torch_matmul_rows(A, X)
    anorm = float(A.abs().sum(1).max())
    eta = (R.abs().amax(0) / (anorm * X.abs().amax(0) + B.abs().amax(0))).max().item()
    out = dict(precision=precision, n=n, nrhs=nrhs, cond=cond, ms=round(ms, 3),
               tflops=round(nominal_flops(n, nrhs) / (ms / 1e3) / 1e12, 3), iters=res.iters,
               fell_back=bool(res.fell_back), lo_info=res.lo_info, eta_reported=res.eta, eta_fp64_device=eta,
               info=int(info), reps=reps, roofline=roof)
    del A, Xt, Bc, Xc, work, R, X, B
    torch.cuda.empty_cache()
    return out


def bench_small(torch, mg, synth, n: int = 1024, reps: int = 20, seed: int = 1024):
    """FP64 posv latency at n = 1024, nrhs = 1 (A = G G^T/n + I)."""
    from paper_2601_14466_amd import _lib
    A0 = synth.torch_gram_spd(n, seed)
    xt = synth.torch_normal((n, 1), seed + 1)
    B0 = (A0 @ xt).T.contiguous()
    A, B = A0.clone(), B0.clone()
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    h = mg.handle()
    h.set_block_size(0)
    wb = ctypes.c_size_t()
    _lib.call("mg_potrs_buffer_size", h.h, _lib.MG_F64, n, 1, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=A.device)
    times = []
    for r in range(reps + 3):
        A.copy_(A0)
        B.copy_(B0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.call("mg_posv", h.sync_stream(), _lib.MG_F64, n, 1, _p(A), n, _p(B), n, _p(work), wb.value, _p(info))
        e1.record()
        torch.cuda.synchronize()
        if r >= 3:
            times.append(e0.elapsed_time(e1))
    ms = _median(times)
    return dict(n=n, nrhs=1, us=round(ms * 1e3, 1), tflops=round(nominal_flops(n, 1) / (ms / 1e3) / 1e12, 3),
                info=int(info))


def bench_batched(torch, mg, synth, dtype, reps: int = 10, seed: int = 2026):
    """4096 SPD systems, n_i uniform on [16, 512], nrhs = 1, A_i = G_i G_i^T/n_i + I,
    solved by one graph-replayed persistent launch; A_i restored outside the
    timed region before every replay."""
    import numpy as np
    sizes = [int(v) for v in synth.batch_sizes(4096, seed)]
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed + 1)
    offs = np.concatenate([[0], np.cumsum([k * k for k in sizes])])
    boffs = np.concatenate([[0], np.cumsum(sizes)])
    A0 = torch.empty(int(offs[-1]), dtype=torch.float64, device=dev)
    B0 = torch.empty(int(boffs[-1]), dtype=torch.float64, device=dev)
    for k, nk in enumerate(sizes):
        G = torch.randn((nk, nk), generator=gen, device=dev, dtype=torch.float64)
        Ak = G @ G.T / nk + torch.eye(nk, device=dev, dtype=torch.float64)
        Ak = torch.tril(Ak) + torch.tril(Ak, -1).T
        xk = torch.randn((nk,), generator=gen, device=dev, dtype=torch.float64)
        A0[int(offs[k]):int(offs[k + 1])] = Ak.reshape(-1)
        B0[int(boffs[k]):int(boffs[k + 1])] = Ak @ xk
    A0 = A0.to(dtype)
    B0 = B0.to(dtype)
    A, B = A0.clone(), B0.clone()
    es = A.element_size()
    ap = torch.tensor([A.data_ptr() + int(o) * es for o in offs[:-1]], dtype=torch.int64, device=dev)
    bp = torch.tensor([B.data_ptr() + int(o) * es for o in boffs[:-1]], dtype=torch.int64, device=dev)
    ld = torch.tensor(sizes, dtype=torch.int64, device=dev)
    info = torch.zeros(len(sizes), dtype=torch.int32, device=dev)
    plan = mg.BatchPlan(sizes, nrhs=1, dtype=dtype, autotune=True)
    times = []
    for r in range(reps + 2):
        A.copy_(A0)
        B.copy_(B0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.solve_raw(ap, ld, bp, ld, info)
        e1.record()
        torch.cuda.synchronize()
        if r >= 2:
            times.append(e0.elapsed_time(e1))
    ms = _median(times)
    # adjoint of the same solve (mg_posv_batched_backward) from its factors
    # and solutions, upstream gradient ~ N(0,1): one launch
    G = torch.randn(int(boffs[-1]), generator=gen, device=dev, dtype=torch.float64).to(dtype)
    GB = torch.empty_like(G)
    GA = torch.empty(int(offs[-1]), dtype=dtype, device=dev)
    gp = torch.tensor([G.data_ptr() + int(o) * es for o in boffs[:-1]], dtype=torch.int64, device=dev)
    gbp = torch.tensor([GB.data_ptr() + int(o) * es for o in boffs[:-1]], dtype=torch.int64, device=dev)
    gap = torch.tensor([GA.data_ptr() + int(o) * es for o in offs[:-1]], dtype=torch.int64, device=dev)
    from paper_2601_14466_amd import _lib
    btimes = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.call("mg_posv_batched_backward", mg.handle().sync_stream(), plan.p, _p(ap), _p(ld), _p(bp), _p(ld),
                  _p(gp), _p(ld), _p(gbp), _p(ld), _p(gap), _p(ld), _lib.MG_GRAD_SYM, _p(info))
        e1.record()
        torch.cuda.synchronize()
        if r >= 1:
            btimes.append(e0.elapsed_time(e1))
    bms = _median(btimes)
    bbytes = sum(k * (k + 1) // 2 + k * k + 3 * k for k in sizes) * es   # read L, write gA, vectors
    backward = dict(ms=round(bms, 4), bad=int((~torch.isfinite(GA)).sum()),
                    roofline=roofline_obj("k_batched_backward (one launch)",
                                          sum(6.0 * k * k for k in sizes), bbytes, bms, 1,
                                          FP64_PEAK_TFLOPS if dtype == torch.float64 else FP32_PEAK_TFLOPS))
    flops = sum(nominal_flops(k, 1) for k in sizes)
    # each system's lower triangle read and L written over it, b read and x written
    nbytes = sum(k * (k + 1) + 2 * k for k in sizes) * es
    peak = FP64_PEAK_TFLOPS if dtype == torch.float64 else FP32_PEAK_TFLOPS
    out = dict(dtype="f64" if dtype == torch.float64 else "f32", batch=len(sizes), ms=round(ms, 4),
               systems_per_s=round(len(sizes) / (ms / 1e3), 1), tflops=round(flops / (ms / 1e3) / 1e12, 3),
               info_nonzero=int((info != 0).sum()), plan=plan.info(),
               roofline=roofline_obj("k_batched_posv (one replay)", flops, nbytes, ms, 1, peak),
               backward=backward)
    del plan, A, B, A0, B0, G, GB, GA
    torch.cuda.empty_cache()
    return out


def bench_adjoint(torch, mg, synth, n: int = 8192, nrhs: int = 64, reps: int = 5, seed: int = 8192):
    """Forward posv and hand-written backward (gB = A^{-1} gX, symmetric gA)
    at n = 8192, nrhs = 64, A = G G^T/n + I."""
    from paper_2601_14466_amd import _lib
    A0 = synth.torch_gram_spd(n, seed)
    Bc0 = synth.torch_normal((nrhs, n), seed + 1)      # column-major n x nrhs
    W = synth.torch_normal((nrhs, n), seed + 2)
    A, Bc = A0.clone(), Bc0.clone()
    gB = torch.empty_like(Bc)
    gA = torch.empty_like(A0)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    h = mg.handle()
    h.set_block_size(0)
    wb = ctypes.c_size_t()
    _lib.call("mg_potrs_buffer_size", h.h, _lib.MG_F64, n, nrhs, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=A.device)
    fw, bw = [], []
    h.set_profiling(True, kinds=[_lib.MG_PROF_ADJOINT])
    h.profile(_lib.MG_PROF_ADJOINT, reset=True)
    for r in range(reps + 1):
        A.copy_(A0)
        Bc.copy_(Bc0)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        _lib.call("mg_posv", h.sync_stream(), _lib.MG_F64, n, nrhs, _p(A), n, _p(Bc), n, _p(work), wb.value, _p(info))
        ev[1].record()
        _lib.call("mg_posv_backward", h.sync_stream(), n, nrhs, _p(A), n, _p(Bc), n, _p(W), n, _p(gB), n, _p(gA), n,
                  _lib.MG_GRAD_SYM, _p(work), wb.value, _p(info))
        ev[2].record()
        torch.cuda.synchronize()
        if r >= 1:
            fw.append(ev[0].elapsed_time(ev[1]))
            bw.append(ev[1].elapsed_time(ev[2]))
    ad = h.profile(_lib.MG_PROF_ADJOINT, reset=True)
    h.set_profiling(False)
    f, b = _median(fw), _median(bw)
    bflops = 2.0 * n * n * nrhs + 4.0 * n * n * nrhs
    roof = (roofline_obj("k_syr2k_grad", ad["flops"], ad["bytes"], ad["ms"], ad["launches"], FP64_PEAK_TFLOPS)
            if ad["launches"] else None)
    return dict(n=n, nrhs=nrhs, forward_ms=round(f, 3), backward_ms=round(b, 3),
                forward_tflops=round(nominal_flops(n, nrhs) / (f / 1e3) / 1e12, 3),
                backward_tflops=round(bflops / (b / 1e3) / 1e12, 3), info=int(info), roofline=roof)


def bench_potrf_backward(torch, mg, synth, n: int = 8192, reps: int = 3, seed: int = 8300):
    """Adjoint of the factorisation itself (mg_potrf_backward) at n = 8192:
    P = Phi(L^T gL), two backward sweeps with n right-hand sides, the
    symmetrisation.  TF/s counts n^3/3 + 2 n^3."""
    from paper_2601_14466_amd import _lib
    A = synth.torch_gram_spd(n, seed)
    L, info = mg.potrf(A)
    Lc = L.T.contiguous() if not L.T.is_contiguous() else L.T
    Gc = synth.torch_normal((n, n), seed + 1)        # only its lower triangle is read
    gA = torch.empty((n, n), dtype=torch.float64, device=A.device)
    h = mg.handle()
    wb = ctypes.c_size_t()
    _lib.call("mg_potrf_backward_buffer_size", h.h, n, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=A.device)
    ts = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.call("mg_potrf_backward", h.sync_stream(), n, _p(Lc), n, _p(Gc), n, _p(gA), n, _lib.MG_GRAD_SYM,
                  _p(work), wb.value, _p(info))
        e1.record()
        torch.cuda.synchronize()
        if r >= 1:
            ts.append(e0.elapsed_time(e1))
    t = _median(ts)
    fl = n ** 3 / 3 + 2.0 * n ** 3
    out = dict(n=n, ms=round(t, 3), tflops=round(fl / (t / 1e3) / 1e12, 3), info=int(info))
    del A, L, Lc, Gc, gA, work
    torch.cuda.empty_cache()
    return out


def bench_gp(torch, mg, synth, n: int = 16384, nrhs: int = 1, reps: int = 3, seed: int = 7700):
    """Gaussian-process marginal log likelihood (factor, solve, log det and
    the per-column combination) at n = 16384 for one observation vector,
    A = G G^T/n + delta I (cond 1e4), nonzero mean.  TFLOP/s uses the posv
    nominal flops."""
    from paper_2601_14466_amd import _lib
    A0 = synth.torch_gram_spd_cond(n, seed, 1e4)
    Yc = synth.torch_normal((nrhs, n), seed + 1)         # column-major n x nrhs
    Mc = synth.torch_normal((nrhs, n), seed + 2)
    A = A0.clone()
    Al = torch.empty_like(Yc)
    ll = torch.empty(nrhs, dtype=torch.float64, device=A.device)
    info = torch.zeros((), dtype=torch.int32, device=A.device)
    h = mg.handle()
    h.set_block_size(0)
    wb = ctypes.c_size_t()
    _lib.call("mg_gp_loglik_buffer_size", h.h, n, nrhs, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=A.device)
    ts = []
    for r in range(reps + 1):
        A.copy_(A0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.call("mg_gp_loglik", h.sync_stream(), n, nrhs, _p(A), n, _p(Yc), n, _p(Mc), n, _p(Al), n, _p(ll),
                  _p(work), wb.value, _p(info))
        e1.record()
        torch.cuda.synchronize()
        if r >= 1:
            ts.append(e0.elapsed_time(e1))
    t = _median(ts)
    return dict(n=n, nrhs=nrhs, ms=round(t, 3), tflops=round(nominal_flops(n, nrhs) / (t / 1e3) / 1e12, 3),
                loglik=float(ll[0]), info=int(info))


def bench_gp_grad(torch, mg, synth, n: int = 4096, nrhs: int = 1, reps: int = 3, seed: int = 7800):
    """Gradient of the GP log likelihood from a stored factor (A^{-1} by the
    two sweeps with n right-hand sides, then the symmetric combination) at
    n = 4096.  TFLOP/s counts the 2 n^3 flops of the two triangular solves
    against n right-hand sides."""
    from paper_2601_14466_amd import _lib
    A = synth.torch_gram_spd(n, seed)
    Y = synth.torch_normal((n, nrhs), seed + 1)
    ll, alpha, L, info = mg.gp_loglik(A, Y)
    Lc = L.T.contiguous()
    Ac = alpha.T.contiguous()
    g = torch.ones(nrhs, dtype=torch.float64, device=A.device)
    gA = torch.empty((n, n), dtype=torch.float64, device=A.device)
    gY = torch.empty((nrhs, n), dtype=torch.float64, device=A.device)
    h = mg.handle()
    wb = ctypes.c_size_t()
    _lib.call("mg_gp_loglik_grad_buffer_size", h.h, n, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=A.device)
    ts = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _lib.call("mg_gp_loglik_grad", h.sync_stream(), n, nrhs, _p(Lc), n, _p(Ac), n, _p(g), _p(gA), n, _p(gY), n,
                  None, n, _p(work), wb.value, _p(info))
        e1.record()
        torch.cuda.synchronize()
        if r >= 1:
            ts.append(e0.elapsed_time(e1))
    t = _median(ts)
    return dict(n=n, nrhs=nrhs, ms=round(t, 3), tflops=round(2.0 * n ** 3 / (t / 1e3) / 1e12, 3), info=int(info))


def cpu_baseline(torch, synth, n: int = 6144, nrhs: int = 16, reps: int = 3, seed: int = 4242):
    """The CPU oracle (plain C, FP64, OpenMP) on a bounded sample of the
    headline recipe: median of `reps` posv runs at order n."""
    import oracle  # CPU oracle: baseline leg only
    A = synth.torch_gram_spd_cond(n, seed, 1e4)
    Xt = synth.torch_normal((n, nrhs), seed + 1)
    B = (A @ Xt).cpu().numpy()
    Ah = A.cpu().numpy()
    del A, Xt
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        X, info = oracle.posv(Ah, B)
        ts.append(time.perf_counter() - t0)
    dt = _median(ts)
    return dict(value=nominal_flops(n, nrhs) / dt / 1e12, unit="TFLOP/s", cores=oracle.num_threads(),
                kind="oracle", sample=f"oracle posv (plain C FP64) on the same recipe at n={n}, nrhs={nrhs}, "
                                      f"median of {reps}: {dt:.2f} s", seconds=dt, runs_s=[round(t, 3) for t in ts],
                info=int(info))


def cpu_library_context(torch, synth, n: int = 8192, nrhs: int = 16, reps: int = 3, seed: int = 4243):
    """Context line, not a target: LAPACK dpotrf + dpotrs from the host's
    scipy (OpenBLAS) on the same recipe, median of `reps`."""
    import numpy as np
    try:
        from scipy.linalg import lapack
    except ImportError:
        return None
    A = synth.torch_gram_spd_cond(n, seed, 1e4)
    Xt = synth.torch_normal((n, nrhs), seed + 1)
    B = np.asfortranarray((A @ Xt).cpu().numpy())
    Ah = np.asfortranarray(A.cpu().numpy())
    del A, Xt
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((d.get("num_threads") or 0) for d in threadpool_info()) or None
    except Exception:
        pass
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        c, inf1 = lapack.dpotrf(Ah, lower=1, clean=0, overwrite_a=0)
        x, inf2 = lapack.dpotrs(c, B, lower=1)
        ts.append(time.perf_counter() - t0)
    dt = _median(ts)
    return dict(value=nominal_flops(n, nrhs) / dt / 1e12, unit="TFLOP/s", threads=threads,
                kind="scipy-openblas dpotrf+dpotrs", sample=f"n={n}, nrhs={nrhs}, median of {reps}: {dt:.3f} s",
                info=int(inf1) or int(inf2))


def lu_flops(n: int, nrhs: int) -> float:
    """Nominal flops of getrf (LAWN 41: 2n^3/3 - n^2/2 + 5n/6) plus getrs (2 n^2 nrhs)."""
    return 2.0 * n ** 3 / 3 - n ** 2 / 2 + 5.0 * n / 6 + 2.0 * n * n * nrhs


def bench_lu(torch, mg, synth, n: int, nrhs: int = 16, reps: int = 3, seed: int = 7100):
    """The general solve (mg_gesv: pivoted LU + the two sweeps), FP64, on a
    Gaussian A (entries N(0,1)) and B = A X_true; each rep factors its own
    pre-staged copy.  Only the trailing-update kind is bracketed by events in
    the timed reps; the per-kind breakdown comes from one extra rep."""
    from paper_2601_14466_amd import _lib
    dev = torch.device("cuda", 0)
    log(f"[bench] lu: generating n={n} nrhs={nrhs}")
    A0 = synth.torch_normal((n, n), seed + n)
    Xt = synth.torch_normal((n, nrhs), seed + 1 + n)
    B0 = A0 @ Xt
    A0c = A0.T.contiguous()                    # column-major A
    B0c = B0.T.contiguous()
    h = mg.handle()
    wb = ctypes.c_size_t()
    _lib.call("mg_gesv_buffer_size", h.h, n, nrhs, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=dev)
    free, _ = torch.cuda.mem_get_info()
    ncopy = max(1, min(reps + 1, int(0.7 * free // (A0c.numel() * 8 + B0c.numel() * 8))))
    As = [A0c.clone() for _ in range(ncopy)]
    Bs = [B0c.clone() for _ in range(ncopy)]
    ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
    infos = torch.zeros(ncopy, dtype=torch.int32, device=dev)

    def run(j):
        _lib.call("mg_gesv", h.sync_stream(), n, nrhs, ctypes.c_void_p(As[j].data_ptr()), n,
                  ctypes.c_void_p(ipiv.data_ptr()), ctypes.c_void_p(Bs[j].data_ptr()), n,
                  ctypes.c_void_p(work.data_ptr()), wb.value, ctypes.c_void_p(infos[j:j + 1].data_ptr()))

    def restage():
        for j in range(ncopy):
            As[j].copy_(A0c)
            Bs[j].copy_(B0c)
        torch.cuda.synchronize()

    run(0)                                     # warm-up
    restage()
    h.set_profiling(True, kinds=[_lib.MG_PROF_LU_UPDATE])
    h.profile(_lib.MG_PROF_LU_UPDATE, reset=True)
    ts = []
    for i in range(reps):
        j = i % ncopy
        if i >= ncopy:
            As[j].copy_(A0c)
            Bs[j].copy_(B0c)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run(j)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    up = h.profile(_lib.MG_PROF_LU_UPDATE, reset=True)
    info = int(infos.max())
    X = Bs[(reps - 1) % ncopy].T
    R = B0 - A0 @ X
    anorm = float(A0.abs().sum(1).max())
    eta = (R.abs().amax(0) / (anorm * X.abs().amax(0) + B0.abs().amax(0))).max().item()
    # per-kind breakdown, one more rep with the panel and solve kinds bracketed too
    restage()
    kinds = [_lib.MG_PROF_LU_PANEL, _lib.MG_PROF_LU_UPDATE, _lib.MG_PROF_SOLVE]
    h.set_profiling(True, kinds=kinds)
    for k in kinds:
        h.profile(k, reset=True)
    run(0)
    torch.cuda.synchronize()
    kms = {name: round(h.profile(k, reset=True)["ms"], 3) for name, k in zip(("panel", "update", "solve"), kinds)}
    h.set_profiling(False)
    ms = _median(ts)
    del As, Bs
    return dict(n=n, nrhs=nrhs, ms=round(ms, 3), runs_ms=[round(t, 3) for t in ts],
                tflops=round(lu_flops(n, nrhs) / (ms / 1e3) / 1e12, 3), eta_fp64_device=eta, info=info,
                kernel_ms=kms,
                roofline=(roofline_obj("k_gemm_sub<true> (LU trailing update, rank 256/512)", up["flops"], up["bytes"],
                                       up["ms"], up["launches"], FP64_PEAK_TFLOPS) if up["launches"] else None))


def bench_zposv(torch, mg, synth, n: int = 16384, nrhs: int = 16, reps: int = 3, seed: int = 7700):
    """Complex128 Hermitian posv (mg_zposv) on A = G G^H / n + delta I (G
    complex Gaussian, cond ~ 1e4 as the real recipe) and B = A X_true, each
    rep on a pre-staged copy.  TFLOP/s counts the real flops of complex
    arithmetic, 4 (n^3/3 + 2 n^2 nrhs); the path itself runs the real
    factorisation of the 2n x 2n blocked form (twice that count)."""
    from paper_2601_14466_amd import _lib
    dev = torch.device("cuda", 0)
    log(f"[bench] zposv: generating n={n} nrhs={nrhs}")
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed + n)
    G = torch.complex(torch.randn((n, n), generator=gen, device=dev, dtype=torch.float64),
                      torch.randn((n, n), generator=gen, device=dev, dtype=torch.float64)) / (2.0 ** 0.5)
    A0 = torch.matmul(G, G.conj().T.contiguous()) / n
    del G
    v = torch.complex(torch.randn((n, 1), generator=gen, device=dev, dtype=torch.float64),
                      torch.zeros((n, 1), device=dev, dtype=torch.float64))
    for _ in range(50):                       # power iteration for lambda_max
        v = A0 @ v
        v = v / torch.linalg.vector_norm(v)
    lam = float((v.conj().T @ (A0 @ v)).real)
    A0.diagonal().add_(synth.cond_shift(lam, 1e4))
    Xt = torch.complex(torch.randn((n, nrhs), generator=gen, device=dev, dtype=torch.float64),
                       torch.randn((n, nrhs), generator=gen, device=dev, dtype=torch.float64))
    B0 = A0 @ Xt
    A0c, B0c = A0.T.contiguous(), B0.T.contiguous()   # column-major
    h = mg.handle()
    wb = ctypes.c_size_t()
    _lib.call("mg_zposv_buffer_size", h.h, _lib.MG_F64, n, nrhs, ctypes.byref(wb))
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=dev)
    info = torch.zeros((), dtype=torch.int32, device=dev)
    A, B = A0c.clone(), B0c.clone()

    def run():
        _lib.call("mg_zposv", h.sync_stream(), _lib.MG_F64, n, nrhs, ctypes.c_void_p(A.data_ptr()), n,
                  ctypes.c_void_p(B.data_ptr()), n, ctypes.c_void_p(work.data_ptr()), wb.value,
                  ctypes.c_void_p(info.data_ptr()))

    ts = []
    for r in range(reps + 1):
        A.copy_(A0c)
        B.copy_(B0c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            ts.append(e0.elapsed_time(e1))
    X = B.T
    R = B0 - A0 @ X
    anorm = float(A0.abs().sum(1).max())
    eta = (R.abs().amax(0) / (anorm * X.abs().amax(0) + B0.abs().amax(0))).max().item()
    ms = _median(ts)
    cflops = 4.0 * (n ** 3 / 3 + 2.0 * n * n * nrhs)
    return dict(n=n, nrhs=nrhs, dtype="complex128", ms=round(ms, 3), runs_ms=[round(t, 3) for t in ts],
                tflops=round(cflops / (ms / 1e3) / 1e12, 3),
                real_path_tflops=round(nominal_flops(2 * n, nrhs) / (ms / 1e3) / 1e12, 3),
                eta_fp64_device=eta, info=int(info))


LEGS = ("mixed_fp32", "mixed_bf16", "mixed_fp32_n65536", "small_n1024", "batched_f64", "batched_f32", "adjoint_n8192",
        "potrf_backward_n8192",
        "fp64_n8192", "fp64_n16384", "gp_loglik_n16384", "gp_loglik_grad_n4096", "lu_n8192", "lu_n32768",
        "zposv_n16384")


def run_extra(key, torch, mg, synth, args):
    if key == "mixed_fp32":
        return bench_mixed(torch, mg, synth, args.n, 8, 1e4, "fp32", 3, gram=args.mixed_input == "gram")
    if key == "mixed_bf16":
        return bench_mixed(torch, mg, synth, args.n, 8, 1e2, "bf16", 3, gram=args.mixed_input == "gram")
    if key == "mixed_fp32_n65536":
        return bench_mixed(torch, mg, synth, 65536, 8, 1e4, "fp32", 1)
    if key == "small_n1024":
        return bench_small(torch, mg, synth)
    if key == "batched_f64":
        return bench_batched(torch, mg, synth, torch.float64)
    if key == "batched_f32":
        return bench_batched(torch, mg, synth, torch.float32)
    if key == "adjoint_n8192":
        return bench_adjoint(torch, mg, synth)
    if key == "potrf_backward_n8192":
        return bench_potrf_backward(torch, mg, synth)
    if key in ("fp64_n8192", "fp64_n16384"):
        n = int(key.split("_n")[1])
        r = bench_fp64(torch, mg, synth, n, 16, 5, 2)
        tr = r["trailing"]
        return dict(n=n, nrhs=16, ms=round(r["ms_step"], 3), tflops=round(r["tflops"], 3), nb=r["nb"],
                    eta_fp64_device=r["eta_fp64_device"], info=r["info"], solve=r["solve"],
                    kernel_ms={k: round(v["ms"], 3) for k, v in r["prof"].items()},
                    roofline=(roofline_obj("k_syrk_lower<double, true, 4, false>", tr["flops"], tr["bytes"],
                                           tr["ms"], tr["launches"], FP64_PEAK_TFLOPS) if tr["launches"] else None))
    if key == "gp_loglik_n16384":
        return bench_gp(torch, mg, synth)
    if key == "gp_loglik_grad_n4096":
        return bench_gp_grad(torch, mg, synth)
    if key in ("lu_n8192", "lu_n32768"):
        return bench_lu(torch, mg, synth, int(key.split("_n")[1]))
    if key == "zposv_n16384":
        return bench_zposv(torch, mg, synth)
    raise ValueError(key)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--nb", type=int, default=0, help="potrf block size (0: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision, batched, adjoint and n=1024 measurements")
    ap.add_argument("--mixed-input", choices=("haar", "gram"), default="haar",
                    help="input of the n = 32768 mixed legs (gram: no QR in the generator, for counter runs)")
    ap.add_argument("--only", choices=LEGS, default=None,
                    help="run one extra measurement alone (no headline leg, no CPU baseline), e.g. for profiling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "a multi-GPU layout is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2601_14466_amd as mg
    import synth
    if not torch.cuda.is_available():
        print("bench.py: no ROCm device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    mg.load()
    if args.only:
        out = run_extra(args.only, torch, mg, synth, args)
        log(f"[bench] {args.only}: {out}")
        print(json.dumps({"extra": args.only, **out}), flush=True)
        return

    r = bench_fp64(torch, mg, synth, args.n, args.nrhs, args.steps, args.warmup, args.nb)
    log(f"[bench] fp64 n={args.n}: {r['ms_step']:.2f} ms/step, {r['tflops']:.2f} TFLOP/s, eta {r['eta_fp64_device']:.2e}")
    extras = None
    if not args.no_extras:
        extras = {}
        for key in LEGS:
            extras[key] = run_extra(key, torch, mg, synth, args)
            log(f"[bench] {key}: {extras[key]}")
    cpu = cpu_lib = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(torch, synth)
        log(f"[bench] cpu baseline: {cpu['value'] * 1e3:.2f} GFLOP/s on {cpu['cores']} threads")
        cpu_lib = cpu_library_context(torch, synth)
        log(f"[bench] cpu library context: {cpu_lib}")
    tr = r["trailing"]
    roof = None
    if r["trailing_tflops"] is not None:
        traffic = syrk_traffic_bytes() if (args.n == 32768 and r["nb"] == 512) else None
        roof = dict(bound="mfma", achieved=round(r["trailing_tflops"], 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(r["trailing_tflops"] / FP64_PEAK_TFLOPS, 4), traffic=traffic,
                    kernel="k_syrk_lower<double, true, 4, false>", launches=tr["launches"],
                    flops_per_launch=tr["flops"] / tr["launches"],
                    algorithmic_bytes_per_launch=tr["bytes"] / tr["launches"],
                    avg_launch_ms=tr["ms"] / tr["launches"])
    line = {
        "metric": METRIC,
        "value": round(r["tflops"], 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 posv (potrf+potrs), n={args.n}, nrhs={args.nrhs}, "
                               "A = G G^T/n + delta I with cond(A) ~ 1e4, B = A X_true",
                   "n": args.n, "nrhs": args.nrhs, "nb": r["nb"], "lookahead": True,
                   "parallelism": "single GPU"},
        "eta_max": r["eta_fp64_device"],
        "info": r["info"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_library_context": cpu_lib,
        "solve": r["solve"],
        # event-summed kernel time per kind, from one extra step after the timed region
        "kernel_ms": {k: round(v["ms"], 3) for k, v in r["prof"].items()},
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
