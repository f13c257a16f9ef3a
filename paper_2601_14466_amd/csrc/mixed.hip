// mixed.hip -- mixed-precision Cholesky solve with FP64 iterative refinement.
//
// The paper (JAXMg, "Software design", potrs bullet) fixes the problem, a
// Cholesky solve of an SPD system; it says nothing about precision, so the
// scheme is the classic one for SPD systems (Langou et al., SC'06):
//   1. A_w = fl32(A) (lower triangle), factored by potrf in binary32 storage:
//      diagonal blocks in FP64 arithmetic, panel TRSM and trailing update on
//      the FP32 matrix pipe (with lo = BF16 the trailing-update operands are
//      rounded to bfloat16 first, products and sums stay FP32).
//   2. x = solve_w(fl32(b)), widened to FP64.
//   3. repeat: r = b - A x in FP64 with the original A; eta_j =
//      |r_j|_inf / (|A|_inf |x_j|_inf + |b_j|_inf); stop when every column
//      has eta_j <= tol; otherwise d = solve_w(fl32(r)), x += d in FP64.
//   4. Stop without convergence after max_iter corrections, or when the
//      largest eta fails to halve twice in a row; then (or on a breakdown of
//      the low-precision factor) solve in FP64 if the caller allows it.
// One device-to-host copy of the per-column eta per iteration is the only
// synchronisation.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

// ---------------------------------------------------------------- casts
// W = fl32(A) on the lower triangle (column j, rows j..n-1).
__global__ __launch_bounds__(256) void k_cast_lower_f64_f32(const double* __restrict__ A, int64_t lda,
                                                            float* __restrict__ W, int64_t ldw, int64_t n) {
    const int64_t j = blockIdx.y;
    for (int64_t i = j + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        W[idx(i, j, ldw)] = (float)A[idx(i, j, lda)];
}

// copy the lower triangle of A (FP64) into W (FP64)
__global__ __launch_bounds__(256) void k_copy_lower_f64(const double* __restrict__ A, int64_t lda,
                                                        double* __restrict__ W, int64_t ldw, int64_t n) {
    const int64_t j = blockIdx.y;
    for (int64_t i = j + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        W[idx(i, j, ldw)] = A[idx(i, j, lda)];
}

// D (n x nrhs, ld n, FP32) = fl32(S) ; S FP64 with leading dimension lds
__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ S, int64_t lds, float* __restrict__ D,
                                                int64_t n, int64_t nrhs) {
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, r = e / n;
        D[e] = (float)S[idx(i, r, lds)];
    }
}

// X (FP64, ldx) = widen(D) when add == 0, X += widen(D) when add == 1
__global__ __launch_bounds__(256) void k_widen(const float* __restrict__ D, double* __restrict__ X, int64_t ldx,
                                               int64_t n, int64_t nrhs, int add) {
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, r = e / n;
        const double d = (double)D[e];
        X[idx(i, r, ldx)] = add ? X[idx(i, r, ldx)] + d : d;
    }
}

// copy an n x nrhs FP64 block between leading dimensions
__global__ __launch_bounds__(256) void k_copy_block(const double* __restrict__ S, int64_t lds, double* __restrict__ D,
                                                    int64_t ldd, int64_t n, int64_t nrhs) {
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, r = e / n;
        D[idx(i, r, ldd)] = S[idx(i, r, lds)];
    }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t cnt, unsigned long long v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

// ------------------------------------------------------- residual / norms
// R = B - A X (A symmetric, lower triangle stored), FP64, and the per-column
// maxima |r|, |x|, |b| (as ordered bit patterns: non-negative doubles order
// like unsigned integers, so atomicMax is exact and order-independent).
// With absmode != 0 the kernel instead accumulates the row sums of |A| into
// colmax[0] as max over rows (|A|_inf of the symmetric matrix) and ignores
// B, X, R.
// One workgroup per 64-row strip; it walks the 64 x 64 tiles (I, J) of the
// whole row, reading the stored tile A(I, J) for J <= I and the transpose of
// the stored tile A(J, I) for J > I, each staged through LDS with coalesced
// column reads.
constexpr int RS = 64;        // strip height / tile width
constexpr int RQ = 4;         // threads per row (right-hand-side groups)

template <int RPT>
__global__ __launch_bounds__(256) void k_sym_residual(const double* __restrict__ A, int64_t lda, int64_t n,
                                                      int64_t nrhs, const double* __restrict__ X, int64_t ldx,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ R, int64_t ldr,
                                                      unsigned long long* __restrict__ colmax, int absmode) {
    __shared__ double Ts[RS][RS + 1];          // tile, Ts[row][col] in strip-local orientation
    __shared__ double Xs[RS][RQ * RPT];        // x rows of tile J
    const int tid = threadIdx.x, row = tid & (RS - 1), q = tid >> 6;
    const int64_t I0 = (int64_t)blockIdx.x * RS;
    const int64_t nt = (n + RS - 1) / RS;
    double acc[RPT];
    double asum = 0.0;
    for (int64_t rc0 = 0; rc0 < (absmode ? 1 : nrhs); rc0 += RQ * RPT) {
#pragma unroll
        for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
        for (int64_t Jt = 0; Jt < nt; ++Jt) {
            const int64_t J0 = Jt * RS;
            __syncthreads();
            // stage the tile: for J <= I the block A(I0.., J0..); else A(J0.., I0..)^T
            for (int e = tid; e < RS * RS; e += 256) {
                const int a = e & (RS - 1), b = e >> 6;  // a walks the contiguous (row) direction
                double v = 0.0;
                if (Jt <= (int64_t)blockIdx.x) {
                    const int64_t gi = I0 + a, gj = J0 + b;      // Ts[a][b] = A(gi, gj)
                    if (gi < n && gj < n) v = (gi >= gj) ? A[idx(gi, gj, lda)] : A[idx(gj, gi, lda)];
                    Ts[a][b] = v;
                } else {
                    const int64_t gi = J0 + a, gj = I0 + b;      // Ts[b][a] = A(gi, gj) = A_sym(I0+b, J0+a)
                    if (gi < n && gj < n) v = A[idx(gi, gj, lda)];
                    Ts[b][a] = v;
                }
            }
            if (!absmode) {
                for (int e = tid; e < RS * RQ * RPT; e += 256) {
                    const int c = e % RS, r = e / RS;
                    const int64_t gc = J0 + c, gr = rc0 + r;
                    Xs[c][r] = (gc < n && gr < nrhs) ? X[idx(gc, gr, ldx)] : 0.0;
                }
            }
            __syncthreads();
            if (absmode) {
                if (q == 0)
                    for (int c = 0; c < RS; ++c) asum += fabs(Ts[row][c]);
            } else {
                for (int c = 0; c < RS; ++c) {
                    const double a = Ts[row][c];
#pragma unroll
                    for (int r = 0; r < RPT; ++r) acc[r] = fma(a, Xs[c][q * RPT + r], acc[r]);
                }
            }
        }
        const int64_t gi = I0 + row;
        if (absmode) {
            if (q == 0 && gi < n) atomicMax(&colmax[0], (unsigned long long)__double_as_longlong(asum));
        } else if (gi < n) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int64_t gr = rc0 + q * RPT + r;
                if (gr < nrhs) {
                    const double b = B[idx(gi, gr, ldb)];
                    const double x = X[idx(gi, gr, ldx)];
                    const double res = b - acc[r];
                    R[idx(gi, gr, ldr)] = res;
                    atomicMax(&colmax[3 * gr + 0], (unsigned long long)__double_as_longlong(fabs(res)));
                    atomicMax(&colmax[3 * gr + 1], (unsigned long long)__double_as_longlong(fabs(x)));
                    atomicMax(&colmax[3 * gr + 2], (unsigned long long)__double_as_longlong(fabs(b)));
                }
            }
        }
    }
}

// eta_j from the column maxima: eta[j] = rmax / (anorm * xmax + bmax)
__global__ void k_eta(const unsigned long long* __restrict__ colmax, const unsigned long long* __restrict__ anorm,
                      int64_t nrhs, double* __restrict__ eta) {
    for (int64_t r = threadIdx.x; r < nrhs; r += blockDim.x) {
        const double rm = __longlong_as_double((long long)colmax[3 * r + 0]);
        const double xm = __longlong_as_double((long long)colmax[3 * r + 1]);
        const double bm = __longlong_as_double((long long)colmax[3 * r + 2]);
        const double an = __longlong_as_double((long long)anorm[0]);
        const double den = an * xm + bm;
        eta[r] = (rm != rm || xm != xm) ? (double)NAN : (den > 0.0 ? rm / den : (rm > 0.0 ? (double)INFINITY : 0.0));
    }
}

// ------------------------------------------------------------ workspace
struct MixedWork {
    size_t bytes = 0;
    size_t o_aw = 0, o_r = 0, o_d = 0, o_y = 0, o_cm = 0, o_an = 0, o_eta = 0, o_info = 0;
};

static MixedWork mixed_layout(int64_t n, int64_t nrhs, int fallback) {
    MixedWork w;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = align_up(o + b, 256);
        return at;
    };
    const size_t nn = (size_t)n * (size_t)n;
    w.o_aw = take(std::max(nn * 4, fallback ? nn * 8 : (size_t)0));  // FP32 factor, or the FP64 fallback copy
    w.o_r = take((size_t)n * nrhs * 8);
    w.o_d = take((size_t)n * nrhs * 4);
    w.o_y = take(potrs_work_bytes(n, nrhs, 8));  // potrs workspace (FP32 or FP64 fallback)
    w.o_cm = take((size_t)(3 * nrhs + 1) * 8);
    w.o_an = take(8);
    w.o_eta = take((size_t)std::max<int64_t>(nrhs, 1) * 8);
    w.o_info = take(8);
    w.bytes = o;
    return w;
}

size_t mixed_work_bytes(int64_t n, int64_t nrhs, int fallback) { return mixed_layout(n, nrhs, fallback).bytes; }

static inline unsigned grid1(int64_t tot) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(tot, 256)), 65535); }

static mg_status sym_residual(hipStream_t st, const double* A, int64_t lda, int64_t n, int64_t nrhs, const double* X,
                              int64_t ldx, const double* B, int64_t ldb, double* R, unsigned long long* colmax,
                              int absmode) {
    const dim3 grid((unsigned)cdiv(n, RS)), block(256);
    const int64_t per = absmode ? 1 : std::min<int64_t>(nrhs, RQ * 16);
    if (per <= RQ * 1)
        hipLaunchKernelGGL((k_sym_residual<1>), grid, block, 0, st, A, lda, n, nrhs, X, ldx, B, ldb, R, n, colmax, absmode);
    else if (per <= RQ * 2)
        hipLaunchKernelGGL((k_sym_residual<2>), grid, block, 0, st, A, lda, n, nrhs, X, ldx, B, ldb, R, n, colmax, absmode);
    else if (per <= RQ * 4)
        hipLaunchKernelGGL((k_sym_residual<4>), grid, block, 0, st, A, lda, n, nrhs, X, ldx, B, ldb, R, n, colmax, absmode);
    else
        hipLaunchKernelGGL((k_sym_residual<8>), grid, block, 0, st, A, lda, n, nrhs, X, ldx, B, ldb, R, n, colmax, absmode);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

mg_status posv_mixed_impl(mg_handle_t h, int lo, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                          const double* B, int64_t ldb, double* X, int64_t ldx, const mg_ir_opts* o, void* work,
                          mg_ir_result* res, int32_t* info) {
    hipStream_t st = h->stream;
    std::memset(res, 0, sizeof(*res));
    mg_status rc = set_info_zero(st, info);
    if (rc) return rc;
    if (n == 0 || nrhs == 0) {
        MG_HIP(hipStreamSynchronize(st));
        return MG_OK;
    }
    const MixedWork L = mixed_layout(n, nrhs, o->fallback);
    char* base = (char*)work;
    float* Aw = (float*)(base + L.o_aw);
    double* R = (double*)(base + L.o_r);
    float* D = (float*)(base + L.o_d);
    void* Yw = (void*)(base + L.o_y);
    unsigned long long* cm = (unsigned long long*)(base + L.o_cm);
    unsigned long long* an = (unsigned long long*)(base + L.o_an);
    double* eta_d = (double*)(base + L.o_eta);
    int32_t* info_lo = (int32_t*)(base + L.o_info);

    const int saved_trail = h->trail_lo;
    h->trail_lo = (lo == MG_PREC_BF16) ? 2 : 1;
    // 1. working copy and low-precision factor
    hipLaunchKernelGGL(k_cast_lower_f64_f32, dim3(grid1(n), (unsigned)n), dim3(256), 0, st, A, lda, Aw, n, n);
    MG_LAUNCH_CHECK();
    rc = potrf_impl<float>(h, n, Aw, n, info_lo);
    h->trail_lo = saved_trail;
    if (rc) return rc;
    int32_t hinfo = 0;
    MG_HIP(hipMemcpyAsync(&hinfo, info_lo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    res->lo_info = hinfo;
    bool converged = false;
    std::vector<double> eta((size_t)nrhs);
    if (hinfo == 0) {
        // 2. first solve in working precision
        hipLaunchKernelGGL(k_to_f32, dim3(grid1(n * nrhs)), dim3(256), 0, st, B, ldb, D, n, nrhs);
        MG_LAUNCH_CHECK();
        if ((rc = potrs_impl<float>(h, n, nrhs, Aw, n, D, n, (float*)Yw, nullptr))) return rc;
        hipLaunchKernelGGL(k_widen, dim3(grid1(n * nrhs)), dim3(256), 0, st, D, X, ldx, n, nrhs, 0);
        MG_LAUNCH_CHECK();
        // |A|_inf once
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, an, (int64_t)1, 0ull);
        MG_LAUNCH_CHECK();
        if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, an, 1))) return rc;
        double prev = INFINITY;
        int slow = 0;
        for (int it = 0;; ++it) {
            // 3. FP64 residual and per-column backward error
            hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, cm, 3 * nrhs, 0ull);
            MG_LAUNCH_CHECK();
            if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, cm, 0))) return rc;
            hipLaunchKernelGGL(k_eta, dim3(1), dim3(256), 0, st, cm, an, nrhs, eta_d);
            MG_LAUNCH_CHECK();
            MG_HIP(hipMemcpyAsync(eta.data(), eta_d, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
            MG_HIP(hipStreamSynchronize(st));
            double e = 0.0;
            bool bad = false;
            for (double v : eta) {
                if (v != v) bad = true;
                e = std::max(e, v);
            }
            res->eta = bad ? (double)NAN : e;
            res->iters = it;
            if (!bad && e <= o->tol) {
                converged = true;
                break;
            }
            if (bad || it >= o->max_iter) break;
            if (it > 0 && !(e <= 0.5 * prev)) ++slow;
            else slow = 0;
            if (slow >= 2) break;
            prev = e;
            // 4. correction in working precision, update in FP64
            hipLaunchKernelGGL(k_to_f32, dim3(grid1(n * nrhs)), dim3(256), 0, st, R, n, D, n, nrhs);
            MG_LAUNCH_CHECK();
            if ((rc = potrs_impl<float>(h, n, nrhs, Aw, n, D, n, (float*)Yw, nullptr))) return rc;
            hipLaunchKernelGGL(k_widen, dim3(grid1(n * nrhs)), dim3(256), 0, st, D, X, ldx, n, nrhs, 1);
            MG_LAUNCH_CHECK();
        }
    }
    if (!converged) {
        if (!o->fallback) {
            res->fell_back = 0;
            return MG_OK;
        }
        // 5. FP64 fallback on a copy of A (A itself is const)
        res->fell_back = 1;
        double* Ad = (double*)(base + L.o_aw);
        hipLaunchKernelGGL(k_copy_lower_f64, dim3(grid1(n), (unsigned)n), dim3(256), 0, st, A, lda, Ad, n, n);
        MG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_copy_block, dim3(grid1(n * nrhs)), dim3(256), 0, st, B, ldb, X, ldx, n, nrhs);
        MG_LAUNCH_CHECK();
        if ((rc = potrf_impl<double>(h, n, Ad, n, info))) return rc;
        if ((rc = potrs_impl<double>(h, n, nrhs, Ad, n, X, ldx, (double*)Yw, info))) return rc;
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, cm, 3 * nrhs, 0ull);
        MG_LAUNCH_CHECK();
        if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, cm, 0))) return rc;
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, an, (int64_t)1, 0ull);
        MG_LAUNCH_CHECK();
        if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, an, 1))) return rc;
        hipLaunchKernelGGL(k_eta, dim3(1), dim3(256), 0, st, cm, an, nrhs, eta_d);
        MG_LAUNCH_CHECK();
        MG_HIP(hipMemcpyAsync(eta.data(), eta_d, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        double e = 0.0;
        for (double v : eta) e = (v != v || v > e) ? v : e;
        res->eta = e;
    }
    return MG_OK;
}

}  // namespace mg
