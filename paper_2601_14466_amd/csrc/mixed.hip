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
// W = A (converted to W's type) on the lower triangle (column j, rows
// j..n-1): the binary32 working copy, and the FP64 copy of the fallback.
// Workgroup b converts columns b and n - 1 - b (n + 1 entries together, the
// same for every workgroup, so no launch is empty or long); workgroups are
// strided over the (n + 1) / 2 pairs.
template <typename D>
__global__ __launch_bounds__(256) void k_copy_lower(const double* __restrict__ A, int64_t lda, D* __restrict__ W,
                                                    int64_t ldw, int64_t n) {
    for (int64_t b = blockIdx.x; b < (n + 1) / 2; b += gridDim.x) {
        const int64_t j2 = n - 1 - b;
        for (int64_t i = b + threadIdx.x; i < n; i += 256) W[idx(i, b, ldw)] = (D)A[idx(i, b, lda)];
        if (j2 != b)
            for (int64_t i = j2 + threadIdx.x; i < n; i += 256) W[idx(i, j2, ldw)] = (D)A[idx(i, j2, lda)];
    }
}

static inline dim3 lower_grid(int64_t n) {
    return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + 1) / 2), 65535));
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

// X (n x nrhs, ldx) := quiet NaN: the result of a solve that produced none
__global__ __launch_bounds__(256) void k_fill_nan(double* __restrict__ X, int64_t ldx, int64_t n, int64_t nrhs) {
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        X[idx(e % n, e / n, ldx)] = (double)NAN;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t cnt, unsigned long long v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

// ------------------------------------------------------- residual / norms
// R = B - A X (A symmetric, lower triangle stored), FP64, and the per-column
// maxima |r|, |x|, |b| (as ordered bit patterns: non-negative doubles order
// like unsigned integers, so atomicMax is exact and order-independent).
// With absmode != 0 the kernels instead produce the row sums of |A| and their
// maximum (|A|_inf of the symmetric matrix) in colmax[0].
//
// Pass 1 (k_sym_rowprod): the grid is (64-row strips) x RSPLIT column ranges.
// Each workgroup's four waves take the 64 x 64 tiles of its range in turn;
// a lane owns one row of the strip and streams that row of the tile from
// memory: stored tiles (J <= I) down their columns (coalesced across lanes);
// tiles above the diagonal (J > I) are the transposed stored tile, read in
// coalesced 16 x 4 pieces and transposed through a per-wave LDS buffer (no
// workgroup barrier).  The x values of the tile arrive one per lane and are
// broadcast by readlane.  The four waves' sums are added in a fixed order and written as one
// partial per (strip, range).
// Pass 2 (k_sym_finish): R = B - sum of the partials over the ranges (fixed
// order), and the column maxima.  The result does not depend on the launch.
constexpr int RS = 64;      // strip height / tile width
constexpr int RSPLIT = 8;   // column ranges per strip
constexpr int RRPT = 8;     // right-hand sides per pass

// partial sums: RSPLIT ranges x n rows x (up to) RRPT right-hand sides
size_t residual_part_bytes(int64_t n, int64_t nrhs) {
    (void)nrhs;
    return (size_t)RSPLIT * (size_t)n * RRPT * 8;
}

template <int RPT>
__global__ __launch_bounds__(256) void k_sym_rowprod(const double* __restrict__ A, int64_t lda, int64_t n,
                                                     int64_t nrhs, int64_t rc0, const double* __restrict__ X,
                                                     int64_t ldx, double* __restrict__ Pp, int absmode) {
    __shared__ double red[4][RPT][RS];
    __shared__ double tr[4][RS][17];  // per wave: a transposed 64 x 16 piece of a tile above the diagonal
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t strip = blockIdx.x, I0 = strip * RS;
    const int64_t nt = (n + RS - 1) / RS;
    const int64_t per = (nt + RSPLIT - 1) / RSPLIT;
    const int64_t jb = blockIdx.y * per, je = jb + per < nt ? jb + per : nt;
    const int64_t gi = I0 + lane;
    const bool rin = gi < n;
    const int64_t gic = rin ? gi : I0;  // clamped row for loads
    double acc[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) acc[r] = 0.0;
    for (int64_t Jt = jb + w; Jt < je; Jt += 4) {
        const int64_t J0 = Jt * RS;
        const int jw = (int)(n - J0 < RS ? n - J0 : RS);
        double xv[RPT];
        if (!absmode) {
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                xv[r] = (lane < jw && rc0 + r < nrhs) ? X[idx(J0 + lane, rc0 + r, ldx)] : 0.0;
        }
        // element (gi, J0 + c) of the symmetric matrix: below the diagonal of
        // the stored triangle it is A[gi + (J0 + c) lda], above it A[(J0 + c) + gi lda]
        const bool below = Jt < strip, above = Jt > strip;
#pragma unroll
        for (int c0 = 0; c0 < RS; c0 += 16) {
            double av[16];
            if (above) {
                // Stored rows J0 + c0 .. + 15 of columns I0 .. I0 + 63, read
                // sixteen rows by four columns per instruction (coalesced),
                // transposed through this wave's LDS piece so that lane b
                // receives its row's sixteen values.  Read directly, each
                // lane would walk its own column: 64 cache lines per load.
                const int a = lane & 15, b0 = lane >> 4;
                const bool aok = c0 + a < jw;
                double tv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int64_t gi2 = I0 + 4 * q + b0;
                    tv[q] = (aok && gi2 < n) ? A[idx(J0 + c0 + a, gi2, lda)] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) tr[w][4 * q + b0][a] = tv[q];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int c = 0; c < 16; ++c) av[c] = tr[w][lane][c];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    const int cc = c0 + c;
                    const int64_t gj = J0 + (cc < jw ? cc : 0);
                    const double v = (below || gic >= gj) ? A[idx(gic, gj, lda)] : A[idx(gj, gic, lda)];
                    av[c] = (cc < jw && rin) ? v : 0.0;
                }
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                if (absmode) {
                    acc[0] += fabs(av[c]);
                } else {
#pragma unroll
                    for (int r = 0; r < RPT; ++r) acc[r] = fma(av[c], readlane(xv[r], c0 + c), acc[r]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) red[w][r][lane] = acc[r];
    __syncthreads();
    if (w == 0 && rin) {
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            Pp[((size_t)blockIdx.y * n + gi) * RPT + r] = ((red[0][r][lane] + red[1][r][lane]) + red[2][r][lane]) +
                                                          red[3][r][lane];
    }
}

template <int RPT>
__global__ __launch_bounds__(256) void k_sym_finish(int64_t n, int64_t nrhs, int64_t rc0, const double* __restrict__ X,
                                                    int64_t ldx, const double* __restrict__ B, int64_t ldb,
                                                    double* __restrict__ R, int64_t ldr, const double* __restrict__ Pp,
                                                    unsigned long long* __restrict__ colmax, int absmode) {
    for (int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x; gi < n; gi += (int64_t)gridDim.x * 256) {
        if (absmode) {
            double sm = 0.0;
            for (int sp = 0; sp < RSPLIT; ++sp) sm += Pp[((size_t)sp * n + gi) * RPT];
            atomicMax(&colmax[0], (unsigned long long)__double_as_longlong(sm));
            continue;
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int64_t gr = rc0 + r;
            if (gr >= nrhs) break;
            double sm = 0.0;
            for (int sp = 0; sp < RSPLIT; ++sp) sm += Pp[((size_t)sp * n + gi) * RPT + r];
            const double b = B[idx(gi, gr, ldb)];
            const double x = X[idx(gi, gr, ldx)];
            const double res = b - sm;
            R[idx(gi, gr, ldr)] = res;
            atomicMax(&colmax[3 * gr + 0], (unsigned long long)__double_as_longlong(fabs(res)));
            atomicMax(&colmax[3 * gr + 1], (unsigned long long)__double_as_longlong(fabs(x)));
            atomicMax(&colmax[3 * gr + 2], (unsigned long long)__double_as_longlong(fabs(b)));
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
    size_t o_aw = 0, o_r = 0, o_d = 0, o_y = 0, o_cm = 0, o_an = 0, o_eta = 0, o_info = 0, o_p16 = 0, o_rp = 0;
};

static MixedWork mixed_layout(int64_t n, int64_t nrhs, int fallback, int lo) {
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
    // per-column eta, then one slot whose first word is the working-precision
    // solves' info (MG_INFO_SOLVE_ABORTED after a sweep gave up); read back together
    w.o_eta = take((size_t)(std::max<int64_t>(nrhs, 1) + 1) * 8);
    w.o_info = take(8);
    w.o_rp = take(residual_part_bytes(n, nrhs));  // residual partial sums
    // bfloat16 mode: two row-major bfloat16 copies of a block column panel
    // (n x 512 each), alternating between consecutive block columns
    if (lo == MG_PREC_BF16) w.o_p16 = take(bf16_panel_bytes(n));
    w.bytes = o;
    return w;
}

size_t mixed_work_bytes(int64_t n, int64_t nrhs, int fallback, int lo) {
    return mixed_layout(n, nrhs, fallback, lo).bytes;
}

static inline unsigned grid1(int64_t tot) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(tot, 256)), 65535); }

static mg_status sym_residual(hipStream_t st, const double* A, int64_t lda, int64_t n, int64_t nrhs, const double* X,
                              int64_t ldx, const double* B, int64_t ldb, double* R, unsigned long long* colmax,
                              int absmode, double* Pp) {
    const dim3 grid((unsigned)cdiv(n, RS), RSPLIT), block(256);
    const unsigned gf = (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(n, 256)), 4096);
    for (int64_t rc0 = 0; rc0 < (absmode ? 1 : nrhs); rc0 += RRPT) {
        const int64_t cnt = absmode ? 1 : std::min<int64_t>(RRPT, nrhs - rc0);
        if (cnt <= 1) {
            hipLaunchKernelGGL((k_sym_rowprod<1>), grid, block, 0, st, A, lda, n, nrhs, rc0, X, ldx, Pp, absmode);
            MG_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_sym_finish<1>), dim3(gf), block, 0, st, n, nrhs, rc0, X, ldx, B, ldb, R, n, Pp,
                               colmax, absmode);
        } else if (cnt <= 2) {
            hipLaunchKernelGGL((k_sym_rowprod<2>), grid, block, 0, st, A, lda, n, nrhs, rc0, X, ldx, Pp, absmode);
            MG_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_sym_finish<2>), dim3(gf), block, 0, st, n, nrhs, rc0, X, ldx, B, ldb, R, n, Pp,
                               colmax, absmode);
        } else if (cnt <= 4) {
            hipLaunchKernelGGL((k_sym_rowprod<4>), grid, block, 0, st, A, lda, n, nrhs, rc0, X, ldx, Pp, absmode);
            MG_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_sym_finish<4>), dim3(gf), block, 0, st, n, nrhs, rc0, X, ldx, B, ldb, R, n, Pp,
                               colmax, absmode);
        } else {
            hipLaunchKernelGGL((k_sym_rowprod<8>), grid, block, 0, st, A, lda, n, nrhs, rc0, X, ldx, Pp, absmode);
            MG_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_sym_finish<8>), dim3(gf), block, 0, st, n, nrhs, rc0, X, ldx, B, ldb, R, n, Pp,
                               colmax, absmode);
        }
        MG_LAUNCH_CHECK();
    }
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
    const MixedWork L = mixed_layout(n, nrhs, o->fallback, lo);
    char* base = (char*)work;
    float* Aw = (float*)(base + L.o_aw);
    double* R = (double*)(base + L.o_r);
    float* D = (float*)(base + L.o_d);
    void* Yw = (void*)(base + L.o_y);
    unsigned long long* cm = (unsigned long long*)(base + L.o_cm);
    unsigned long long* an = (unsigned long long*)(base + L.o_an);
    double* eta_d = (double*)(base + L.o_eta);
    int32_t* info_lo = (int32_t*)(base + L.o_info);
    int32_t* info_sw = (int32_t*)(eta_d + nrhs);  // working-precision solves
    double* Pp = (double*)(base + L.o_rp);

    const int saved_trail = h->trail_lo;
    h->trail_lo = (lo == MG_PREC_BF16) ? 2 : 1;
    h->bf16_panel = (lo == MG_PREC_BF16) ? (void*)(base + L.o_p16) : nullptr;
    // 1. working copy and low-precision factor
    hipLaunchKernelGGL(k_copy_lower<float>, lower_grid(n), dim3(256), 0, st, A, lda, Aw, n, n);
    MG_LAUNCH_CHECK();
    rc = potrf_impl<float>(h, n, Aw, n, info_lo);
    h->trail_lo = saved_trail;
    h->bf16_panel = nullptr;
    if (rc) return rc;
    if ((rc = set_info_zero(st, info_sw))) return rc;
    int32_t hinfo = 0;
    MG_HIP(hipMemcpyAsync(&hinfo, info_lo, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    res->lo_info = hinfo;
    bool converged = false;
    std::vector<double> eta((size_t)nrhs + 1);
    if (hinfo == 0) {
        // 2. first solve in working precision
        hipLaunchKernelGGL(k_to_f32, dim3(grid1(n * nrhs)), dim3(256), 0, st, B, ldb, D, n, nrhs);
        MG_LAUNCH_CHECK();
        if ((rc = potrs_impl<float>(h, n, nrhs, Aw, n, D, n, (float*)Yw, info_sw))) return rc;
        hipLaunchKernelGGL(k_widen, dim3(grid1(n * nrhs)), dim3(256), 0, st, D, X, ldx, n, nrhs, 0);
        MG_LAUNCH_CHECK();
        // |A|_inf once
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, an, (int64_t)1, 0ull);
        MG_LAUNCH_CHECK();
        if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, an, 1, Pp))) return rc;
        double prev = INFINITY;
        int slow = 0;
        for (int it = 0;; ++it) {
            // 3. FP64 residual and per-column backward error
            hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, cm, 3 * nrhs, 0ull);
            MG_LAUNCH_CHECK();
            if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, cm, 0, Pp))) return rc;
            hipLaunchKernelGGL(k_eta, dim3(1), dim3(256), 0, st, cm, an, nrhs, eta_d);
            MG_LAUNCH_CHECK();
            MG_HIP(hipMemcpyAsync(eta.data(), eta_d, sizeof(double) * (nrhs + 1), hipMemcpyDeviceToHost, st));
            MG_HIP(hipStreamSynchronize(st));
            int32_t sw = 0;
            std::memcpy(&sw, &eta[(size_t)nrhs], sizeof(sw));
            if (sw != 0) {
                // a working-precision sweep gave up waiting: X is not a solution
                hipLaunchKernelGGL(k_fill_nan, dim3(grid1(n * nrhs)), dim3(256), 0, st, X, ldx, n, nrhs);
                MG_LAUNCH_CHECK();
                MG_HIP(hipStreamSynchronize(st));
                res->eta = (double)NAN;
                res->iters = it;
                return MG_ERR_ABORTED;
            }
            double e = 0.0;
            bool bad = false;
            for (int64_t r = 0; r < nrhs; ++r) {
                const double v = eta[(size_t)r];
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
            if ((rc = potrs_impl<float>(h, n, nrhs, Aw, n, D, n, (float*)Yw, info_sw))) return rc;
            hipLaunchKernelGGL(k_widen, dim3(grid1(n * nrhs)), dim3(256), 0, st, D, X, ldx, n, nrhs, 1);
            MG_LAUNCH_CHECK();
        }
    }
    if (!converged) {
        if (!o->fallback) {
            res->fell_back = 0;
            if (hinfo != 0) {
                // the low-precision factor broke down and no FP64 solve is
                // allowed: there is no solution to return
                hipLaunchKernelGGL(k_fill_nan, dim3(grid1(n * nrhs)), dim3(256), 0, st, X, ldx, n, nrhs);
                MG_LAUNCH_CHECK();
                MG_HIP(hipStreamSynchronize(st));
                res->eta = (double)NAN;
            }
            return MG_OK;
        }
        // 5. FP64 fallback on a copy of A (A itself is const)
        res->fell_back = 1;
        double* Ad = (double*)(base + L.o_aw);
        hipLaunchKernelGGL(k_copy_lower<double>, lower_grid(n), dim3(256), 0, st, A, lda, Ad, n, n);
        MG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_copy_block, dim3(grid1(n * nrhs)), dim3(256), 0, st, B, ldb, X, ldx, n, nrhs);
        MG_LAUNCH_CHECK();
        if ((rc = potrf_impl<double>(h, n, Ad, n, info))) return rc;
        if ((rc = potrs_impl<double>(h, n, nrhs, Ad, n, X, ldx, (double*)Yw, info))) return rc;
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, cm, 3 * nrhs, 0ull);
        MG_LAUNCH_CHECK();
        if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, cm, 0, Pp))) return rc;
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, an, (int64_t)1, 0ull);
        MG_LAUNCH_CHECK();
        if ((rc = sym_residual(st, A, lda, n, nrhs, X, ldx, B, ldb, R, an, 1, Pp))) return rc;
        hipLaunchKernelGGL(k_eta, dim3(1), dim3(256), 0, st, cm, an, nrhs, eta_d);
        MG_LAUNCH_CHECK();
        int32_t finfo = 0;
        MG_HIP(hipMemcpyAsync(eta.data(), eta_d, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
        MG_HIP(hipMemcpyAsync(&finfo, info, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        double e = 0.0;
        for (int64_t r = 0; r < nrhs; ++r) {
            const double v = eta[(size_t)r];
            e = (v != v || v > e) ? v : e;
        }
        res->eta = e;
        if (finfo == MG_INFO_SOLVE_ABORTED) return MG_ERR_ABORTED;
    }
    return MG_OK;
}

}  // namespace mg
