// lu.hip -- the paper's general solve (JAXMg, "Software design", lu_solve
// bullet: A x = b for a general nonsingular A through a pivoted LU
// factorisation): P A = L U by Gaussian elimination with partial pivoting,
// then the row interchanges and the two triangular solves.  FP64.
//
// Blocked right-looking factorisation over block columns of LU_NB = 64:
//   1. k_getf2_panel: the panel (rows k0..n-1, columns k0..k0+63) with
//      partial pivoting, a cooperative launch of G workgroups that each keep
//      256 consecutive rows of the panel in LDS, one row per thread.  For
//      every column j each workgroup publishes its largest |entry| (the first
//      row on ties) with that row's values, and the owner of row j publishes
//      row j, to a double-buffered slot array; the workgroups meet at one
//      grid barrier and all pick the same winner: the owners of rows j and p
//      exchange them, and every row below j is scaled by the pivot and
//      updated with the pivot row (a local rank-1 update).  Pivot choice and
//      the order of each entry's updates are those of column-by-column
//      elimination.
//   2. k_lu_swap_cols: the panel's interchanges applied to the columns left
//      of it.
//   3. k_lu_row_block: per 64 columns right of the panel, the interchanges
//      (the block row's rows and every row they touch go through LDS), then
//      U12 = L11^{-1} A12 by forward substitution with the unit lower L11
//      (one lane per column), stored over A12 and transposed into a
//      workspace, the operand layout of the update.
//   4. k_gemm_sub: A22 -= L21 U12 on the FP64 matrix pipe (128 x 128 output
//      tiles of four 64 x 64 wave quarters, operands streamed from memory
//      straight into registers through a ring of four k-steps, as the
//      Cholesky trailing update but over the whole tile grid).
// info: the first k (1-based) whose pivot is exactly zero; elimination goes
// on past it (that column is not scaled), as LAPACK's xGETRF.
//
// The solve (getrs): the interchanges ipiv are turned into one row
// permutation (k_lu_perm_lists per 64 interchanges in parallel, then
// k_lu_perm_apply composing them in order), and the triangular sweeps of
// potrs run with the unit lower and the upper factor, the forward sweep
// reading row perm[i] of B for row i.
#include <algorithm>
#include <climits>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

constexpr int LU_NB = 64;                    // block column width
constexpr int LU_ROWS = 256;                 // panel rows per workgroup (one per thread)
constexpr int LU_HDR = 2;                    // slot header: |value|, row
constexpr int LU_SLOT = LU_HDR + LU_NB;      // doubles per slot
constexpr int LU_LIST = 2 * LU_NB;           // rows one block of 64 interchanges can touch
constexpr int LU_LIST_WORDS = 1 + 2 * LU_LIST;  // count, destination rows, source rows
constexpr int LU_SPIN_LIMIT = 1 << 24;       // default polls before a barrier wait gives up

struct LuSync {
    unsigned count;  // grid-barrier arrivals since the start of the factorisation
    int err;         // set when a barrier wait gave up
    int bad;         // the solve: an interchange outside 1..n was ignored
    int pad;
};

__device__ __forceinline__ double ld_dev(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_dev(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// (v, r) pairs: larger v wins, the smaller r on ties.  v < 0 marks "no candidate".
__device__ __forceinline__ void argmax_merge(double& v, int& r, double ov, int orr) {
    if (ov > v || (ov == v && orr < r)) {
        v = ov;
        r = orr;
    }
}
__device__ __forceinline__ void wave_argmax(double& v, int& r) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int orr = __shfl_xor(r, off, 64);
        argmax_merge(v, r, ov, orr);
    }
}

__global__ void k_lu_reset(LuSync* sy) {
    if (threadIdx.x == 0) *sy = LuSync{0u, 0, 0, 0};
}

// Panel factorisation (cooperative launch of G = ceil(m / 256) workgroups).
// base: barrier arrivals of earlier panels of this factorisation.
// slots: 2 x (G + 1) x LU_SLOT doubles (slot G: row j).
__global__ __launch_bounds__(256, 1) void k_getf2_panel(double* __restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                        int nbw, double* slots, LuSync* sy, unsigned base,
                                                        int32_t* __restrict__ ipiv, int32_t* __restrict__ info,
                                                        int spin_limit) {
    __shared__ double P[LU_ROWS][LU_NB + 1];
    __shared__ double urow[LU_NB], jrow[LU_NB];
    __shared__ double red_v[2][4];
    __shared__ int red_r[2][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, G = gridDim.x, wg = blockIdx.x;
    const int64_t m = n - k0;
    const int64_t row0 = (int64_t)wg * LU_ROWS;  // first panel row (relative to k0) of this workgroup
    const int R = (int)(m - row0 < LU_ROWS ? m - row0 : LU_ROWS);
    for (int c = 0; c < nbw; ++c)
        if (tid < R) P[tid][c] = A[idx(k0 + row0 + tid, k0 + c, lda)];
    __syncthreads();
    bool gave_up = false;
    for (int j = 0; j < nbw; ++j) {
        double* sl = slots + (size_t)(j & 1) * (G + 1) * LU_SLOT;
        // ---- this workgroup's candidate: rows >= j, NaN entries never win
        double v = -1.0;
        int r = INT_MAX;
        if (tid < R && row0 + tid >= j) {
            const double a = fabs(P[tid][j]);
            if (a == a) {
                v = a;
                r = tid;
            }
        }
        wave_argmax(v, r);
        if (lane == 0) {
            red_v[0][w] = v;
            red_r[0][w] = r;
        }
        __syncthreads();
        v = red_v[0][0];
        r = red_r[0][0];
#pragma unroll
        for (int q = 1; q < 4; ++q) argmax_merge(v, r, red_v[0][q], red_r[0][q]);
        // ---- publish it, and row j by its owner
        double* me = sl + (size_t)wg * LU_SLOT;
        if (tid == 0) {
            me[0] = v;
            me[1] = v >= 0.0 ? (double)(row0 + r) : -1.0;
        }
        if (v >= 0.0 && tid < nbw) me[LU_HDR + tid] = P[r][tid];
        const bool ownj = j >= row0 && j < row0 + R;
        if (ownj && tid < nbw) sl[(size_t)G * LU_SLOT + LU_HDR + tid] = P[j - row0][tid];
        // ---- grid barrier: every thread's stores are made visible at device
        // scope, then one arrival per workgroup; the wait is bounded (a flag
        // set by any workgroup that gave up ends every other wait)
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            atomicAdd(&sy->count, 1u);
            const unsigned target = base + (unsigned)(j + 1) * (unsigned)G;
            for (int spins = 0;; ++spins) {
                if (spin_limit == 0 && G > 1) {  // forced give-up (host setting)
                    atomicExch(&sy->err, 1);
                    break;
                }
                if (__hip_atomic_load(&sy->count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
                if (gave_up || spins > spin_limit || ld_dev(&sy->err) != 0) {
                    atomicExch(&sy->err, 1);
                    gave_up = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        __threadfence();
        // ---- the winner over all workgroups (every workgroup alike): headers
        // from the slots; row j's values meanwhile
        double hv = -1.0;
        int hr = INT_MAX;
        if (tid < G) {
            const double a = ld_dev(&sl[(size_t)tid * LU_SLOT]);
            const double rr = ld_dev(&sl[(size_t)tid * LU_SLOT + 1]);
            if (a >= 0.0 && rr >= (double)j && rr < (double)m) {
                hv = a;
                hr = (int)rr;
            }
        }
        if (tid < nbw) jrow[tid] = ld_dev(&sl[(size_t)G * LU_SLOT + LU_HDR + tid]);
        wave_argmax(hv, hr);
        if (lane == 0) {
            red_v[1][w] = hv;
            red_r[1][w] = hr;
        }
        __syncthreads();
        hv = red_v[1][0];
        hr = red_r[1][0];
#pragma unroll
        for (int q = 1; q < 4; ++q) argmax_merge(hv, hr, red_v[1][q], red_r[1][q]);
        // a NaN diagonal entry stays the pivot (a sequential scan starting
        // from it never replaces it); so does row j when nothing else qualifies
        const int64_t p = (hv < 0.0 || jrow[j] != jrow[j]) ? (int64_t)j : (int64_t)hr;
        const int pw = (int)(p / LU_ROWS);  // workgroup whose slot holds row p
        if (tid < nbw) urow[tid] = (p == j) ? jrow[tid] : ld_dev(&sl[(size_t)pw * LU_SLOT + LU_HDR + tid]);
        __syncthreads();
        const double piv = urow[j];
        if (wg == 0 && tid == 0) {
            ipiv[k0 + j] = (int32_t)(k0 + p + 1);
            if (piv == 0.0 && *info == 0) *info = (int32_t)(k0 + j + 1);
        }
        // ---- interchange rows j and p (their owners), then eliminate below j
        if (p != j) {
            if (ownj && tid < nbw) P[j - row0][tid] = urow[tid];
            if (p >= row0 && p < row0 + R && tid < nbw) P[p - row0][tid] = jrow[tid];
        }
        __syncthreads();
        if (piv != 0.0 && tid < R && row0 + tid > j) {
            const double l = P[tid][j] / piv;
            P[tid][j] = l;
            for (int c = j + 1; c < nbw; ++c) P[tid][c] = P[tid][c] - l * urow[c];
        }
        __syncthreads();
    }
    for (int c = 0; c < nbw; ++c)
        if (tid < R) A[idx(k0 + row0 + tid, k0 + c, lda)] = P[tid][c];
}

// One wave: the net row permutation of the interchanges s = 0..cw-1 (row
// c0 + s with row ipiv[c0 + s] - 1, in order), as (destination, source)
// pairs -- after the interchanges, row dst[t] holds what row src[t] held
// before them.  Entries 0..cw-1 are rows c0..c0+cw-1 (src = dst when a row
// is not moved), entries cw.. the other rows touched, in order of first
// touch.  Entries outside 1..n are skipped and flagged.  Lane q keeps
// entries q (pa) and cw + q (pb) in registers.  Returns the count.
__device__ int lu_swap_list(const int32_t* __restrict__ ipiv, int64_t n, int64_t c0, int cw, int* dst, int* src,
                            bool& bad) {
    const int lane = threadIdx.x & 63;
    const int pv = lane < cw ? ipiv[c0 + lane] - 1 : 0;
    int pa_dst = (int)(c0 + lane), pa_src = pa_dst;
    int pb_dst = -1, pb_src = -1;
    int cnt = 0;
    bad = false;
    for (int s = 0; s < cw; ++s) {
        const int r2 = __shfl(pv, s, 64);
        const int r1 = (int)c0 + s;
        if (r2 < 0 || r2 >= n) {
            bad = true;
            continue;
        }
        if (r2 == r1) continue;
        const bool in_a = r2 >= c0 && r2 < c0 + cw;
        int q;
        if (in_a) {
            q = r2 - (int)c0;
        } else {
            const unsigned long long hit = __ballot(lane < cnt && pb_dst == r2);
            if (hit) {
                q = __ffsll((long long)hit) - 1;
            } else {
                q = cnt;
                if (lane == cnt) pb_dst = pb_src = r2;
                ++cnt;
            }
        }
        const int v1 = __shfl(pa_src, s, 64);
        const int v2 = in_a ? __shfl(pa_src, q, 64) : __shfl(pb_src, q, 64);
        if (lane == s) pa_src = v2;
        if (lane == q) {
            if (in_a) pa_src = v1;
            else pb_src = v1;
        }
    }
    if (lane < cw) {
        dst[lane] = pa_dst;
        src[lane] = pa_src;
    }
    if (lane < cnt) {
        dst[cw + lane] = pb_dst;
        src[cw + lane] = pb_src;
    }
    return cw + cnt;
}

// Interchanges of the panel at k0 (nbw of them) applied to columns
// [0, ncols): 64 columns per workgroup, every touched value read into LDS
// before any is written.
__global__ __launch_bounds__(256) void k_lu_swap_cols(double* __restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                      int nbw, int64_t ncols, const int32_t* __restrict__ ipiv) {
    __shared__ double V[LU_LIST][65];
    __shared__ int sdst[LU_LIST], ssrc[LU_LIST];
    __shared__ int s_cnt;
    const int tid = threadIdx.x;
    if (tid < 64) {
        bool bad;
        const int cnt = lu_swap_list(ipiv, n, k0, nbw, sdst, ssrc, bad);
        if (tid == 0) s_cnt = cnt;
    }
    __syncthreads();
    const int cnt = s_cnt;
    const int64_t cb = (int64_t)blockIdx.x * 64;
    const int cw = (int)(ncols - cb < 64 ? ncols - cb : 64);
    for (int e = tid; e < LU_LIST * 64; e += 256) {
        const int t = e & (LU_LIST - 1), c = e >> 7;
        if (t < cnt && c < cw && sdst[t] != ssrc[t]) V[t][c] = A[idx(ssrc[t], cb + c, lda)];
    }
    __syncthreads();
    for (int e = tid; e < LU_LIST * 64; e += 256) {
        const int t = e & (LU_LIST - 1), c = e >> 7;
        if (t < cnt && c < cw && sdst[t] != ssrc[t]) A[idx(sdst[t], cb + c, lda)] = V[t][c];
    }
}

// Block row right of a full-width panel at k0 (64 interchanges), 64 columns
// per workgroup starting at column k0 + 64 + 64 * blockIdx.x: the panel's
// interchanges, then U12 = L11^{-1} A12 (L11 = the panel's unit lower
// 64 x 64 block) by forward substitution, one lane per column of wave 0,
// stored over A12 and as U12^T into Ut (column j - (k0 + 64) of U12 is row
// j - (k0 + 64) of Ut; leading dimension ldu).
__global__ __launch_bounds__(256) void k_lu_row_block(double* __restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                      const int32_t* __restrict__ ipiv, double* __restrict__ Ut,
                                                      int64_t ldu) {
    constexpr int nbw = LU_NB;
    __shared__ double V[LU_LIST][65];
    __shared__ double Lt[LU_NB][LU_NB + 1];  // Lt[c][r] = L11(r, c), r > c
    __shared__ int sdst[LU_LIST], ssrc[LU_LIST];
    __shared__ int s_cnt;
    const int tid = threadIdx.x;
    if (tid < 64) {
        bool bad;
        const int cnt = lu_swap_list(ipiv, n, k0, nbw, sdst, ssrc, bad);
        if (tid == 0) s_cnt = cnt;
    }
    const int64_t cb = k0 + nbw + (int64_t)blockIdx.x * 64;
    const int cw = (int)(n - cb < 64 ? n - cb : 64);
    for (int e = tid; e < LU_NB * LU_NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r > c) Lt[c][r] = A[idx(k0 + r, k0 + c, lda)];
    }
    __syncthreads();
    const int cnt = s_cnt;
    // every touched row's values (the block row's own rows included) into V
    for (int e = tid; e < LU_LIST * 64; e += 256) {
        const int t = e & (LU_LIST - 1), c = e >> 7;
        if (t < cnt && c < cw) V[t][c] = A[idx(ssrc[t], cb + c, lda)];
    }
    __syncthreads();
    // rows below the block row that received another row's values
    for (int e = tid; e < LU_LIST * 64; e += 256) {
        const int t = e & (LU_LIST - 1), c = e >> 7;
        if (t >= nbw && t < cnt && c < cw && sdst[t] != ssrc[t]) A[idx(sdst[t], cb + c, lda)] = V[t][c];
    }
    // V[0..64) holds the interchanged block row; substitution down each column
    if (tid < 64) {
        double b[LU_NB];
#pragma unroll
        for (int r = 0; r < LU_NB; ++r) b[r] = V[r][tid];
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) {
            const double uc = b[c];
#pragma unroll
            for (int r = c + 1; r < LU_NB; ++r) b[r] = b[r] - Lt[c][r] * uc;
        }
#pragma unroll
        for (int r = 0; r < LU_NB; ++r) V[r][tid] = b[r];
        if (tid < cw) {
            const int64_t jc = cb + tid - (k0 + LU_NB);
#pragma unroll
            for (int r = 0; r < LU_NB; ++r) Ut[idx(jc, r, ldu)] = b[r];
        }
    }
    __syncthreads();
    for (int e = tid; e < LU_NB * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (c < cw) A[idx(k0 + r, cb + c, lda)] = V[r][c];
    }
}

// C (m x nn, ldc) -= X (m x kdim, ldx) Zt^T with Zt nn x kdim (ldz): 128 x 128
// output tiles over the whole grid, tiles taken column by column with
// consecutive runs per XCD; each wave computes a 64 x 64 quarter, C loaded
// up front (the k-loop is short), operands through a ring of four k-steps.
// The host keeps every byte offset below 2^31 and kdim a multiple of 16.
__global__ __launch_bounds__(256, 2) void k_gemm_sub(double* __restrict__ C, int64_t ldc, const double* __restrict__ X,
                                                     int64_t ldx, const double* __restrict__ Zt, int64_t ldz, int64_t m,
                                                     int64_t nn, int kdim) {
    constexpr int ES = 8, RG = 4;
    const int64_t TI = (m + 127) / 128, TJ = (nn + 127) / 128, ntiles = TI * TJ;
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;
    const int64_t I = t % TI, J = t / TI;
    const int tid = threadIdx.x, l = tid & 63, i = l & 15, g = l >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w >> 1, wc = w & 1;
    const int64_t sr0 = I * 128 + 64 * wr, sc0 = J * 128 + 64 * wc;
    if (sr0 >= m || sc0 >= nn) return;
    const int lc = (int)ldc, lx = (int)ldx, lz = (int)ldz;
    const int rmax = (int)(m - 1 - sr0 < 63 ? m - 1 - sr0 : 63);
    const int cmax = (int)(nn - 1 - sc0 < 63 ? nn - 1 - sc0 : 63);
    const __amdgpu_buffer_rsrc_t crs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(C + idx(sr0, sc0, ldc)), (short)0, 0x7fffffff, 0x00020000);
    // local indices clamped into the quarter: loads stay in bounds, stores are masked
    auto c_in = [&](int bi, int bj, int r) { return 16 * bi + i <= rmax && 16 * bj + tcol<double>(g, r) <= cmax; };
    auto c_off = [&](int bi, int bj, int r) {
        const int rr = min(16 * bi + i, rmax), cc = min(16 * bj + tcol<double>(g, r), cmax);
        return (rr + cc * lc) * ES;
    };
    // accumulators hold X Zt^T - C (negated as they are stored)
    f64x4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[bi][bj][r] =
                    -__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(crs, c_off(bi, bj, r), 0, 0));
    const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc((void*)X, (short)0, 0x7fffffff, 0x00020000);
    const __amdgpu_buffer_rsrc_t zrs = __builtin_amdgcn_make_buffer_rsrc((void*)Zt, (short)0, 0x7fffffff, 0x00020000);
    int xo[4], zo[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        xo[b] = ((int)sr0 + min(16 * b + i, rmax) + g * lx) * ES;
        zo[b] = ((int)sc0 + min(16 * b + i, cmax) + g * lz) * ES;
    }
    const int nks = kdim / 4;
    double xq[RG][4], zq[RG][4];
    auto fetch = [&](int slot, int kn) {
        const int kk = kn < nks ? kn : nks - 1;  // steps past the end re-read the last one
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            xq[slot][b] =
                __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(xrs, xo[b], kk * 4 * lx * ES, 0));
            zq[slot][b] =
                __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(zrs, zo[b], kk * 4 * lz * ES, 0));
        }
    };
#pragma unroll
    for (int p = 0; p < RG - 1; ++p) fetch(p, p);
    for (int ks = 0; ks < nks; ks += RG) {
#pragma unroll
        for (int s = 0; s < RG; ++s) {
            fetch((s + RG - 1) % RG, ks + s + RG - 1);
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mma_xzt(acc[bi][bj], xq[s][bi], zq[s][bj]);
        }
    }
    typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (c_in(bi, bj, r))
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, -acc[bi][bj][r]), crs,
                                                          c_off(bi, bj, r), 0, 0);
}

// After the factorisation: a panel barrier that gave up turns A into quiet
// NaNs and info into MG_INFO_SOLVE_ABORTED.
__global__ __launch_bounds__(256) void k_lu_check(double* A, int64_t lda, int64_t n, const LuSync* sy, int32_t* info) {
    if (ld_dev(&sy->err) == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = MG_INFO_SOLVE_ABORTED;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * 256)
        A[idx(e % n, e / n, lda)] = (double)NAN;
}

// ---------------------------------------------------------------- solve

// Per 64 interchanges (one wave each): their (destination, source) list.
__global__ __launch_bounds__(64) void k_lu_perm_lists(const int32_t* __restrict__ ipiv, int64_t n, int* lists,
                                                      LuSync* sy, const int32_t* info) {
    if (info && *info != 0) return;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const int cw = (int)(n - c0 < 64 ? n - c0 : 64);
    int* L = lists + (size_t)blockIdx.x * LU_LIST_WORDS;
    bool bad;
    const int cnt = lu_swap_list(ipiv, n, c0, cw, L + 1, L + 1 + LU_LIST, bad);
    if (threadIdx.x == 0) {
        L[0] = cnt;
        if (bad) atomicExch(&sy->bad, 1);
    }
}

// One workgroup: perm = the composition of the lists in order, starting
// from the identity (after all interchanges row i of B holds row perm[i] of
// the original B).
__global__ __launch_bounds__(256) void k_lu_perm_apply(int32_t* __restrict__ perm, int64_t n, const int* lists,
                                                       int nlists, const int32_t* info) {
    if (info && *info != 0) return;
    const int tid = threadIdx.x;
    for (int64_t i = tid; i < n; i += 256) perm[i] = (int32_t)i;
    __syncthreads();
    for (int b = 0; b < nlists; ++b) {
        const int* L = lists + (size_t)b * LU_LIST_WORDS;
        const int cnt = L[0];
        int v = 0, d = 0;
        const bool act = tid < cnt && L[1 + tid] != L[1 + LU_LIST + tid];
        if (act) {
            d = L[1 + tid];
            v = perm[L[1 + LU_LIST + tid]];
        }
        __syncthreads();
        if (act) perm[d] = v;
        __syncthreads();
    }
}

// After the sweeps: an ignored interchange outside 1..n turns B into quiet
// NaNs and info into MG_INFO_BAD_PIVOT.
__global__ __launch_bounds__(256) void k_lu_solve_check(double* B, int64_t ldb, int64_t n, int64_t nrhs,
                                                        const LuSync* sy, int32_t* info) {
    if (info && *info != 0) return;
    if (ld_dev(&sy->bad) == 0) return;
    __syncthreads();
    if (info && threadIdx.x == 0) *info = MG_INFO_BAD_PIVOT;
    for (int64_t e = threadIdx.x; e < n * nrhs; e += 256) B[idx(e % n, e / n, ldb)] = (double)NAN;
}

// ------------------------------------------------------------- host side

static int panel_groups(int64_t m) { return (int)cdiv(m, LU_ROWS); }

size_t getrf_work_bytes(int64_t n) {
    if (n == 0) return 0;
    const int gmax = panel_groups(n);
    return align_up((size_t)2 * (gmax + 1) * LU_SLOT * 8, 256) + 256 + align_up((size_t)n * LU_NB * 8, 256);
}

mg_status getrf_impl(mg_handle_t h, int64_t n, double* A, int64_t lda, int32_t* ipiv, void* work, int32_t* info) {
    hipStream_t st = h->stream;
    mg_status rc = set_info_zero(st, info);
    if (rc != MG_OK || n == 0) return rc;
    // 32-bit buffer offsets of the update's operands and C quarters
    if (((n + (int64_t)(LU_NB + 64) * lda) * 8 >= ((int64_t)1 << 31) - 65536) ||
        ((int64_t)n * LU_NB * 8 >= ((int64_t)1 << 31) - 65536))
        return MG_ERR_UNSUPPORTED;
    if (panel_groups(n) > h->cu_count) return MG_ERR_UNSUPPORTED;  // co-residency of the cooperative panel
    char* base = (char*)work;
    double* slots = (double*)base;
    LuSync* sy = (LuSync*)(base + align_up((size_t)2 * (panel_groups(n) + 1) * LU_SLOT * 8, 256));
    double* Ut = (double*)((char*)sy + 256);
    int lim = h->spin_limit < 0 ? LU_SPIN_LIMIT : h->spin_limit;
    hipLaunchKernelGGL(k_lu_reset, dim3(1), dim3(64), 0, st, sy);
    MG_LAUNCH_CHECK();
    unsigned arrivals = 0;
    for (int64_t k0 = 0; k0 < n; k0 += LU_NB) {
        int nbw = (int)std::min<int64_t>(LU_NB, n - k0);
        const int64_t m = n - k0;
        const int G = panel_groups(m);
        if ((rc = prof_begin(h, MG_PROF_LU_PANEL, st))) return rc;
        void* args[] = {(void*)&A,  (void*)&lda,      (void*)&n,    (void*)&k0,   (void*)&nbw, (void*)&slots,
                        (void*)&sy, (void*)&arrivals, (void*)&ipiv, (void*)&info, (void*)&lim};
        MG_HIP(hipLaunchCooperativeKernel((const void*)k_getf2_panel, dim3(G), dim3(256), args, 0, st));
        const double md = (double)m, bd = (double)nbw;
        if ((rc = prof_end(h, MG_PROF_LU_PANEL, md * bd * bd - bd * bd * bd / 3.0, 2.0 * md * bd * 8.0, st)))
            return rc;
        arrivals += (unsigned)G * (unsigned)nbw;
        if (k0 > 0) {
            hipLaunchKernelGGL(k_lu_swap_cols, dim3((unsigned)cdiv(k0, 64)), dim3(256), 0, st, A, lda, n, k0, nbw, k0,
                               (const int32_t*)ipiv);
            MG_LAUNCH_CHECK();
        }
        const int64_t nr = n - k0 - nbw;
        if (nr > 0) {
            // nr > 0 implies a full-width panel (nbw == LU_NB)
            hipLaunchKernelGGL(k_lu_row_block, dim3((unsigned)cdiv(nr, 64)), dim3(256), 0, st, A, lda, n, k0,
                               (const int32_t*)ipiv, Ut, nr);
            MG_LAUNCH_CHECK();
            const int64_t tiles = cdiv(nr, 128) * cdiv(nr, 128);
            if ((rc = prof_begin(h, MG_PROF_LU_UPDATE, st))) return rc;
            hipLaunchKernelGGL(k_gemm_sub, dim3((unsigned)(8 * cdiv(tiles, 8))), dim3(256), 0, st,
                               A + idx(k0 + nbw, k0 + nbw, lda), lda, (const double*)(A + idx(k0 + nbw, k0, lda)), lda,
                               (const double*)Ut, nr, nr, nr, LU_NB);
            MG_LAUNCH_CHECK();
            const double nd = (double)nr;
            if ((rc = prof_end(h, MG_PROF_LU_UPDATE, 2.0 * nd * nd * LU_NB, (2.0 * nd * nd + 2.0 * nd * LU_NB) * 8.0,
                               st)))
                return rc;
        }
    }
    hipLaunchKernelGGL(k_lu_check, dim3((unsigned)std::min<int64_t>(cdiv(n * n, 256), 1024)), dim3(256), 0, st, A,
                       lda, n, (const LuSync*)sy, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

static size_t lists_bytes(int64_t n) { return align_up((size_t)cdiv(n, 64) * LU_LIST_WORDS * 4, 256); }

size_t getrs_work_bytes(int64_t n, int64_t nrhs) {
    if (n == 0 || nrhs == 0) return 0;
    return align_up((size_t)n * nrhs * 8, 256) + 2 * sweep_words_bytes(nrhs) + 256 + align_up((size_t)n * 4, 256) +
           lists_bytes(n);
}

mg_status getrs_impl(mg_handle_t h, int64_t n, int64_t nrhs, const double* LU, int64_t lda, const int32_t* ipiv,
                     double* B, int64_t ldb, void* work, int32_t* info) {
    if (n == 0 || nrhs == 0) return MG_OK;
    hipStream_t st = h->stream;
    mg_status rc;
    char* p = (char*)work;
    double* Y = (double*)p;
    p += align_up((size_t)n * nrhs * 8, 256);
    void* words = p;
    p += 2 * sweep_words_bytes(nrhs);
    LuSync* sy = (LuSync*)p;
    p += 256;
    int32_t* perm = (int32_t*)p;
    p += align_up((size_t)n * 4, 256);
    int* lists = (int*)p;
    if ((rc = prof_begin(h, MG_PROF_SOLVE, st))) return rc;
    hipLaunchKernelGGL(k_lu_reset, dim3(1), dim3(64), 0, st, sy);
    MG_LAUNCH_CHECK();
    const int nl = (int)cdiv(n, 64);
    hipLaunchKernelGGL(k_lu_perm_lists, dim3((unsigned)nl), dim3(64), 0, st, ipiv, n, lists, sy,
                       (const int32_t*)info);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_lu_perm_apply, dim3(1), dim3(256), 0, st, perm, n, (const int*)lists, nl,
                       (const int32_t*)info);
    MG_LAUNCH_CHECK();
    if ((rc = lu_sweeps(h, n, nrhs, LU, lda, perm, B, ldb, Y, words, info))) return rc;
    hipLaunchKernelGGL(k_lu_solve_check, dim3(1), dim3(256), 0, st, B, ldb, n, nrhs, (const LuSync*)sy, info);
    MG_LAUNCH_CHECK();
    const double nd = (double)n;
    return prof_end(h, MG_PROF_SOLVE, 2.0 * nd * nd * (double)nrhs, (nd * nd + 4.0 * nd * (double)nrhs) * 8.0, st);
}

}  // namespace mg
