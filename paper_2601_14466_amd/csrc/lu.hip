// lu.hip -- the paper's general solve (JAXMg, "Software design", lu_solve
// bullet: A x = b for a general nonsingular A through a pivoted LU
// factorisation): P A = L U by Gaussian elimination with partial pivoting,
// then the row interchanges and the two triangular solves.  FP64.
//
// Two-level blocked right-looking factorisation: outer block columns of
// nb2 = 256 or 512 (512 from n = 16384; the handle's block size selects
// either), each factored as inner panels of LU_NB = 64.
//   1. k_getf2_panel: the inner panel (rows k0..n-1, 64 columns) with partial
//      pivoting, a cooperative launch of G workgroups that each keep 256
//      consecutive rows of the panel in LDS, one row per thread.  For every
//      column j each workgroup publishes its largest |entry| (the first row
//      on ties; reduced by DPP moves and the gfx950 row swaps) with that
//      row's values, and the owner of row j publishes row j, into write-once
//      slots (one per column and workgroup, reset to a sentinel before the
//      panel); every workgroup polls the G headers until all are written,
//      picks the same winner, fetches its row, and the owners of rows j and
//      p exchange them before the local rank-1 update.  Pivot choice and the
//      order of each entry's updates are those of column-by-column
//      elimination.
//   2. k_lu_swap_cols: the panel's interchanges applied to the columns left
//      of it and to those right of the outer block column (which no update
//      of this outer block has reached yet, so moving their rows keeps them
//      consistent).
//   3. k_lu_row_block (with interchanges): the rest of the outer block row,
//      U12 = L11^{-1} A12 by forward substitution with the panel's unit lower
//      L11 (one lane per column), then k_gemm_sub<false>: the rank-64 update
//      of the rest of the outer block column, so the next inner panel sees
//      every earlier one.
//   4. After the inner panels, the outer block row right of the outer
//      block: U12 = L11^{-1} A12 with the nb2 x nb2 unit lower L11, by 64-row
//      blocks (k_lu_row_block without interchanges, then a rank-64
//      k_gemm_sub<false> of the rows below inside the outer block).
//   5. k_gemm_sub<true>: A22 -= L21 U12 of rank nb2 on the FP64 matrix pipe
//      over the trailing matrix (128 x 128 output tiles of four 64 x 64 wave
//      quarters in bands of 8 tile rows, operands streamed from memory
//      straight into registers through a ring of four k-steps, C folded into
//      the k-loop).
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

constexpr int LU_NB = 64;                       // inner panel width
constexpr int LU_NB2 = 512;                     // widest outer block (rank of the trailing update)
constexpr int LU_ROWS = 256;                    // panel rows per workgroup (one per thread)
constexpr int LU_HDR = 2;                       // slot header: |value|, row
constexpr int LU_SLOT = LU_HDR + LU_NB;         // doubles per slot
constexpr int LU_LIST = 2 * LU_NB;              // rows one block of 64 interchanges can touch
constexpr int LU_LIST_WORDS = 1 + 2 * LU_LIST;  // count, destination rows, source rows
constexpr int LU_SPIN_LIMIT = 1 << 22;          // default polls before a wait gives up

struct LuSync {
    int err;  // set when a panel wait gave up
    int bad;  // the solve: an interchange outside 1..n was ignored
    int pad[2];
};

// Panel slots are write-once per panel: reset to a signalling NaN (never
// produced by arithmetic; published values are canonicalised so that an
// input NaN cannot carry this payload), written with device-coherent stores
// and polled with device-coherent loads until no value is the sentinel.
__device__ __forceinline__ double lu_sentinel() { return __builtin_bit_cast(double, 0x7ff4d1e5a1f00d01ull); }
__device__ __forceinline__ bool lu_is_sentinel(double v) {
    return __builtin_bit_cast(unsigned long long, v) == 0x7ff4d1e5a1f00d01ull;
}
__device__ __forceinline__ double lu_canon(double v) { return v == v ? v : (double)NAN; }
__device__ __forceinline__ double ld_dev(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_dev(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// (v, r) pairs: larger v wins, the smaller r on ties.  v < 0 marks "no candidate".
__device__ __forceinline__ void argmax_merge(double& v, int& r, double ov, int orr) {
    if (ov > v || (ov == v && orr < r)) {
        v = ov;
        r = orr;
    }
}

// A double moved across lanes by a DPP pattern (both halves; every lane
// reads a valid lane for the patterns used here).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// max(v over the pairs of rows of 16 lanes that a permlane swap exchanges)
template <bool B32>
__device__ __forceinline__ double swap_max_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    const auto l = B32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                       : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = B32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                       : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double d0 = __builtin_bit_cast(double, ((unsigned long long)h[0] << 32) | l[0]);
    const double d1 = __builtin_bit_cast(double, ((unsigned long long)h[1] << 32) | l[1]);
    return fmax(d0, d1);
}
// Largest v of the wave (no NaN among the values): quad, half-row and row
// steps by DPP, then the two gfx950 row swaps.
__device__ __forceinline__ double wave_max_f64(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));   // quad_perm [1,0,3,2]
    v = fmax(v, dpp_f64<0x4E>(v));   // quad_perm [2,3,0,1]
    v = fmax(v, dpp_f64<0x141>(v));  // row_half_mirror
    v = fmax(v, dpp_f64<0x140>(v));  // row_mirror
    v = swap_max_f64<false>(v);
    return swap_max_f64<true>(v);
}
// Workgroup argmax of (v, r) over 256 threads (v >= 0 candidates, -1 none):
// each wave takes its largest v and, among the lanes holding it, the first
// lane's r (callers number r in lane order, so that is the smallest r); the
// four wave results meet in LDS.  Every thread returns the same pair.
__device__ __forceinline__ void block_argmax(double v, int r, double* rv, int* rr, double& ov, int& orr) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double m = wave_max_f64(v);
    const unsigned long long hit = __ballot(v == m);
    const int first = __ffsll((long long)hit) - 1;
    const int rw = __builtin_amdgcn_readlane(r, first);
    if (lane == 0) {
        rv[w] = m;
        rr[w] = m >= 0.0 ? rw : INT_MAX;
    }
    __syncthreads();
    ov = rv[0];
    orr = rr[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) argmax_merge(ov, orr, rv[q], rr[q]);
}

__global__ void k_lu_reset(LuSync* sy) {
    if (threadIdx.x == 0) *sy = LuSync{0, 0, {0, 0}};
}

__global__ __launch_bounds__(256) void k_lu_fill_sentinel(double* p, int64_t cnt) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256)
        p[e] = lu_sentinel();
}

// Panel factorisation (cooperative launch of G = ceil(m / 256) workgroups,
// thread t of workgroup q holding panel row 256 q + t in LDS).
// cur: this panel's slots, LU_NB x gs entries of LU_SLOT doubles (entry
// (j, q): workgroup q's candidate for column j; entry (j, gs - 1): row j);
// nxt: the next panel's slots, whose entries this launch resets (workgroup q
// those of workgroup q, workgroup 0 also the row-j entries).
__global__ __launch_bounds__(256, 1) void k_getf2_panel(double* __restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                        int nbw, double* cur, double* nxt, int gs, LuSync* sy,
                                                        int32_t* __restrict__ ipiv, int32_t* __restrict__ info,
                                                        int spin_limit) {
    __shared__ double P[LU_ROWS][LU_NB + 1];
    __shared__ double urow[LU_NB], jrow[LU_NB], wrow[LU_NB];
    __shared__ double red_v[2][4];
    __shared__ int red_r[2][4];
    const int tid = threadIdx.x, G = gridDim.x, wg = blockIdx.x;
    const int jslot = gs - 1;
    const int64_t m = n - k0;
    const int64_t row0 = (int64_t)wg * LU_ROWS;  // first panel row (relative to k0) of this workgroup
    const int R = (int)(m - row0 < LU_ROWS ? m - row0 : LU_ROWS);
    for (int e = tid; e < LU_NB * LU_SLOT; e += 256) {
        const int j = e / LU_SLOT, x = e - j * LU_SLOT;
        nxt[((size_t)j * gs + wg) * LU_SLOT + x] = lu_sentinel();
        if (wg == 0) nxt[((size_t)j * gs + jslot) * LU_SLOT + x] = lu_sentinel();
    }
    for (int c = 0; c < nbw; ++c)
        if (tid < R) P[tid][c] = A[idx(k0 + row0 + tid, k0 + c, lda)];
    __syncthreads();
    // a spin limit of 0 (host setting) gives up every wait of a panel with
    // more than one workgroup, without waiting
    bool gave_up = spin_limit == 0 && G > 1;
    if (gave_up && tid == 0) atomicExch(&sy->err, 1);
    double piv_prev = 0.0;
    // Column j's step in three parts: (1) the candidate and its header, which
    // the other workgroups wait for, go out first; (2) then the rank-1 update
    // of columns j + 1.. by the previous pivot row, deferred from step j - 1,
    // overlaps that round trip, after which the candidate row and row j are
    // complete and published; (3) the winner, the interchange, and the
    // scaling of column j with the update of column j + 1 only (all the next
    // candidate needs).
    for (int j = 0; j < nbw; ++j) {
        double* E = cur + (size_t)j * gs * LU_SLOT;  // column j's entries
        // ---- (1) this workgroup's candidate: rows >= j, NaN entries never win
        double v = -1.0;
        if (tid < R && row0 + tid >= j) {
            const double a = fabs(P[tid][j]);
            if (a == a) v = a;
        }
        double bv;
        int br;
        block_argmax(v, tid, red_v[0], red_r[0], bv, br);
        double* me = E + (size_t)wg * LU_SLOT;
        const bool ownj = j >= row0 && j < row0 + R;
        if (tid == 0) {
            st_dev(&me[0], bv);
            st_dev(&me[1], bv >= 0.0 ? (double)(row0 + br) : -1.0);
        }
        // ---- (2) the deferred update a_rc -= l_r u_c, c > j, by pivot j - 1
        // (urow and the multipliers l_r = P[r][j - 1] of step j - 1)
        if (j > 0 && piv_prev != 0.0 && tid < R && row0 + tid > j - 1) {
            const double l = P[tid][j - 1];
#pragma unroll 8
            for (int c = j + 1; c < nbw; ++c) P[tid][c] = P[tid][c] - l * urow[c];
        }
        __syncthreads();
        if (bv >= 0.0 && tid < nbw) st_dev(&me[LU_HDR + tid], lu_canon(P[br][tid]));
        if (ownj && tid < nbw) st_dev(&E[(size_t)jslot * LU_SLOT + LU_HDR + tid], lu_canon(P[j - row0][tid]));
        // ---- (3) every workgroup's header (a thread each), polled until written
        double hv = -1.0;
        int hr = INT_MAX;
        for (int spins = 0;; ++spins) {
            bool ok = true;
            hv = -1.0;
            hr = INT_MAX;
            if (tid < G) {
                const double a = ld_dev(&E[(size_t)tid * LU_SLOT]);
                const double rr = ld_dev(&E[(size_t)tid * LU_SLOT + 1]);
                ok = !lu_is_sentinel(a) && !lu_is_sentinel(rr);
                if (a >= 0.0 && rr >= (double)j && rr < (double)m) {
                    hv = a;
                    hr = (int)rr;
                }
            }
            if (__syncthreads_and(ok) || gave_up) break;
            if ((spins & 31) == 31) {
                const int e = (tid == 0) ? ld_dev(&sy->err) : 0;
                if (__syncthreads_or(spins > spin_limit || e != 0)) {
                    gave_up = true;
                    if (tid == 0) atomicExch(&sy->err, 1);
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        // the winner (every workgroup alike; workgroup q's rows follow q)
        double gv;
        int gr;
        block_argmax(hv, hr, red_v[1], red_r[1], gv, gr);
        const int pw = gv >= 0.0 ? gr / LU_ROWS : 0;  // workgroup whose slot holds the candidate row
        // row j and the candidate row, polled until written
        for (int spins = 0;; ++spins) {
            bool ok = true;
            if (tid < nbw) {
                const double jr = ld_dev(&E[(size_t)jslot * LU_SLOT + LU_HDR + tid]);
                const double wr = gv >= 0.0 ? ld_dev(&E[(size_t)pw * LU_SLOT + LU_HDR + tid]) : 0.0;
                ok = !lu_is_sentinel(jr) && !lu_is_sentinel(wr);
                jrow[tid] = jr;
                wrow[tid] = wr;
            }
            if (__syncthreads_and(ok) || gave_up) break;
            if ((spins & 31) == 31) {
                const int e = (tid == 0) ? ld_dev(&sy->err) : 0;
                if (__syncthreads_or(spins > spin_limit || e != 0)) {
                    gave_up = true;
                    if (tid == 0) atomicExch(&sy->err, 1);
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        // a NaN diagonal entry stays the pivot (a sequential scan starting
        // from it never replaces it); so does row j when nothing qualifies
        const int64_t p = (gv < 0.0 || jrow[j] != jrow[j]) ? (int64_t)j : (int64_t)gr;
        if (tid < nbw) urow[tid] = (p == j) ? jrow[tid] : wrow[tid];
        __syncthreads();
        const double piv = urow[j];
        if (wg == 0 && tid == 0) {
            ipiv[k0 + j] = (int32_t)(k0 + p + 1);
            if (piv == 0.0 && *info == 0) *info = (int32_t)(k0 + j + 1);
        }
        // interchange rows j and p (their owners), then scale column j and
        // update column j + 1; the other columns wait for step j + 1
        if (p != j) {
            if (ownj && tid < nbw) P[j - row0][tid] = urow[tid];
            if (p >= row0 && p < row0 + R && tid < nbw) P[p - row0][tid] = jrow[tid];
        }
        __syncthreads();
        if (piv != 0.0 && tid < R && row0 + tid > j) {
            const double l = P[tid][j] / piv;
            P[tid][j] = l;
            if (j + 1 < nbw) P[tid][j + 1] = P[tid][j + 1] - l * urow[j + 1];
        }
        piv_prev = piv;
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

// Interchanges of the panel at k0 (nbw of them) applied to the columns
// [0, nleft) and [cr0, n): 64 columns per workgroup, every touched value read
// into LDS before any is written.
__global__ __launch_bounds__(256) void k_lu_swap_cols(double* __restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                      int nbw, int64_t nleft, int64_t cr0,
                                                      const int32_t* __restrict__ ipiv) {
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
    const int64_t ncols = nleft + (n - cr0);
    const int64_t cb = (int64_t)blockIdx.x * 64;
    const int cw = (int)(ncols - cb < 64 ? ncols - cb : 64);
    auto col = [&](int c) { return cb + c < nleft ? cb + c : cb + c - nleft + cr0; };
    for (int e = tid; e < LU_LIST * 64; e += 256) {
        const int t = e & (LU_LIST - 1), c = e >> 7;
        if (t < cnt && c < cw && sdst[t] != ssrc[t]) V[t][c] = A[idx(ssrc[t], col(c), lda)];
    }
    __syncthreads();
    for (int e = tid; e < LU_LIST * 64; e += 256) {
        const int t = e & (LU_LIST - 1), c = e >> 7;
        if (t < cnt && c < cw && sdst[t] != ssrc[t]) A[idx(sdst[t], col(c), lda)] = V[t][c];
    }
}

// Block row of a full-width panel at k0 (rows k0..k0+63) over the columns
// [c0, c0 + ncols), 64 per workgroup: with SWAPS, the panel's interchanges
// first (the block row's rows and every row they touch go through LDS; the
// touched rows below the block row are written back); then
// U12 = L11^{-1} A12 (L11 = the panel's unit lower 64 x 64 block) by forward
// substitution, one lane per column of wave 0, stored over A12 and, when Ut
// is given, transposed into Ut (row j - c0 holds column j's 64 values).
__global__ __launch_bounds__(256) void k_lu_row_block(double* __restrict__ A, int64_t lda, int64_t n, int64_t k0,
                                                      int64_t c0, int64_t ncols, int swaps,
                                                      const int32_t* __restrict__ ipiv, double* __restrict__ Ut,
                                                      int64_t ldu) {
    constexpr int nbw = LU_NB;
    __shared__ double V[LU_LIST][65];
    __shared__ double Lt[LU_NB][LU_NB + 1];  // Lt[c][r] = L11(r, c), r > c
    __shared__ int sdst[LU_LIST], ssrc[LU_LIST];
    __shared__ int s_cnt;
    const int tid = threadIdx.x;
    if (swaps && tid < 64) {
        bool bad;
        const int cnt = lu_swap_list(ipiv, n, k0, nbw, sdst, ssrc, bad);
        if (tid == 0) s_cnt = cnt;
    }
    const int64_t cb = c0 + (int64_t)blockIdx.x * 64;
    const int cw = (int)(c0 + ncols - cb < 64 ? c0 + ncols - cb : 64);
    for (int e = tid; e < LU_NB * LU_NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r > c) Lt[c][r] = A[idx(k0 + r, k0 + c, lda)];
    }
    __syncthreads();
    if (swaps) {
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
    } else {
        for (int e = tid; e < LU_NB * 64; e += 256) {
            const int r = e & 63, c = e >> 6;
            if (c < cw) V[r][c] = A[idx(k0 + r, cb + c, lda)];
        }
        __syncthreads();
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
    }
    __syncthreads();
    for (int e = tid; e < LU_NB * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (c < cw) A[idx(k0 + r, cb + c, lda)] = V[r][c];
    }
    // U12^T: column j - c0 of the block row is row j - c0 of Ut (lanes
    // along the block row's columns, so each store is contiguous)
    if (Ut) {
        for (int e = tid; e < LU_NB * 64; e += 256) {
            const int c = e & 63, r = e >> 6;
            if (c < cw) Ut[idx(cb + c - c0, r, ldu)] = V[r][c];
        }
    }
}

// C (m x nn, ldc) -= X Z with X m x kdim (column-major, ldx) and Z kdim x nn
// (column-major, ldz: the block row U12 as it lies in A; with ZT, Z^T given
// instead, nn x kdim column-major, read along its rows like X).  128 x 128 output
// tiles, each XCD taking a contiguous run of tiles numbered in bands of 8
// tile rows, column by column inside a band (the workgroups an XCD holds at
// once cover an 8 x 8 patch and share its operand blocks in L2); each wave
// computes a 64 x 64 quarter.  Operands stream straight into registers
// through a ring of four k-steps: lane (i, g) of k-step s reads X row
// 16 b + i, column 4 s + g, and Z column 16 b + i, row 4 s + g (32 contiguous
// bytes of a column per 4 lanes; with ZT row 16 b + i, column 4 s + g of
// Z^T).  FOLD (rank 256 / 512): C is folded into the
// k-loop one 16 x 16 piece at a time; otherwise (rank 64) C is loaded up
// front.  The accumulators hold X Z - C and are negated as they are stored.
// The host keeps every byte offset below 2^31 and kdim a multiple of 16
// (of 256 with FOLD).
template <bool FOLD, bool ZT>
__global__ __launch_bounds__(256, 2) void k_gemm_sub(double* __restrict__ C, int64_t ldc, const double* __restrict__ X,
                                                     int64_t ldx, const double* __restrict__ Z, int64_t ldz, int64_t m,
                                                     int64_t nn, int kdim) {
    constexpr int ES = 8, RG = 4;
    const int64_t TI = (m + 127) / 128, TJ = (nn + 127) / 128, ntiles = TI * TJ;
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;
    const int64_t band = t / (8 * TJ), rem = t - band * 8 * TJ;
    const int64_t bh = TI - band * 8 < 8 ? TI - band * 8 : 8;
    const int64_t I = __builtin_amdgcn_readfirstlane((int)(band * 8 + rem % bh));
    const int64_t J = __builtin_amdgcn_readfirstlane((int)(rem / bh));
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
    auto c_load = [&](int bi, int bj, int r) -> double {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(crs, c_off(bi, bj, r), 0, 0));
    };
    f64x4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] = FOLD ? 0.0 : -c_load(bi, bj, r);
    const __amdgpu_buffer_rsrc_t xrs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(X + sr0), (short)0, 0x7fffffff, 0x00020000);
    // ZT: Z given transposed (nn x kdim, leading dimension ldz), read like X
    const __amdgpu_buffer_rsrc_t zrs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(ZT ? Z + sc0 : Z + idx(0, sc0, ldz)), (short)0, 0x7fffffff, 0x00020000);
    int xo[4], zo[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        xo[b] = (min(16 * b + i, rmax) + g * lx) * ES;
        zo[b] = ZT ? (min(16 * b + i, cmax) + g * lz) * ES : (min(16 * b + i, cmax) * lz + g) * ES;
    }
    const int nks = kdim / 4;
    double xq[RG][4], zq[RG][4];
    auto fetch = [&](int slot, int kn) {
        const int kk = kn < nks ? kn : nks - 1;  // steps past the end re-read the last one
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            xq[slot][b] =
                __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(xrs, xo[b], kk * 4 * lx * ES, 0));
            zq[slot][b] = __builtin_bit_cast(
                double, __builtin_amdgcn_raw_buffer_load_b64(zrs, zo[b], kk * 4 * (ZT ? lz : 1) * ES, 0));
        }
    };
#pragma unroll
    for (int p = 0; p < RG - 1; ++p) fetch(p, p);
    auto body = [&](int ks) {
#pragma unroll
        for (int s = 0; s < RG; ++s) {
            fetch((s + RG - 1) % RG, ks + s + RG - 1);
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mma_xzt(acc[bi][bj], xq[s][bi], zq[s][bj]);
        }
    };
    if constexpr (FOLD) {
        const int per_q = nks / (16 * RG);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            f64x4 cv;
#pragma unroll
            for (int r = 0; r < 4; ++r) cv[r] = c_load(q >> 2, q & 3, r);
            for (int u = 0; u < per_q; ++u) body((q * per_q + u) * RG);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[q >> 2][q & 3][r] -= cv[r];
        }
    } else {
        for (int ks = 0; ks < nks; ks += RG) body(ks);
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

// After the factorisation: a panel wait that gave up turns A into quiet
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

// Workspace: two slot sets (LU_NB x (G + 1) entries each, G the first
// panel's workgroups) and the sync words.
static size_t slot_set_doubles(int64_t n) { return (size_t)LU_NB * (panel_groups(n) + 1) * LU_SLOT; }

// Workspace: the two slot sets, the sync words, and U12^T of an outer block
// row (n x LU_NB2).
size_t getrf_work_bytes(int64_t n) {
    if (n == 0) return 0;
    return align_up(2 * slot_set_doubles(n) * 8, 256) + 256 + align_up((size_t)n * LU_NB2 * 8, 256);
}

template <bool FOLD, bool ZT = false>
static mg_status gemm_sub(hipStream_t st, double* C, int64_t ldc, const double* X, int64_t ldx, const double* Z,
                          int64_t ldz, int64_t m, int64_t nn, int kdim) {
    if (m <= 0 || nn <= 0) return MG_OK;
    const int64_t tiles = cdiv(m, 128) * cdiv(nn, 128);
    hipLaunchKernelGGL((k_gemm_sub<FOLD, ZT>), dim3((unsigned)(8 * cdiv(tiles, 8))), dim3(256), 0, st, C, ldc, X, ldx,
                       Z, ldz, m, nn, kdim);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

// C (m x nn, ldc) -= X (m x kdim, ldx) Z (kdim x nn, ldz), kdim % 16 == 0 (a
// multiple of 256: the C-folding variant); the caller keeps every byte
// offset below 2^31.
mg_status gemm_sub_f64(hipStream_t st, double* C, int64_t ldc, const double* X, int64_t ldx, const double* Z,
                       int64_t ldz, int64_t m, int64_t nn, int64_t kdim) {
    if (kdim % 16 != 0) return MG_ERR_UNSUPPORTED;
    return kdim % 256 == 0 ? gemm_sub<true>(st, C, ldc, X, ldx, Z, ldz, m, nn, (int)kdim)
                           : gemm_sub<false>(st, C, ldc, X, ldx, Z, ldz, m, nn, (int)kdim);
}

mg_status getrf_impl(mg_handle_t h, int64_t n, double* A, int64_t lda, int32_t* ipiv, void* work, int32_t* info) {
    hipStream_t st = h->stream;
    mg_status rc = set_info_zero(st, info);
    if (rc != MG_OK || n == 0) return rc;
    // 32-bit buffer offsets of the update's operands (X: up to 512 columns from its
    // base row; Z and C: 64 columns from a wave's base column)
    if ((n + (int64_t)(LU_NB2 + 64) * lda) * 8 >= ((int64_t)1 << 31) - 65536) return MG_ERR_UNSUPPORTED;
    const int64_t nb2 = (h->nb == 256 || h->nb == 512) ? h->nb : (n >= 16384 ? 512 : 256);
    if (panel_groups(n) > h->cu_count) return MG_ERR_UNSUPPORTED;  // co-residency of the cooperative panel
    const int gs = panel_groups(n) + 1;
    double* sets[2] = {(double*)work, (double*)work + slot_set_doubles(n)};
    LuSync* sy = (LuSync*)((char*)work + align_up(2 * slot_set_doubles(n) * 8, 256));
    double* Ut = (double*)((char*)sy + 256);
    int lim = h->spin_limit < 0 ? LU_SPIN_LIMIT : h->spin_limit;
    hipLaunchKernelGGL(k_lu_reset, dim3(1), dim3(64), 0, st, sy);
    MG_LAUNCH_CHECK();
    const int64_t nfill = (int64_t)(2 * slot_set_doubles(n));
    hipLaunchKernelGGL(k_lu_fill_sentinel, dim3((unsigned)std::min<int64_t>(cdiv(nfill, 256), 1024)), dim3(256), 0,
                       st, sets[0], nfill);
    MG_LAUNCH_CHECK();
    int set = 0;
    for (int64_t K0 = 0; K0 < n; K0 += nb2) {
        const int64_t W = std::min<int64_t>(nb2, n - K0);  // < nb2 only for the last outer block
        const int64_t kend = K0 + W;
        // the outer block column, inner panel by inner panel; the columns
        // right of it only take the interchanges (no update of this outer
        // block has reached them yet, so moving their rows is consistent)
        for (int64_t k0 = K0; k0 < kend; k0 += LU_NB) {
            int nbw = (int)std::min<int64_t>(LU_NB, kend - k0);
            const int64_t m = n - k0;
            const int G = panel_groups(m);
            if ((rc = prof_begin(h, MG_PROF_LU_PANEL, st))) return rc;
            double* cur = sets[set];
            double* nxt = sets[set ^ 1];
            int gsv = gs;
            void* args[] = {(void*)&A,   (void*)&lda, (void*)&n,  (void*)&k0,   (void*)&nbw,  (void*)&cur,
                            (void*)&nxt, (void*)&gsv, (void*)&sy, (void*)&ipiv, (void*)&info, (void*)&lim};
            MG_HIP(hipLaunchCooperativeKernel((const void*)k_getf2_panel, dim3(G), dim3(256), args, 0, st));
            const double md = (double)m, bd = (double)nbw;
            if ((rc = prof_end(h, MG_PROF_LU_PANEL, md * bd * bd - bd * bd * bd / 3.0, 2.0 * md * bd * 8.0, st)))
                return rc;
            set ^= 1;
            const int64_t nsw = k0 + (n - kend);
            if (nsw > 0) {
                hipLaunchKernelGGL(k_lu_swap_cols, dim3((unsigned)cdiv(nsw, 64)), dim3(256), 0, st, A, lda, n, k0, nbw,
                                   k0, kend, (const int32_t*)ipiv);
                MG_LAUNCH_CHECK();
            }
            const int64_t k1 = k0 + nbw;
            if (k1 >= kend) continue;  // nbw == LU_NB below
            hipLaunchKernelGGL(k_lu_row_block, dim3((unsigned)cdiv(kend - k1, 64)), dim3(256), 0, st, A, lda, n, k0,
                               k1, kend - k1, 1, (const int32_t*)ipiv, (double*)nullptr, (int64_t)1);
            MG_LAUNCH_CHECK();
            // rank-64 update of the rest of the outer block column
            if ((rc = prof_begin(h, MG_PROF_TRAILING_NARROW, st))) return rc;
            if ((rc = gemm_sub<false>(st, A + idx(k1, k1, lda), lda, A + idx(k1, k0, lda), lda, A + idx(k0, k1, lda),
                                      lda, n - k1, kend - k1, LU_NB)))
                return rc;
            const double a1 = (double)(n - k1) * (double)(kend - k1);
            if ((rc = prof_end(h, MG_PROF_TRAILING_NARROW, 2.0 * LU_NB * a1,
                               (2.0 * a1 + LU_NB * (double)(n - k1 + kend - k1)) * 8.0, st)))
                return rc;
        }
        const int64_t mr = n - kend;
        if (mr <= 0) continue;
        // the outer block row right of it: U12 = L11^{-1} A12 with the
        // nb2 x nb2 unit lower L11, by 64-row blocks (substitution, then a
        // rank-64 update of the block rows below inside the outer block)
        for (int64_t k0 = K0; k0 < kend; k0 += LU_NB) {
            hipLaunchKernelGGL(k_lu_row_block, dim3((unsigned)cdiv(mr, 64)), dim3(256), 0, st, A, lda, n, k0, kend, mr,
                               0, (const int32_t*)ipiv, Ut + (k0 - K0) * mr, mr);
            MG_LAUNCH_CHECK();
            const int64_t k1 = k0 + LU_NB;
            if (k1 < kend) {
                if ((rc = prof_begin(h, MG_PROF_TRAILING_NARROW, st))) return rc;
                if ((rc = gemm_sub<false>(st, A + idx(k1, kend, lda), lda, A + idx(k1, k0, lda), lda,
                                          A + idx(k0, kend, lda), lda, kend - k1, mr, LU_NB)))
                    return rc;
                const double a2 = (double)(kend - k1) * (double)mr;
                if ((rc = prof_end(h, MG_PROF_TRAILING_NARROW, 2.0 * LU_NB * a2,
                                   (2.0 * a2 + LU_NB * (double)(kend - k1 + mr)) * 8.0, st)))
                    return rc;
            }
        }
        // rank-nb2 update of the trailing matrix
        if ((rc = prof_begin(h, MG_PROF_LU_UPDATE, st))) return rc;
        if ((rc = gemm_sub<true, true>(st, A + idx(kend, kend, lda), lda, A + idx(kend, K0, lda), lda,
                                       (const double*)Ut, mr, mr, mr, (int)W)))
            return rc;
        const double md = (double)mr;
        if ((rc = prof_end(h, MG_PROF_LU_UPDATE, 2.0 * (double)W * md * md, (2.0 * md * md + 2.0 * (double)W * md) * 8.0,
                           st)))
            return rc;
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
