// potrf.hip -- blocked right-looking Cholesky A = L L^T (lower, column-major)
// on gfx950.  Paper: JAXMg "Software design", potrs bullet (Cholesky solve);
// the block size is the paper's tile size T_A.
//
// Step k of the factorisation (block columns of width nb):
//   1. k_factor_block : L_kk = chol(A_kk), one workgroup, FP64 arithmetic.
//   2. k_trsm_panel   : L_ik = A_ik L_kk^{-T} for the m = n - (k+1) nb rows
//                       below, one wave per 16 or 32 rows, MFMA + shuffle solves.
//   3. k_syrk_lower   : lower(A_22) -= L_ik L_ik^T, FP64 MFMA on 128 x 128
//                       tiles (about n^3/3 of the n^3/3 + O(n^2) flops).
#include <algorithm>
#include <cmath>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

__global__ void k_set_info_zero(int32_t* info) {
    if (threadIdx.x == 0) *info = 0;
}

mg_status set_info_zero(hipStream_t s, int32_t* info) {
    hipLaunchKernelGGL(k_set_info_zero, dim3(1), dim3(64), 0, s, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Diagonal-block factor.  One workgroup of W = 4 waves factors the s x s block
// at A (s <= FB_MAX = 128) in place, right-looking over 16-wide block columns,
// FP64 arithmetic whatever the storage type S (the mixed-precision path keeps
// the diagonal blocks in FP64).
//   - Wave w owns tile rows ra = w and rb = 7 - w of the lower triangle: 9
//     tiles of 16 x 16 held in registers for the whole factorisation.  Slot t
//     holds tile (ra, t) for t <= ra and tile (rb, 8 - t) otherwise, so in
//     the unrolled slot loops every tile column is a compile-time constant and
//     only the two row bases are run-time values (this keeps the LDS operand
//     addresses in immediates and the kernel free of register spills).
//   - Step j: the owner of (j, j) has factored it (factor16) and published
//     L_jj pre-scaled by its pivots.  Barrier.  Owners of tiles (I, j), I > j,
//     solve them (solve16s) and publish them to the LDS copy of block column
//     j.  Barrier.  Every wave applies column j to its tiles (I, J), J > j
//     (4 MFMAs each, both operands from LDS), starting with column j + 1; the
//     owner of (j + 1, j + 1) factors it as soon as its own update is in,
//     while the other waves are still updating.
//   - The tiles are written back to A once, at the end.
// On a non-positive pivot, *info = col0 + local column (1-based).
// ---------------------------------------------------------------------------
constexpr int FB_MAX = 128;  // largest block this kernel factors

// Factor the diagonal tile d (tile (j, j) of the block) in registers and
// publish it to LDS scaled by its pivots; returns 0 or the failing local
// column (1-based, within the block).
template <typename C>
__device__ __forceinline__ int factor_publish(V4<C>& d, int j, C* Lsc, C* piv) {
    const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int f = factor16<C>(d);
    if (f) return 16 * j + f;
    C pv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) pv[c] = readlane(d[treg<C>(c)], tgrp<C>(c) * 16 + c);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = tcol<C>(g, r);
        C p = pv[tcol<C>(0, r)];
#pragma unroll
        for (int gg = 1; gg < 4; ++gg)
            if (g == gg) p = pv[tcol<C>(gg, r)];
        Lsc[i * 17 + col] = (i > col) ? d[r] / p : (C)0;
        if (i == col) piv[col] = p;
    }
    return 0;
}

// One wave's part of k_factor_block, with its two tile rows ra = RA and
// rb = NTM - 1 - RA as compile-time constants: every slot test in the
// unrolled slot loops then folds away, so the diagonal tile's slot is known
// when it is factored (no select chain over the nine slots, no per-column
// mask reloads).
template <typename S, int W, int SMAX, int RA>
__device__ __forceinline__ void factor_block_wave(S* __restrict__ A, int64_t lda, int s, int64_t col0, int32_t* info,
                                                  double* Pc, double* Lsc, double* piv, int* fail) {
    typedef double C;
    constexpr int NTM = SMAX / 16;  // tile rows at most
    constexpr int TPW = NTM + 1;    // tiles per wave
    constexpr int ra = RA, rb = NTM - 1 - RA;
    const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int nt = (s + 15) >> 4;
    const C* xa = Pc + (16 * ra + i) * 17 + g;  // LDS row bases of the two owned tile rows
    const C* xb = Pc + (16 * rb + i) * 17 + g;
    const C* zc = Pc + i * 17 + g;

    V4<C> acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t <= ra) {
            if (ra < nt) load_tile<S, C>(acc[t], A, lda, 16 * ra, 16 * t, s, s, ra == t, ra == t);
            else acc[t] = V4<C>{0, 0, 0, 0};
        } else {
            if (rb < nt) load_tile<S, C>(acc[t], A, lda, 16 * rb, 16 * (NTM - t), s, s, rb == NTM - t, rb == NTM - t);
            else acc[t] = V4<C>{0, 0, 0, 0};
        }
    }

    // the owner of (jj, jj) factors it: slot jj (row ra) or NTM - jj (row rb)
#define MG_FACTOR_OWNED(jj)                                                                  \
    do {                                                                                     \
        const int td_ = ((jj) == ra) ? (jj) : NTM - (jj);                                     \
        V4<C> d_ = acc[0];                                                                   \
        _Pragma("unroll") for (int t = 1; t < TPW; ++t) if (t == td_) d_ = acc[t];           \
        const int f_ = factor_publish<C>(d_, (jj), Lsc, piv);                                \
        if (f_ && l == 0) *fail = f_;                                                         \
        _Pragma("unroll") for (int t = 0; t < TPW; ++t) if (t == td_) acc[t] = d_;           \
    } while (0)
    // acc[t] -= L(I, j) L(J, j)^T, operands from the LDS copy of column j
#define MG_APPLY(t, xr, J)                                                                   \
    _Pragma("unroll") for (int ks = 0; ks < 4; ++ks)                                         \
        acc[t] = mma_xzt(acc[t], (xr)[4 * ks], -zc[(16 * (J)) * 17 + 4 * ks])

    // step j = -1 only factors tile (0, 0)
    for (int j = -1; j < nt; ++j) {
        if (j >= 0) {
            __syncthreads();  // L_jj published (or failure flagged)
            if (*fail) {
                if (threadIdx.x == 0) *info = (int32_t)(col0 + *fail);
                return;
            }
            // ---- solve the owned tiles (I, j), I > j, and publish them (one
            // code path for both owned rows)
            for (int h = 0; h < 2; ++h) {
                const int I = h ? rb : ra;
                if (I <= j || I >= nt) continue;
                const int ts = h ? NTM - j : j;
                V4<C> y = acc[0];
#pragma unroll
                for (int t = 1; t < TPW; ++t)
                    if (t == ts) y = acc[t];
                solve16s<C, 17>(y, Lsc, piv);
#pragma unroll
                for (int r = 0; r < 4; ++r) Pc[(16 * I + i) * 17 + tcol<C>(g, r)] = y[r];
#pragma unroll
                for (int t = 0; t < TPW; ++t)
                    if (t == ts) acc[t] = y;
            }
            __syncthreads();  // block column j in LDS; L_jj no longer read
            // ---- apply column j to column j + 1
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                if (t <= ra) {
                    if (ra < nt && t == j + 1) MG_APPLY(t, xa, t);
                } else {
                    if (rb < nt && NTM - t == j + 1) MG_APPLY(t, xb, NTM - t);
                }
            }
        }
        // ---- factor (j+1, j+1) if owned, while the others keep updating
        if (j + 1 < nt && (j + 1 == ra || j + 1 == rb)) MG_FACTOR_OWNED(j + 1);
        if (j >= 0) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                if (t <= ra) {
                    if (ra < nt && t > j + 1) MG_APPLY(t, xa, t);
                } else {
                    if (rb < nt && NTM - t > j + 1) MG_APPLY(t, xb, NTM - t);
                }
                __builtin_amdgcn_sched_barrier(0);  // one tile's operands live at a time
            }
        }
    }
#undef MG_APPLY
#undef MG_FACTOR_OWNED
    // ---- write the factor back (diagonal tiles: lower part only)
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t <= ra) {
            if (ra < nt) store_tile<S, C>(acc[t], A, lda, 16 * ra, 16 * t, s, s, ra == t);
        } else {
            if (rb < nt) store_tile<S, C>(acc[t], A, lda, 16 * rb, 16 * (NTM - t), s, s, rb == NTM - t);
        }
    }
}

template <typename S, int W, int SMAX>
// (At most 256 registers per wave, VGPRs and AGPRs together: the look-ahead
// runs this kernel while the trailing update holds two 256-register waves on
// every SIMD, and a wave that needs more than half a SIMD's registers can
// only start once the update drains a whole SIMD, which starved it for
// milliseconds at a time.)
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2))) void k_factor_block(S* __restrict__ A, int64_t lda, int s, int64_t col0,
                                                         int32_t* info) {
    typedef double C;
    constexpr int NTM = SMAX / 16;  // tile rows at most
    static_assert(2 * W == NTM && W == 4, "four waves of two tile rows");
    __shared__ C Pc[SMAX * 17];     // block column j: row r, column c at r*17 + c
    __shared__ C Lsc[16 * 17];      // L_jj scaled by columns (0 on and above the diagonal)
    __shared__ C piv[16];
    __shared__ int fail;
    if (*info != 0) return;
    if (threadIdx.x == 0) fail = 0;
    // every wave runs the same sequence of barriers in its own instance
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
        case 0: factor_block_wave<S, W, SMAX, 0>(A, lda, s, col0, info, Pc, Lsc, piv, &fail); break;
        case 1: factor_block_wave<S, W, SMAX, 1>(A, lda, s, col0, info, Pc, Lsc, piv, &fail); break;
        case 2: factor_block_wave<S, W, SMAX, 2>(A, lda, s, col0, info, Pc, Lsc, piv, &fail); break;
        default: factor_block_wave<S, W, SMAX, 3>(A, lda, s, col0, info, Pc, Lsc, piv, &fail); break;
    }
}

// bfloat16 rounding (nearest-even on the bit pattern) of a binary32 value,
// widened back to binary32; used for the BF16 trailing-update operands.
__device__ __forceinline__ float round_bf16(float x) {
    unsigned u = __builtin_bit_cast(unsigned, x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    return __builtin_bit_cast(float, u);
}
__device__ __forceinline__ double lo_round(double x, int) { return x; }
__device__ __forceinline__ float lo_round(float x, int bf16) { return bf16 ? round_bf16(x) : x; }

// ---------------------------------------------------------------------------
// Panel TRSM: X = P L^{-T} in place for the m x NB panel P, L = L_kk (NB x NB
// lower, NB <= FB_MAX).  The NB/16 (NB/16 + 1)/2 lower 16 x 16 tiles of L_kk
// are staged once per workgroup in LDS (diagonal tiles pre-scaled by their
// pivots), laid out so that each MFMA operand is one conflict-free LDS read.
// Each wave owns RB (1 or 2) 16-row blocks of the panel, whose NB/16 tiles
// it keeps in registers and carries through the same steps side by side
// (the solve is a chain of dependent latencies; two independent chains fill
// each other's stalls): tile t receives -X_p L_tp^T from every solved tile p < t
// (the k index of step ks in lane group g is tcol(g, ks), exactly the column
// tile p keeps in its register ks, so that operand comes straight from
// registers), then is solved against L_tt by substitution (solve16s / solve16s2).
// Exact for integer data with power-of-two pivots.
// ---------------------------------------------------------------------------
template <typename S, int NB, int RB>
// (At most 256 registers per wave, for the same reason as k_factor_block.)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_trsm_panel(S* __restrict__ P, const S* __restrict__ Lkk,
                                                    int64_t lda, int64_t m, const int32_t* info,
                                                    __bf16* __restrict__ Pq, int ldq) {
    constexpr int NT = NB / 16, NTT = NT * (NT + 1) / 2;
    __shared__ S Lt[NTT][16 * 17];  // tile (t, p), p <= t, at t (t + 1) / 2 + p: row r, column c at r*17 + c
    __shared__ S Pv[NT][16];        // pivots of the diagonal tiles
    if (*info != 0) return;
    for (int e = threadIdx.x; e < NT * 16; e += blockDim.x) {
        const int b = e >> 4, c = e & 15;
        Pv[b][c] = Lkk[idx(16 * b + c, 16 * b + c, lda)];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NTT * 256; e += blockDim.x) {
        const int tt = e >> 8, rr = (e >> 4) & 15, cc = e & 15;
        int t = 0;
        while ((t + 1) * (t + 2) / 2 <= tt) ++t;
        const int p = tt - t * (t + 1) / 2;
        S v;
        if (p < t) v = Lkk[idx(16 * t + rr, 16 * p + cc, lda)];
        else v = (rr > cc) ? Lkk[idx(16 * t + rr, 16 * t + cc, lda)] / Pv[t][cc] : (S)0;
        Lt[tt][rr * 17 + cc] = v;
    }
    __syncthreads();
    // each wave solves RB 16-row blocks side by side (rows R and R + 16)
    static_assert(RB == 1 || RB == 2, "one or two row blocks per wave");
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int64_t R = ((int64_t)blockIdx.x * 4 + w) * 16 * RB;
    if (R >= m) return;
    V4<S> x[NT], u[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        load_tile<S, S>(x[t], P, lda, R, 16 * t, m, NB, false, false);
        if constexpr (RB == 2) load_tile<S, S>(u[t], P, lda, R + 16, 16 * t, m, NB, false, false);  // rows past m load as 0
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int p = 0; p < t; ++p) {
            const S* Z = Lt[t * (t + 1) / 2 + p] + i * 17;
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const S zv = -Z[tcol<S>(g, ks)];
                x[t] = mma_xzt(x[t], x[p][ks], zv);
                if constexpr (RB == 2) u[t] = mma_xzt(u[t], u[p][ks], zv);
            }
        }
        if constexpr (RB == 2) solve16s2<S, 17>(x[t], u[t], Lt[t * (t + 1) / 2 + t], Pv[t]);
        else solve16s<S, 17>(x[t], Lt[t * (t + 1) / 2 + t], Pv[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        store_tile<S, S>(x[t], P, lda, R, 16 * t, m, NB, false);
        if constexpr (RB == 2) store_tile<S, S>(u[t], P, lda, R + 16, 16 * t, m, NB, false);
    }
    if constexpr (sizeof(S) == 4) {
        // bfloat16 mode: the solved rows also go to the block column's
        // row-major bfloat16 copy (a lane's four values are four consecutive
        // columns: one 8-byte store), rounded to nearest even (round_bf16)
        if (Pq) {
#pragma unroll
            for (int h2 = 0; h2 < RB; ++h2) {
                const int64_t row = R + 16 * h2 + i;
                if (row >= m) continue;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const V4<S>& y = h2 ? u[t] : x[t];
                    unsigned q[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) q[r] = __builtin_bit_cast(unsigned, round_bf16(y[r])) >> 16;
                    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
                    const u32x2 v = {q[0] | (q[1] << 16), q[2] | (q[3] << 16)};
                    *(u32x2*)(Pq + row * ldq + 16 * t + tcol<S>(g, 0)) = v;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Trailing update lower(C) -= P P^T, C m x m, P m x kdim (kdim % 16 == 0),
// restricted to the 128 x 128 lower tiles of tile columns [j0, j0 + wj).
// A workgroup owns one tile; each of its four waves owns a 64 x 64 quarter
// (4 x 4 MFMA tiles, 64 accumulators per lane) and streams its own operand
// rows of P from L1/L2 straight into registers through buffer loads (scalar
// resource + 32-bit lane offsets), three k-steps ahead of the MFMAs in a
// four-slot register ring.  There is no LDS staging and no barrier: waves
// never wait for each other, and two waves per SIMD keep the matrix pipe
// busy while the other waits on memory.  When kdim % 256 == 0 the C tile is
// not loaded up front: its 16 x 16 pieces are fetched one at a time during
// the k-loop and folded into the accumulators, so C's HBM reads overlap the
// MFMAs.  Quarters entirely above the diagonal exit at once.  With bf16 set
// (binary32 storage only) each operand is rounded to bfloat16 before its
// MFMA, so the products are those of bfloat16 inputs accumulated in FP32.
// Tile order is XCD-aware: workgroup b runs on XCD b % 8, and each XCD
// receives a contiguous run of tiles, numbered so that the workgroups it
// holds at once share panel rows in its L2.
// ---------------------------------------------------------------------------
constexpr int SY_BM = 128;

__host__ __device__ __forceinline__ void lower_tile_coords(int64_t t, int64_t& I, int64_t& J) {
    int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    I = r;
    J = t - r * (r + 1) / 2;
}

// Lower tiles (I, J), I >= J, of a T x T tile grid restricted to tile columns
// [j0, j0 + wj): numbered row by row.  Rows I - j0 < wj hold I - j0 + 1
// tiles, later rows hold wj.
__host__ __device__ __forceinline__ int64_t slab_tiles(int64_t T, int64_t j0, int64_t wj) {
    const int64_t h = T - j0;
    const int64_t w = wj < h ? wj : h;
    return w * (w + 1) / 2 + (h - w) * w;
}
__host__ __device__ __forceinline__ void slab_tile_coords(int64_t t, int64_t j0, int64_t wj, int64_t& I, int64_t& J) {
    const int64_t tri = wj * (wj + 1) / 2;
    if (t < tri) {
        lower_tile_coords(t, I, J);
    } else {
        const int64_t u = t - tri;
        I = wj + u / wj;
        J = u % wj;
    }
    I += j0;
    J += j0;
}

// The whole lower triangle of a TT x TT tile grid in grouped order: bands of
// SY_GROUP tile rows; inside a band, its full columns of SY_GROUP tiles come
// first (column by column), then the band's own diagonal triangle (row by
// row).  Workgroups resident together on one XCD then cover a square patch
// of the triangle and share both its panel row blocks and its panel column
// blocks in L2, instead of one row block and many column blocks.
constexpr int SY_GROUP = 8;
struct TileIJ {
    int64_t I, J;
};
__host__ __device__ __forceinline__ int64_t band_start(int64_t b) {
    return (int64_t)SY_GROUP * SY_GROUP * b * (b - 1) / 2 + b * (int64_t)(SY_GROUP * (SY_GROUP + 1) / 2);
}
__host__ __device__ __forceinline__ TileIJ grouped_tile_coords(int64_t t, int64_t TT) {
    constexpr double G = SY_GROUP;
    int64_t b = (int64_t)((sqrt((G + 1) * (G + 1) / 4 + 2.0 * (double)t) - (G + 1) / 2) / G);
    if (b < 0) b = 0;
    while (b > 0 && band_start(b) > t) --b;
    while (band_start(b + 1) <= t) ++b;
    const int64_t u = t - band_start(b), r0 = b * SY_GROUP, h = TT - r0 < SY_GROUP ? TT - r0 : SY_GROUP;
    if (u < h * r0) return {r0 + u % h, u / h};
    int64_t I, J;
    lower_tile_coords(u - h * r0, I, J);
    return {r0 + I, r0 + J};
}

// Tile t of the trailing update over tile columns [j0, j0 + wj) of a T x T
// grid: grouped order when the slab is the whole remaining triangle (the
// large updates), row order for narrow slabs (whose few column blocks stay
// in L2 anyway).
__host__ __device__ __forceinline__ TileIJ trailing_tile_coords(int64_t t, int64_t T, int64_t j0, int64_t wj) {
    TileIJ c;
    if (wj >= T - j0) {
        c = grouped_tile_coords(t, T - j0);
        c.I += j0;
        c.J += j0;
    } else {
        slab_tile_coords(t, j0, wj, c.I, c.J);
    }
    return c;
}

// The same on the device, with the result held in scalar registers: the
// inputs are uniform, and making that explicit keeps the tile's buffer
// resources scalar (tile indices stay below 2^31).
__device__ __forceinline__ void trailing_tile(int64_t t, int64_t T, int64_t j0, int64_t wj, int64_t& I, int64_t& J) {
    const TileIJ c = trailing_tile_coords(t, T, j0, wj);
    I = __builtin_amdgcn_readfirstlane((int)c.I);
    J = __builtin_amdgcn_readfirstlane((int)c.J);
}


// Raw buffer access: a 128-bit resource (base, byte extent) that the compiler
// keeps in scalar registers, plus a 32-bit per-lane byte offset.  Loads at or
// beyond the extent return 0 instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int64_t bytes) {
    const int nr = (int)(bytes < 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : bytes));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nr, 0x00020000);
}
__device__ __forceinline__ double buf_ld(double*, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ float buf_ld(float*, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

template <typename S, bool FOLD, int RG, bool BF>
__global__ __launch_bounds__(256, 2) void k_syrk_lower(S* __restrict__ Cm, const S* __restrict__ P,
                                                       int64_t lda, int64_t m, int kdim, int64_t j0, int64_t wj,
                                                       const int32_t* info) {
    if (*info != 0) return;
    const int64_t T = (m + SY_BM - 1) / SY_BM;
    const int64_t ntiles = slab_tiles(T, j0, wj);
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;
    int64_t I, J;
    trailing_tile(t, T, j0, wj, I, J);
    constexpr int ES = (int)sizeof(S);
    const int tid = threadIdx.x, l = tid & 63, i = l & 15, g = l >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w >> 1, wc = w & 1;
    const int64_t sr0 = I * SY_BM + 64 * wr, sc0 = J * SY_BM + 64 * wc;
    // quarters above the diagonal or past the block's edge hold no output
    if (sr0 + 63 < sc0 || sr0 >= m || sc0 >= m) return;
    const int ld = (int)lda;  // the host keeps every byte offset below 2^31
    const int rmax = (int)(m - 1 - sr0 < 63 ? m - 1 - sr0 : 63);
    const int cmax = (int)(m - 1 - sc0 < 63 ? m - 1 - sc0 : 63);
    const int dd = (int)(sr0 - sc0 < 64 ? sr0 - sc0 : 64);  // >= 64: no entry of the quarter is above the diagonal
    // C quarter at (sr0, sc0).  Local row / column indices are clamped into
    // the block, so every load stays inside it (entries of a diagonal
    // quarter above the diagonal are read and discarded); stores are masked.
    const __amdgpu_buffer_rsrc_t crs = buf_rsrc(Cm + idx(sr0, sc0, lda), 0x7fffffff);
    auto c_in = [&](int bi, int bj, int r) {
        const int rr = 16 * bi + i, cc = 16 * bj + tcol<S>(g, r);
        return rr <= rmax && cc <= cmax && rr + dd >= cc;
    };
    auto c_off = [&](int bi, int bj, int r) {
        const int rr = min(16 * bi + i, rmax), cc = min(16 * bj + tcol<S>(g, r), cmax);
        return (rr + cc * ld) * ES;
    };
    auto c_load = [&](int bi, int bj, int r) -> S {
        const S v = buf_ld((S*)nullptr, crs, c_off(bi, bj, r), 0);
        return c_in(bi, bj, r) ? v : (S)0;
    };
    // The accumulators hold P P^T - C: products are added with their own
    // sign and the result is negated as it is stored (round-to-nearest is
    // symmetric, so this equals C - P P^T accumulated in the same order).
    V4<S> acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] = FOLD ? (S)0 : -c_load(bi, bj, r);
    // Operands: panel rows sr0 + 16 b + i (x) and sc0 + 16 b + i (z) of
    // column 4 kn + g; rows past the block are clamped to its last row
    // (they only feed outputs that are never stored).
    const __amdgpu_buffer_rsrc_t prs = buf_rsrc(P, 0x7fffffff);
    int xo[4], zo[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        xo[b] = ((int)sr0 + min(16 * b + i, rmax) + g * ld) * ES;
        zo[b] = ((int)sc0 + min(16 * b + i, cmax) + g * ld) * ES;
    }
    const int nks = kdim / 4;
    // ring of RG k-steps of operands; step kn lives in slot kn % RG and is
    // fetched RG - 1 steps before its MFMAs (RG = 8 for binary32, whose
    // MFMAs take half as long, so that the prefetch still covers a round
    // trip to memory)
    static_assert(RG == 4 || RG == 8, "ring of 4 or 8 k-steps");
    S xq[RG][4], zq[RG][4];
    auto fetch = [&](int slot, int kn) {
        const int soff = (kn < nks ? kn : nks - 1) * 4 * ld * ES;  // steps past the end re-read the last one
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            xq[slot][b] = buf_ld((S*)nullptr, prs, xo[b], soff);
            zq[slot][b] = buf_ld((S*)nullptr, prs, zo[b], soff);
        }
    };
#pragma unroll
    for (int p = 0; p < RG - 1; ++p) fetch(p, p);
    // k-steps ks .. ks + RG - 1 (ks % RG == 0)
    auto body = [&](int ks) {
#pragma unroll
        for (int s = 0; s < RG; ++s) {
            fetch((s + RG - 1) % RG, ks + s + RG - 1);
            S xv[4], zv[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                xv[b] = BF ? lo_round(xq[s][b], 1) : xq[s][b];
                zv[b] = BF ? lo_round(zq[s][b], 1) : zq[s][b];
            }
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mma_xzt(acc[bi][bj], xv[bi], zv[bj]);
        }
    };
    if constexpr (FOLD) {
        // C is folded in one 16 x 16 tile at a time, spread over the k-loop:
        // the load of tile q is issued, nks / 16 k-steps of MFMAs run, then
        // it is subtracted.  C's HBM traffic thus overlaps the matrix pipe
        // instead of forming a prologue that every resident workgroup issues
        // at once.
        const int per_q = nks / (16 * RG);  // the host keeps nks a multiple of 16 RG
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            V4<S> cv;
#pragma unroll
            for (int r = 0; r < 4; ++r) cv[r] = c_load(q >> 2, q & 3, r);
            for (int u = 0; u < per_q; ++u) body((q * per_q + u) * RG);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[q >> 2][q & 3][r] -= cv[r];
        }
    } else {
        for (int ks = 0; ks < nks; ks += RG) body(ks);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (c_in(bi, bj, r)) buf_st(-acc[bi][bj][r], crs, c_off(bi, bj, r), 0);
}

// ---------------------------------------------------------------------------
// bfloat16 trailing update (mixed precision, bfloat16 mode): lower(C) -= P P^T
// with C in binary32 and P given as a row-major bfloat16 copy Pt (m x kdim,
// row stride ldp, kdim % 32 == 0), products of bfloat16 inputs
// accumulated in FP32 on the 16x16x32 bfloat16 matrix instruction.  Same
// tiling, tile order, buffer-resource addressing and four-slot operand ring
// as k_syrk_lower; each lane loads 8 consecutive k of one row (16 bytes) per
// operand and k-step.  The C tile is loaded up front (short k-loop).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mma_xzt_bf16(f32x4 acc, bf16x8 x, bf16x8 z) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(z, x, acc, 0, 0, 0);
}

// bfloat16 trailing update with the operands staged through LDS.  The
// register-ring form above keeps only three 32-wide k-steps in flight, so at
// bfloat16 MFMA rates (a k-step is ~0.1 us of matrix-pipe time per wave)
// nearly every step waits for a round trip to memory.  Here the tile's two
// 128-row operand blocks move in chunks of 64 k: all of a chunk's loads are
// issued at once into registers (4 x 16 bytes per thread and operand),
// written to padded LDS rows (16 bytes of padding per row: the 16 rows a
// quarter-wave reads sit in distinct banks), and the four waves multiply from
// LDS while the next chunk's loads are in flight.  Three workgroups share a
// CU (37 KB of LDS each), so one's C read and first chunk overlap the
// others' products, and a workgroup holds its CU for one tile only, so the narrow
// kernels of the panel chain find CUs as tiles finish.  Operand rows past the
// block read as zero (the buffer resource ends at the panel's last row);
// their products feed only outputs that are never stored.  Interior quarters
// (every entry inside the block and below the diagonal) address C with one
// per-lane offset plus uniform ones; diagonal and edge quarters take the
// clamped, masked path of k_syrk_lower_bf16.  The MFMA sequence per output
// tile is that kernel's, so the result is bitwise the same.
constexpr int BFL_KC = 64;                   // k per LDS chunk
constexpr int BFL_LD = BFL_KC * 2 + 16;      // LDS row stride in bytes
constexpr int BFL_PC = BFL_KC / 8;           // 16-byte pieces per row of a chunk
constexpr int BFL_U = 128 * BFL_PC / 256;    // pieces per thread and operand
constexpr int BFL_RS = 256 / BFL_PC;         // rows between a thread's pieces

__global__ __launch_bounds__(256, 3) void k_syrk_lower_bf16l(float* __restrict__ Cm, const __bf16* __restrict__ Pt,
                                                             int64_t lda, int64_t m, int kdim, int ldp, int64_t j0,
                                                             int64_t wj, const int32_t* info) {
    __shared__ __attribute__((aligned(16))) unsigned char Xs[128 * BFL_LD];
    __shared__ __attribute__((aligned(16))) unsigned char Zs[128 * BFL_LD];
    if (*info != 0) return;
    const int64_t T = (m + SY_BM - 1) / SY_BM;
    const int64_t ntiles = slab_tiles(T, j0, wj);
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;  // uniform across the workgroup
    int64_t I, J;
    trailing_tile(t, T, j0, wj, I, J);
    constexpr int ES = 4;
    const int tid = threadIdx.x, l = tid & 63, i = l & 15, g = l >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w >> 1, wc = w & 1;
    const int ld = (int)lda;
    // chunk c: thread tid moves piece tid % BFL_PC of rows tid / BFL_PC +
    // BFL_RS u of both blocks; rows at or past m lie beyond the resource and
    // read 0
    const __amdgpu_buffer_rsrc_t prs = buf_rsrc(Pt, m * ldp * 2);
    const int pvo = ((tid / BFL_PC) * ldp + (tid % BFL_PC) * 8) * 2;
    const int xso = (int)(I * SY_BM) * ldp * 2, zso = (int)(J * SY_BM) * ldp * 2;
    u32x4 sx[BFL_U], sz[BFL_U];
    auto gload = [&](int c) {
#pragma unroll
        for (int u = 0; u < BFL_U; ++u) {
            const int so = (BFL_RS * u * ldp + c * BFL_KC) * 2;
            sx[u] = __builtin_amdgcn_raw_buffer_load_b128(prs, pvo, xso + so, 0);
            sz[u] = __builtin_amdgcn_raw_buffer_load_b128(prs, pvo, zso + so, 0);
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int u = 0; u < BFL_U; ++u) {
            const int row = tid / BFL_PC + BFL_RS * u, pc = tid % BFL_PC;
            *(u32x4*)(Xs + row * BFL_LD + pc * 16) = sx[u];
            *(u32x4*)(Zs + row * BFL_LD + pc * 16) = sz[u];
        }
    };
    gload(0);
    const int64_t sr0 = I * SY_BM + 64 * wr, sc0 = J * SY_BM + 64 * wc;
    // quarters above the diagonal or past the block's edge hold no output but
    // still take part in the loads and barriers
    const bool active = !(sr0 + 63 < sc0 || sr0 >= m || sc0 >= m);
    const int rmax = active ? (int)(m - 1 - sr0 < 63 ? m - 1 - sr0 : 63) : 0;
    const int cmax = active ? (int)(m - 1 - sc0 < 63 ? m - 1 - sc0 : 63) : 0;
    const int dd = (int)(sr0 - sc0 < 64 ? sr0 - sc0 : 64);
    const bool interior = active && rmax == 63 && cmax == 63 && dd >= 64;
    const __amdgpu_buffer_rsrc_t crs = buf_rsrc(Cm + idx(active ? sr0 : 0, active ? sc0 : 0, lda), 0x7fffffff);
    // C entry (16 bi + i, 16 bj + 4 g + r) of the quarter: per-lane part
    // (i + 4 g ld), uniform parts 16 bi and (16 bj + r) ld
    auto c_in = [&](int li, int lg, int bi, int bj, int r) {
        const int rr = 16 * bi + li, cc = 16 * bj + tcol<float>(lg, r);
        return rr <= rmax && cc <= cmax && rr + dd >= cc;
    };
    auto c_off = [&](int li, int lg, int bi, int bj, int r) {
        const int rr = min(16 * bi + li, rmax), cc = min(16 * bj + tcol<float>(lg, r), cmax);
        return (rr + cc * ld) * ES;
    };
    f32x4 acc[4][4];
    if (interior) {
        const int cvo = (i + 4 * g * ld) * ES;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[bi][bj][r] = -buf_ld((float*)nullptr, crs, cvo + 16 * bi * ES, (16 * bj + r) * ld * ES);
    } else {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[bi][bj][r] = (active && c_in(i, g, bi, bj, r))
                                         ? -buf_ld((float*)nullptr, crs, c_off(i, g, bi, bj, r), 0)
                                         : 0.0f;
    }
    const int nch = kdim / BFL_KC;
    for (int c = 0; c < nch; ++c) {
        lstore();
        __syncthreads();
        if (c + 1 < nch) gload(c + 1);
        if (active) {
#pragma unroll
            for (int s = 0; s < BFL_KC / 32; ++s) {
                bf16x8 xv[4], zv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    xv[b] = *(const bf16x8*)(Xs + (64 * wr + 16 * b + i) * BFL_LD + (32 * s + 8 * g) * 2);
                    zv[b] = *(const bf16x8*)(Zs + (64 * wc + 16 * b + i) * BFL_LD + (32 * s + 8 * g) * 2);
                }
#pragma unroll
                for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mma_xzt_bf16(acc[bi][bj], xv[bi], zv[bj]);
            }
        }
        __syncthreads();
    }
    if (!active) return;
    // the store's offsets are recomputed from lane indices the compiler
    // cannot see through, so none of the load's 64 offsets stays live
    // across the k-loop
    int li = i, lg = g;
    asm volatile("" : "+v"(li), "+v"(lg));
    if (interior) {
        const int cvo = (li + 4 * lg * ld) * ES;
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    buf_st(-acc[bi][bj][r], crs, cvo + 16 * bi * ES, (16 * bj + r) * ld * ES);
    } else {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (c_in(li, lg, bi, bj, r)) buf_st(-acc[bi][bj][r], crs, c_off(li, lg, bi, bj, r), 0);
    }
}

__global__ __launch_bounds__(256, 2) void k_syrk_lower_bf16(float* __restrict__ Cm, const __bf16* __restrict__ Pt,
                                                            int64_t lda, int64_t m, int kdim, int ldp, int64_t j0,
                                                            int64_t wj, const int32_t* info) {
    if (*info != 0) return;
    const int64_t T = (m + SY_BM - 1) / SY_BM;
    const int64_t ntiles = slab_tiles(T, j0, wj);
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;
    int64_t I, J;
    trailing_tile(t, T, j0, wj, I, J);
    constexpr int ES = 4;
    const int tid = threadIdx.x, l = tid & 63, i = l & 15, g = l >> 4;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w >> 1, wc = w & 1;
    const int64_t sr0 = I * SY_BM + 64 * wr, sc0 = J * SY_BM + 64 * wc;
    if (sr0 + 63 < sc0 || sr0 >= m || sc0 >= m) return;
    const int ld = (int)lda;
    const int rmax = (int)(m - 1 - sr0 < 63 ? m - 1 - sr0 : 63);
    const int cmax = (int)(m - 1 - sc0 < 63 ? m - 1 - sc0 : 63);
    const int dd = (int)(sr0 - sc0 < 64 ? sr0 - sc0 : 64);
    const __amdgpu_buffer_rsrc_t crs = buf_rsrc(Cm + idx(sr0, sc0, lda), 0x7fffffff);
    auto c_in = [&](int bi, int bj, int r) {
        const int rr = 16 * bi + i, cc = 16 * bj + tcol<float>(g, r);
        return rr <= rmax && cc <= cmax && rr + dd >= cc;
    };
    auto c_off = [&](int bi, int bj, int r) {
        const int rr = min(16 * bi + i, rmax), cc = min(16 * bj + tcol<float>(g, r), cmax);
        return (rr + cc * ld) * ES;
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v = buf_ld((float*)nullptr, crs, c_off(bi, bj, r), 0);
                acc[bi][bj][r] = c_in(bi, bj, r) ? -v : 0.0f;
            }
    // operand rows (clamped into the block) of the row-major panel; k-step
    // kn covers k = 32 kn .. 32 kn + 31, lane group g its 8 entries 8 g ..
    const __amdgpu_buffer_rsrc_t prs = buf_rsrc(Pt, 0x7fffffff);
    int xo[4], zo[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        xo[b] = (((int)sr0 + min(16 * b + i, rmax)) * ldp + 8 * g) * 2;
        zo[b] = (((int)sc0 + min(16 * b + i, cmax)) * ldp + 8 * g) * 2;
    }
    const int nks = kdim / 32;
    bf16x8 xq[4][4], zq[4][4];
    auto fetch = [&](int slot, int kn) {
        const int soff = (kn < nks ? kn : nks - 1) * 64;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            xq[slot][b] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(prs, xo[b], soff, 0));
            zq[slot][b] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(prs, zo[b], soff, 0));
        }
    };
    fetch(0, 0);
    fetch(1, 1);
    fetch(2, 2);
    for (int ks = 0; ks < nks; ks += 4) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            fetch((s + 3) & 3, ks + s + 3);
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mma_xzt_bf16(acc[bi][bj], xq[s][bi], zq[s][bj]);
        }
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (c_in(bi, bj, r)) buf_st(-acc[bi][bj][r], crs, c_off(bi, bj, r), 0);
}

// ---------------------------------------------------------------------------
// Host driver.
// ---------------------------------------------------------------------------
int64_t potrf_block_size(mg_handle_t h, int64_t n, int es) {
    (void)es;
    if (h && h->nb > 0) return h->nb;
    // measured switch points (FP64 posv, look-ahead on): 64 is fastest up to
    // n = 4096, 128 at 6144-8192, 256 at 12288, 512 at 24576 and above
    if (n >= 24576) return 512;
    if (n >= 10240) return 256;
    if (n >= 5120) return 128;
    return 64;
}

constexpr int64_t TRSM_TWO_ROWS = 12288;  // panel rows from which waves take two row blocks

template <typename S>
static mg_status launch_trsm(hipStream_t st, int64_t nb, S* P, const S* Lkk, int64_t lda, int64_t m,
                             const int32_t* info, bool latency, __bf16* Pq = nullptr, int ldq = 0) {
    // Tall panels (the look-ahead regime, where the solve shares the chip
    // with the trailing update) take two row blocks per wave, halving the
    // wave-time the solve holds; short ones one, for the shortest latency.
    // latency: the caller's schedule is bound by the panel chain, not by the
    // trailing update (bfloat16 mode), so every panel takes one row block
    // per wave.
    const dim3 block(256);
    const bool two = m >= TRSM_TWO_ROWS && !latency;
    const dim3 grid((unsigned)cdiv(m, two ? 128 : 64));
    if (nb == 64 && two) hipLaunchKernelGGL((k_trsm_panel<S, 64, 2>), grid, block, 0, st, P, Lkk, lda, m, info, Pq, ldq);
    else if (nb == 64) hipLaunchKernelGGL((k_trsm_panel<S, 64, 1>), grid, block, 0, st, P, Lkk, lda, m, info, Pq, ldq);
    else if (nb == 128 && two) hipLaunchKernelGGL((k_trsm_panel<S, 128, 2>), grid, block, 0, st, P, Lkk, lda, m, info, Pq, ldq);
    else if (nb == 128) hipLaunchKernelGGL((k_trsm_panel<S, 128, 1>), grid, block, 0, st, P, Lkk, lda, m, info, Pq, ldq);
    else return MG_ERR_UNSUPPORTED;
    MG_LAUNCH_CHECK();
    return MG_OK;
}

template <typename S>
mg_status syrk_lower_launch(hipStream_t st, S* Cm, const S* P, int64_t lda, int64_t m, int64_t kdim,
                            const int32_t* info, int64_t j0 = 0, int64_t wj = -1, int bf16 = 0) {
    const int64_t T = cdiv(m, SY_BM);
    if (wj < 0) wj = T - j0;
    if (j0 >= T || wj <= 0) return MG_OK;
    const int64_t ntiles = slab_tiles(T, j0, wj);
    const int64_t grid = 8 * cdiv(ntiles, 8);
    // every byte offset the kernel forms from P or from a quarter's corner
    // must fit in 31 bits
    if ((m + (kdim + 64) * lda) * (int64_t)sizeof(S) >= ((int64_t)1 << 31) - 65536 || kdim % 16 != 0)
        return MG_ERR_UNSUPPORTED;
#define MG_SYRK(FOLD_, RG_, BF_)                                                                             \
    hipLaunchKernelGGL((k_syrk_lower<S, FOLD_, RG_, BF_>), dim3((unsigned)grid), dim3(256), 0, st, Cm, P, lda, m, \
                       (int)kdim, j0, wj, info)
    // rank-256/512 updates fold C into the k-loop (which needs kdim a
    // multiple of 16 ring depths); binary32 rank-512 updates use the deeper
    // ring (not with bfloat16 rounding, which would then spill), and so do
    // binary32 updates of other ranks that are a multiple of 8 ring steps;
    // the bfloat16 rounding of binary32 operands is a template switch
    if constexpr (sizeof(S) == 4) {
        if (kdim % 512 == 0 && !bf16) {
            MG_SYRK(true, 8, false);
        } else if (kdim % 256 == 0) {
            if (bf16) MG_SYRK(true, 4, true);
            else MG_SYRK(true, 4, false);
        } else if (kdim % 32 == 0) {
            // narrow slabs (the panel chain's rank-128 updates) are latency
            // bound: the deeper ring keeps seven k-steps in flight
            if (bf16) MG_SYRK(false, 8, true);
            else MG_SYRK(false, 8, false);
        } else {
            if (bf16) MG_SYRK(false, 4, true);
            else MG_SYRK(false, 4, false);
        }
    } else {
        if (kdim % 256 == 0) MG_SYRK(true, 4, false);
        else MG_SYRK(false, 4, false);
    }
#undef MG_SYRK
    MG_LAUNCH_CHECK();
    return MG_OK;
}

constexpr int BF_LDP = 512;  // row stride of the bfloat16 panel copies (elements)

// Factor of the diagonal block at k0 (width min(nb, n - k0)).
template <typename T>
static mg_status diag_step(mg_handle_t h, hipStream_t st, T* A, int64_t lda, int64_t n, int64_t k0, int64_t nb,
                           int32_t* info) {
    const int64_t kb = std::min(nb, n - k0);
    mg_status rc;
    if ((rc = prof_begin(h, MG_PROF_DIAG, st))) return rc;
    hipLaunchKernelGGL((k_factor_block<T, FB_MAX / 32, FB_MAX>), dim3(1), dim3(2 * FB_MAX), 0, st,
                       A + idx(k0, k0, lda), lda, (int)kb, k0, info);
    MG_LAUNCH_CHECK();
    const double b = (double)kb;
    return prof_end(h, MG_PROF_DIAG, b * b * b / 3 + b * b / 2 + b / 6, b * (b + 1) * sizeof(T), st);
}

// Panel rows [r0, r0 + m) of block column k0 (width kb) solved against its
// factored diagonal block; rows are independent, so any split of the panel's
// rows gives bitwise the same result.
template <typename T>
static mg_status panel_rows(mg_handle_t h, hipStream_t st, T* A, int64_t lda, int64_t k0, int64_t kb, int64_t r0,
                            int64_t m, int32_t* info, __bf16* Pq = nullptr) {
    if (m <= 0) return MG_OK;
    mg_status rc;
    if ((rc = prof_begin(h, MG_PROF_TRSM, st))) return rc;
    if ((rc = launch_trsm<T>(st, kb, A + idx(r0, k0, lda), A + idx(k0, k0, lda), lda, m, info, h->trail_lo == 2, Pq,
                             BF_LDP)))
        return rc;
    const double b = (double)kb;
    return prof_end(h, MG_PROF_TRSM, (double)m * b * b, 2.0 * m * b * sizeof(T), st);
}

// Pq (bfloat16 mode): where the solved rows' bfloat16 copy goes (row stride
// BF_LDP), or null.
template <typename T>
static mg_status panel_step(mg_handle_t h, hipStream_t st, T* A, int64_t lda, int64_t n, int64_t k0, int64_t nb,
                           int32_t* info, __bf16* Pq = nullptr) {
    // factor the diagonal block at k0 and solve the panel below it
    const int64_t kb = std::min(nb, n - k0);
    mg_status rc;
    if ((rc = diag_step<T>(h, st, A, lda, n, k0, nb, info))) return rc;
    return panel_rows<T>(h, st, A, lda, k0, kb, k0 + kb, n - k0 - kb, info, Pq);
}

template <typename T>
static mg_status trailing(mg_handle_t h, hipStream_t st, T* A, int64_t lda, int64_t n, int64_t k0, int64_t nb,
                         const int32_t* info, int64_t j0, int64_t wj);

// bfloat16 mode: the row-major bfloat16 copy of block column k0's panel
// (block columns of 256 or 512 only), or null.  Row r >= k0 of the block
// column sits at row r - k0 of the copy, whose row stride is BF_LDP; each
// 128-wide step of the column packs its columns for the rows below its
// diagonal block as soon as they are solved.  Three buffers rotate over
// consecutive block columns: the chain stream writes column k + 3's only
// after waiting for the update stream's rest_a(k + 1), which that stream
// runs after rest_b(k), the last reader of column k's copy.
template <typename T>
static __bf16* bf16_panel(mg_handle_t h, int64_t n, int64_t k0, int64_t nb) {
    if constexpr (sizeof(T) != 4) {
        return nullptr;
    } else {
        if (h->trail_lo != 2 || !h->bf16_panel || nb % 256 != 0 || nb > BF_LDP) return nullptr;
        return (__bf16*)h->bf16_panel + (size_t)((k0 / nb) % 3) * (size_t)n * BF_LDP;
    }
}

// lower(C) -= P P^T over tile columns [j0, j0 + wj) of the m x m binary32
// matrix C (lda), P the m x kdim row-major bfloat16 copy at Pt (row stride
// ldp): the LDS-staged kernel, or the register-ring one where a rank or size
// does not fit its chunks and offsets.
static mg_status bf16_update(hipStream_t st, float* C, int64_t lda, const __bf16* Pt, int ldp, int64_t m,
                             int64_t kdim, int64_t j0, int64_t wj, const int32_t* info) {
    const int64_t T_ = cdiv(m, SY_BM);
    if (wj < 0) wj = T_ - j0;
    if (m <= 0 || j0 >= T_ || wj <= 0) return MG_OK;
    const int64_t ntiles = slab_tiles(T_, j0, wj);
    const dim3 grid((unsigned)(8 * cdiv(ntiles, 8)));
    if ((m + (kdim + 64) * lda) * 4 >= ((int64_t)1 << 31) - 65536 || kdim % 32 != 0) return MG_ERR_UNSUPPORTED;
    if (kdim % BFL_KC == 0 && (m + 128) * ldp * 2 < ((int64_t)1 << 31))
        hipLaunchKernelGGL(k_syrk_lower_bf16l, grid, dim3(256), 0, st, C, Pt, lda, m, (int)kdim, ldp, j0, wj, info);
    else if ((m + 1) * ldp * 2 < ((int64_t)1 << 31))
        hipLaunchKernelGGL(k_syrk_lower_bf16, grid, dim3(256), 0, st, C, Pt, lda, m, (int)kdim, ldp, j0, wj, info);
    else
        return MG_ERR_UNSUPPORTED;
    MG_LAUNCH_CHECK();
    return MG_OK;
}

// Block column [k0, k0 + nb) factored completely (diagonal block and the
// panel below it).  For nb <= 128 this is one panel_step; wider columns are
// factored right-looking in sub-steps of 128: the columns after each
// sub-step receive its update (a 128-wide slab of the trailing update)
// before their own panel step.  The caller then applies the whole panel to
// the trailing matrix in one rank-nb update, which divides the passes over
// the trailing matrix's HBM-resident entries by nb / 128.  In bfloat16 mode
// each sub-step's solved columns are packed into the block column's
// bfloat16 copy (rows below its diagonal block) and its slab runs on the
// bfloat16 matrix instruction from that copy.
template <typename T>
static mg_status panel_block(mg_handle_t h, hipStream_t st, T* A, int64_t lda, int64_t n, int64_t k0, int64_t nb,
                             int32_t* info) {
    const int64_t nbi = std::min<int64_t>(nb, FB_MAX), end = std::min(n, k0 + nb);
    __bf16* Pb = bf16_panel<T>(h, n, k0, nb);
    mg_status rc;
    for (int64_t k1 = k0; k1 < end; k1 += nbi) {
        const int64_t e = k1 + nbi, rest = end - e;
        // bfloat16 mode: the panel solve also writes this step's columns,
        // rows e .. n - 1, into the copy (a step with rows below it is a
        // full 128 columns)
        __bf16* Pq = (Pb && e < n) ? Pb + (size_t)(e - k0) * BF_LDP + (size_t)(k1 - k0) : nullptr;
        if ((rc = panel_step<T>(h, st, A, lda, n, k1, nbi, info, Pq))) return rc;
        if (!Pb) {
            if (rest > 0 && (rc = trailing<T>(h, st, A, lda, n, k1, nbi, info, 0, cdiv(rest, SY_BM)))) return rc;
            continue;
        }
        if (rest <= 0) continue;
        const int64_t mq = n - e;
        if ((rc = prof_begin(h, MG_PROF_TRAILING_NARROW, st))) return rc;
        const int64_t wj = cdiv(rest, SY_BM);
        if ((rc = bf16_update(st, (float*)(A + idx(e, e, lda)), lda, Pq, BF_LDP, mq, nbi, 0, wj, info))) return rc;
        const double c1 = (double)std::min(mq, wj * SY_BM), md = (double)mq, b = (double)nbi;
        const double elems = c1 * md - c1 * (c1 - 1) / 2;
        if ((rc = prof_end(h, MG_PROF_TRAILING_NARROW, 2.0 * b * elems, (2.0 * elems + md * b) * sizeof(T), st)))
            return rc;
    }
    return MG_OK;
}

template <typename T>
static mg_status trailing(mg_handle_t h, hipStream_t st, T* A, int64_t lda, int64_t n, int64_t k0, int64_t nb,
                         const int32_t* info, int64_t j0, int64_t wj) {
    // lower(A22) -= P P^T over tile columns [j0, j0 + wj) of the trailing matrix
    const int64_t kb = std::min(nb, n - k0), e = k0 + kb, m = n - e;
    const int64_t T_ = cdiv(m, SY_BM);
    if (wj < 0) wj = T_ - j0;
    if (m <= 0 || j0 >= T_ || wj <= 0) return MG_OK;
    mg_status rc;
    // rank-256/512 updates run the C-folding kernel variant, narrower ones the other
    const int kind = (kb % 256 == 0) ? MG_PROF_TRAILING : MG_PROF_TRAILING_NARROW;
    if ((rc = prof_begin(h, kind, st))) return rc;
    const __bf16* Pb = kb == nb ? bf16_panel<T>(h, n, k0, nb) : nullptr;
    if (Pb) {
        // bfloat16 mode, full block column: its rows below the block were
        // packed by panel_block
        if ((rc = bf16_update(st, (float*)(A + idx(e, e, lda)), lda, Pb + (size_t)kb * BF_LDP, BF_LDP, m, kb, j0, wj,
                              info)))
            return rc;
    } else if ((rc = syrk_lower_launch<T>(st, A + idx(e, e, lda), A + idx(e, k0, lda), lda, m, kb, info, j0, wj,
                                          h->trail_lo == 2 ? 1 : 0))) {
        return rc;
    }
    // algorithmic work of this slab: columns c0..c1 of the lower triangle
    const double c0 = (double)std::min(m, j0 * SY_BM), c1 = (double)std::min(m, (j0 + wj) * SY_BM);
    const double md = (double)m, b = (double)kb;
    const double elems = (c1 - c0) * md - (c1 * (c1 - 1) - c0 * (c0 - 1)) / 2;  // lower entries in the slab
    return prof_end(h, kind, 2.0 * b * elems, (2.0 * elems + (md - c0) * b) * sizeof(T), st);
}

// The two streams of the look-ahead schedule (created by mg_create, and again
// at the next factorisation after the mode changes).  In
// mode 2 the bulk stream is created with a CU mask that leaves one CU per XCD
// out (mask bits 33 x for x = 0..7: one per group of 32 consecutive bits and
// one per residue mod 8, so one per XCD whichever way the bits map to XCDs),
// so that the one-workgroup diagonal factor on the chain stream finds a CU
// the bulk update does not occupy.  A CU-masked stream synchronises with the
// legacy default stream, which the schedule never uses.
mg_status ensure_streams(mg_handle_t h) {
    if (h->side && h->side_mode == h->lookahead) return MG_OK;
    if (h->side) {
        MG_HIP(hipStreamSynchronize(h->side));
        MG_HIP(hipStreamDestroy(h->side));
        h->side = nullptr;
    }
    if (h->lookahead == 2 && h->cu_count >= 64) {
        const int words = std::min(64, (h->cu_count + 31) / 32);
        uint32_t mask[64];
        for (int k = 0; k < words; ++k) {
            const int nbits = std::min(32, h->cu_count - 32 * k);
            mask[k] = nbits >= 32 ? 0xffffffffu : ((1u << nbits) - 1u);
        }
        for (int x = 0; x < 8; ++x) {
            const int bit = 33 * x;
            if (bit < h->cu_count) mask[bit >> 5] &= ~(1u << (bit & 31));
        }
        MG_HIP(hipExtStreamCreateWithCUMask(&h->side, (uint32_t)words, mask));
    } else {
        MG_HIP(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    }
    h->side_mode = h->lookahead;
    if (h->chain) return MG_OK;
    MG_HIP(hipStreamCreateWithFlags(&h->chain, hipStreamNonBlocking));
    MG_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    MG_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    MG_HIP(hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming));
    MG_HIP(hipEventCreateWithFlags(&h->ev_rest, hipEventDisableTiming));
    return MG_OK;
}

template <typename T>
mg_status potrf_impl(mg_handle_t h, int64_t n, T* A, int64_t lda, int32_t* info) {
    hipStream_t st = h->stream;
    mg_status rc = set_info_zero(st, info);
    if (rc != MG_OK || n == 0) return rc;
    const int64_t nb = potrf_block_size(h, n, (int)sizeof(T));
    const int64_t nsteps = cdiv(n, nb);
    const int64_t wnext = nb / SY_BM;  // tile columns in the next block column
    if (!h->lookahead || nsteps < 3 || nb % SY_BM != 0) {
        for (int64_t k0 = 0; k0 < n; k0 += nb) {
            if ((rc = panel_block<T>(h, st, A, lda, n, k0, nb, info))) return rc;
            if ((rc = trailing<T>(h, st, A, lda, n, k0, nb, info, 0, -1))) return rc;
        }
        return MG_OK;
    }
    // Look-ahead: a chain stream updates the next block column with panel k,
    // then factors it and solves its panel while the second stream applies
    // panel k to everything to the right of that column, the block column
    // after next first:
    //   chain : wait(ev_rest) -> next(k) -> [ev_panel] -> panel(k+1)
    //   side  : wait(ev_panel) -> rest_a(k) -> [ev_rest] -> rest_b(k)
    // next(k+1) writes only block column k+2, which rest_a(k) finishes, so
    // the chain resumes while rest_b(k) still runs and the update stream
    // never idles on it.  The remainder is released only once next(k) is
    // done, so the one-workgroup diagonal factor of block k+1 becomes
    // runnable together with it and is dispatched before the remainder's
    // workgroups fill the chip.  Both streams are the handle's own,
    // non-blocking, and fork from / join into the caller's stream by events
    // (the side stream's last work precedes the chain's last ev_rest wait
    // or, for the final step, is empty).
    if ((rc = ensure_streams(h))) return rc;
    hipStream_t ch = h->chain;
    MG_HIP(hipEventRecord(h->ev_fork, st));
    MG_HIP(hipStreamWaitEvent(ch, h->ev_fork, 0));
    MG_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    if ((rc = panel_block<T>(h, ch, A, lda, n, 0, nb, info))) return rc;
    for (int64_t k = 0; k + 1 < nsteps; ++k) {
        const int64_t k0 = k * nb;
        if ((rc = trailing<T>(h, ch, A, lda, n, k0, nb, info, 0, wnext))) return rc;
        MG_HIP(hipEventRecord(h->ev_panel, ch));             // panel k applied to block column k+1
        MG_HIP(hipStreamWaitEvent(h->side, h->ev_panel, 0));
        if ((rc = trailing<T>(h, h->side, A, lda, n, k0, nb, info, wnext, wnext))) return rc;
        MG_HIP(hipEventRecord(h->ev_rest, h->side));         // block column k+2 has every update but panel k+1's
        if ((rc = trailing<T>(h, h->side, A, lda, n, k0, nb, info, 2 * wnext, -1))) return rc;
        if ((rc = panel_block<T>(h, ch, A, lda, n, k0 + nb, nb, info))) return rc;
        MG_HIP(hipStreamWaitEvent(ch, h->ev_rest, 0));
    }
    MG_HIP(hipEventRecord(h->ev_rest, h->side));             // the side stream's last rest_b
    MG_HIP(hipStreamWaitEvent(ch, h->ev_rest, 0));
    MG_HIP(hipEventRecord(h->ev_join, ch));
    MG_HIP(hipStreamWaitEvent(st, h->ev_join, 0));
    return MG_OK;
}

template mg_status potrf_impl<double>(mg_handle_t, int64_t, double*, int64_t, int32_t*);
template mg_status potrf_impl<float>(mg_handle_t, int64_t, float*, int64_t, int32_t*);
template mg_status syrk_lower_launch<double>(hipStream_t, double*, const double*, int64_t, int64_t, int64_t,
                                             const int32_t*, int64_t, int64_t, int);
template mg_status syrk_lower_launch<float>(hipStream_t, float*, const float*, int64_t, int64_t, int64_t,
                                            const int32_t*, int64_t, int64_t, int);

}  // namespace mg
