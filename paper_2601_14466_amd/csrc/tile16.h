// tile16.h -- wave-level building blocks on 16x16 tiles for gfx950 (CDNA4).
//
// A 16x16 tile Y is held by one 64-lane wave in "row-per-lane" layout:
//   lane l = 16*g + i (i = l % 16, g = l / 16) holds, in register r = 0..3,
//   Y[i][tcol<C>(g, r)].
// Row i lives in the 4 lanes {i, 16+i, 32+i, 48+i}; a register r of the four
// lane groups covers four columns.  Loading or storing a tile of a
// column-major matrix in this layout is coalesced: each register moves four
// 128-byte column segments (16 consecutive rows each).
//
// The layout is the transpose of the MFMA 16x16x4 result.  The instruction
// computes D[row][col] += sum_k A[row][k] B[k][col] with lane l supplying
// A[l%16][l/16] and B[l/16][l%16].  Lane l receives D[row][l%16] in register
// r, where measured on gfx950
//   f32 (v_mfma_f32_16x16x4_f32): row = 4*(l/16) + r
//   f64 (v_mfma_f64_16x16x4_f64): row = 4*r + l/16
// so tcol is 4g + r for float and 4r + g for double.  Reading D as Y^T gives
//   Y += X Z^T   with lane l supplying x = X[l%16][k_l], z = Z[l%16][k_l]
// where k_l is any bijection between (lane group, step) and the k range that
// both operands share.  Everything below uses that form.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mg {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef f64x4 type; };
template <> struct Vec4<float> { typedef f32x4 type; };
template <typename T> using V4 = typename Vec4<T>::type;

// Column held by register r of lane group g, and its inverse.
template <typename C> __host__ __device__ constexpr int tcol(int g, int r);
template <> __host__ __device__ constexpr int tcol<float>(int g, int r) { return 4 * g + r; }
template <> __host__ __device__ constexpr int tcol<double>(int g, int r) { return 4 * r + g; }
template <typename C> __host__ __device__ constexpr int tgrp(int c);   // lane group owning column c
template <typename C> __host__ __device__ constexpr int treg(int c);   // register holding column c
template <> __host__ __device__ constexpr int tgrp<float>(int c) { return c >> 2; }
template <> __host__ __device__ constexpr int treg<float>(int c) { return c & 3; }
template <> __host__ __device__ constexpr int tgrp<double>(int c) { return c & 3; }
template <> __host__ __device__ constexpr int treg<double>(int c) { return c >> 2; }

// Y (tile layout, accumulator) += X Z^T over one k-step: lane supplies
// x = X[i][k_l] and z = Z[i][k_l].
__device__ __forceinline__ f64x4 mma_xzt(f64x4 acc, double x, double z) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(z, x, acc, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_xzt(f32x4 acc, float x, float z) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(z, x, acc, 0, 0, 0);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ double shfl(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float shfl(float v, int src) { return __shfl(v, src, 64); }

// Row broadcast: every lane (i, g) receives the value of lane (i, G), G a
// wave-uniform lane group (rows of 16 lanes; a constant in the unrolled
// loops that call it, so the selects fold away).  Two gfx950 lane swaps instead
// of an LDS permute: permlane16_swap pairs rows 0/1 and 2/3, giving either
// (R0 R0 R2 R2) or (R1 R1 R3 R3); permlane32_swap of that pairs the halves,
// giving one row in all four.
__device__ __forceinline__ unsigned rowbcast_u32(unsigned v, int G) {
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    const unsigned x = (G & 1) ? a[1] : a[0];
    const auto b = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (G & 2) ? b[1] : b[0];
}
__device__ __forceinline__ float rowbcast(float v, int G) {
    return __builtin_bit_cast(float, rowbcast_u32(__builtin_bit_cast(unsigned, v), G));
}
__device__ __forceinline__ double rowbcast(double v, int G) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = rowbcast_u32((unsigned)b, G), hi = rowbcast_u32((unsigned)(b >> 32), G);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Broadcast lane `src` (wave-uniform) through the scalar unit.
__device__ __forceinline__ float readlane(float v, int src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double readlane(double v, int src) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__host__ __device__ __forceinline__ size_t idx(int64_t i, int64_t j, int64_t ld) {
    return (size_t)i + (size_t)j * (size_t)ld;
}

// Load the 16x16 tile at (r0, c0) of column-major M into tile layout.
// Rows >= rmax or columns >= cmax read as 0, except that on the diagonal of a
// diagonal tile (diag_pad) they read as 1, so padding behaves like identity.
// With lower_only, entries strictly above the tile diagonal are not read (0).
template <typename S, typename C>
__device__ __forceinline__ void load_tile(V4<C>& y, const S* M, int64_t ld, int64_t r0, int64_t c0,
                                          int64_t rmax, int64_t cmax, bool lower_only, bool diag_pad) {
    const int l = lane_id(), i = l & 15, g = l >> 4;
    const int64_t row = r0 + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int jj = tcol<C>(g, r);
        const int64_t col = c0 + jj;
        C v = 0;
        if (row < rmax && col < cmax && (!lower_only || i >= jj))
            v = (C)M[idx(row, col, ld)];
        else if (diag_pad && i == jj)
            v = 1;
        y[r] = v;
    }
}

// Store a tile; rows >= rmax / columns >= cmax are skipped; with lower_only
// only entries on or below the tile diagonal are written.
template <typename S, typename C>
__device__ __forceinline__ void store_tile(const V4<C>& y, S* M, int64_t ld, int64_t r0, int64_t c0,
                                           int64_t rmax, int64_t cmax, bool lower_only) {
    const int l = lane_id(), i = l & 15, g = l >> 4;
    const int64_t row = r0 + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int jj = tcol<C>(g, r);
        const int64_t col = c0 + jj;
        if (row < rmax && col < cmax && (!lower_only || i >= jj))
            M[idx(row, col, ld)] = (S)y[r];
    }
}

// p^(-1/2) for p > 0: the hardware estimate refined by two Newton steps on
// FMAs (y += y/2 (1 - p y^2)), within one unit in the last place; exact when
// p is an even power of two (the Newton residual is then exact and the step
// lands on 2^-k).  Replaces a square root followed by a division on the
// factor's critical path.
__device__ __forceinline__ double rsqrt_nr(double p) {
    double y = __builtin_amdgcn_rsq(p);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double py = p * y;
        y = __builtin_fma(0.5 * y, __builtin_fma(-py, y, 1.0), y);
    }
    return y;
}
__device__ __forceinline__ float rsqrt_nr(float p) {
    float y = __builtin_amdgcn_rsqf(p);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const float py = p * y;
        y = __builtin_fmaf(0.5f * y, __builtin_fmaf(-py, y, 1.0f), y);
    }
    return y;
}

// In-register Cholesky of a 16x16 SPD tile (lower part significant).  Column
// by column: column c is scaled by p^(-1/2) (its diagonal entry becomes
// p p^(-1/2)), and the columns to its right receive the rank-1 update; the
// lane shuffles that fetch L[j][c] are issued starting with the register that
// holds column c + 1.  With PIVOT_AHEAD the next column is also formed
// directly, in every lane group:
//   Y[i][c+1] - L[i][c] L[c+1][c],
// from its row broadcast taken before the update and the lane read of
// L[c+1][c]. It uses the same fused multiply-add as the lanes' update, so it
// is bitwise the value the lanes end up holding; its entry c+1 is the next
// pivot. The chain from column to column then runs through lane reads and
// FMAs only, and the shuffles have a column of slack. Without PIVOT_AHEAD
// (for callers whose register cap leaves no room for the carried column),
// each column is broadcast from the updated registers.  Returns 0, or c+1 for
// the first local column whose pivot is not > 0 (NaN included); the decision
// is uniform across the wave.  The columns after a failing one are computed
// on meaningless values (no exit per column, so the compiler can schedule
// across columns) and, like the entries above the diagonal, are unspecified.
template <typename C, bool PIVOT_AHEAD = true>
__device__ __forceinline__ int factor16(V4<C>& y) {
    const int l = lane_id(), i = l & 15, g = l >> 4;
    int fail = 0;
    C p = readlane(y[treg<C>(0)], tgrp<C>(0) * 16);  // pivot of column c
    C vc = rowbcast(y[treg<C>(0)], tgrp<C>(0));      // column c: Y[i][c] in lane group g, row i
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int gc = tgrp<C>(c), rc = treg<C>(c);
        if constexpr (!PIVOT_AHEAD) {
            p = readlane(y[rc], gc * 16 + c);
            vc = rowbcast(y[rc], gc);
        }
        if (fail == 0 && !(p > (C)0)) fail = c + 1;
        const C rs = rsqrt_nr(p);
        const C lic = (i > c) ? vc * rs : (i == c ? p * rs : (C)0);
        C vn = (C)0;
        if (PIVOT_AHEAD && c < 15) {
            const C yb = rowbcast(y[treg<C>(c + 1)], tgrp<C>(c + 1));  // Y[i][c+1] before the update
            const C lnc = readlane(lic, c + 1);                           // L[c+1][c]
            vn = __builtin_fma(-lic, lnc, yb);
        }
        y[rc] = (g == gc) ? lic : y[rc];
        const int rn = c < 15 ? treg<C>(c + 1) : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = (rn + q) & 3;
            const int j = tcol<C>(g, r);
            const C ljc = shfl(lic, j);         // L[j][c] sits in lane j (group 0)
            // (the carried column must equal this value bit for bit: same fma)
            const C t = PIVOT_AHEAD ? __builtin_fma(-lic, ljc, y[r]) : y[r] - lic * ljc;
            y[r] = (j > c) ? t : y[r];
        }
        if constexpr (PIVOT_AHEAD) {
            if (c < 15) {
                vc = vn;
                p = readlane(vn, c + 1);
            }
        }
    }
    return fail;
}

// X = Y L^{-T} with L pre-scaled by columns: Lsc[j*LDL + c] = L(j,c)/L(c,c)
// for j > c, exactly 0 elsewhere (relied on: see below), and piv[c] = L(c,c).  Column c of Y is final after
// the updates from the columns before it; it is broadcast along its row and
// applied to the columns after it (one shuffle and up to four FMAs), and each
// column is divided by its pivot once at the end.  Exact for integer data
// with power-of-two pivots.
template <typename C, int LDL, bool GUARDED = false>
__device__ __forceinline__ void solve16s(V4<C>& y, const C* Lsc, const C* piv) {
    const int l = lane_id(), i = l & 15, g = l >> 4;
#pragma unroll
    for (int c = 0; c < 15; ++c) {
        const int gc = tgrp<C>(c), rc = treg<C>(c);
        const C yc = rowbcast(y[rc], gc);  // (updated) Y[i][c]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = tcol<C>(g, r);
            if constexpr (GUARDED) {
                if (j > c) y[r] = y[r] - yc * Lsc[j * LDL + c];
            } else {
                // Applied to every column: Lsc holds exact zeros for j <= c,
                // so those columns keep their (finite) values.  A guard on
                // j > c differs between lane groups, and the compiler turns
                // it into a branch with the LDS read of L inside, unhoisted,
                // which left every step waiting for LDS.  The guarded form
                // holds fewer values in registers, for callers that are
                // short of them.
                y[r] = y[r] - yc * Lsc[j * LDL + c];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = y[r] / piv[tcol<C>(g, r)];
}

// solve16s on two independent tiles at once (same L): their dependency
// chains interleave, so one wave hides most of the latency of either.
template <typename C, int LDL>
__device__ __forceinline__ void solve16s2(V4<C>& y, V4<C>& u, const C* Lsc, const C* piv) {
    const int l = lane_id(), g = (l & 63) >> 4;
#pragma unroll
    for (int c = 0; c < 15; ++c) {
        const int gc = tgrp<C>(c), rc = treg<C>(c);
        const C yc = rowbcast(y[rc], gc), uc = rowbcast(u[rc], gc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // guarded (unlike solve16s): with two tiles in flight, hoisting
            // every read of L would take this past 256 registers per wave
            const int j = tcol<C>(g, r);
            if (j > c) {
                const C lv = Lsc[j * LDL + c];
                y[r] = y[r] - yc * lv;
                u[r] = u[r] - uc * lv;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const C pv = piv[tcol<C>(g, r)];
        y[r] = y[r] / pv;
        u[r] = u[r] / pv;
    }
}

// Column-scaled copy of a lower-triangular 16x16 L held in LDS (Ls, row-major
// with leading dimension LDL): Lsc(j,c) = L(j,c)/L(c,c) for j > c, 0
// elsewhere; piv[c] = L(c,c).  One thread per entry; callers synchronise.
template <typename C, int LDL>
__device__ __forceinline__ void scale_lower16(const C* Ls, C* Lsc, C* piv, int t) {
    if (t < 256) {
        const int j = t >> 4, c = t & 15;
        Lsc[j * LDL + c] = (j > c) ? Ls[j * LDL + c] / Ls[c * LDL + c] : (C)0;
        if (j == c) piv[c] = Ls[c * LDL + c];
    }
}

// Write a factored diagonal tile (tile layout) into LDS as Ls[row*LDL+col],
// zeroing the strict upper part.
template <typename C, int LDL>
__device__ __forceinline__ void tile_to_lds_lower(const V4<C>& y, C* Ls) {
    const int l = lane_id(), i = l & 15, g = l >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = tcol<C>(g, r);
        Ls[i * LDL + j] = (i >= j) ? y[r] : (C)0;
    }
}

}  // namespace mg
