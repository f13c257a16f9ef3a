// potrf.hip -- blocked right-looking Cholesky A = L L^T (lower, column-major)
// on gfx950.  Paper: JAXMg "Software design", potrs bullet (Cholesky solve);
// the block size is the paper's tile size T_A.
//
// Step k of the factorisation (block columns of width nb):
//   1. k_factor_block : L_kk = chol(A_kk), one workgroup, FP64 arithmetic.
//   2. k_trsm_panel   : L_ik = A_ik L_kk^{-T} for the m = n - (k+1) nb rows
//                       below, one wave per 16 rows, MFMA + shuffle solves.
//   3. k_syrk_lower   : lower(A_22) -= L_ik L_ik^T, MFMA with LDS-staged
//                       128 x 128 tiles (about n^3/3 of the n^3/3 + O(n^2) flops).
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
// Diagonal-block factor.  One workgroup of W waves factors the s x s block at
// A (s <= 512) in place.  Left-looking over 16-wide block columns j: every
// tile (I, j), I >= j, first receives -sum_{p<j} L_Ip L_jp^T on MFMA (FP64
// accumulate), then the diagonal tile is factored in registers (factor16)
// and the tiles below it are solved against it (solve16).  S is the storage
// type, arithmetic is FP64 (the mixed-precision path keeps the diagonal
// blocks in FP64).  On a non-positive pivot, *info = col0 + local column.
// ---------------------------------------------------------------------------
template <typename S, int W>
__global__ __launch_bounds__(64 * W) void k_factor_block(S* __restrict__ A, int64_t lda, int s,
                                                         int64_t col0, int32_t* info) {
    typedef double C;
    __shared__ C Ls[16 * 17];
    __shared__ int fail;
    if (*info != 0) return;
    const int w = threadIdx.x >> 6;
    const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int nt = (s + 15) >> 4;
    if (threadIdx.x == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < nt; ++j) {
        // update phase: tile (I, j) -= sum_{p<j} L_Ip L_jp^T; the diagonal tile
        // (always the first tile of wave 0) is factored right away, the others
        // are parked back in A until L_jj is known.
        const int64_t rj = 16 * j + i;
        const bool vj = rj < s;
        for (int I = j + w; I < nt; I += W) {
            V4<C> acc;
            load_tile<S, C>(acc, A, lda, 16 * I, 16 * j, s, s, I == j, I == j);
            const int64_t ri = 16 * I + i;
            const bool vi = ri < s;
            for (int p = 0; p < j; ++p) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int64_t kk = 16 * p + 4 * ks + g;
                    const C x = vi ? (C)A[idx(ri, kk, lda)] : (C)0;
                    const C z = vj ? (C)A[idx(rj, kk, lda)] : (C)0;
                    acc = mma_xzt(acc, x, -z);
                }
            }
            if (I == j) {
                const int f = factor16<C>(acc);
                if (f) {
                    if (l == 0) fail = 16 * j + f;
                } else {
                    tile_to_lds_lower<C, 17>(acc, Ls);
                    store_tile<S, C>(acc, A, lda, 16 * j, 16 * j, s, s, true);
                }
            } else {
                store_tile<S, C>(acc, A, lda, 16 * I, 16 * j, s, s, false);
            }
        }
        __syncthreads();
        if (fail) {
            if (threadIdx.x == 0) *info = (int32_t)(col0 + fail);
            return;
        }
        // solve phase: L_Ij = (updated tile) L_jj^{-T}
        for (int I = j + 1 + w; I < nt; I += W) {
            V4<C> acc;
            load_tile<S, C>(acc, A, lda, 16 * I, 16 * j, s, s, false, false);
            solve16<C, 17>(acc, Ls);
            store_tile<S, C>(acc, A, lda, 16 * I, 16 * j, s, s, false);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Panel TRSM: X = P L^{-T} in place for the m x NB panel P, L = L_kk (NB x NB
// lower).  Each wave owns 16 panel rows and walks the NB columns in chunks of
// four 16-wide tiles held in registers:
//   - the chunk first receives -X_p L_jp^T for every earlier tile p (the
//     wave's own solved tiles, re-read from L1/L2 where it stored them, and
//     rows of L_kk shared by every wave), four independent MFMA chains;
//   - inside the chunk, tile t takes the update from tiles p < t straight from
//     registers (the k index of step ks in lane group g is 16p + tcol(g, ks),
//     exactly the column that tile p keeps in register ks), then solve16
//     against the diagonal 16 x 16 block of L_kk held in LDS.
// ---------------------------------------------------------------------------
template <typename S, int NB>
__global__ __launch_bounds__(256) void k_trsm_panel(S* __restrict__ P, const S* __restrict__ Lkk,
                                                    int64_t lda, int64_t m, const int32_t* info) {
    constexpr int NT = NB / 16;
    __shared__ S Ld[NT][16 * 17];
    if (*info != 0) return;
    for (int e = threadIdx.x; e < NT * 256; e += blockDim.x) {
        const int b = e >> 8, rr = (e >> 4) & 15, cc = e & 15;
        Ld[b][rr * 17 + cc] = (rr >= cc) ? Lkk[idx(16 * b + rr, 16 * b + cc, lda)] : (S)0;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int64_t R = ((int64_t)blockIdx.x * 4 + w) * 16;
    if (R >= m) return;
    const bool vrow = R + i < m;
    for (int jc = 0; jc < NT; jc += 4) {
        V4<S> x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) load_tile<S, S>(x[t], P, lda, R, 16 * (jc + t), m, NB, false, false);
        for (int p = 0; p < jc; ++p) {
            S xp[4];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                xp[ks] = vrow ? P[idx(R + i, 16 * p + tcol<S>(g, ks), lda)] : (S)0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const S z = Lkk[idx(16 * (jc + t) + i, 16 * p + tcol<S>(g, ks), lda)];
                    x[t] = mma_xzt(x[t], xp[ks], -z);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int p = 0; p < t; ++p) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const S z = Lkk[idx(16 * (jc + t) + i, 16 * (jc + p) + tcol<S>(g, ks), lda)];
                    x[t] = mma_xzt(x[t], x[p][ks], -z);
                }
            }
            solve16<S, 17>(x[t], Ld[jc + t]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) store_tile<S, S>(x[t], P, lda, R, 16 * (jc + t), m, NB, false);
    }
}

// ---------------------------------------------------------------------------
// Trailing update lower(C) -= P P^T, C m x m, P m x kdim (kdim % 16 == 0).
// 128 x 128 output tiles over the lower triangle only; 4 waves in a 2 x 2
// arrangement, each owning 64 x 64 = 4 x 4 MFMA tiles (64 accumulators per
// lane).  P is staged through LDS in 16-column chunks, double buffered: the
// next chunk's global loads are in flight while the current one feeds the
// MFMAs.  Tile order is XCD-aware: workgroup b runs on XCD b % 8, and each
// XCD receives a contiguous run of row-major lower tiles so that the panel
// rows they share stay in that XCD's L2.
// ---------------------------------------------------------------------------
constexpr int SY_BM = 128;
constexpr int SY_KC = 16;
constexpr int SY_LD = SY_BM + 4;

__device__ __forceinline__ void lower_tile_coords(int64_t t, int64_t& I, int64_t& J) {
    int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    I = r;
    J = t - r * (r + 1) / 2;
}

template <typename S>
__global__ __launch_bounds__(256, 2) void k_syrk_lower(S* __restrict__ Cm, const S* __restrict__ P,
                                                       int64_t lda, int64_t m, int kdim,
                                                       const int32_t* info) {
    __shared__ S As[2][SY_KC][SY_LD];
    __shared__ S Bs[2][SY_KC][SY_LD];
    if (*info != 0) return;
    const int64_t T = (m + SY_BM - 1) / SY_BM;
    const int64_t ntiles = T * (T + 1) / 2;
    const int64_t per = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntiles) return;
    int64_t I, J;
    lower_tile_coords(t, I, J);
    const bool diag = (I == J);
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, i = l & 15, g = l >> 4;
    const int wr = w >> 1, wc = w & 1;
    const bool active = !(diag && wr == 0 && wc == 1);
    const int64_t rowA0 = I * SY_BM, rowB0 = J * SY_BM;

    const int lr = tid & 127, lk = (tid >> 7) * 8;
    const bool va = rowA0 + lr < m, vb = rowB0 + lr < m;
    const S* pa = P + (rowA0 + lr) + (int64_t)lk * lda;
    const S* pb = P + (rowB0 + lr) + (int64_t)lk * lda;
    S ra[8], rb[8];

    V4<S> acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = V4<S>{0, 0, 0, 0};

    const int nk = kdim / SY_KC;
    auto gload = [&](int kc) {
        const size_t off = (size_t)kc * SY_KC * (size_t)lda;
#pragma unroll
        for (int q = 0; q < 8; ++q) ra[q] = va ? pa[off + (size_t)q * lda] : (S)0;
        if (!diag) {
#pragma unroll
            for (int q = 0; q < 8; ++q) rb[q] = vb ? pb[off + (size_t)q * lda] : (S)0;
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) As[buf][lk + q][lr] = ra[q];
        if (!diag) {
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[buf][lk + q][lr] = rb[q];
        }
    };

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) gload(kc + 1);
        if (active) {
            const S(*Xs)[SY_LD] = As[buf];
            const S(*Zs)[SY_LD] = diag ? As[buf] : Bs[buf];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = 4 * ks + g;
                S xv[4], zv[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) xv[b] = Xs[kk][64 * wr + 16 * b + i];
#pragma unroll
                for (int b = 0; b < 4; ++b) zv[b] = Zs[kk][64 * wc + 16 * b + i];
#pragma unroll
                for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mma_xzt(acc[bi][bj], xv[bi], zv[bj]);
            }
        }
        if (kc + 1 < nk) lstore(buf ^ 1);
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        const int64_t row = rowA0 + 64 * wr + 16 * bi + i;
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t col = rowB0 + 64 * wc + 16 * bj + tcol<S>(g, r);
                if (row < m && col < m && (!diag || row >= col)) {
                    S* c = Cm + idx(row, col, lda);
                    *c = *c - acc[bi][bj][r];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host driver.
// ---------------------------------------------------------------------------
int64_t potrf_block_size(mg_handle_t h, int64_t n, int es) {
    (void)es;
    if (h && h->nb > 0) return h->nb;
    if (n >= 8192) return 256;
    if (n >= 2048) return 128;
    return 64;
}

template <typename S>
static mg_status launch_trsm(hipStream_t st, int64_t nb, S* P, const S* Lkk, int64_t lda, int64_t m,
                             const int32_t* info) {
    const dim3 grid((unsigned)cdiv(m, 64)), block(256);
    switch (nb) {
        case 64: hipLaunchKernelGGL((k_trsm_panel<S, 64>), grid, block, 0, st, P, Lkk, lda, m, info); break;
        case 128: hipLaunchKernelGGL((k_trsm_panel<S, 128>), grid, block, 0, st, P, Lkk, lda, m, info); break;
        case 256: hipLaunchKernelGGL((k_trsm_panel<S, 256>), grid, block, 0, st, P, Lkk, lda, m, info); break;
        default: return MG_ERR_UNSUPPORTED;
    }
    MG_LAUNCH_CHECK();
    return MG_OK;
}

template <typename S>
mg_status syrk_lower_launch(hipStream_t st, S* Cm, const S* P, int64_t lda, int64_t m, int64_t kdim,
                            const int32_t* info) {
    const int64_t T = cdiv(m, SY_BM);
    const int64_t ntiles = T * (T + 1) / 2;
    const int64_t grid = 8 * cdiv(ntiles, 8);
    hipLaunchKernelGGL((k_syrk_lower<S>), dim3((unsigned)grid), dim3(256), 0, st, Cm, P, lda, m, (int)kdim,
                       info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

template <typename T>
mg_status potrf_impl(mg_handle_t h, int64_t n, T* A, int64_t lda, int32_t* info) {
    hipStream_t st = h->stream;
    mg_status rc = set_info_zero(st, info);
    if (rc != MG_OK || n == 0) return rc;
    const int64_t nb = potrf_block_size(h, n, (int)sizeof(T));
    for (int64_t k0 = 0; k0 < n; k0 += nb) {
        const int64_t kb = std::min(nb, n - k0);
        T* Akk = A + idx(k0, k0, lda);
        if ((rc = prof_begin(h, MG_PROF_DIAG))) return rc;
        hipLaunchKernelGGL((k_factor_block<T, 16>), dim3(1), dim3(1024), 0, st, Akk, lda, (int)kb, k0, info);
        MG_LAUNCH_CHECK();
        const double b = (double)kb;
        if ((rc = prof_end(h, MG_PROF_DIAG, b * b * b / 3 + b * b / 2 + b / 6, b * (b + 1) * sizeof(T))))
            return rc;
        const int64_t m = n - k0 - kb;
        if (m <= 0) break;
        T* P = A + idx(k0 + kb, k0, lda);
        if ((rc = prof_begin(h, MG_PROF_TRSM))) return rc;
        if ((rc = launch_trsm<T>(st, nb, P, Akk, lda, m, info))) return rc;
        if ((rc = prof_end(h, MG_PROF_TRSM, (double)m * b * b, 2.0 * m * b * sizeof(T)))) return rc;
        if ((rc = prof_begin(h, MG_PROF_TRAILING))) return rc;
        if ((rc = syrk_lower_launch<T>(st, A + idx(k0 + kb, k0 + kb, lda), P, lda, m, kb, info))) return rc;
        // algorithmic traffic: read the panel once, read+write the lower triangle once
        const double md = (double)m;
        if ((rc = prof_end(h, MG_PROF_TRAILING, b * md * (md + 1),
                           (md * b + md * (md + 1)) * sizeof(T))))
            return rc;
    }
    return MG_OK;
}

template mg_status potrf_impl<double>(mg_handle_t, int64_t, double*, int64_t, int32_t*);
template mg_status potrf_impl<float>(mg_handle_t, int64_t, float*, int64_t, int32_t*);
template mg_status syrk_lower_launch<double>(hipStream_t, double*, const double*, int64_t, int64_t, int64_t,
                                             const int32_t*);
template mg_status syrk_lower_launch<float>(hipStream_t, float*, const float*, int64_t, int64_t, int64_t,
                                            const int32_t*);

}  // namespace mg
