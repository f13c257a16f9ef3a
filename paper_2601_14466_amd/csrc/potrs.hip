// potrs.hip -- X = A^{-1} B from the Cholesky factor: L Y = B, then L^T X = Y.
// Paper: JAXMg "Software design", potrs bullet (b is N x N_RHS).
//
// Both sweeps are blocked by JB = 64 rows and take one launch per block,
// right-looking, so every launch is parallel over the rows it updates:
//   forward step j : every workgroup solves L_jj Y_j = B_j (64 x 64 lower in
//                    LDS, 16 right-hand sides per wave, the solved value
//                    broadcast by the scalar unit), workgroup 0 stores Y_j in
//                    the workspace, and all workgroups apply
//                    B_i -= L_ij Y_j to the rows below (coalesced: one thread
//                    per row, consecutive rows on consecutive lanes).
//   backward step j: every workgroup solves L_jj^T X_j = Y_j, workgroup 0
//                    stores X_j into B, and all apply Y_i -= L_ji^T X_j to the
//                    rows above; L_ji^T is staged through LDS in 64 x 64 tiles
//                    so the global reads stay column-contiguous.
// The two sweeps read the lower triangle once each (HBM-bound: the
// arithmetic intensity is nrhs/4 flop per byte in FP64).
#include <algorithm>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

constexpr int JB = 64;     // rows per block step
constexpr int RCH = 64;    // right-hand sides handled per pass
constexpr int RPT = 16;    // right-hand sides per thread / per wave

size_t potrs_work_bytes(int64_t n, int64_t nrhs, int es) {
    return (size_t)n * (size_t)nrhs * (size_t)es;
}

// Load the jb x jb lower-triangular diagonal block at L(j0, j0) into LDS,
// row-major with leading dimension JB + 1, strict upper part zero.
template <typename T>
__device__ __forceinline__ void load_diag_block(T* Ls, const T* L, int64_t lda, int64_t j0, int jb) {
    for (int e = threadIdx.x; e < JB * JB; e += blockDim.x) {
        const int rr = e & (JB - 1), cc = e >> 6;  // consecutive threads: consecutive rows
        T v = 0;
        if (rr < jb && cc < jb && rr >= cc) v = L[idx(j0 + rr, j0 + cc, lda)];
        Ls[rr * (JB + 1) + cc] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd_step(const T* __restrict__ L, int64_t lda, int64_t n,
                                                       int64_t nrhs, T* __restrict__ B, int64_t ldb,
                                                       T* __restrict__ Y, int64_t ldy, int64_t j0, int jb,
                                                       const int32_t* info) {
    __shared__ T Ls[JB * (JB + 1)];
    __shared__ T Ys[JB * RCH];
    if (info && *info != 0) return;
    load_diag_block(Ls, L, lda, j0, jb);
    __syncthreads();
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int64_t rc0 = 0; rc0 < nrhs; rc0 += RCH) {
        const int nr = (int)std::min<int64_t>(RCH, nrhs - rc0);
        // --- diagonal solve, wave w takes right-hand sides [16w, 16w+16)
        if (RPT * w < nr) {
            T v[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int col = RPT * w + r;
                v[r] = (lane < jb && col < nr) ? B[idx(j0 + lane, rc0 + col, ldb)] : (T)0;
            }
            for (int c = 0; c < jb; ++c) {
                const T rinv = (T)1 / Ls[c * (JB + 1) + c];
                const T lic = Ls[lane * (JB + 1) + c];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const T yc = readlane(v[r], c) * rinv;
                    if (lane == c) v[r] = yc;
                    else if (lane > c) v[r] = v[r] - lic * yc;
                }
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int col = RPT * w + r;
                Ys[lane * RCH + col] = v[r];
                if (blockIdx.x == 0 && lane < jb && col < nr) Y[idx(j0 + lane, rc0 + col, ldy)] = v[r];
            }
        }
        __syncthreads();
        // --- update of the rows below: B_i -= L_ij Y_j
        const int tpr = (nr + RPT - 1) / RPT;        // threads per row
        const int rpw = 256 / tpr;                   // rows per workgroup
        const int q = tid % tpr;
        const int64_t row = j0 + jb + (int64_t)blockIdx.x * rpw + tid / tpr;
        if (tid / tpr < rpw && row < n) {
            T acc[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int col = RPT * q + r;
                acc[r] = col < nr ? B[idx(row, rc0 + col, ldb)] : (T)0;
            }
            for (int c = 0; c < jb; ++c) {
                const T a = L[idx(row, j0 + c, lda)];
#pragma unroll
                for (int r = 0; r < RPT; ++r) acc[r] = acc[r] - a * Ys[c * RCH + RPT * q + r];
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int col = RPT * q + r;
                if (col < nr) B[idx(row, rc0 + col, ldb)] = acc[r];
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd_step(const T* __restrict__ L, int64_t lda, int64_t n,
                                                       int64_t nrhs, T* __restrict__ B, int64_t ldb,
                                                       T* __restrict__ Y, int64_t ldy, int64_t j0, int jb,
                                                       const int32_t* info) {
    __shared__ T Ls[JB * (JB + 1)];
    __shared__ T Xs[JB * RCH];
    __shared__ T Lt[64 * (JB + 1)];  // Lt[rr][c] = L(j0 + c, r0 + rr)
    if (info && *info != 0) return;
    load_diag_block(Ls, L, lda, j0, jb);
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const bool have_rows = r0 < j0;
    if (have_rows) {
        for (int e = tid; e < 64 * JB; e += blockDim.x) {
            const int c = e & (JB - 1), rr = e >> 6;  // consecutive threads: consecutive c (contiguous)
            T v = 0;
            if (c < jb && r0 + rr < j0) v = L[idx(j0 + c, r0 + rr, lda)];
            Lt[rr * (JB + 1) + c] = v;
        }
    }
    __syncthreads();
    (void)n;
    for (int64_t rc0 = 0; rc0 < nrhs; rc0 += RCH) {
        const int nr = (int)std::min<int64_t>(RCH, nrhs - rc0);
        if (RPT * w < nr) {
            T v[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int col = RPT * w + r;
                v[r] = (lane < jb && col < nr) ? Y[idx(j0 + lane, rc0 + col, ldy)] : (T)0;
            }
            for (int c = jb - 1; c >= 0; --c) {
                const T rinv = (T)1 / Ls[c * (JB + 1) + c];
                const T lci = Ls[c * (JB + 1) + lane];   // L(c, lane), zero for lane > c
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const T xc = readlane(v[r], c) * rinv;
                    if (lane == c) v[r] = xc;
                    else if (lane < c) v[r] = v[r] - lci * xc;
                }
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int col = RPT * w + r;
                Xs[lane * RCH + col] = v[r];
                if (blockIdx.x == 0 && lane < jb && col < nr) B[idx(j0 + lane, rc0 + col, ldb)] = v[r];
            }
        }
        __syncthreads();
        if (have_rows) {
            const int tpr = (nr + RPT - 1) / RPT;
            const int rr = tid / tpr, q = tid % tpr;
            const int64_t row = r0 + rr;
            if (rr < 64 && row < j0) {
                T acc[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int col = RPT * q + r;
                    acc[r] = col < nr ? Y[idx(row, rc0 + col, ldy)] : (T)0;
                }
                for (int c = 0; c < jb; ++c) {
                    const T a = Lt[rr * (JB + 1) + c];
#pragma unroll
                    for (int r = 0; r < RPT; ++r) acc[r] = acc[r] - a * Xs[c * RCH + RPT * q + r];
                }
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int col = RPT * q + r;
                    if (col < nr) Y[idx(row, rc0 + col, ldy)] = acc[r];
                }
            }
        }
        __syncthreads();
    }
}

template <typename T>
mg_status potrs_impl(mg_handle_t h, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B, int64_t ldb,
                     T* Y, const int32_t* info) {
    if (n == 0 || nrhs == 0) return MG_OK;
    hipStream_t st = h->stream;
    const int64_t ldy = n;
    const int64_t nblk = cdiv(n, JB);
    const int tpr = (int)((std::min<int64_t>(nrhs, RCH) + RPT - 1) / RPT);
    const int rpw = 256 / tpr;
    mg_status rc;
    if ((rc = prof_begin(h, MG_PROF_SOLVE))) return rc;
    for (int64_t jbk = 0; jbk < nblk; ++jbk) {
        const int64_t j0 = jbk * JB;
        const int jb = (int)std::min<int64_t>(JB, n - j0);
        const int64_t below = n - j0 - jb;
        const int64_t grid = std::max<int64_t>(1, cdiv(below, rpw));
        hipLaunchKernelGGL((k_trsv_fwd_step<T>), dim3((unsigned)grid), dim3(256), 0, st, L, lda, n, nrhs, B, ldb,
                           Y, ldy, j0, jb, info);
        MG_LAUNCH_CHECK();
    }
    for (int64_t jbk = nblk - 1; jbk >= 0; --jbk) {
        const int64_t j0 = jbk * JB;
        const int jb = (int)std::min<int64_t>(JB, n - j0);
        const int64_t grid = std::max<int64_t>(1, cdiv(j0, 64));
        hipLaunchKernelGGL((k_trsv_bwd_step<T>), dim3((unsigned)grid), dim3(256), 0, st, L, lda, n, nrhs, B, ldb,
                           Y, ldy, j0, jb, info);
        MG_LAUNCH_CHECK();
    }
    const double nd = (double)n;
    return prof_end(h, MG_PROF_SOLVE, 2.0 * nd * nd * (double)nrhs,
                    (nd * (nd + 1) + 4.0 * nd * (double)nrhs) * sizeof(T));
}

template mg_status potrs_impl<double>(mg_handle_t, int64_t, int64_t, const double*, int64_t, double*, int64_t,
                                      double*, const int32_t*);
template mg_status potrs_impl<float>(mg_handle_t, int64_t, int64_t, const float*, int64_t, float*, int64_t,
                                     float*, const int32_t*);

}  // namespace mg
