// potrs.hip -- X = A^{-1} B from the Cholesky factor: L Y = B, then L^T X = Y.
// Paper: JAXMg "Software design", potrs bullet (b is N x N_RHS).
//
// Both sweeps are blocked by JB = 64 rows and take one launch per block,
// right-looking, so each launch is parallel over the rows it updates:
//   forward step j : every workgroup solves L_jj Y_j = B_j, workgroup 0 keeps
//                    Y_j in the workspace, and every workgroup applies
//                    B_i -= L_ij Y_j to its own 64 rows below the block.
//   backward step j: every workgroup solves L_jj^T X_j = Y_j, workgroup 0
//                    stores X_j into B, and every workgroup applies
//                    Y_i -= L_ji^T X_j to its own 64 rows above the block.
// The diagonal solve is a substitution in registers: a lane per row, the four
// waves splitting the right-hand sides, each step's pivot row broadcast by
// the scalar unit (readlane).  L_jj is staged pre-scaled by its pivots
// (column c divided by L_cc for the forward sweep, row c for the backward one,
// diagonal set to 0), so a step is one readlane and one FMA per value and the
// division by the pivot happens once per value at the end.  Integer data with
// power-of-two pivots stays exact under this scaling.
// The 64 x 64 block of L that a workgroup applies is staged through LDS with
// all of its global loads in flight together (column-contiguous for both
// sweeps).  Each sweep reads the lower triangle once: HBM-bound, arithmetic
// intensity nrhs/4 flop per byte in FP64.
#include <algorithm>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

constexpr int JB = 64;       // rows per block step
constexpr int LDP = JB + 1;  // LDS leading dimension (bank spread)

size_t potrs_work_bytes(int64_t n, int64_t nrhs, int es) {
    return (size_t)n * (size_t)nrhs * (size_t)es;
}

// L_jj (jb x jb lower, identity-padded to 64 x 64) into Ls[r*LDP + c] scaled
// by its pivots: by column (Ls(r,c) = L(r,c)/L(c,c)) when by_row is false,
// by row (Ls(r,c) = L(r,c)/L(r,r)) when it is true; the diagonal of Ls is 0
// and piv holds L(c,c).
template <typename T, bool by_row>
__device__ __forceinline__ void stage_diag(T* Ls, T* piv, const T* L, int64_t lda, int64_t j0, int jb) {
    const int tid = threadIdx.x;
    T v[JB * JB / 256];
#pragma unroll
    for (int q = 0; q < JB * JB / 256; ++q) {
        const int e = tid + 256 * q;
        const int rr = e & (JB - 1), cc = e >> 6;
        v[q] = (rr < jb && cc < jb && rr >= cc) ? L[idx(j0 + rr, j0 + cc, lda)] : (T)(rr == cc ? 1 : 0);
        if (rr == cc) piv[rr] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < JB * JB / 256; ++q) {
        const int e = tid + 256 * q;
        const int rr = e & (JB - 1), cc = e >> 6;
        Ls[rr * LDP + cc] = (rr == cc) ? (T)0 : v[q] / piv[by_row ? rr : cc];
    }
}

// Lt[rr*LDP + c] = L(rbase + rr, cbase + c) when transpose == false (panel
// rows), or L(cbase + c, rbase + rr) when transpose == true (the block row of
// L read as L^T); out-of-range entries are 0.
template <typename T, bool transpose>
__device__ __forceinline__ void stage_panel(T* Lt, const T* L, int64_t lda, int64_t rbase, int64_t rlim,
                                            int64_t cbase, int clim) {
    const int tid = threadIdx.x;
    T v[JB * JB / 256];
#pragma unroll
    for (int q = 0; q < JB * JB / 256; ++q) {
        const int e = tid + 256 * q;
        // consecutive threads walk the contiguous direction of the column-major source
        const int a = e & (JB - 1), b = e >> 6;
        const int rr = transpose ? b : a, c = transpose ? a : b;
        const bool ok = rbase + rr < rlim && c < clim;
        v[q] = ok ? (transpose ? L[idx(cbase + c, rbase + rr, lda)] : L[idx(rbase + rr, cbase + c, lda)]) : (T)0;
    }
#pragma unroll
    for (int q = 0; q < JB * JB / 256; ++q) {
        const int e = tid + 256 * q;
        const int a = e & (JB - 1), b = e >> 6;
        const int rr = transpose ? b : a, c = transpose ? a : b;
        Lt[rr * LDP + c] = v[q];
    }
}

// Forward step j.  RPT right-hand sides per wave, 4*RPT per pass.
template <typename T, int RPT>
__global__ __launch_bounds__(256) void k_trsv_fwd(const T* __restrict__ L, int64_t lda, int64_t n, int64_t nrhs,
                                                  T* __restrict__ B, int64_t ldb, T* __restrict__ Y, int64_t ldy,
                                                  int64_t j0, int jb, const int32_t* info) {
    constexpr int RCH = 4 * RPT;
    __shared__ T Ls[JB * LDP];
    __shared__ T Lp[JB * LDP];
    __shared__ T piv[JB];
    __shared__ T Ys[JB * RCH];
    if (info && *info != 0) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t row0 = j0 + jb + (int64_t)blockIdx.x * JB;
    const bool have_rows = row0 < n;
    stage_diag<T, false>(Ls, piv, L, lda, j0, jb);
    if (have_rows) stage_panel<T, false>(Lp, L, lda, row0, n, j0, jb);
    __syncthreads();
    const T pl = piv[lane];
    const int64_t row = row0 + lane;
    for (int64_t rc0 = 0; rc0 < nrhs; rc0 += RCH) {
        const int cb = (int)rc0 + RPT * w;  // first right-hand side of this wave
        // ---- diagonal solve L_jj y = b for the wave's RPT columns
        T v[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            v[r] = (lane < jb && cb + r < nrhs) ? B[idx(j0 + lane, cb + r, ldb)] : (T)0;
#pragma unroll 8
        for (int c = 0; c < JB; ++c) {
            const T lic = Ls[lane * LDP + c];   // L(lane,c)/L(c,c), 0 unless lane > c
#pragma unroll
            for (int r = 0; r < RPT; ++r) v[r] = v[r] - lic * readlane(v[r], c);
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            v[r] = v[r] / pl;
            Ys[lane * RCH + RPT * w + r] = v[r];
            if (blockIdx.x == 0 && lane < jb && cb + r < nrhs) Y[idx(j0 + lane, cb + r, ldy)] = v[r];
        }
        __syncthreads();
        // ---- B_i -= L_ij Y_j for the workgroup's 64 rows
        if (have_rows && row < n) {
            T acc[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) acc[r] = (cb + r < nrhs) ? B[idx(row, cb + r, ldb)] : (T)0;
#pragma unroll 8
            for (int c = 0; c < JB; ++c) {
                const T a = Lp[lane * LDP + c];
#pragma unroll
                for (int r = 0; r < RPT; ++r) acc[r] = acc[r] - a * Ys[c * RCH + RPT * w + r];
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (cb + r < nrhs) B[idx(row, cb + r, ldb)] = acc[r];
        }
        __syncthreads();
    }
}

// Backward step j.
template <typename T, int RPT>
__global__ __launch_bounds__(256) void k_trsv_bwd(const T* __restrict__ L, int64_t lda, int64_t n, int64_t nrhs,
                                                  T* __restrict__ B, int64_t ldb, T* __restrict__ Y, int64_t ldy,
                                                  int64_t j0, int jb, const int32_t* info) {
    constexpr int RCH = 4 * RPT;
    __shared__ T Ls[JB * LDP];
    __shared__ T Lt[JB * LDP];
    __shared__ T piv[JB];
    __shared__ T Xs[JB * RCH];
    if (info && *info != 0) return;
    (void)n;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t r0 = (int64_t)blockIdx.x * JB;
    const bool have_rows = r0 < j0;
    stage_diag<T, true>(Ls, piv, L, lda, j0, jb);
    if (have_rows) stage_panel<T, true>(Lt, L, lda, r0, j0, j0, jb);
    __syncthreads();
    const T pl = piv[lane];
    const int64_t row = r0 + lane;
    for (int64_t rc0 = 0; rc0 < nrhs; rc0 += RCH) {
        const int cb = (int)rc0 + RPT * w;
        T v[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            v[r] = (lane < jb && cb + r < nrhs) ? Y[idx(j0 + lane, cb + r, ldy)] : (T)0;
#pragma unroll 8
        for (int c = JB - 1; c >= 0; --c) {
            const T lci = Ls[c * LDP + lane];  // L(c,lane)/L(c,c), 0 unless lane < c
#pragma unroll
            for (int r = 0; r < RPT; ++r) v[r] = v[r] - lci * readlane(v[r], c);
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            v[r] = v[r] / pl;
            Xs[lane * RCH + RPT * w + r] = v[r];
            if (blockIdx.x == 0 && lane < jb && cb + r < nrhs) B[idx(j0 + lane, cb + r, ldb)] = v[r];
        }
        __syncthreads();
        if (have_rows && row < j0) {
            T acc[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) acc[r] = (cb + r < nrhs) ? Y[idx(row, cb + r, ldy)] : (T)0;
#pragma unroll 8
            for (int c = 0; c < JB; ++c) {
                const T a = Lt[lane * LDP + c];
#pragma unroll
                for (int r = 0; r < RPT; ++r) acc[r] = acc[r] - a * Xs[c * RCH + RPT * w + r];
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (cb + r < nrhs) Y[idx(row, cb + r, ldy)] = acc[r];
        }
        __syncthreads();
    }
}

template <typename T, int RPT>
static mg_status sweep(hipStream_t st, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B, int64_t ldb, T* Y,
                       const int32_t* info) {
    const int64_t nblk = cdiv(n, JB);
    for (int64_t jbk = 0; jbk < nblk; ++jbk) {
        const int64_t j0 = jbk * JB;
        const int jb = (int)std::min<int64_t>(JB, n - j0);
        const int64_t grid = std::max<int64_t>(1, cdiv(n - j0 - jb, JB));
        hipLaunchKernelGGL((k_trsv_fwd<T, RPT>), dim3((unsigned)grid), dim3(256), 0, st, L, lda, n, nrhs, B, ldb, Y,
                           n, j0, jb, info);
        MG_LAUNCH_CHECK();
    }
    for (int64_t jbk = nblk - 1; jbk >= 0; --jbk) {
        const int64_t j0 = jbk * JB;
        const int jb = (int)std::min<int64_t>(JB, n - j0);
        const int64_t grid = std::max<int64_t>(1, cdiv(j0, JB));
        hipLaunchKernelGGL((k_trsv_bwd<T, RPT>), dim3((unsigned)grid), dim3(256), 0, st, L, lda, n, nrhs, B, ldb, Y,
                           n, j0, jb, info);
        MG_LAUNCH_CHECK();
    }
    return MG_OK;
}

template <typename T>
mg_status potrs_impl(mg_handle_t h, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B, int64_t ldb, T* Y,
                     const int32_t* info) {
    if (n == 0 || nrhs == 0) return MG_OK;
    hipStream_t st = h->stream;
    mg_status rc;
    if ((rc = prof_begin(h, MG_PROF_SOLVE, st))) return rc;
    if (nrhs <= 4) rc = sweep<T, 1>(st, n, nrhs, L, lda, B, ldb, Y, info);
    else if (nrhs <= 8) rc = sweep<T, 2>(st, n, nrhs, L, lda, B, ldb, Y, info);
    else if (nrhs <= 16) rc = sweep<T, 4>(st, n, nrhs, L, lda, B, ldb, Y, info);
    else if (nrhs <= 32) rc = sweep<T, 8>(st, n, nrhs, L, lda, B, ldb, Y, info);
    else rc = sweep<T, 16>(st, n, nrhs, L, lda, B, ldb, Y, info);
    if (rc) return rc;
    const double nd = (double)n;
    return prof_end(h, MG_PROF_SOLVE, 2.0 * nd * nd * (double)nrhs,
                    (nd * (nd + 1) + 4.0 * nd * (double)nrhs) * sizeof(T), st);
}

template mg_status potrs_impl<double>(mg_handle_t, int64_t, int64_t, const double*, int64_t, double*, int64_t,
                                      double*, const int32_t*);
template mg_status potrs_impl<float>(mg_handle_t, int64_t, int64_t, const float*, int64_t, float*, int64_t,
                                     float*, const int32_t*);

}  // namespace mg
