// chol_adjoint.hip -- reverse-mode derivative of the Cholesky factorisation
// itself: given gL = df/dL for L = chol(A), the gradient of f with respect
// to A.
//
// The paper puts the solver inside differentiable programs ("Statement of
// need") but states no adjoint.  From A = L L^T, L^{-1} dA L^{-T} =
// L^{-1} dL + (L^{-1} dL)^T with L^{-1} dL lower triangular, so
// dL = L Phi(L^{-1} dA L^{-T}) with Phi = lower triangle, diagonal halved,
// and df = <gL, dL> = <L^{-T} Phi(L^T gL) L^{-1}, dA> (Murray 2016).  With
// S = L^{-T} P L^{-1}, P = Phi(L^T gL):
//   MG_GRAD_SYM   : gA = (S + S^T)/2 (dA symmetric), full n x n;
//   MG_GRAD_LOWER : gradient with respect to the lower-triangle entries:
//                   S_ij + S_ji below the diagonal, S_ii on it; the strict
//                   upper triangle of gA is not written.
// Steps on the GPU (W: an n x n workspace):
//   1. W = P (lower, zeros above) by k_phi_ltgl: 64 x 64 output tiles, the
//      32-row k-slices of L and gL staged through LDS (the next slice fetched
//      into registers during the products), products on the FP64 matrix
//      pipe;
//   2. gA <- Q = L^{-T} P by the backward sweep with n right-hand sides;
//   3. W <- Q^T (k_transpose, 64 x 64 tiles through LDS);
//   4. gA <- R = L^{-T} Q^T = S^T by the backward sweep;
//   5. gA <- sym(R) in place (k_sym_pairs: one thread per pair (i, j), so
//      the two halves are written from the same two values).
// Where n is a multiple of 64 (and the offsets fit), steps 2-4 are done as
// right solves with L by 64-column blocks on the matrix pipe instead of
// sweeps: gA <- P^T, gA <- gA L^-1 = Q^T, W <- Q, W <- W L^-1 = R^T, and gA
// is formed from R^T by k_sym_tiles (transposes and pairs tile-wise through
// LDS).
#include <algorithm>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

constexpr int PT = 64;        // output tile of P
constexpr int PK = 32;        // k rows staged per step
constexpr int PLD = PT + 1;   // LDS leading dimension

// W(r, c) = Phi(L^T gL)(r, c) for the PT x PT tile (I, J) of an n x n grid:
// sum over k >= r of L(k, r) gL(k, c) for r > c, half of it for r == c, and 0
// above the diagonal.  L(k, r) is read only for k >= r and gL(k, c) only for
// k >= c (their strict upper triangles are never read).
__global__ __launch_bounds__(256) void k_phi_ltgl(const double* __restrict__ L, int64_t lda,
                                                  const double* __restrict__ GL, int64_t ldgl, int64_t n,
                                                  double* __restrict__ W, int64_t ldw, const int32_t* info) {
    if (info && *info != 0) return;
    const int64_t T = (n + PT - 1) / PT;
    const int64_t I = blockIdx.x % T, J = blockIdx.x / T;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, i = l & 15, g = l >> 4;
    const int64_t r0 = I * PT, c0 = J * PT;
    if (I < J) {  // strictly above the diagonal: zeros
        for (int e = tid; e < PT * PT; e += 256) {
            const int64_t r = r0 + (e & (PT - 1)), c = c0 + (e >> 6);
            if (r < n && c < n) W[idx(r, c, ldw)] = 0.0;
        }
        return;
    }
    __shared__ double Ls[PK][PLD], Gs[PK][PLD];
    f64x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0, 0, 0, 0};
    // the k-slices are software-pipelined: slice kb + PK is fetched into
    // registers while slice kb is multiplied from LDS
    constexpr int QN = PK * PT / 256;
    double lv[QN], gv[QN];
    auto fetch = [&](int64_t kb) {
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int e = tid + 256 * q, kk = e % PK, c = e / PK;
            const int64_t k = kb + kk, rr = r0 + c, cc = c0 + c;
            lv[q] = (k < n && rr < n && k >= rr) ? L[idx(k, rr, lda)] : 0.0;
            gv[q] = (k < n && cc < n && k >= cc) ? GL[idx(k, cc, ldgl)] : 0.0;
        }
    };
    // rows k < r0 contribute nothing (L(k, r) = 0 for k < r)
    fetch(r0);
    for (int64_t kb = r0; kb < n; kb += PK) {
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int e = tid + 256 * q, kk = e % PK, c = e / PK;
            Ls[kk][c] = lv[q];
            Gs[kk][c] = gv[q];
        }
        __syncthreads();
        if (kb + PK < n) fetch(kb + PK);
        // wave w: rows 16 w .. 16 w + 15 of the tile, all 64 columns
#pragma unroll
        for (int ks = 0; ks < PK / 4; ++ks) {
            const int kk = 4 * ks + g;
            const double xv = Ls[kk][16 * w + i];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mma_xzt(acc[t], xv, Gs[kk][16 * t + i]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = r0 + 16 * w + i, col = c0 + 16 * t + tcol<double>(g, r);
            if (row >= n || col >= n) continue;
            W[idx(row, col, ldw)] = row > col ? acc[t][r] : (row == col ? 0.5 * acc[t][r] : 0.0);
        }
}

// D = S^T (n x n), 64 x 64 tiles through LDS (coalesced reads and writes).
__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ S, int64_t lds, double* __restrict__ D,
                                                   int64_t ldd, int64_t n, const int32_t* info) {
    if (info && *info != 0) return;
    __shared__ double tile[PT][PLD];
    const int64_t T = (n + PT - 1) / PT;
    const int64_t I = blockIdx.x % T, J = blockIdx.x / T;
    const int tid = threadIdx.x;
    for (int e = tid; e < PT * PT; e += 256) {
        const int rr = e & (PT - 1), cc = e >> 6;
        const int64_t r = I * PT + rr, c = J * PT + cc;
        tile[cc][rr] = (r < n && c < n) ? S[idx(r, c, lds)] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < PT * PT; e += 256) {
        const int rr = e & (PT - 1), cc = e >> 6;   // D(J*PT + rr, I*PT + cc) = S(I*PT + cc, J*PT + rr)
        const int64_t r = J * PT + rr, c = I * PT + cc;
        if (r < n && c < n) D[idx(r, c, ldd)] = tile[rr][cc];
    }
}

// In place on R (= S^T): mode 0 writes (R_ij + R_ji)/2 to both (i, j) and
// (j, i); mode 1 writes R_ij + R_ji below the diagonal and R_ii on it, and
// leaves the strict upper triangle alone.  One thread per pair i >= j.
// NaN everywhere it writes when info != 0.
__global__ __launch_bounds__(256) void k_sym_pairs(double* R, int64_t ldr, int64_t n, int mode, const int32_t* info) {
    const bool bad = info && *info != 0;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = j + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
            const double a = R[idx(i, j, ldr)], b = R[idx(j, i, ldr)];
            if (bad) {
                R[idx(i, j, ldr)] = (double)NAN;
                if (mode == 0 && i != j) R[idx(j, i, ldr)] = (double)NAN;
            } else if (i == j) {
                R[idx(i, i, ldr)] = a;
            } else if (mode == 0) {
                const double v = 0.5 * (a + b);
                R[idx(i, j, ldr)] = v;
                R[idx(j, i, ldr)] = v;
            } else {
                R[idx(i, j, ldr)] = a + b;
            }
        }
}

// gA from R^T (W, n x n) without the transpose: tile pair (I, J), I >= J,
// of a T x T grid per workgroup, both tiles of W staged through LDS so that
// every read and write is coalesced.  Mode 0 writes (R_ij + R_ji)/2 to both
// (i, j) and (j, i); mode 1 writes R_ij + R_ji below the diagonal and R_ii
// on it and leaves the strict upper triangle alone (the expressions are
// symmetric in R and R^T).  NaN wherever it writes when info != 0.
__global__ __launch_bounds__(256) void k_sym_tiles(const double* __restrict__ W, int64_t ldw, double* __restrict__ G,
                                                   int64_t ldg, int64_t n, int mode, const int32_t* info) {
    __shared__ double a[PT][PLD], b[PT][PLD];  // a[c][r] = W(I*PT + r, J*PT + c); b[c][r] = W(J*PT + r, I*PT + c)
    const int64_t T = (n + PT - 1) / PT;
    const int64_t I = blockIdx.x % T, J = blockIdx.x / T;
    if (I < J) return;
    const bool bad = info && *info != 0;
    const int tid = threadIdx.x;
    for (int e = tid; e < PT * PT; e += 256) {
        const int rr = e & (PT - 1), cc = e >> 6;
        const int64_t r1 = I * PT + rr, c1 = J * PT + cc, r2 = J * PT + rr, c2 = I * PT + cc;
        a[cc][rr] = (r1 < n && c1 < n) ? W[idx(r1, c1, ldw)] : 0.0;
        b[cc][rr] = (r2 < n && c2 < n) ? W[idx(r2, c2, ldw)] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < PT * PT; e += 256) {
        const int rr = e & (PT - 1), cc = e >> 6;
        // entry (i, j) = (I*PT + rr, J*PT + cc) of the lower tile: W(i, j) = a[cc][rr], W(j, i) = b[rr][cc]
        const int64_t i = I * PT + rr, j = J * PT + cc;
        if (i < n && j < n && i >= j) {
            const double v = a[cc][rr], t = b[rr][cc];
            if (bad) G[idx(i, j, ldg)] = (double)NAN;
            else if (i == j) G[idx(i, j, ldg)] = v;
            else G[idx(i, j, ldg)] = mode == 0 ? 0.5 * (v + t) : v + t;
        }
        // entry (j', i') = (J*PT + rr, I*PT + cc) of the upper tile (mode 0): W(j', i') = b[cc][rr],
        // W(i', j') = a[rr][cc]
        const int64_t j2 = J * PT + rr, i2 = I * PT + cc;
        if (mode == 0 && j2 < n && i2 < n && i2 > j2)
            G[idx(j2, i2, ldg)] = bad ? (double)NAN : 0.5 * (a[rr][cc] + b[cc][rr]);
    }
}

// D = S^T for n x n FP64 matrices (skipped when *info != 0).
mg_status transpose_f64(hipStream_t st, const double* S, int64_t lds, double* D, int64_t ldd, int64_t n,
                        const int32_t* info) {
    if (n <= 0) return MG_OK;
    const int64_t T = cdiv(n, PT);
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)(T * T)), dim3(256), 0, st, S, lds, D, ldd, n, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

size_t potrf_backward_work_bytes(int64_t n) {
    return n == 0 ? 0
                  : align_up((size_t)n * (size_t)n * 8, 256) +
                        std::max(2 * sweep_words_bytes(n), right_solve_lower_work_bytes(n));
}

mg_status potrf_backward_impl(mg_handle_t h, int64_t n, const double* L, int64_t lda, const double* GL,
                              int64_t ldgl, double* GA, int64_t ldga, int mode, void* work, int32_t* info) {
    if (n == 0) return MG_OK;
    hipStream_t st = h->stream;
    double* W = (double*)work;
    char* words = (char*)work + align_up((size_t)n * (size_t)n * 8, 256);
    const int64_t T = cdiv(n, PT);
    hipLaunchKernelGGL(k_phi_ltgl, dim3((unsigned)(T * T)), dim3(256), 0, st, L, lda, GL, ldgl, n, W, n, info);
    MG_LAUNCH_CHECK();
    mg_status rc;
    if (right_solve_lower_ok(n, n, lda, std::max<int64_t>(n, ldga))) {
        // Blocked: the two solves as right solves with L on the matrix pipe,
        // Q^T = P^T L^-1 and R^T = Q L^-1 (the gradient is symmetric in S and
        // S^T = R, so R^T serves as well as R).
        double* Zw = (double*)words;
        const dim3 tg((unsigned)(T * T));
        hipLaunchKernelGGL(k_transpose, tg, dim3(256), 0, st, W, n, GA, ldga, n, info);  // GA = P^T
        MG_LAUNCH_CHECK();
        if ((rc = right_solve_lower(st, n, n, L, lda, GA, ldga, Zw))) return rc;          // GA = Q^T
        hipLaunchKernelGGL(k_transpose, tg, dim3(256), 0, st, GA, ldga, W, n, n, info);  // W = Q
        MG_LAUNCH_CHECK();
        if ((rc = right_solve_lower(st, n, n, L, lda, W, n, Zw))) return rc;              // W = R^T
        hipLaunchKernelGGL(k_sym_tiles, tg, dim3(256), 0, st, W, n, GA, ldga, n, mode, info);  // GA from R^T
        MG_LAUNCH_CHECK();
        return MG_OK;
    } else {
        if ((rc = trsm_lt_impl<double>(h, n, n, L, lda, W, n, GA, ldga, words, info))) return rc;  // Q = L^-T P
        hipLaunchKernelGGL(k_transpose, dim3((unsigned)(T * T)), dim3(256), 0, st, GA, ldga, W, n, n, info);
        MG_LAUNCH_CHECK();
        if ((rc = trsm_lt_impl<double>(h, n, n, L, lda, W, n, GA, ldga, words + sweep_words_bytes(n), info)))
            return rc;  // R = L^-T Q^T = S^T
    }
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 64));
    const unsigned gy = (unsigned)std::min<int64_t>(std::max<int64_t>(1, n), 4096);
    hipLaunchKernelGGL(k_sym_pairs, dim3(gx, gy), dim3(256), 0, st, GA, ldga, n, mode, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

}  // namespace mg
