// adjoint.hip -- reverse-mode derivative of X = A^{-1} B (A = L L^T SPD).
//
// The paper (JAXMg, "Statement of need") places these solves inside
// differentiable programs but states no adjoint; it follows from
// dX = A^{-1} (dB - dA X):
//   gB = A^{-1} gX                       (two triangular solves with the stored L)
//   gA = -gB X^T                         (unconstrained A)
// Reported forms:
//   MG_GRAD_SYM   : gA = -1/2 (gB X^T + X gB^T), the full symmetric matrix;
//   MG_GRAD_LOWER : the gradient with respect to the stored lower triangle
//                   (the entries the solver reads): -(gB X^T + X gB^T)(i,j)
//                   for i > j, -(gB X^T)(i,i) on the diagonal; the strict
//                   upper triangle of gA is not written.
// The rank-2 nrhs product runs on the FP64 matrix pipe as one product
// U V^T with U = [gB | X], V = [X | gB] (n x 2 nrhs each) over the lower
// triangle only: a 128 x 128 tile per workgroup, 64 x 64 per wave, operands
// streamed from L1/L2 into registers; the symmetric form mirrors each value.
#include <algorithm>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

// gA tile (I, J), I >= J: alpha_off * sum_k U(i,k) V(j,k) below the diagonal,
// alpha_diag on it.  Only entries with i >= j are computed into memory; with
// mirror set each strictly-lower value is also written to (j, i), so the
// symmetric result is exactly symmetric (the two halves of a diagonal tile
// would otherwise be summed in different orders).  After a failed
// factorisation or an aborted solve (info != 0) the same entries receive NaN.
__global__ __launch_bounds__(256, 2) void k_syr2k_grad(const double* __restrict__ G, int64_t ldg,
                                                       const double* __restrict__ X, int64_t ldx, int64_t n,
                                                       int64_t nrhs, double* __restrict__ GA, int64_t ldga,
                                                       double alpha_off, double alpha_diag, int mirror,
                                                       const int32_t* info) {
    const bool bad = info && *info != 0;
    const int64_t T = (n + 127) / 128;
    const int64_t t = blockIdx.x;
    if (t >= T * (T + 1) / 2) return;
    int64_t r0 = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r0 * (r0 + 1) / 2 > t) --r0;
    while ((r0 + 1) * (r0 + 2) / 2 <= t) ++r0;
    const int64_t I = r0, J = t - r0 * (r0 + 1) / 2;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, i = l & 15, g = l >> 4;
    const int wr = w >> 1, wc = w & 1;
    const int64_t sr0 = I * 128 + 64 * wr, sc0 = J * 128 + 64 * wc;
    if (sr0 + 63 < sc0) return;
    f64x4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f64x4{0, 0, 0, 0};
    const int64_t K = bad ? 0 : 2 * nrhs;
    // U(i,k) = G(i,k) for k < nrhs, X(i,k-nrhs) after; V(j,k) = X(j,k), then G(j,k-nrhs)
    for (int64_t k0 = 0; k0 < K; k0 += 4) {
        const int64_t k = k0 + g;
        const bool kin = k < K;
        const bool first = k < nrhs;
        const int64_t kk = first ? k : k - nrhs;
        double xv[4], zv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t ra = sr0 + 16 * b + i, rb = sc0 + 16 * b + i;
            xv[b] = (kin && ra < n) ? (first ? G[idx(ra, kk, ldg)] : X[idx(ra, kk, ldx)]) : 0.0;
            zv[b] = (kin && rb < n) ? (first ? X[idx(rb, kk, ldx)] : G[idx(rb, kk, ldg)]) : 0.0;
        }
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mma_xzt(acc[bi][bj], xv[bi], zv[bj]);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = sr0 + 16 * bi + i, col = sc0 + 16 * bj + tcol<double>(g, r);
                if (row < n && col < n && row >= col) {
                    const double v = bad ? (double)NAN : (row == col ? alpha_diag : alpha_off) * acc[bi][bj][r];
                    GA[idx(row, col, ldga)] = v;
                    if (mirror && row > col) GA[idx(col, row, ldga)] = v;
                }
            }
}

__global__ __launch_bounds__(256) void k_copy_rhs(const double* __restrict__ S, int64_t lds, double* __restrict__ D,
                                                  int64_t ldd, int64_t n, int64_t nrhs) {
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, r = e / n;
        D[idx(i, r, ldd)] = S[idx(i, r, lds)];
    }
}

// gB := NaN when the factorisation failed or a sweep gave up (info != 0).
__global__ __launch_bounds__(256) void k_nan_on_info(double* __restrict__ D, int64_t ldd, int64_t n, int64_t nrhs,
                                                     const int32_t* info) {
    if (!info || *info == 0) return;
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        D[idx(e % n, e / n, ldd)] = (double)NAN;
}

mg_status posv_backward_impl(mg_handle_t h, int64_t n, int64_t nrhs, const double* L, int64_t lda,
                             const double* X, int64_t ldx, const double* GX, int64_t ldgx, double* GB,
                             int64_t ldgb, double* GA, int64_t ldga, int mode, void* work, int32_t* info) {
    if (n == 0) return MG_OK;
    hipStream_t st = h->stream;
    mg_status rc;
    if (nrhs > 0) {
        const unsigned g1 = (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(n * nrhs, 256)), 65535);
        hipLaunchKernelGGL(k_copy_rhs, dim3(g1), dim3(256), 0, st, GX, ldgx, GB, ldgb, n, nrhs);
        MG_LAUNCH_CHECK();
        if ((rc = potrs_impl<double>(h, n, nrhs, L, lda, GB, ldgb, (double*)work, info))) return rc;
        hipLaunchKernelGGL(k_nan_on_info, dim3(g1), dim3(256), 0, st, GB, ldgb, n, nrhs, (const int32_t*)info);
        MG_LAUNCH_CHECK();
    }
    const int64_t T = cdiv(n, 128);
    const bool lower = mode == MG_GRAD_LOWER;
    const int64_t grid = T * (T + 1) / 2;
    if ((rc = prof_begin(h, MG_PROF_ADJOINT, st))) return rc;
    hipLaunchKernelGGL(k_syr2k_grad, dim3((unsigned)grid), dim3(256), 0, st, GB, ldgb, X, ldx, n, nrhs, GA, ldga,
                       lower ? -1.0 : -0.5, -0.5, lower ? 0 : 1, (const int32_t*)info);
    MG_LAUNCH_CHECK();
    const double nd = (double)n;
    return prof_end(h, MG_PROF_ADJOINT, 2.0 * nd * nd * 2.0 * (double)nrhs,
                    (nd * nd + 2.0 * nd * 2.0 * (double)nrhs) * 8.0, st);
}

}  // namespace mg
