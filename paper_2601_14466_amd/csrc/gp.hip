// gp.hip -- Gaussian-process marginal log likelihood on the Cholesky path.
//
// The paper's application section (Research Impact Statement, "Scientific
// applications", Cholesky solve) writes the marginal log likelihood of
// observations y with mean m under covariance A = K + Sigma as
//   log L = -1/2 (y - m)^T A^{-1} (y - m) - 1/2 log det A - N/2 log(2 pi),
// so it needs one solve against A and A's log determinant.  Both come from a
// single factorisation here: A = L L^T in place (potrf), alpha = A^{-1}(y - m)
// by the two triangular sweeps (potrs), log det A = 2 sum_j log L_jj, and one
// workgroup per column forms (y - m)^T alpha in a fixed summation order and
// combines the three terms.  Columns of Y are independent observation
// vectors sharing the covariance.
//
// Gradient: d log L / dA = (alpha alpha^T - A^{-1}) / 2 (A symmetric, the
// log-det term contributing -A^{-1}/2), d log L / dy = -alpha and
// d log L / dm = alpha.  A^{-1} = L^{-T} L^{-1} I comes from the same two
// sweeps with n right-hand sides.
#include <algorithm>
#include <cmath>

#include "mg_internal.h"

using namespace mg;

namespace mg {

// Alpha = Y - M (M may be null: zero mean), n x nrhs, column-major.
__global__ __launch_bounds__(256) void k_gp_center(const double* __restrict__ Y, int64_t ldy,
                                                   const double* __restrict__ M, int64_t ldm,
                                                   double* __restrict__ Al, int64_t lda_, int64_t n, int64_t nrhs) {
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, j = e / n;
        const double mv = M ? M[i + j * ldm] : 0.0;
        Al[i + j * lda_] = Y[i + j * ldy] - mv;
    }
}

// One workgroup per column j: q = sum_i (y_ij - m_ij) alpha_ij, each thread
// over rows tid, tid + 256, ... in order, then a fixed tree over the 256
// partial sums; loglik[j] = -q/2 - logdet/2 - n/2 log(2 pi), NaN after a
// failed factorisation.
__global__ __launch_bounds__(256) void k_gp_combine(const double* __restrict__ Y, int64_t ldy,
                                                    const double* __restrict__ M, int64_t ldm,
                                                    const double* __restrict__ Al, int64_t lda_, int64_t n,
                                                    const double* __restrict__ logdet, double* __restrict__ loglik,
                                                    const int32_t* __restrict__ info) {
    __shared__ double part[256];
    const int64_t j = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double mv = M ? M[i + j * ldm] : 0.0;
        s += (Y[i + j * ldy] - mv) * Al[i + j * lda_];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double two_pi_log = 1.8378770664093454835606594728112353;  // log(2 pi)
        loglik[j] = (*info != 0) ? (double)NAN : -0.5 * part[0] - 0.5 * (*logdet) - 0.5 * (double)n * two_pi_log;
    }
}

__global__ void k_gp_zero(double* v, int64_t k) {
    for (int64_t e = threadIdx.x; e < k; e += blockDim.x) v[e] = 0.0;
}

// X = I (n x n, leading dimension n): the right-hand side whose solve is A^{-1}
__global__ __launch_bounds__(256) void k_gp_eye(double* __restrict__ X, int64_t n) {
    const int64_t tot = n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        X[e] = (e % n == e / n) ? 1.0 : 0.0;
}

// gA = sum_r g_r (alpha_r alpha_r^T) / 2 - (sum_r g_r) A^{-1} / 2, the
// gradient of sum_r g_r log L_r with respect to the symmetric A (full n x n).
// A^{-1} is taken from its lower entries for both (i, j) and (j, i), so gA is
// exactly symmetric; the sums over r run in a fixed order.  NaN everywhere
// after a failed factorisation.
__global__ __launch_bounds__(256) void k_gp_grad_a(const double* __restrict__ Ainv, int64_t n,
                                                   const double* __restrict__ Al, int64_t lda_, int64_t nrhs,
                                                   const double* __restrict__ g, double* __restrict__ gA, int64_t ldg,
                                                   const int32_t* __restrict__ info) {
    const bool bad = *info != 0;
    const int64_t tot = n * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, j = e / n;
        const int64_t hi = i > j ? i : j, lo = i > j ? j : i;
        double outer = 0.0, gs = 0.0;
        for (int64_t r = 0; r < nrhs; ++r) {
            outer += g[r] * (Al[i + r * lda_] * Al[j + r * lda_]);
            gs += g[r];
        }
        gA[i + j * ldg] = bad ? (double)NAN : 0.5 * outer - 0.5 * gs * Ainv[hi + lo * n];
    }
}

// gY = -g_r alpha_r and (when gM is given) gM = +g_r alpha_r, column r
__global__ __launch_bounds__(256) void k_gp_grad_y(const double* __restrict__ Al, int64_t lda_, int64_t n,
                                                   int64_t nrhs, const double* __restrict__ g,
                                                   double* __restrict__ gY, int64_t ldgy, double* __restrict__ gM,
                                                   int64_t ldgm, const int32_t* __restrict__ info) {
    const bool bad = *info != 0;
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e % n, r = e / n;
        const double v = bad ? (double)NAN : g[r] * Al[i + r * lda_];
        gY[i + r * ldgy] = -v;
        if (gM) gM[i + r * ldgm] = v;
    }
}

static size_t gp_grad_work_bytes(int64_t n) {
    if (n == 0) return 0;
    // A^{-1}, then the sweeps' space, then the blocked solves' diagonal inverses
    return align_up((size_t)n * (size_t)n * 8, 256) + potrs_work_bytes(n, n, 8) + right_solve_lower_work_bytes(n);
}

static size_t gp_work_bytes(int64_t n, int64_t nrhs) {
    if (n == 0 || nrhs == 0) return 0;
    return potrs_work_bytes(n, nrhs, 8) + 256;  // sweeps' workspace, then the log determinant
}

}  // namespace mg

extern "C" {

mg_status mg_gp_loglik_buffer_size(mg_handle_t h, int64_t n, int64_t nrhs, size_t* bytes) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (!bytes) return -4;
    *bytes = gp_work_bytes(n, nrhs);
    return MG_OK;
}

mg_status mg_gp_loglik(mg_handle_t h, int64_t n, int64_t nrhs, double* A, int64_t lda, const double* Y, int64_t ldy,
                       const double* M, int64_t ldm, double* Alpha, int64_t ldalpha, double* loglik, void* work,
                       size_t work_bytes, int32_t* info) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    const bool any = n > 0 && nrhs > 0;
    if (!A && n > 0) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (!Y && any) return -6;
    if (ldy < std::max<int64_t>(1, n)) return -7;
    if (M && ldm < std::max<int64_t>(1, n)) return -9;
    if (!Alpha && any) return -10;
    if (ldalpha < std::max<int64_t>(1, n)) return -11;
    if (!loglik && nrhs > 0) return -12;
    const size_t need = gp_work_bytes(n, nrhs);
    if (need > 0 && !work) return -13;
    if (work_bytes < need) return -14;
    if (!info) return -15;
    mg_status rc;
    if ((rc = potrf_impl<double>(h, n, A, lda, info))) return rc;  // info = 0 when n == 0
    if (!any) {
        if (nrhs > 0) {
            // n == 0: log L = 0 for every column (empty sum, det of the empty
            // matrix 1); a fill kernel, not a memset, so that graph capture
            // of the call records no memset node
            hipLaunchKernelGGL(k_gp_zero, dim3(1), dim3(256), 0, h->stream, loglik, nrhs);
            MG_LAUNCH_CHECK();
        }
        return MG_OK;
    }
    hipStream_t st = h->stream;
    const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n * nrhs + 255) / 256), 4096);
    hipLaunchKernelGGL(k_gp_center, dim3(grid), dim3(256), 0, st, Y, ldy, M, ldm, Alpha, ldalpha, n, nrhs);
    MG_LAUNCH_CHECK();
    if ((rc = potrs_impl<double>(h, n, nrhs, A, lda, Alpha, ldalpha, (double*)work, info))) return rc;
    double* ld = (double*)((char*)work + potrs_work_bytes(n, nrhs, 8));
    if ((rc = mg_logdet(h, MG_F64, n, A, lda, ld, info))) return rc;
    hipLaunchKernelGGL(k_gp_combine, dim3((unsigned)nrhs), dim3(256), 0, st, Y, ldy, M, ldm, Alpha, ldalpha, n, ld,
                       loglik, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

mg_status mg_gp_loglik_grad_buffer_size(mg_handle_t h, int64_t n, size_t* bytes) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (!bytes) return -3;
    *bytes = gp_grad_work_bytes(n);
    return MG_OK;
}

mg_status mg_gp_loglik_grad(mg_handle_t h, int64_t n, int64_t nrhs, const double* L, int64_t lda, const double* Alpha,
                            int64_t ldalpha, const double* g, double* gA, int64_t ldga, double* gY, int64_t ldgy,
                            double* gM, int64_t ldgm, void* work, size_t work_bytes, int32_t* info) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    const bool any = n > 0 && nrhs > 0;
    if (!L && n > 0) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (!Alpha && any) return -6;
    if (ldalpha < std::max<int64_t>(1, n)) return -7;
    if (!g && nrhs > 0) return -8;
    if (!gA && n > 0) return -9;
    if (ldga < std::max<int64_t>(1, n)) return -10;
    if (!gY && any) return -11;
    if (ldgy < std::max<int64_t>(1, n)) return -12;
    if (gM && ldgm < std::max<int64_t>(1, n)) return -14;
    const size_t need = gp_grad_work_bytes(n);
    if (need > 0 && !work) return -15;
    if (work_bytes < need) return -16;
    if (!info) return -17;
    if (n == 0) return MG_OK;
    if ((n + 15) / 16 > 65535) return MG_ERR_UNSUPPORTED;  // right-hand-side passes of the sweeps (grid y)
    hipStream_t st = h->stream;
    double* Ainv = (double*)work;
    double* Yw = (double*)((char*)work + align_up((size_t)n * (size_t)n * 8, 256));
    const unsigned gsq = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n * n + 255) / 256), 8192);
    hipLaunchKernelGGL(k_gp_eye, dim3(gsq), dim3(256), 0, st, Ainv, n);
    MG_LAUNCH_CHECK();
    mg_status rc;
    const double* Ai = Ainv;
    if (right_solve_lower_ok(n, n, lda, n)) {
        // blocked right solves with L on the matrix pipe: I L^-1 = L^-1, then
        // L^-T L^-1 = A^{-1} from its transpose
        double* Zw = (double*)((char*)Yw + potrs_work_bytes(n, n, 8));
        if ((rc = right_solve_lower(st, n, n, L, lda, Ainv, n, Zw))) return rc;
        if ((rc = transpose_f64(st, Ainv, n, Yw, n, n, info))) return rc;
        if ((rc = right_solve_lower(st, n, n, L, lda, Yw, n, Zw))) return rc;
        Ai = Yw;
    } else if ((rc = potrs_impl<double>(h, n, n, L, lda, Ainv, n, Yw, info))) {  // A^{-1} = L^{-T} L^{-1} I
        return rc;
    }
    hipLaunchKernelGGL(k_gp_grad_a, dim3(gsq), dim3(256), 0, st, Ai, n, Alpha, ldalpha, nrhs, g, gA, ldga, info);
    MG_LAUNCH_CHECK();
    if (any) {
        const unsigned gy = (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n * nrhs + 255) / 256), 4096);
        hipLaunchKernelGGL(k_gp_grad_y, dim3(gy), dim3(256), 0, st, Alpha, ldalpha, n, nrhs, g, gY, ldgy, gM, ldgm,
                           info);
        MG_LAUNCH_CHECK();
    }
    return MG_OK;
}

}  // extern "C"
