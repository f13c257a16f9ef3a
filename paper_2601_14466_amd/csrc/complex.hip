// complex.hip -- the complex Hermitian positive-definite solve (the paper's
// routines take complex64 and complex128 as well as the real types;
// "Software design").
//
// gfx950 has no complex matrix instruction, so the complex problem is carried
// by the real one it is equivalent to.  Writing every complex entry
// a = a_r + i a_i as the 2 x 2 real block [[a_r, -a_i], [a_i, a_r]] turns an
// n x n Hermitian A into a 2n x 2n real symmetric M, positive definite when
// A is, with the product of complex matrices mapping to the product of their
// blocked forms.  If A = L L^H, the blocked form of L is lower triangular
// with positive diagonal (its diagonal blocks are l_jj I) and its product
// with its transpose is M; by uniqueness of the Cholesky factor it IS the
// real factor of M.  So the real factorisation of M (the tuned FP64 or FP32
// path, on the matrix pipe) yields L exactly up to rounding: l_ij is
// M-factor(2i, 2j) + i M-factor(2i + 1, 2j).  Complex vectors need no
// conversion: an interleaved complex column (real, imaginary, real, ...) is
// the even column of its blocked form, so a complex n x nrhs B with leading
// dimension ldb is the real 2n x nrhs right-hand side with leading dimension
// 2 ldb, and the real solve leaves X in the same storage.
//
// Cost: the real factorisation does (2n)^3 / 3 flops against the 4 n^3 / 3
// real flops of complex arithmetic, and M takes twice A's bytes; in exchange
// the complex path runs at the real path's matrix-pipe rate.
#include <algorithm>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

// Lower triangle of the blocked form of the complex lower triangle Z (n x n,
// interleaved pairs, leading dimension ldz in complex elements) into M
// (2n x 2n, leading dimension ldm): blocks below the diagonal in full, the
// diagonal blocks as [[z_r, .], [0, z_r]] (the imaginary part of a diagonal
// entry is not read: Hermitian diagonals are real).
template <typename T>
__global__ __launch_bounds__(256) void k_z_embed(const T* __restrict__ Z, int64_t ldz, int64_t n, T* __restrict__ M,
                                                 int64_t ldm) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int64_t j = blockIdx.y; j <= i && j < n; j += gridDim.y) {
        const T zr = Z[2 * idx(i, j, ldz)];
        const T zi = i == j ? (T)0 : Z[2 * idx(i, j, ldz) + 1];
        M[idx(2 * i, 2 * j, ldm)] = zr;
        M[idx(2 * i + 1, 2 * j, ldm)] = zi;
        if (i > j) M[idx(2 * i, 2 * j + 1, ldm)] = -zi;
        M[idx(2 * i + 1, 2 * j + 1, ldm)] = zr;
    }
}

// The complex lower triangle of the real factor of M back into Z: entry
// (i, j), i >= j, from M's column 2j rows 2i and 2i + 1 (the diagonal's
// imaginary part written as 0).  The strict upper triangle of Z is not
// touched.
template <typename T>
__global__ __launch_bounds__(256) void k_z_extract(const T* __restrict__ M, int64_t ldm, int64_t n, T* __restrict__ Z,
                                                   int64_t ldz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int64_t j = blockIdx.y; j <= i && j < n; j += gridDim.y) {
        Z[2 * idx(i, j, ldz)] = M[idx(2 * i, 2 * j, ldm)];
        Z[2 * idx(i, j, ldz) + 1] = i == j ? (T)0 : M[idx(2 * i + 1, 2 * j, ldm)];
    }
}

// Real column k (1-based) of M fails when complex column ceil(k / 2) does.
__global__ void k_z_info(int32_t* info) {
    if (threadIdx.x == 0 && *info > 0) *info = (*info + 1) / 2;
}

static dim3 z_grid(int64_t n) {
    return dim3((unsigned)cdiv(n, 256), (unsigned)std::min<int64_t>(std::max<int64_t>(n, 1), 65535));
}

static size_t m_bytes(int64_t n, int es) { return align_up((size_t)4 * n * n * es, 256); }

size_t zposv_work_bytes(int64_t n, int64_t nrhs, int es) {
    if (n == 0) return 0;
    return m_bytes(n, es) + potrs_work_bytes(2 * n, nrhs, es);
}

template <typename T>
static mg_status embed(hipStream_t st, const T* Z, int64_t ldz, int64_t n, T* M) {
    hipLaunchKernelGGL((k_z_embed<T>), z_grid(n), dim3(256), 0, st, Z, ldz, n, M, 2 * n);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

// op: 0 factor (A -> L), 1 solve with a given L, 2 factor and solve.
template <typename T>
mg_status zposv_impl(mg_handle_t h, int op, int64_t n, int64_t nrhs, T* A, int64_t lda, T* B, int64_t ldb, void* work,
                     int32_t* info) {
    hipStream_t st = h->stream;
    mg_status rc;
    if (op != 1 && (rc = set_info_zero(st, info))) return rc;
    if (n == 0) return MG_OK;
    T* M = (T*)work;
    T* Y = (T*)((char*)work + m_bytes(n, (int)sizeof(T)));
    if ((rc = embed<T>(st, A, lda, n, M))) return rc;
    if (op != 1) {
        if ((rc = potrf_impl<T>(h, 2 * n, M, 2 * n, info))) return rc;
    }
    if (op != 0 && nrhs > 0) {
        if ((rc = potrs_impl<T>(h, 2 * n, nrhs, M, 2 * n, B, 2 * ldb, Y, info))) return rc;
    }
    if (op != 1) {
        hipLaunchKernelGGL((k_z_extract<T>), z_grid(n), dim3(256), 0, st, (const T*)M, 2 * n, n, A, lda);
        MG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_z_info, dim3(1), dim3(64), 0, st, info);
        MG_LAUNCH_CHECK();
    }
    return MG_OK;
}

template mg_status zposv_impl<double>(mg_handle_t, int, int64_t, int64_t, double*, int64_t, double*, int64_t, void*,
                                      int32_t*);
template mg_status zposv_impl<float>(mg_handle_t, int, int64_t, int64_t, float*, int64_t, float*, int64_t, void*,
                                     int32_t*);

}  // namespace mg
