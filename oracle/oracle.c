/*
 * oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously-correct CPU implementation of what the solver
 * computes.  Only the test suite, the package smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library, and neither side includes or links the other.
 *
 * The paper (JAXMg, "Software design", the potrs bullet) states the problem:
 * solve A x = b for a symmetric positive-definite A through a Cholesky
 * factorisation, optionally returning log det A.  It delegates the algorithm
 * to a closed library, so every routine here is the textbook definition:
 *
 *   or_potrf   : the unique lower-triangular L with positive diagonal and
 *                A = L L^T, column by column (Golub & Van Loan, "gaxpy"
 *                Cholesky): column j of L is column j of A minus the sum of
 *                the previous columns scaled by row j, divided by the square
 *                root of its diagonal entry.  Summation over k runs in
 *                increasing k.  Failure index (LAPACK convention): the first
 *                1-based column whose pivot is not > 0 (NaN included).
 *   or_potrs   : forward substitution L y = b, then back substitution
 *                L^T x = y, one right-hand-side column at a time.
 *   or_residual: r = b - A x with A symmetric, read from its lower triangle,
 *                accumulated in x87 extended precision (64-bit significand);
 *                eta_j = |r_j|_inf / (|A|_inf |x_j|_inf + |b_j|_inf), the
 *                Rigal-Gaches normwise backward error of column j.
 *   or_logdet  : log det A = 2 sum_j log L_jj (the paper's optional output).
 *   or_potrf_lo_blocked: the low-precision factor of the mixed-precision
 *                reading (the paper is silent on precision): right-looking
 *                blocks of nb columns; each diagonal block is promoted to
 *                FP64, factored by or_potrf and stored rounded to binary32;
 *                the panel below it is solved by substitution in binary32;
 *                the trailing matrix receives the block's rank-nb product
 *                with its operands rounded to the working precision
 *                (binary32, or bfloat16 when lo == 2) and the products
 *                summed in binary32.
 *   or_posv_ir : mixed-precision iterative refinement (the paper is silent;
 *                this is the classic scheme of Langou et al., SC'06): factor
 *                a single-precision copy, solve, then repeat
 *                r = b - A x (FP64), d = solve_lo(r), x += d.
 *   or_posv_backward: adjoint of X = A^{-1} B:  gB = A^{-1} gX and
 *                gA = -1/2 (gB X^T + X gB^T) (symmetric convention), or the
 *                gradient with respect to the lower-triangle parameters.
 *   or_getrf / or_getrs: the paper's general solve (lu_solve): P A = L U by
 *                Gaussian elimination with partial pivoting (column by
 *                column: the row with the largest |entry| on or below the
 *                diagonal, the first one on ties, is swapped into place;
 *                L unit lower, U upper, stored over A; ipiv[k] = 1-based row
 *                swapped with row k); info = first k whose pivot is exactly
 *                zero (elimination goes on past it, as LAPACK's xGETRF).
 *                getrs applies the swaps to B, then L y = P b, U x = y.
 *   or_zpotrf / or_zpotrs: the complex Hermitian case of the same solve (the
 *                paper lists complex64 and complex128 for its routines): A =
 *                L L^H with L lower, real positive diagonal; column j of L:
 *                L_jj = sqrt(Re a_jj - sum_{k<j} |l_jk|^2), l_ij = (a_ij -
 *                sum_{k<j} l_ik conj(l_jk)) / L_jj (the imaginary part of the
 *                diagonal is not read, as LAPACK's ZPOTRF); info as or_potrf.
 *                zpotrs: L y = b, then L^H x = y.  or_residual_z: the
 *                per-column normwise backward error of A X = B with the full
 *                Hermitian A rebuilt from its lower triangle, |.| the complex
 *                modulus, in extended precision.
 *   or_potrf_backward: adjoint of L = chol(A) (the paper is silent; the
 *                result is Murray, "Differentiation of the Cholesky
 *                decomposition", 2016).  From A = L L^T,
 *                L^{-1} dA L^{-T} = L^{-1} dL + (L^{-1} dL)^T with L^{-1} dL
 *                lower triangular, so dL = L Phi(L^{-1} dA L^{-T}), Phi taking
 *                the lower triangle with the diagonal halved.  For a scalar
 *                f with gradient gL (lower) with respect to L,
 *                df = <Phi(L^T gL), L^{-1} dA L^{-T}>, hence
 *                S = L^{-T} Phi(L^T gL) L^{-1} and, dA being symmetric,
 *                gA = (S + S^T)/2 (mode 0), or the gradient with respect to
 *                the lower-triangle parameters (mode 1: S_ij + S_ji below
 *                the diagonal, S_ii on it).
 *
 * Storage: column-major, element (i, j) at A[i + j*lda]; only the lower
 * triangle of A is read and the strict upper triangle is never written.
 * Build with -ffp-contract=off so that every a - b*c is two roundings, as
 * written.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define AT(M, ld, i, j) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/* ------------------------------------------------------------------ potrf */
int64_t or_potrf(int64_t n, double *A, int64_t lda)
{
    for (int64_t j = 0; j < n; ++j) {
        /* column j of A, rows j..n-1, minus sum_{k<j} L(:,k) * L(j,k),
         * k increasing; the row range is split across threads */
        int64_t m = n - j;
#pragma omp parallel if (m * j > 65536)
        {
            int nt = omp_get_num_threads(), t = omp_get_thread_num();
            int64_t i0 = j + (m * t) / nt, i1 = j + (m * (t + 1)) / nt;
            for (int64_t k = 0; k < j; ++k) {
                double ljk = AT(A, lda, j, k);
                for (int64_t i = i0; i < i1; ++i)
                    AT(A, lda, i, j) = AT(A, lda, i, j) - AT(A, lda, i, k) * ljk;
            }
        }
        double d = AT(A, lda, j, j);
        if (!(d > 0.0))
            return j + 1;
        d = sqrt(d);
        AT(A, lda, j, j) = d;
        for (int64_t i = j + 1; i < n; ++i)
            AT(A, lda, i, j) = AT(A, lda, i, j) / d;
    }
    return 0;
}

/* ------------------------------------------------------------------ potrs */
static void trsv_lower(int64_t n, const double *L, int64_t lda, double *b)
{
    /* L y = b: y_j = (b_j - sum_{k<j} L_jk y_k) / L_jj, increasing k */
    for (int64_t j = 0; j < n; ++j) {
        double t = b[j];
        for (int64_t k = 0; k < j; ++k)
            t = t - AT(L, lda, j, k) * b[k];
        b[j] = t / AT(L, lda, j, j);
    }
}

static void trsv_lower_trans(int64_t n, const double *L, int64_t lda, double *b)
{
    /* L^T x = y: x_j = (y_j - sum_{k>j} L_kj x_k) / L_jj, increasing k */
    for (int64_t j = n - 1; j >= 0; --j) {
        double t = b[j];
        for (int64_t k = j + 1; k < n; ++k)
            t = t - AT(L, lda, k, j) * b[k];
        b[j] = t / AT(L, lda, j, j);
    }
}

void or_potrs(int64_t n, int64_t nrhs, const double *L, int64_t lda,
              double *B, int64_t ldb)
{
#pragma omp parallel for schedule(dynamic, 1) if (nrhs > 1 && n > 256)
    for (int64_t r = 0; r < nrhs; ++r) {
        double *b = B + (size_t)r * (size_t)ldb;
        trsv_lower(n, L, lda, b);
        trsv_lower_trans(n, L, lda, b);
    }
}

int64_t or_posv(int64_t n, int64_t nrhs, double *A, int64_t lda,
                double *B, int64_t ldb)
{
    int64_t info = or_potrf(n, A, lda);
    if (info == 0)
        or_potrs(n, nrhs, A, lda, B, ldb);
    return info;
}

/* --------------------------------------------------------------- log det */
double or_logdet(int64_t n, const double *L, int64_t lda)
{
    long double s = 0.0L;
    for (int64_t j = 0; j < n; ++j)
        s += logl((long double)AT(L, lda, j, j));
    return (double)(2.0L * s);
}

/* ------------------------------------------------------- residual and eta */
/* |A|_inf of the symmetric matrix whose lower triangle is stored. */
double or_sym_norm_inf(int64_t n, const double *A, int64_t lda)
{
    long double *rs = (long double *)calloc((size_t)(n > 0 ? n : 1), sizeof(long double));
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = j; i < n; ++i) {
            long double a = fabsl((long double)AT(A, lda, i, j));
            rs[i] += a;
            if (i != j)
                rs[j] += a;
        }
    }
    long double m = 0.0L;
    for (int64_t i = 0; i < n; ++i)
        if (rs[i] > m)
            m = rs[i];
    free(rs);
    return (double)m;
}

/*
 * R = B - A X (A symmetric, lower triangle stored), in long double.
 * Two passes keep every inner loop on a contiguous column segment:
 *   pass 1: rows i >= j of each column j (the stored lower part, diagonal
 *           included) act on x_j;
 *   pass 2: the strict lower part read as the upper part, i.e. entry (i, j)
 *           with i > j also acts on x_i in row j.
 * R may be NULL.  eta[r] receives the normwise backward error of column r.
 * Returns |A|_inf.
 */
double or_residual(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                   const double *X, int64_t ldx, const double *B, int64_t ldb,
                   double *R, int64_t ldr, double *eta)
{
    if (nrhs <= 0)
        return 0.0;
    size_t nn = (size_t)(n > 0 ? n : 1);
    long double *acc = (long double *)malloc(nn * (size_t)nrhs * sizeof(long double));
    long double *up = (long double *)calloc(nn * (size_t)nrhs, sizeof(long double));
    const int64_t RB = 64;
    int64_t nblk = (n + RB - 1) / RB;

    /* pass 1: acc(i, r) = b(i, r) - sum_{j <= i} A(i, j) x(j, r) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        int64_t i0 = blk * RB, i1 = i0 + RB < n ? i0 + RB : n;
        for (int64_t r = 0; r < nrhs; ++r)
            for (int64_t i = i0; i < i1; ++i)
                acc[(size_t)r * nn + (size_t)i] = (long double)AT(B, ldb, i, r);
        for (int64_t j = 0; j < i1; ++j) {
            int64_t ib = j > i0 ? j : i0;
            for (int64_t r = 0; r < nrhs; ++r) {
                long double xj = (long double)AT(X, ldx, j, r);
                long double *a = acc + (size_t)r * nn;
                for (int64_t i = ib; i < i1; ++i)
                    a[i] -= (long double)AT(A, lda, i, j) * xj;
            }
        }
    }
    /* pass 2: up(j, r) = sum_{i > j} A(i, j) x(i, r) */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t r = 0; r < nrhs; ++r) {
            long double s = 0.0L;
            for (int64_t i = j + 1; i < n; ++i)
                s += (long double)AT(A, lda, i, j) * (long double)AT(X, ldx, i, r);
            up[(size_t)r * nn + (size_t)j] = s;
        }
    }
    double anorm = or_sym_norm_inf(n, A, lda);
    for (int64_t r = 0; r < nrhs; ++r) {
        long double rmax = 0.0L, xmax = 0.0L, bmax = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            long double ri = acc[(size_t)r * nn + (size_t)i] - up[(size_t)r * nn + (size_t)i];
            if (R)
                AT(R, ldr, i, r) = (double)ri;
            if (fabsl(ri) > rmax) rmax = fabsl(ri);
            long double xi = fabsl((long double)AT(X, ldx, i, r));
            long double bi = fabsl((long double)AT(B, ldb, i, r));
            if (xi > xmax) xmax = xi;
            if (bi > bmax) bmax = bi;
            if (ri != ri || xi != xi) rmax = (long double)NAN;
        }
        long double den = (long double)anorm * xmax + bmax;
        if (eta)
            eta[r] = (double)(den > 0.0L ? rmax / den : (rmax > 0.0L ? INFINITY : 0.0));
    }
    free(acc);
    free(up);
    return anorm;
}

/* --------------------------------------------- mixed precision refinement */
/* Round a binary32 value to bfloat16 (8-bit significand), nearest-even, on
 * the bit pattern, and return it widened back to binary32.  Infinities and
 * NaNs pass through unchanged; a finite value above the largest bfloat16
 * number (by at least half an ulp) becomes an infinity. */
float or_round_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u)
        return x;
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    float y;
    memcpy(&y, &u, 4);
    return y;
}

/* or_round_bf16 over an array (bit patterns in and out untouched by any
 * host-side conversion). */
void or_round_bf16_array(int64_t n, const float *in, float *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = or_round_bf16(in[i]);
}

/* Low-precision Cholesky of the binary32 copy W (lower, in place).  Every
 * arithmetic step is single precision; with lo == 2 each factor entry is
 * rounded to bfloat16 before it enters a product of the Schur-complement
 * sum.  Same column algorithm as or_potrf. */
int64_t or_potrf_lo(int64_t n, float *W, int64_t ldw, int lo)
{
    for (int64_t j = 0; j < n; ++j) {
        int64_t m = n - j;
#pragma omp parallel if (m * j > 65536)
        {
            int nt = omp_get_num_threads(), t = omp_get_thread_num();
            int64_t i0 = j + (m * t) / nt, i1 = j + (m * (t + 1)) / nt;
            for (int64_t k = 0; k < j; ++k) {
                float b = AT(W, ldw, j, k);
                if (lo == 2) b = or_round_bf16(b);
                for (int64_t i = i0; i < i1; ++i) {
                    float a = AT(W, ldw, i, k);
                    if (lo == 2) a = or_round_bf16(a);
                    AT(W, ldw, i, j) = AT(W, ldw, i, j) - a * b;
                }
            }
        }
        float d = AT(W, ldw, j, j);
        if (!(d > 0.0f))
            return j + 1;
        d = sqrtf(d);
        AT(W, ldw, j, j) = d;
        for (int64_t i = j + 1; i < n; ++i)
            AT(W, ldw, i, j) = AT(W, ldw, i, j) / d;
    }
    return 0;
}

/* Blocked low-precision factor of the binary32 copy W (lower, in place),
 * block width nb >= 1:
 *   for each block column [k0, k1):
 *     1. W_kk (FP32) -> FP64, Cholesky by or_potrf, stored rounded to FP32;
 *        a failing pivot returns k0 + its local column (1-based);
 *     2. rows i >= k1: L_ic = (W_ic - sum_{k0<=p<c} L_ip L_cp) / L_cc for
 *        c = k0 .. k1-1, every operation in binary32, p increasing;
 *     3. lower trailing entries (i >= j >= k1):
 *        W_ij = W_ij - s,  s = sum_{p=k0}^{k1-1} r(L_ip) r(L_jp)
 *        accumulated in binary32 from 0, p increasing, where r rounds to
 *        bfloat16 when lo == 2 and is the identity otherwise.
 * With nb >= n the whole matrix is one diagonal block: the result is the
 * FP64 factor of fl32(A) rounded to binary32. */
int64_t or_potrf_lo_blocked(int64_t n, float *W, int64_t ldw, int lo, int64_t nb)
{
    if (nb < 1)
        nb = 1;
    double *D = (double *)malloc((size_t)nb * (size_t)nb * sizeof(double));
    for (int64_t k0 = 0; k0 < n; k0 += nb) {
        int64_t kb = n - k0 < nb ? n - k0 : nb, k1 = k0 + kb;
        for (int64_t j = 0; j < kb; ++j)
            for (int64_t i = j; i < kb; ++i)
                D[i + j * kb] = (double)AT(W, ldw, k0 + i, k0 + j);
        int64_t f = or_potrf(kb, D, kb);
        if (f != 0) {
            free(D);
            return k0 + f;
        }
        for (int64_t j = 0; j < kb; ++j)
            for (int64_t i = j; i < kb; ++i)
                AT(W, ldw, k0 + i, k0 + j) = (float)D[i + j * kb];
#pragma omp parallel for schedule(static) if ((n - k1) * kb > 65536)
        for (int64_t i = k1; i < n; ++i) {
            for (int64_t c = k0; c < k1; ++c) {
                float t = AT(W, ldw, i, c);
                for (int64_t p = k0; p < c; ++p)
                    t = t - AT(W, ldw, i, p) * AT(W, ldw, c, p);
                AT(W, ldw, i, c) = t / AT(W, ldw, c, c);
            }
        }
#pragma omp parallel for schedule(dynamic, 16) if ((n - k1) * kb > 65536)
        for (int64_t j = k1; j < n; ++j) {
            for (int64_t i = j; i < n; ++i) {
                float s = 0.0f;
                for (int64_t p = k0; p < k1; ++p) {
                    float a = AT(W, ldw, i, p), b = AT(W, ldw, j, p);
                    if (lo == 2) {
                        a = or_round_bf16(a);
                        b = or_round_bf16(b);
                    }
                    s = s + a * b;
                }
                AT(W, ldw, i, j) = AT(W, ldw, i, j) - s;
            }
        }
    }
    free(D);
    return 0;
}

/* Forward then back substitution in binary32. */
void or_potrs_lo(int64_t n, int64_t nrhs, const float *L, int64_t ldl,
                 float *B, int64_t ldb)
{
    for (int64_t r = 0; r < nrhs; ++r) {
        float *b = B + (size_t)r * (size_t)ldb;
        for (int64_t j = 0; j < n; ++j) {
            float t = b[j];
            for (int64_t k = 0; k < j; ++k)
                t = t - AT(L, ldl, j, k) * b[k];
            b[j] = t / AT(L, ldl, j, j);
        }
        for (int64_t j = n - 1; j >= 0; --j) {
            float t = b[j];
            for (int64_t k = j + 1; k < n; ++k)
                t = t - AT(L, ldl, k, j) * b[k];
            b[j] = t / AT(L, ldl, j, j);
        }
    }
}

/* FP64 residual (plain double, increasing column order) and per-column eta
 * used by the refinement loop's stopping test. */
static double ir_residual(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                          const double *X, int64_t ldx, const double *B, int64_t ldb,
                          double anorm, double *R, double *eta_max)
{
    double emax = 0.0;
    for (int64_t r = 0; r < nrhs; ++r) {
        double rmax = 0.0, xmax = 0.0, bmax = 0.0;
        int bad = 0;
        for (int64_t i = 0; i < n; ++i) {
            double t = AT(B, ldb, i, r);
            for (int64_t j = 0; j < n; ++j) {
                double a = i >= j ? AT(A, lda, i, j) : AT(A, lda, j, i);
                t = t - a * AT(X, ldx, j, r);
            }
            R[(size_t)r * (size_t)n + (size_t)i] = t;
            if (fabs(t) > rmax) rmax = fabs(t);
            if (fabs(AT(X, ldx, i, r)) > xmax) xmax = fabs(AT(X, ldx, i, r));
            if (fabs(AT(B, ldb, i, r)) > bmax) bmax = fabs(AT(B, ldb, i, r));
            if (t != t) bad = 1;
        }
        double den = anorm * xmax + bmax;
        double e = bad ? INFINITY : (den > 0.0 ? rmax / den : (rmax > 0.0 ? INFINITY : 0.0));
        if (e > emax || e != e) emax = e;
    }
    *eta_max = emax;
    return emax;
}

/*
 * Mixed-precision solve with iterative refinement.
 *   1. W = fl32(A); factor W in low precision (lo = 1: binary32,
 *      lo = 2: bfloat16 operands in the Schur-complement products): the
 *      blocked factor or_potrf_lo_blocked with block nb when nb > 0, the
 *      column algorithm or_potrf_lo (every operation in binary32) when
 *      nb == 0.
 *   2. x = solve_lo(fl32(b)), widened to FP64.
 *   3. repeat: r = b - A x in FP64; stop when max_j eta_j <= tol;
 *      otherwise d = solve_lo(fl32(r)) and x = x + d in FP64.
 *   4. Non-convergence: max_iter corrections without reaching tol, or the
 *      largest eta failing to halve on two consecutive iterations.
 *   5. On a low-precision breakdown or non-convergence: plain FP64 solve,
 *      *fell_back = 1.
 * hist (NULL, or max_iter + 1 entries) receives the largest eta of every
 * residual evaluated by the refinement loop, in order (entry k: after k
 * corrections); *nhist receives how many were written.
 * Returns the FP64 info of the fallback (0 unless A itself is not SPD).
 */
int64_t or_posv_ir(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double *X, int64_t ldx,
                   int lo, double tol, int max_iter, int64_t nb,
                   int *iters, int *fell_back, double *eta_final,
                   double *hist, int *nhist)
{
    if (nhist)
        *nhist = 0;
    *iters = 0;
    *fell_back = 0;
    *eta_final = 0.0;
    if (n == 0 || nrhs == 0)
        return 0;
    size_t nn = (size_t)n;
    float *W = (float *)malloc(nn * nn * sizeof(float));
    float *d = (float *)malloc(nn * (size_t)nrhs * sizeof(float));
    double *R = (double *)malloc(nn * (size_t)nrhs * sizeof(double));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i < n; ++i)
            W[i + j * nn] = (float)AT(A, lda, i, j);
    int converged = 0;
    int64_t finfo = nb > 0 ? or_potrf_lo_blocked(n, W, n, lo, nb) : or_potrf_lo(n, W, n, lo);
    if (finfo == 0) {
        for (int64_t r = 0; r < nrhs; ++r)
            for (int64_t i = 0; i < n; ++i)
                d[i + r * nn] = (float)AT(B, ldb, i, r);
        or_potrs_lo(n, nrhs, W, n, d, n);
        for (int64_t r = 0; r < nrhs; ++r)
            for (int64_t i = 0; i < n; ++i)
                AT(X, ldx, i, r) = (double)d[i + r * nn];
        double anorm = or_sym_norm_inf(n, A, lda);
        double prev = INFINITY, prev2 = INFINITY, e = INFINITY;
        int slow = 0;
        for (int it = 0;; ++it) {
            ir_residual(n, nrhs, A, lda, X, ldx, B, ldb, anorm, R, &e);
            *eta_final = e;
            if (hist && nhist)
                hist[(*nhist)++] = e;
            if (e <= tol) { converged = 1; *iters = it; break; }
            if (it >= max_iter || e != e) { *iters = it; break; }
            if (it > 0 && !(e <= 0.5 * prev)) ++slow; else slow = 0;
            if (slow >= 2) { *iters = it; break; }
            prev2 = prev;
            prev = e;
            for (int64_t r = 0; r < nrhs; ++r)
                for (int64_t i = 0; i < n; ++i)
                    d[i + r * nn] = (float)R[i + r * nn];
            or_potrs_lo(n, nrhs, W, n, d, n);
            for (int64_t r = 0; r < nrhs; ++r)
                for (int64_t i = 0; i < n; ++i)
                    AT(X, ldx, i, r) = AT(X, ldx, i, r) + (double)d[i + r * nn];
        }
        (void)prev2;
    }
    int64_t info = 0;
    if (!converged) {
        *fell_back = 1;
        double *Ac = (double *)malloc(nn * nn * sizeof(double));
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = j; i < n; ++i)
                Ac[i + j * nn] = AT(A, lda, i, j);
        for (int64_t r = 0; r < nrhs; ++r)
            for (int64_t i = 0; i < n; ++i)
                AT(X, ldx, i, r) = AT(B, ldb, i, r);
        info = or_posv(n, nrhs, Ac, n, X, ldx);
        free(Ac);
        if (info == 0) {
            double anorm = or_sym_norm_inf(n, A, lda), e;
            ir_residual(n, nrhs, A, lda, X, ldx, B, ldb, anorm, R, &e);
            *eta_final = e;
        }
    }
    free(W);
    free(d);
    free(R);
    return info;
}

/* ------------------------------------------------------------- adjoint */
/*
 * X = A^{-1} B with A = L L^T.  Given gX = dloss/dX:
 *   gB = A^{-1} gX                      (two triangular solves with L)
 *   mode 0: gA = -1/2 (gB X^T + X gB^T) (full symmetric matrix)
 *   mode 1: gradient with respect to the stored lower triangle:
 *           gA(i, j) = -(gB X^T + X gB^T)(i, j) for i > j,
 *           gA(i, i) = -(gB X^T)(i, i), strict upper set to 0.
 * Follows from dX = A^{-1}(dB - dA X).
 */
void or_posv_backward(int64_t n, int64_t nrhs, const double *L, int64_t lda,
                      const double *X, int64_t ldx, const double *GX, int64_t ldgx,
                      double *GB, int64_t ldgb, double *GA, int64_t ldga, int mode)
{
    for (int64_t r = 0; r < nrhs; ++r)
        for (int64_t i = 0; i < n; ++i)
            AT(GB, ldgb, i, r) = AT(GX, ldgx, i, r);
    or_potrs(n, nrhs, L, lda, GB, ldgb);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < n; ++i) {
            double s1 = 0.0, s2 = 0.0;
            for (int64_t r = 0; r < nrhs; ++r) {
                s1 = s1 + AT(GB, ldgb, i, r) * AT(X, ldx, j, r);
                s2 = s2 + AT(X, ldx, i, r) * AT(GB, ldgb, j, r);
            }
            double v;
            if (mode == 0)
                v = -0.5 * (s1 + s2);
            else if (i > j)
                v = -(s1 + s2);
            else if (i == j)
                v = -s1;
            else
                v = 0.0;
            AT(GA, ldga, i, j) = v;
        }
    }
}

void or_potrf_backward(int64_t n, const double *L, int64_t lda, const double *GL, int64_t ldgl,
                       double *GA, int64_t ldga, int mode)
{
    if (n <= 0)
        return;
    double *P = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    /* P = Phi(L^T GL): (L^T GL)_ij = sum_{k >= max(i,j)} L_ki GL_kj, lower part
     * only, diagonal halved (GL is lower triangular: only k >= j counts) */
#pragma omp parallel for schedule(dynamic)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i < n; ++i) {
            double s = 0.0;
            for (int64_t k = i; k < n; ++k)
                s = s + AT(L, lda, k, i) * AT(GL, ldgl, k, j);
            AT(P, n, i, j) = (i == j) ? 0.5 * s : s;
        }
    /* Y = P L^{-1}: each row y of P solves y L = p, i.e. L^T y^T = p^T
     * (back substitution on the row) */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        for (int64_t c = n - 1; c >= 0; --c) {
            double v = AT(P, n, r, c);
            for (int64_t k = c + 1; k < n; ++k)
                v = v - AT(P, n, r, k) * AT(L, lda, k, c);
            AT(P, n, r, c) = v / AT(L, lda, c, c);
        }
    }
    /* S = L^{-T} Y: each column solved by back substitution with L^T */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        trsv_lower_trans(n, L, lda, &AT(P, n, 0, c));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            double v;
            if (mode == 0)
                v = 0.5 * (AT(P, n, i, j) + AT(P, n, j, i));
            else if (i > j)
                v = AT(P, n, i, j) + AT(P, n, j, i);
            else if (i == j)
                v = AT(P, n, i, i);
            else
                continue;
            AT(GA, ldga, i, j) = v;
        }
    free(P);
}

int64_t or_getrf(int64_t n, double *A, int64_t lda, int32_t *ipiv)
{
    int64_t info = 0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        double best = fabs(AT(A, lda, k, k));
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(AT(A, lda, i, k)) > best) {
                best = fabs(AT(A, lda, i, k));
                p = i;
            }
        ipiv[k] = (int32_t)(p + 1);
        if (p != k)
            for (int64_t j = 0; j < n; ++j) {
                double t = AT(A, lda, k, j);
                AT(A, lda, k, j) = AT(A, lda, p, j);
                AT(A, lda, p, j) = t;
            }
        double piv = AT(A, lda, k, k);
        if (piv == 0.0) {
            if (info == 0)
                info = k + 1;
            continue;
        }
        for (int64_t i = k + 1; i < n; ++i)
            AT(A, lda, i, k) = AT(A, lda, i, k) / piv;
#pragma omp parallel for schedule(static) if ((n - k) * (n - k) > 65536)
        for (int64_t j = k + 1; j < n; ++j) {
            double ukj = AT(A, lda, k, j);
            for (int64_t i = k + 1; i < n; ++i)
                AT(A, lda, i, j) = AT(A, lda, i, j) - AT(A, lda, i, k) * ukj;
        }
    }
    return info;
}

void or_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda, const int32_t *ipiv,
              double *B, int64_t ldb)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double *b = &AT(B, ldb, 0, r);
        for (int64_t k = 0; k < n; ++k) {
            int64_t p = ipiv[k] - 1;
            if (p != k) {
                double t = b[k];
                b[k] = b[p];
                b[p] = t;
            }
        }
        for (int64_t i = 0; i < n; ++i) { /* L y = P b, L unit lower */
            double v = b[i];
            for (int64_t k = 0; k < i; ++k)
                v = v - AT(LU, lda, i, k) * b[k];
            b[i] = v;
        }
        for (int64_t i = n - 1; i >= 0; --i) { /* U x = y */
            double v = b[i];
            for (int64_t k = i + 1; k < n; ++k)
                v = v - AT(LU, lda, i, k) * b[k];
            b[i] = v / AT(LU, lda, i, i);
        }
    }
}

/* residual of a general (non-symmetric) system in extended precision:
 * eta_j = |b_j - A x_j|inf / (|A|inf |x_j|inf + |b_j|inf), |A|inf the
 * largest row sum of |A| */
double or_residual_gen(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                       const double *X, int64_t ldx, const double *B, int64_t ldb, double *eta)
{
    long double anorm = 0.0L;
    for (int64_t i = 0; i < n; ++i) {
        long double s = 0.0L;
        for (int64_t j = 0; j < n; ++j)
            s += fabsl((long double)AT(A, lda, i, j));
        if (s > anorm)
            anorm = s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        long double rmax = 0.0L, xmax = 0.0L, bmax = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            long double s = (long double)AT(B, ldb, i, r);
            for (int64_t j = 0; j < n; ++j)
                s -= (long double)AT(A, lda, i, j) * (long double)AT(X, ldx, j, r);
            if (fabsl(s) > rmax)
                rmax = fabsl(s);
            if (fabsl((long double)AT(X, ldx, i, r)) > xmax)
                xmax = fabsl((long double)AT(X, ldx, i, r));
            if (fabsl((long double)AT(B, ldb, i, r)) > bmax)
                bmax = fabsl((long double)AT(B, ldb, i, r));
        }
        long double den = anorm * xmax + bmax;
        eta[r] = (double)(den > 0.0L ? rmax / den : 0.0L);
    }
    return (double)anorm;
}

/* ---------------------------------------------------- complex Hermitian */
int64_t or_zpotrf(int64_t n, double complex *A, int64_t lda)
{
    for (int64_t j = 0; j < n; ++j) {
        /* column j, rows j..n-1, minus sum_{k<j} L(i,k) conj(L(j,k)), k increasing */
        int64_t m = n - j;
#pragma omp parallel if (m * j > 65536)
        {
            int nt = omp_get_num_threads(), t = omp_get_thread_num();
            int64_t i0 = j + (m * t) / nt, i1 = j + (m * (t + 1)) / nt;
            for (int64_t k = 0; k < j; ++k) {
                double complex cjk = conj(AT(A, lda, j, k));
                for (int64_t i = i0; i < i1; ++i)
                    AT(A, lda, i, j) = AT(A, lda, i, j) - AT(A, lda, i, k) * cjk;
            }
        }
        /* the diagonal is real: its imaginary part is neither read nor kept */
        double d = creal(AT(A, lda, j, j));
        if (!(d > 0.0))
            return j + 1;
        d = sqrt(d);
        AT(A, lda, j, j) = d;
        for (int64_t i = j + 1; i < n; ++i)
            AT(A, lda, i, j) = AT(A, lda, i, j) / d;
    }
    return 0;
}

void or_zpotrs(int64_t n, int64_t nrhs, const double complex *L, int64_t lda, double complex *B, int64_t ldb)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        double complex *b = &AT(B, ldb, 0, r);
        for (int64_t i = 0; i < n; ++i) { /* L y = b */
            double complex v = b[i];
            for (int64_t k = 0; k < i; ++k)
                v = v - AT(L, lda, i, k) * b[k];
            b[i] = v / creal(AT(L, lda, i, i));
        }
        for (int64_t i = n - 1; i >= 0; --i) { /* L^H x = y */
            double complex v = b[i];
            for (int64_t k = i + 1; k < n; ++k)
                v = v - conj(AT(L, lda, k, i)) * b[k];
            b[i] = v / creal(AT(L, lda, i, i));
        }
    }
}

/* entry (i, j) of the Hermitian matrix whose lower triangle is stored */
static long double complex herm_at(const double complex *A, int64_t lda, int64_t i, int64_t j)
{
    if (i == j)
        return (long double)creal(AT(A, lda, i, i));
    if (i > j)
        return (long double complex)AT(A, lda, i, j);
    return conjl((long double complex)AT(A, lda, j, i));
}

double or_residual_z(int64_t n, int64_t nrhs, const double complex *A, int64_t lda,
                     const double complex *X, int64_t ldx, const double complex *B, int64_t ldb, double *eta)
{
    long double anorm = 0.0L;
    for (int64_t i = 0; i < n; ++i) {
        long double s = 0.0L;
        for (int64_t j = 0; j < n; ++j)
            s += cabsl(herm_at(A, lda, i, j));
        if (s > anorm)
            anorm = s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrhs; ++r) {
        long double rmax = 0.0L, xmax = 0.0L, bmax = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            long double complex s = (long double complex)AT(B, ldb, i, r);
            for (int64_t j = 0; j < n; ++j)
                s -= herm_at(A, lda, i, j) * (long double complex)AT(X, ldx, j, r);
            if (cabsl(s) > rmax)
                rmax = cabsl(s);
            if (cabsl((long double complex)AT(X, ldx, i, r)) > xmax)
                xmax = cabsl((long double complex)AT(X, ldx, i, r));
            if (cabsl((long double complex)AT(B, ldb, i, r)) > bmax)
                bmax = cabsl((long double complex)AT(B, ldb, i, r));
        }
        long double den = anorm * xmax + bmax;
        eta[r] = (double)(den > 0.0L ? rmax / den : 0.0L);
    }
    return (double)anorm;
}

int or_num_threads(void)
{
    return omp_get_max_threads();
}
