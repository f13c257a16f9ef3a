/*
 * mg.h -- C ABI of the MI355X (gfx950) dense SPD solver library (libmg.so).
 *
 * The operation is the one the paper (JAXMg, "Software design", the potrs
 * bullet) exposes: solve A X = B for a symmetric positive-definite A through
 * a Cholesky factorisation A = L L^T (potrf) followed by the two triangular
 * solves (potrs), optionally returning log det A.  The paper's tile-size
 * knob T_A ("Software design"; larger tiles help once N is large,
 * "Performance and scaling") is the potrf block size (mg_set_block_size).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major with a leading dimension: element (i, j) of A
 *   is A[i + j*lda].  Only the LOWER triangle (diagonal included) of A is
 *   read; potrf writes L over it and never reads or writes the strict upper
 *   triangle.  Rows n..lda-1 of every column are never touched.
 * - All matrix/vector pointers are DEVICE pointers owned by the caller.  The
 *   library allocates no device memory on these paths; scratch space comes
 *   from the caller through `work` arguments sized by *_buffer_size.
 * - Work is enqueued on the handle's HIP stream (hipStream_t passed as
 *   void*); calls return without synchronising unless stated otherwise.
 * - Return value (host): MG_OK, a negative value -k when the k-th argument
 *   (1-based, in C-signature order) is invalid -- checked before anything is
 *   enqueued -- or a positive MG_ERR_* code for runtime failures.
 * - `info` (device int32): 0 on success; k > 0 when the leading minor of
 *   order k is not positive definite (pivot <= 0 or NaN).  Factorisation
 *   stops there; columns >= k of the result are unspecified.  Kernels
 *   enqueued after a failure see the non-zero info and do nothing.
 *   MG_INFO_SOLVE_ABORTED (negative) when a triangular sweep's bounded wait
 *   for an earlier block gave up (which only a stalled device produces, or
 *   mg_set_sweep_spin_limit(h, 0) on purpose): the solution is then filled
 *   with quiet NaNs.
 */
#ifndef MG_H_
#define MG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mg_status;
typedef struct mg_handle_s *mg_handle_t;

#define MG_OK 0
#define MG_ERR_HIP 1          /* a HIP runtime call or kernel launch failed */
#define MG_ERR_UNSUPPORTED 2  /* dtype, precision or option not supported */
#define MG_ERR_INTERNAL 3     /* inconsistent internal state */
#define MG_ERR_ABORTED 4      /* a synchronising call saw a triangular sweep give up waiting */

#define MG_INFO_SOLVE_ABORTED (-1) /* device info: a sweep's (or the LU panel's) bounded wait gave up */
#define MG_INFO_BAD_PIVOT (-2)     /* device info: mg_getrs met an ipiv entry outside 1..n */

typedef enum { MG_F64 = 0, MG_F32 = 1 } mg_dtype;

/* Library version as major*10000 + minor*100 + patch. */
int32_t mg_version(void);

/* Create a handle bound to the current HIP device and to `stream`
 * (a hipStream_t; NULL = the default stream).  *handle receives the handle.
 * Errors: -1 if handle is NULL; MG_ERR_HIP if the device query fails. */
mg_status mg_create(mg_handle_t *handle, void *stream);
/* Destroy a handle (NULL is accepted).  Releases profiling events only. */
mg_status mg_destroy(mg_handle_t handle);
/* Rebind the handle to another stream.  Errors: -1 if handle is NULL. */
mg_status mg_set_stream(mg_handle_t handle, void *stream);

/* potrf block size nb (the paper's tile size T_A).  0 selects the built-in
 * default for the problem size; otherwise nb must be 64, 128, or a multiple
 * of 256 up to 1024.  Blocks wider than 128 are factored in 128-wide steps
 * (diagonal factor, panel solve, rank-128 update of the rest of the block
 * column), and the trailing matrix receives one rank-nb update per block
 * column.
 * Errors: -1 NULL handle, -2 unsupported nb. */
mg_status mg_set_block_size(mg_handle_t handle, int64_t nb);
/* Look-ahead schedule for potrf (default on): the trailing update of step k
 * is split into the next block column, updated first so that the next
 * diagonal block and panel can be factored right away, and the remainder,
 * applied concurrently.  The two run on two non-blocking streams owned by the
 * handle, which fork from and join into the handle's stream by events.  0
 * runs every step in sequence on the handle's stream; 2 is the look-ahead
 * with the remainder's stream CU-masked to leave one CU per XCD to the
 * next block column's factor (measured no faster; kept as an option).  The
 * result is bitwise the same in every mode.
 * Errors: -1 NULL handle, -2 mode not 0, 1 or 2. */
mg_status mg_set_lookahead(mg_handle_t handle, int32_t enable);

/* Polls a triangular-sweep block makes for an earlier block's result before
 * it gives up (the wait is bounded so that a stalled device cannot hang the
 * call): -1 restores the built-in limit (2^22); 0 makes every block that
 * depends on another give up at once without waiting, which drives the
 * give-up path (info = MG_INFO_SOLVE_ABORTED, NaN solution) from the host for
 * tests; positive values set the limit.  The same value bounds the polls of
 * mg_getrf's panel grid barrier (built-in limit 2^24; 0: every barrier of a
 * panel of more than 256 rows gives up without waiting).
 * Errors: -1 NULL handle, -2 limit outside [-1, 2^30]. */
mg_status mg_set_sweep_spin_limit(mg_handle_t handle, int64_t limit);

/* How the triangular sweeps (potrs and every solve built on it) apply a
 * 64 x 64 diagonal block of L:
 *   MG_SOLVE_INVERSE (default): each block's inverse is formed by the
 *     workgroup that owns the block when it starts, while it still waits for
 *     the blocks before it, and the block's solution is then one product on
 *     the matrix pipe.  The result satisfies the usual backward-error bound
 *     up to a factor of the diagonal blocks' condition number.
 *   MG_SOLVE_SUBSTITUTION: forward/back substitution in registers, 64
 *     dependent steps per block (longer chain); exact whenever the data and
 *     every intermediate are representable, e.g. integer factors with
 *     power-of-two pivots.
 * Errors: -1 NULL handle, -2 unknown mode. */
typedef enum { MG_SOLVE_INVERSE = 0, MG_SOLVE_SUBSTITUTION = 1 } mg_solve_mode;
mg_status mg_set_solve_mode(mg_handle_t handle, mg_solve_mode mode);

/* Block size potrf would use for (dtype, n).  Errors: -1, -2, -3 (n < 0), -4 NULL. */
mg_status mg_get_block_size(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t *nb);

/*
 * potrf: Cholesky factorisation A = L L^T in place (paper: "Software design",
 * potrs bullet; LAPACK xPOTRF semantics, lower).
 *   dtype  MG_F64 or MG_F32 (storage and arithmetic type).
 *   n      order, n >= 0 (n = 0: info is set to 0 and nothing else happens).
 *   A      device, lda x n column-major; lower triangle in, L out.
 *   lda    >= max(1, n).
 *   info   device int32, written (0 or k > 0).
 * Errors: -1 NULL handle, -2 bad dtype, -3 n < 0, -4 A NULL with n > 0,
 *         -5 lda < max(1,n), -6 info NULL.
 */
mg_status mg_potrf(mg_handle_t handle, mg_dtype dtype, int64_t n, void *A, int64_t lda,
                   int32_t *info);

/* Bytes of device workspace mg_potrs / mg_posv need for (dtype, n, nrhs):
 * the intermediate Y = L^{-1} B (n x nrhs) plus 256 bytes of sweep counters
 * (0 when n or nrhs is 0).  The library clears the counters itself at the
 * start of every solve, so the workspace needs no initialisation; two solves
 * in flight at once must not share one workspace.
 * Errors: -1 NULL handle, -2 bad dtype, -3 n < 0, -4 nrhs < 0, -5 NULL out. */
mg_status mg_potrs_buffer_size(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t nrhs,
                               size_t *bytes);

/*
 * potrs: X = A^{-1} B from the factor L of mg_potrf: forward substitution
 * L Y = B, then back substitution L^T X = Y (paper: "Software design",
 * potrs bullet; b is N x N_RHS).  Each sweep is one persistent launch whose
 * workgroups take 64-row blocks in order and wait (boundedly) for the blocks
 * they depend on.
 *   L      device, lda x n, the factor in its lower triangle (strict upper
 *          never read).
 *   B      device, ldb x nrhs, overwritten with X.
 *   work   device scratch of mg_potrs_buffer_size bytes (may be NULL when
 *          that size is 0).
 *   info   optional device int32, in/out (NULL = absent): on entry the info
 *          of a preceding mg_potrf -- when it is non-zero B is left
 *          unmodified; set to MG_INFO_SOLVE_ABORTED when a sweep gives up
 *          (B is then all NaN, which is also what happens with info NULL).
 * Errors: -1 NULL handle, -2 dtype, -3 n < 0, -4 nrhs < 0, -5 L NULL,
 *         -6 lda, -7 B NULL, -8 ldb < max(1,n), -9 work NULL, -10 work too small.
 */
mg_status mg_potrs(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t nrhs, const void *L,
                   int64_t lda, void *B, int64_t ldb, void *work, size_t work_bytes,
                   int32_t *info);

/*
 * posv: factor then solve (potrf + potrs) with no host synchronisation.
 * A is overwritten by L; B by X unless info > 0, in which case B is left
 * unmodified (info = MG_INFO_SOLVE_ABORTED: B is all NaN, as for mg_potrs).
 * Workspace: mg_potrs_buffer_size bytes.
 * Errors: -1 handle, -2 dtype, -3 n, -4 nrhs, -5 A, -6 lda, -7 B, -8 ldb,
 *         -9 work NULL, -10 work too small, -11 info NULL.
 */
mg_status mg_posv(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t nrhs, void *A,
                  int64_t lda, void *B, int64_t ldb, void *work, size_t work_bytes,
                  int32_t *info);

/*
 * posv without allocation.  For callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operation, arguments, results and info convention as
 * mg_posv, with no work argument: the solve's scratch (Y = L^{-1} B and the
 * sweep words, mg_potrs_buffer_size bytes) lives in a library-owned device
 * array of MG_NOALLOC_SCRATCH_BYTES on each GPU, created with the library's
 * code object and held until the process ends; its device address is looked
 * up once per device by mg_create.  The call allocates nothing (the handle's
 * look-ahead streams are created by mg_create; mg_set_lookahead(h, 2)
 * re-creates one at the next factorisation).
 * The array is shared by every call on one GPU and keeps the last call's
 * contents (the sweep words are reset by each call): calls whose work
 * overlaps in time on one GPU -- on different streams or handles -- race on
 * it and give undefined results, so serialise them.
 * Errors: -1 handle, -2 dtype, -3 n < 0, -4 nrhs < 0, -5 A NULL with n > 0,
 * -6 lda, -7 B NULL, -8 ldb < max(1,n), -9 info NULL; MG_ERR_SCRATCH_LIMIT
 * (nothing enqueued) when mg_potrs_buffer_size(dtype, n, nrhs) exceeds
 * MG_NOALLOC_SCRATCH_BYTES, i.e. roughly when n * nrhs * (8 for MG_F64, 4 for
 * MG_F32) > 32 MiB.
 */
#define MG_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
#define MG_ERR_SCRATCH_LIMIT 5 /* mg_posv_noalloc: problem needs more than MG_NOALLOC_SCRATCH_BYTES */
mg_status mg_posv_noalloc(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda,
                          void *B, int64_t ldb, int32_t *info);

/*
 * Mixed precision with iterative refinement.  The paper is silent on
 * precision; this is the classic scheme for SPD systems (Langou et al.,
 * SC'06; Carson & Higham 2018): factor a binary32 copy of A (diagonal blocks
 * in FP64 arithmetic, trailing updates on the FP32 matrix pipe, or with
 * MG_PREC_BF16 with trailing-update operands rounded to bfloat16), solve, then
 * refine: r = b - A x in FP64 with the original A, d = solve_lo(r),
 * x += d, until every column's normwise backward error
 * eta_j = |r_j|inf / (|A|inf |x_j|inf + |b_j|inf) <= tol.  It stops after
 * max_iter corrections or when the largest eta fails to halve twice in a
 * row; then, or when the low-precision factor breaks down, it solves in FP64
 * (fallback != 0) and reports fell_back = 1.
 */
typedef enum { MG_PREC_F32 = 1, MG_PREC_BF16 = 2 } mg_prec;
typedef struct {
    double tol;        /* backward-error target, default 1e-12 */
    int32_t max_iter;  /* refinement steps, default 30 */
    int32_t fallback;  /* 1: solve in FP64 when refinement does not converge (default) */
} mg_ir_opts;
typedef struct {
    int32_t iters;     /* corrections applied */
    int32_t fell_back; /* 1 when the FP64 fallback produced X */
    int32_t lo_info;   /* info of the low-precision factor (0, or the failing column) */
    int32_t reserved;
    double eta;        /* largest per-column backward error of the returned X (FP64 residual) */
} mg_ir_result;

/* Workspace bytes for mg_posv_mixed.  Errors: -1 handle, -2 lo, -3 n < 0,
 * -4 nrhs < 0, -5 NULL out.  The FP64 fallback needs an n x n FP64 copy of
 * A, so the size depends on `fallback`. */
mg_status mg_posv_mixed_buffer_size(mg_handle_t handle, mg_prec lo, int64_t n, int64_t nrhs, int32_t fallback,
                                    size_t *bytes);
/*
 * X = A^{-1} B with a low-precision factor and FP64 refinement.
 *   A      device, FP64, lda x n, lower triangle; NOT modified (the residual
 *          needs it).  B device FP64 ldb x nrhs, not modified.
 *   X      device FP64 ldx x nrhs, receives the solution.
 *   opts   host pointer, NULL for the defaults.
 *   work   device scratch of mg_posv_mixed_buffer_size bytes (it holds the
 *          low-precision factor).
 *   result host pointer, filled on return.
 *   info   device int32: 0, or k > 0 when the FP64 fallback finds A itself
 *          not positive definite.
 * The call synchronises the handle's stream once per refinement step (the
 * stopping test reads eta on the host) and returns after the solve.
 * Without a fallback (opts->fallback == 0): if the low-precision factor
 * breaks down (result->lo_info > 0) there is no solution, X is filled with
 * NaN and result->eta is NaN (info stays 0: A itself was not tested); if
 * refinement stops without converging, X is the last iterate and
 * result->eta its backward error (> tol).  If a triangular sweep gives up
 * waiting (see mg_set_sweep_spin_limit) the call returns MG_ERR_ABORTED
 * with X filled with NaN and result->eta NaN.
 * Errors: -1 handle, -2 lo, -3 n, -4 nrhs, -5 A, -6 lda, -7 B, -8 ldb, -9 X,
 *         -10 ldx, -11 opts (tol < 0 or max_iter < 0), -12 work NULL,
 *         -13 work too small, -14 result NULL, -15 info NULL.
 */
mg_status mg_posv_mixed(mg_handle_t handle, mg_prec lo, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double *X, int64_t ldx, const mg_ir_opts *opts, void *work,
                        size_t work_bytes, mg_ir_result *result, int32_t *info);

/*
 * Adjoint of X = A^{-1} B (reverse mode).  The paper puts these solves inside
 * differentiable programs ("Statement of need") without stating the adjoint;
 * from dX = A^{-1}(dB - dA X):
 *   gB = A^{-1} gX, from the stored factor L (no refactorisation);
 *   MG_GRAD_SYM   : gA = -1/2 (gB X^T + X gB^T), full n x n symmetric;
 *   MG_GRAD_LOWER : gradient with respect to the lower triangle the solver
 *                   reads: gA(i,j) = -(gB X^T + X gB^T)(i,j) for i > j,
 *                   gA(i,i) = -(gB X^T)(i,i); the strict upper triangle of
 *                   gA is not written.
 * FP64 only.  L: lda x n factor from mg_potrf; X: ldx x nrhs forward
 * solution; gX: ldgx x nrhs upstream gradient (read only); gB: ldgb x nrhs
 * output; gA: ldga x n output.  work: mg_potrs_buffer_size(MG_F64, n, nrhs)
 * bytes.  info: optional device int32 of the factorisation, in/out; when it
 * is non-zero gB and the entries of gA the mode writes are NaN; a sweep that
 * gives up sets it to MG_INFO_SOLVE_ABORTED (with the same NaN outputs).
 * Errors: -1 handle, -2 n, -3 nrhs, -4 L, -5 lda, -6 X, -7 ldx, -8 gX, -9 ldgx,
 *         -10 gB, -11 ldgb, -12 gA, -13 ldga, -14 mode, -15 work NULL,
 *         -16 work too small.
 */
typedef enum { MG_GRAD_SYM = 0, MG_GRAD_LOWER = 1 } mg_grad_mode;
mg_status mg_posv_backward(mg_handle_t handle, int64_t n, int64_t nrhs, const double *L, int64_t lda,
                           const double *X, int64_t ldx, const double *gX, int64_t ldgx, double *gB, int64_t ldgb,
                           double *gA, int64_t ldga, mg_grad_mode mode, void *work, size_t work_bytes,
                           int32_t *info);

/*
 * Adjoint of the Cholesky factorisation itself (for callers that use L or
 * log det directly): given gL = df/dL for L = chol(A), the gradient of f with
 * respect to A.  The paper places the solver inside differentiable programs
 * ("Statement of need") without stating this adjoint; from A = L L^T,
 * dL = L Phi(L^{-1} dA L^{-T}) with Phi = lower triangle, diagonal halved,
 * so df = <S, dA> with S = L^{-T} Phi(L^T gL) L^{-1} (Murray 2016):
 *   MG_GRAD_SYM   : gA = (S + S^T)/2, full n x n symmetric;
 *   MG_GRAD_LOWER : gradient with respect to the lower-triangle entries:
 *                   S_ij + S_ji for i > j, S_ii on the diagonal; the strict
 *                   upper triangle of gA is not written.
 * FP64.  L: lda x n factor from mg_potrf (lower triangle read).  gL: ldgl x n,
 * only its lower triangle is read.  gA: ldga x n output (also used as
 * scratch: every entry of its n x n block may be written).  work: device
 * scratch of mg_potrf_backward_buffer_size bytes (an n x n FP64 matrix and
 * the sweep words or the 64 x 64 diagonal inverses).  The two triangular
 * solves it performs (n right-hand sides each) are, when n is a multiple of
 * 64, blocked right solves with L (each 64-column block multiplied by its
 * diagonal block's inverse, then a rank-64 update on the matrix pipe);
 * otherwise sweeps that follow mg_set_solve_mode.  info: optional device int32 of the
 * factorisation, in/out; when it is non-zero the entries of gA the mode
 * writes are NaN; a sweep that gives up sets it to MG_INFO_SOLVE_ABORTED
 * (with the same NaN outputs).
 * Errors: -1 handle, -2 n < 0, -3 L, -4 lda, -5 gL, -6 ldgl, -7 gA, -8 ldga,
 *         -9 mode, -10 work NULL, -11 work too small.
 */
mg_status mg_potrf_backward_buffer_size(mg_handle_t handle, int64_t n, size_t *bytes);
mg_status mg_potrf_backward(mg_handle_t handle, int64_t n, const double *L, int64_t lda, const double *gL,
                            int64_t ldgl, double *gA, int64_t ldga, mg_grad_mode mode, void *work,
                            size_t work_bytes, int32_t *info);

/*
 * Batched posv: many independent SPD systems of uneven order (0..512) solved
 * in one persistent launch replayed from a HIP graph.  The paper's operation
 * applied to a batch (it has no batched form).  A plan fixes the orders, the
 * number of right-hand sides (1..8) and the launch shape:
 *   - the systems are taken longest first (or in input order) from an atomic
 *     counter by a persistent grid of grid_per_cu workgroups per CU;
 *   - two kernel variants: four waves per system (one workgroup per
 *     system, up to three per CU), or eight waves per system with each
 *     block column's tiles and their earlier-column products spread over
 *     the waves (shorter per-system latency, one or two per CU);
 *   - with autotune on (the default) the plan times the candidates
 *     (variant x workgroups per CU x queue order) on synthetic systems of
 *     the same orders once and keeps the fastest; results are cached by
 *     (architecture, dtype, nrhs, batch, order histogram) in cache_path
 *     (NULL: no cache file);
 *   - the graph holds a counter reset and the persistent kernel; each call
 *     copies the caller's pointer/leading-dimension arrays into the plan.
 * Plan creation allocates device memory (descriptor arrays, tuning inputs);
 * mg_posv_batched allocates nothing.
 */
typedef struct mg_batch_plan_s *mg_batch_plan_t;
typedef struct {
    int32_t autotune;     /* 1: time the candidates (default), 0: use the fields below */
    int32_t grid_per_cu;  /* workgroups per CU (1..8; the autotuner tries 1 to 3, or 1 to 2 for variant 1); 0 = default */
    int32_t order;        /* 0 longest first, 1 input order, -1 default */
    const char *cache_path;  /* tuning cache file or NULL */
    int32_t variant;      /* kernel: 0 four waves per system, 1 eight waves (the work of each
                             block column spread over them), -1 default (0) */
} mg_tune_opts;
/* Errors: -1 handle, -2 dtype, -3 batch < 0, -4 n_host NULL or an order
 * outside [0, 512], -5 nrhs outside [1, 8], -7 plan NULL. */
mg_status mg_batch_plan_create(mg_handle_t handle, mg_dtype dtype, int32_t batch, const int64_t *n_host,
                               int32_t nrhs, const mg_tune_opts *opts, mg_batch_plan_t *plan);
/* Chosen kernel variant, launch shape and the tuned replay time (ms, -1 if
 * not tuned); NULL outputs are skipped.  Errors: -1 NULL plan. */
mg_status mg_batch_plan_info(mg_batch_plan_t plan, int32_t *grid_per_cu, int32_t *order, double *tuned_ms,
                             int32_t *variant);
/*
 * Solve every system: A_dev[k] (device pointer, lda_dev[k] x n_k, lower
 * triangle, overwritten by L_k) and B_dev[k] (ldb_dev[k] x nrhs, overwritten
 * by X_k).  A_dev, lda_dev, B_dev, ldb_dev and info_dev are DEVICE arrays of
 * length batch.  info_dev[k]: 0 or the failing column of system k (its B_k is
 * then left unmodified; the other systems are unaffected).  Enqueued on the
 * handle's stream, no host synchronisation.
 * Errors: -1 handle, -2 plan, -3 A_dev, -4 lda_dev, -5 B_dev, -6 ldb_dev, -7 info_dev.
 */
mg_status mg_posv_batched(mg_handle_t handle, mg_batch_plan_t plan, void *const *A_dev, const int64_t *lda_dev,
                          void *const *B_dev, const int64_t *ldb_dev, int32_t *info_dev);
/*
 * Adjoint of mg_posv_batched (reverse mode, every system at once; the paper
 * has no batched form, the per-system adjoint is mg_posv_backward's): for
 * system k, from its factor L_k (as mg_posv_batched left it in A_k), its
 * solution X_k and the upstream gradient gX_k,
 *   gB_k = A_k^{-1} gX_k,
 *   MG_GRAD_SYM   : gA_k = -1/2 (gB_k X_k^T + X_k gB_k^T), full n_k x n_k;
 *   MG_GRAD_LOWER : the gradient with respect to the lower-triangle
 *                   entries (strict upper triangle of gA_k not written).
 * Every argument from L_dev on is a DEVICE array of length batch (pointers,
 * leading dimensions >= n_k, info); the orders, nrhs and dtype are the
 * plan's.  info_dev: the forward call's per-system info; a non-zero entry
 * gives NaN in gB_k and in the entries of gA_k the mode writes.  One
 * persistent launch on the handle's stream (no graph, no host
 * synchronisation, nothing allocated).
 * Errors: -1 handle, -2 plan, -3..-12 NULL arrays (L, ldl, X, ldx, gX,
 * ldgx, gB, ldgb, gA, ldga), -15 mode, -16 info_dev NULL.
 */
mg_status mg_posv_batched_backward(mg_handle_t handle, mg_batch_plan_t plan, const void *const *L_dev,
                                   const int64_t *ldl_dev, const void *const *X_dev, const int64_t *ldx_dev,
                                   const void *const *gX_dev, const int64_t *ldgx_dev, void *const *gB_dev,
                                   const int64_t *ldgb_dev, void *const *gA_dev, const int64_t *ldga_dev,
                                   mg_grad_mode mode, const int32_t *info_dev);
/* Release a plan (NULL accepted). */
mg_status mg_batch_plan_destroy(mg_batch_plan_t plan);

/*
 * logdet: log det A = 2 sum_j log L_jj from the factor (paper: "Software
 * design", potrs bullet: the factorisation can optionally return log det A;
 * used by the Gaussian-process likelihood in "Scientific applications").
 *   out    device double, receives the value (NaN when info != 0).
 *   info   optional device int32 from mg_potrf (NULL = absent).
 * Errors: -1 handle, -2 dtype, -3 n < 0, -4 L NULL, -5 lda, -6 out NULL.
 */
mg_status mg_logdet(mg_handle_t handle, mg_dtype dtype, int64_t n, const void *L, int64_t lda,
                    double *out, const int32_t *info);

/*
 * Gaussian-process marginal log likelihood (paper: Research Impact Statement,
 * "Scientific applications", Cholesky solve): for each column j of Y,
 *   loglik[j] = -1/2 r_j^T A^{-1} r_j - 1/2 log det A - n/2 log(2 pi),
 *   r_j = y_j - m_j,
 * with A = K + Sigma the n x n SPD covariance, FP64.  One factorisation
 * serves every column: A = L L^T in place, alpha_j = A^{-1} r_j by the two
 * triangular sweeps, log det A = 2 sum_j log L_jj, and (r_j, alpha_j) summed
 * in a fixed order (results do not depend on the launch).
 *   A       n x n, column-major, lower triangle read; overwritten by L (the
 *           strict upper triangle is never touched).  Caller-owned.
 *   Y       n x nrhs observations (ldy >= n), read only.
 *   M       n x nrhs means (ldm >= n), read only, or NULL for zero mean.
 *   Alpha   n x nrhs output (ldalpha >= n): A^{-1}(y_j - m_j); holds
 *           y_j - m_j when the factorisation fails.
 *   loglik  device double[nrhs]: the values; NaN when info != 0.
 *   work    device workspace of mg_gp_loglik_buffer_size bytes (0 when n or
 *           nrhs is 0); work may be NULL then.
 *   info    device int32: 0, or the first column (1-based) whose pivot is
 *           not positive (as mg_potrf).  With nrhs == 0 only A is factored;
 *           with n == 0 every loglik is 0.
 * Errors (checked before any launch): -1 handle, -2 n < 0, -3 nrhs < 0,
 * -4 A NULL, -5 lda, -6 Y NULL, -7 ldy, -9 ldm (M given), -10 Alpha NULL,
 * -11 ldalpha, -12 loglik NULL, -13 work NULL, -14 work_bytes too small,
 * -15 info NULL.  Positive values: runtime errors as elsewhere.
 */
mg_status mg_gp_loglik_buffer_size(mg_handle_t handle, int64_t n, int64_t nrhs, size_t *bytes);
mg_status mg_gp_loglik(mg_handle_t handle, int64_t n, int64_t nrhs, double *A, int64_t lda, const double *Y,
                       int64_t ldy, const double *M, int64_t ldm, double *Alpha, int64_t ldalpha, double *loglik,
                       void *work, size_t work_bytes, int32_t *info);

/*
 * Gradient of sum_j g_j loglik[j] (mg_gp_loglik) with respect to A, Y and M,
 * from the factor and alpha that mg_gp_loglik returned (the log-det term's
 * adjoint is -A^{-1}/2, the quadratic term's alpha alpha^T/2):
 *   gA = sum_j g_j alpha_j alpha_j^T / 2 - (sum_j g_j) A^{-1} / 2
 *        (full n x n, exactly symmetric: the gradient with respect to the
 *        symmetric matrix, as MG_GRAD_SYM of mg_posv_backward),
 *   gY[:, j] = -g_j alpha_j,   gM[:, j] = g_j alpha_j.
 * A^{-1} = L^{-T} L^{-1} I is formed by the triangular sweeps with n
 * right-hand sides (O(n^3) work, n^2 doubles of it in the workspace).
 *   L       n x n factor from mg_gp_loglik (lower triangle read), lda >= n.
 *   Alpha   n x nrhs from mg_gp_loglik (ldalpha >= n).
 *   g       device double[nrhs]: the upstream gradient of each loglik.
 *   gA      n x n output (ldga >= n); gY n x nrhs output (ldgy >= n);
 *   gM      n x nrhs output (ldgm >= n) or NULL.
 *   work    device workspace of mg_gp_loglik_grad_buffer_size bytes.
 *   info    device int32 from mg_gp_loglik, in/out; nonzero makes every
 *           output NaN (a sweep that gives up sets MG_INFO_SOLVE_ABORTED).
 * Errors: -1 handle, -2 n < 0, -3 nrhs < 0, -4 L NULL, -5 lda, -6 Alpha NULL,
 * -7 ldalpha, -8 g NULL, -9 gA NULL, -10 ldga, -11 gY NULL, -12 ldgy,
 * -14 ldgm (gM given), -15 work NULL, -16 work_bytes too small, -17 info NULL;
 * MG_ERR_UNSUPPORTED when n > 16 * 65535.
 */
mg_status mg_gp_loglik_grad_buffer_size(mg_handle_t handle, int64_t n, size_t *bytes);
mg_status mg_gp_loglik_grad(mg_handle_t handle, int64_t n, int64_t nrhs, const double *L, int64_t lda,
                            const double *Alpha, int64_t ldalpha, const double *g, double *gA, int64_t ldga,
                            double *gY, int64_t ldgy, double *gM, int64_t ldgm, void *work, size_t work_bytes,
                            int32_t *info);

/*
 * Complex Hermitian positive-definite solve (the paper's routines take
 * complex64 and complex128 as well as the real types; "Software design").
 * Complex matrices are column-major with interleaved (real, imaginary) pairs
 * of the dtype's real type: dtype MG_F64 is complex128, MG_F32 complex64;
 * leading dimensions count complex elements.  Only the lower triangle of A is
 * read, and the imaginary part of its diagonal is ignored (LAPACK ZPOTRF).
 * The factorisation is computed as the real Cholesky factorisation of the
 * 2n x 2n blocked form of A (each entry a as [[Re a, -Im a], [Im a, Re a]]),
 * whose factor is the blocked form of L, on the real FP64 / FP32 path; so the
 * solve needs mg_zposv_buffer_size bytes of workspace (the 2n x 2n real
 * matrix, 4 n^2 real elements, plus the real solve's workspace) for all three
 * calls, and the real path's limits apply at order 2n.
 *   zpotrf: A = L L^H in place (lower triangle; real positive diagonal, its
 *           imaginary part written 0; strict upper triangle untouched).
 *           info (device int32, written): 0, or k > 0 when the leading minor
 *           of order k is not positive definite.
 *   zpotrs: X = A^{-1} B from zpotrf's L; B (n x nrhs) overwritten; info as
 *           mg_potrs (optional, in/out).
 *   zposv:  both; B left unmodified when info > 0.
 * Errors: zposv_buffer_size: -1 handle, -2 dtype, -3 n, -4 nrhs, -5 NULL out.
 *   zpotrf: -1 handle, -2 dtype, -3 n, -4 A NULL, -5 lda < max(1,n), -6 work
 *           NULL, -7 work too small, -8 info NULL.
 *   zpotrs: -1 handle, -2 dtype, -3 n, -4 nrhs, -5 L NULL, -6 lda, -7 B NULL,
 *           -8 ldb < max(1,n), -9 work NULL, -10 work too small.
 *   zposv:  as zpotrs with A for L, and -11 info NULL.
 */
mg_status mg_zposv_buffer_size(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t nrhs, size_t *bytes);
mg_status mg_zpotrf(mg_handle_t handle, mg_dtype dtype, int64_t n, void *A, int64_t lda, void *work,
                    size_t work_bytes, int32_t *info);
mg_status mg_zpotrs(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t nrhs, const void *L, int64_t lda,
                    void *B, int64_t ldb, void *work, size_t work_bytes, int32_t *info);
mg_status mg_zposv(mg_handle_t handle, mg_dtype dtype, int64_t n, int64_t nrhs, void *A, int64_t lda, void *B,
                   int64_t ldb, void *work, size_t work_bytes, int32_t *info);

/*
 * General solve (paper: "Software design", the lu_solve bullet: A x = b for a
 * general A through an LU factorisation with partial pivoting), FP64.
 *
 * getrf: P A = L U in place, LAPACK xGETRF semantics.  L is unit lower (its
 * strict lower triangle stored over A's), U upper (stored over A's upper
 * triangle, diagonal included).  Pivot of column k: the row with the largest
 * |entry| on or below the diagonal, the first such row on ties (an entry that
 * is NaN never wins; a NaN diagonal entry stays the pivot).
 *   n      order, n >= 0.
 *   A      device, lda x n column-major, overwritten by L and U.
 *   ipiv   device int32[n]: row k was interchanged with row ipiv[k] (1-based,
 *          ipiv[k] >= k + 1), in order k = 0..n-1.
 *   work   device scratch of mg_getrf_buffer_size bytes (no initialisation;
 *          not shared by two calls in flight).
 *   info   device int32, written: 0, or k > 0 when U(k,k) (1-based) is exactly
 *          zero -- the factorisation still completes, as LAPACK's; or
 *          MG_INFO_SOLVE_ABORTED when a panel's bounded grid-barrier wait gave
 *          up (A is then all NaN; mg_set_sweep_spin_limit sets the bound, 0
 *          forces the give-up at the first wait of a panel with more than 256
 *          rows).
 * Blocking: 64-wide pivoted panels inside outer block columns of 256 or 512
 * (the rank of the trailing update: 512 from n = 16384, else 256;
 * mg_set_block_size(h, 256 or 512) selects one, other values leave the
 * default).  The result does not depend on it up to rounding; pivots and
 * info are those of column-by-column elimination.
 * Limits (MG_ERR_UNSUPPORTED, nothing enqueued): n > 65536 for the default
 * 256-CU device, or (n + 576 lda) * 8 >= 2^31.
 * Errors: -1 handle, -2 n < 0, -3 A NULL, -4 lda < max(1,n), -5 ipiv NULL,
 *         -6 work NULL, -7 work too small, -8 info NULL.
 */
mg_status mg_getrf_buffer_size(mg_handle_t handle, int64_t n, size_t *bytes);
mg_status mg_getrf(mg_handle_t handle, int64_t n, double *A, int64_t lda, int32_t *ipiv, void *work,
                   size_t work_bytes, int32_t *info);

/*
 * getrs: X = A^{-1} B from mg_getrf's L, U and ipiv: the interchanges applied
 * to B, then L Y = P B and U X = Y by the persistent triangular sweeps of
 * mg_potrs (mg_set_solve_mode applies).
 *   LU     device, lda x n, mg_getrf's output (read only).
 *   ipiv   device int32[n], mg_getrf's output; an entry outside 1..n is
 *          ignored and reported (info = MG_INFO_BAD_PIVOT, B all NaN).
 *   B      device, ldb x nrhs, overwritten with X.
 *   work   device scratch of mg_getrs_buffer_size bytes.
 *   info   optional device int32, in/out (NULL = absent): when non-zero on
 *          entry (a singular U from mg_getrf), B is left unmodified; set to
 *          MG_INFO_SOLVE_ABORTED when a sweep gives up (B all NaN).
 * Errors: -1 handle, -2 n < 0, -3 nrhs < 0, -4 LU NULL, -5 lda, -6 ipiv NULL,
 *         -7 B NULL, -8 ldb < max(1,n), -9 work NULL, -10 work too small.
 */
mg_status mg_getrs_buffer_size(mg_handle_t handle, int64_t n, int64_t nrhs, size_t *bytes);
mg_status mg_getrs(mg_handle_t handle, int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                   const int32_t *ipiv, double *B, int64_t ldb, void *work, size_t work_bytes, int32_t *info);

/*
 * gesv: getrf then getrs, no host synchronisation.  A is overwritten by L and
 * U, ipiv written, B by X unless info > 0 (U singular: B left unmodified).
 * Workspace: mg_gesv_buffer_size bytes (the larger of the two).
 * Errors: -1 handle, -2 n, -3 nrhs, -4 A, -5 lda, -6 ipiv, -7 B, -8 ldb,
 *         -9 work NULL, -10 work too small, -11 info NULL.
 */
mg_status mg_gesv_buffer_size(mg_handle_t handle, int64_t n, int64_t nrhs, size_t *bytes);
mg_status mg_gesv(mg_handle_t handle, int64_t n, int64_t nrhs, double *A, int64_t lda, int32_t *ipiv,
                  double *B, int64_t ldb, void *work, size_t work_bytes, int32_t *info);

/*
 * Profiling.  When enabled, every launch of the kernel kinds below is
 * bracketed by a pair of HIP events on the handle's stream, and the
 * algorithmic work of each launch is accumulated.
 *   MG_PROF_TRAILING  -- trailing update lower(C) -= P P^T of rank k = 256 or
 *                        512 (the kernel variant that folds C into the
 *                        k-loop); flops = 2 k x (lower entries updated)
 *   MG_PROF_DIAG      -- diagonal-block factor; flops = b^3/3 + b^2/2 + b/6
 *   MG_PROF_TRSM      -- panel triangular solve; flops = m b^2
 *   MG_PROF_SOLVE     -- potrs steps; flops = 2 n^2 nrhs in total
 *   MG_PROF_ADJOINT   -- gradient product of mg_posv_backward; flops = 4 n^2 nrhs
 *   MG_PROF_BATCHED   -- one batched replay; flops = nominal posv flops summed
 *                        over the systems
 *   MG_PROF_TRAILING_NARROW -- trailing updates of rank 64 or 128 (inside a
 *                        two-level block column, and the rank-64/128 block
 *                        sizes); flops as MG_PROF_TRAILING
 *   MG_PROF_LU_PANEL  -- mg_getrf's pivoted panel factorisation (m x 64);
 *                        flops = m b^2 - b^3/3
 *   MG_PROF_LU_UPDATE -- mg_getrf's trailing update A22 -= L21 U12 (m x m,
 *                        rank 256); flops = 2 * 256 * m^2 (its rank-64
 *                        updates inside a 256-wide block column count as
 *                        MG_PROF_TRAILING_NARROW)
 * mg_profile_query synchronises on the last recorded event, returns the
 * summed event time (ms), the number of launches and the summed flops and
 * algorithmic bytes, and resets the counter when reset != 0.
 * mg_set_profiling switches every kind on (enable != 0) or off;
 * mg_set_profiling_kinds selects kinds by bit mask (bit k = kind k), so that
 * a timed run can bracket one kernel kind without adding events to the
 * latency-bound look-ahead chain.
 */
#define MG_PROF_TRAILING 0
#define MG_PROF_DIAG 1
#define MG_PROF_TRSM 2
#define MG_PROF_SOLVE 3
#define MG_PROF_ADJOINT 4
#define MG_PROF_BATCHED 5
#define MG_PROF_TRAILING_NARROW 6
#define MG_PROF_LU_PANEL 7
#define MG_PROF_LU_UPDATE 8
#define MG_PROF_KINDS 9
/* Errors: -1 NULL handle. */
mg_status mg_set_profiling(mg_handle_t handle, int32_t enable);
/* Errors: -1 NULL handle, -2 a bit at or above MG_PROF_KINDS. */
mg_status mg_set_profiling_kinds(mg_handle_t handle, uint32_t kinds);
/* Errors: -1 NULL handle, -2 bad kind, -3..-6 NULL outputs. */
mg_status mg_profile_query(mg_handle_t handle, int32_t kind, double *total_ms, int64_t *launches,
                           double *flops, double *bytes, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* MG_H_ */
