// mg_internal.h -- host-side internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <vector>
#include <cstring>

#include "mg.h"

struct mg_prof_counter {
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
    double flops = 0.0;
    double bytes = 0.0;
};

struct mg_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    int cu_count = 256;
    int64_t nb = 0;          // potrf block size (the paper's tile size T_A); 0 = default
    int lookahead = 1;       // 0 serial; 1 look-ahead; 2 look-ahead with one CU per XCD kept for the panel
    int side_mode = 0;       // look-ahead mode the bulk stream was created for
    int trail_lo = 1;        // FP32 trailing update: 1 plain, 2 operands rounded to bfloat16
    int spin_limit = -1;     // potrs sweeps: polls before a wait gives up (-1: the built-in limit)
    int solve_mode = MG_SOLVE_INVERSE;  // potrs sweeps: diagonal blocks by inverse (MFMA) or substitution
    void* bf16_panel = nullptr;  // bfloat16 mode: three n x 512 row-major panel buffers
    uint32_t profiling = 0;  // bit k set: launches of kind k are bracketed by events
    mg_prof_counter prof[MG_PROF_KINDS];
    void* scratch = nullptr;  // device address of the no-allocation scratch array on this device
    // second stream and events for the look-ahead schedule (created by mg_create)
    hipStream_t side = nullptr;   // look-ahead: bulk trailing update
    hipStream_t chain = nullptr;  // look-ahead: next block column and panel chain
    hipEvent_t ev_fork = nullptr, ev_panel = nullptr, ev_rest = nullptr, ev_join = nullptr;
};

namespace mg {

#define MG_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return MG_ERR_HIP;       \
    } while (0)

#define MG_LAUNCH_CHECK() MG_HIP(hipGetLastError())

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Profiling: bracket one launch with an event pair when enabled.
mg_status prof_begin(mg_handle_t h, int kind, hipStream_t st);
mg_status prof_end(mg_handle_t h, int kind, double flops, double bytes, hipStream_t st);

// D = S^T, n x n FP64, 64 x 64 tiles through LDS; skipped when *info != 0.
mg_status transpose_f64(hipStream_t st, const double* S, int64_t lds, double* D, int64_t ldd, int64_t n,
                        const int32_t* info);
// C -= X Z on the FP64 matrix pipe (the general update kernel of the LU).
mg_status gemm_sub_f64(hipStream_t st, double* C, int64_t ldc, const double* X, int64_t ldx, const double* Z,
                       int64_t ldz, int64_t m, int64_t nn, int64_t kdim);
// Y L = C in place (C m x n, L lower n x n, n % 64 == 0) by 64-column blocks;
// Zw: right_solve_lower_work_bytes(n) of device scratch.
bool right_solve_lower_ok(int64_t m, int64_t n, int64_t lda, int64_t ldc);
size_t right_solve_lower_work_bytes(int64_t n);
mg_status right_solve_lower(hipStream_t st, int64_t m, int64_t n, const double* L, int64_t lda, double* C,
                            int64_t ldc, double* Zw);

// Block size used by potrf for order n and element size es.
int64_t potrf_block_size(mg_handle_t h, int64_t n, int es);

// Drivers (enqueue on h->stream, no host synchronisation).
template <typename T>
mg_status potrf_impl(mg_handle_t h, int64_t n, T* A, int64_t lda, int32_t* info);
template <typename T>
mg_status potrs_impl(mg_handle_t h, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B,
                     int64_t ldb, T* ywork, int32_t* info);
size_t potrs_work_bytes(int64_t n, int64_t nrhs, int es);
// Backward sweep alone: Out = L^{-T} In (In, Out distinct); words: sweep_words_bytes(nrhs) bytes.
size_t sweep_words_bytes(int64_t nrhs);
template <typename T>
mg_status trsm_lt_impl(mg_handle_t h, int64_t n, int64_t nrhs, const T* L, int64_t lda, const T* In, int64_t ldi,
                       T* Out, int64_t ldo, void* words, int32_t* info);
size_t mixed_work_bytes(int64_t n, int64_t nrhs, int fallback, int lo);
inline size_t bf16_panel_bytes(int64_t n) { return 3 * (size_t)n * 512 * 2; }
mg_status posv_backward_impl(mg_handle_t h, int64_t n, int64_t nrhs, const double* L, int64_t lda,
                             const double* X, int64_t ldx, const double* GX, int64_t ldgx, double* GB,
                             int64_t ldgb, double* GA, int64_t ldga, int mode, void* work, int32_t* info);
size_t potrf_backward_work_bytes(int64_t n);
mg_status potrf_backward_impl(mg_handle_t h, int64_t n, const double* L, int64_t lda, const double* GL,
                              int64_t ldgl, double* GA, int64_t ldga, int mode, void* work, int32_t* info);
mg_status posv_mixed_impl(mg_handle_t h, int lo, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                          const double* B, int64_t ldb, double* X, int64_t ldx, const mg_ir_opts* o, void* work,
                          mg_ir_result* res, int32_t* info);

// General solve (LU with partial pivoting), FP64.
size_t getrf_work_bytes(int64_t n);
mg_status getrf_impl(mg_handle_t h, int64_t n, double* A, int64_t lda, int32_t* ipiv, void* work, int32_t* info);
size_t getrs_work_bytes(int64_t n, int64_t nrhs);
mg_status getrs_impl(mg_handle_t h, int64_t n, int64_t nrhs, const double* LU, int64_t lda, const int32_t* ipiv,
                     double* B, int64_t ldb, void* work, int32_t* info);
// The two sweeps of an LU solve (forward with the unit lower factor, B's rows
// read through rperm; backward with the upper factor); words: 2 x
// sweep_words_bytes(nrhs) bytes.
mg_status lu_sweeps(mg_handle_t h, int64_t n, int64_t nrhs, const double* LU, int64_t lda, const int32_t* rperm,
                    double* B, int64_t ldb, double* Y, void* words, int32_t* info);

// Complex Hermitian solve through the real 2n x 2n blocked form (op 0 factor,
// 1 solve with a given factor, 2 both); work: zposv_work_bytes.
size_t zposv_work_bytes(int64_t n, int64_t nrhs, int es);
template <typename T>
mg_status zposv_impl(mg_handle_t h, int op, int64_t n, int64_t nrhs, T* A, int64_t lda, T* B, int64_t ldb, void* work,
                     int32_t* info);

mg_status set_info_zero(hipStream_t s, int32_t* info);
// Create (or re-create after a mode change) the look-ahead streams and events.
mg_status ensure_streams(mg_handle_t h);

}  // namespace mg
