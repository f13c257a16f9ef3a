// api.hip -- C ABI entry points: argument validation, handle, profiling,
// posv and logdet.  Every check runs on the host before anything is enqueued.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "mg_internal.h"
#include "tile16.h"

using namespace mg;

namespace mg {

mg_status prof_begin(mg_handle_t h, int kind, hipStream_t st) {
    if (!((h->profiling >> kind) & 1u)) return MG_OK;
    mg_prof_counter& pc = h->prof[kind];
    if (pc.used == pc.start.size()) {
        hipEvent_t a, b;
        MG_HIP(hipEventCreate(&a));
        MG_HIP(hipEventCreate(&b));
        pc.start.push_back(a);
        pc.stop.push_back(b);
    }
    MG_HIP(hipEventRecord(pc.start[pc.used], st));
    return MG_OK;
}

mg_status prof_end(mg_handle_t h, int kind, double flops, double bytes, hipStream_t st) {
    if (!((h->profiling >> kind) & 1u)) return MG_OK;
    mg_prof_counter& pc = h->prof[kind];
    MG_HIP(hipEventRecord(pc.stop[pc.used], st));
    ++pc.used;
    pc.flops += flops;
    pc.bytes += bytes;
    return MG_OK;
}

// log det = 2 sum_j log L_jj, one workgroup, fixed-order tree reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_logdet(const T* L, int64_t lda, int64_t n, double* out,
                                                const int32_t* info) {
    __shared__ double part[256];
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s += log((double)L[idx(j, j, lda)]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (info && *info != 0) ? (double)NAN : 2.0 * part[0];
}

// Scratch of mg_posv_noalloc: Y = L^{-1} B and the sweep words live in this
// file-scope device array (one copy per GPU, created with the code object)
// instead of a caller workspace.  In host code `scratch` names a host-side
// stand-in; its device address on each GPU comes from hipGetSymbolAddress,
// looked up once per device (mg_create) and kept in scratch_addr.
static __device__ __align__(256) unsigned char scratch[MG_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mu;
static void* scratch_addr[MAX_DEVICES];

// Device address of `scratch` on the current device (h->device), looked up on
// the first handle created there.
static mg_status scratch_setup(mg_handle_t h) {
    if (h->device < 0 || h->device >= MAX_DEVICES) return MG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_addr[h->device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MG_ERR_HIP;
        scratch_addr[h->device] = p;
    }
    h->scratch = scratch_addr[h->device];
    return MG_OK;
}

}  // namespace mg

static inline int es_of(mg_dtype dt) { return dt == MG_F64 ? 8 : 4; }
static inline bool dtype_ok(mg_dtype dt) { return dt == MG_F64 || dt == MG_F32; }

extern "C" {

int32_t mg_version(void) { return 10000; }

mg_status mg_create(mg_handle_t* handle, void* stream) {
    if (!handle) return -1;
    *handle = nullptr;
    mg_handle_s* h = new mg_handle_s();
    h->stream = (hipStream_t)stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return MG_ERR_HIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
        h->cu_count = cus;
    mg_status rc = scratch_setup(h);
    if (rc == MG_OK) rc = ensure_streams(h);
    if (rc != MG_OK) {
        mg_destroy(h);
        return rc;
    }
    *handle = h;
    return MG_OK;
}

mg_status mg_destroy(mg_handle_t h) {
    if (!h) return MG_OK;
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
    if (h->ev_rest) (void)hipEventDestroy(h->ev_rest);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->chain) (void)hipStreamDestroy(h->chain);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    for (int k = 0; k < MG_PROF_KINDS; ++k) {
        for (hipEvent_t e : h->prof[k].start) (void)hipEventDestroy(e);
        for (hipEvent_t e : h->prof[k].stop) (void)hipEventDestroy(e);
    }
    delete h;
    return MG_OK;
}

mg_status mg_set_stream(mg_handle_t h, void* stream) {
    if (!h) return -1;
    h->stream = (hipStream_t)stream;
    return MG_OK;
}

mg_status mg_set_block_size(mg_handle_t h, int64_t nb) {
    if (!h) return -1;
    if (!(nb == 0 || nb == 64 || nb == 128 || (nb % 256 == 0 && nb >= 256 && nb <= 1024))) return -2;
    h->nb = nb;
    return MG_OK;
}

mg_status mg_set_sweep_spin_limit(mg_handle_t h, int64_t limit) {
    if (!h) return -1;
    if (limit < -1 || limit > ((int64_t)1 << 30)) return -2;
    h->spin_limit = (int)limit;
    return MG_OK;
}

mg_status mg_set_solve_mode(mg_handle_t h, mg_solve_mode mode) {
    if (!h) return -1;
    if (mode != MG_SOLVE_INVERSE && mode != MG_SOLVE_SUBSTITUTION) return -2;
    h->solve_mode = (int)mode;
    return MG_OK;
}

mg_status mg_set_lookahead(mg_handle_t h, int32_t enable) {
    if (!h) return -1;
    if (enable < 0 || enable > 2) return -2;
    h->lookahead = enable;
    return MG_OK;
}

mg_status mg_get_block_size(mg_handle_t h, mg_dtype dt, int64_t n, int64_t* nb) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (!nb) return -4;
    *nb = potrf_block_size(h, n, es_of(dt));
    return MG_OK;
}

mg_status mg_potrf(mg_handle_t h, mg_dtype dt, int64_t n, void* A, int64_t lda, int32_t* info) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (!A && n > 0) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (!info) return -6;
    return dt == MG_F64 ? potrf_impl<double>(h, n, (double*)A, lda, info)
                        : potrf_impl<float>(h, n, (float*)A, lda, info);
}

mg_status mg_potrs_buffer_size(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, size_t* bytes) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (!bytes) return -5;
    *bytes = potrs_work_bytes(n, nrhs, es_of(dt));
    return MG_OK;
}

static mg_status check_solve_args(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, const void* A,
                                  int64_t lda, const void* B, int64_t ldb, const void* work, size_t work_bytes) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (!A && n > 0) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    const size_t need = potrs_work_bytes(n, nrhs, es_of(dt));
    if (need > 0 && !work) return -9;
    if (work_bytes < need) return -10;
    return MG_OK;
}

mg_status mg_potrs(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, const void* L, int64_t lda, void* B,
                   int64_t ldb, void* work, size_t work_bytes, int32_t* info) {
    mg_status rc = check_solve_args(h, dt, n, nrhs, L, lda, B, ldb, work, work_bytes);
    if (rc) return rc;
    return dt == MG_F64
               ? potrs_impl<double>(h, n, nrhs, (const double*)L, lda, (double*)B, ldb, (double*)work, info)
               : potrs_impl<float>(h, n, nrhs, (const float*)L, lda, (float*)B, ldb, (float*)work, info);
}

mg_status mg_posv(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, void* A, int64_t lda, void* B,
                  int64_t ldb, void* work, size_t work_bytes, int32_t* info) {
    mg_status rc = check_solve_args(h, dt, n, nrhs, A, lda, B, ldb, work, work_bytes);
    if (rc) return rc;
    if (!info) return -11;
    if (dt == MG_F64) {
        if ((rc = potrf_impl<double>(h, n, (double*)A, lda, info))) return rc;
        return potrs_impl<double>(h, n, nrhs, (const double*)A, lda, (double*)B, ldb, (double*)work, info);
    }
    if ((rc = potrf_impl<float>(h, n, (float*)A, lda, info))) return rc;
    return potrs_impl<float>(h, n, nrhs, (const float*)A, lda, (float*)B, ldb, (float*)work, info);
}

mg_status mg_posv_noalloc(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, void* A, int64_t lda, void* B,
                          int64_t ldb, int32_t* info) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (!A && n > 0) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    if (!info) return -9;
    if (potrs_work_bytes(n, nrhs, es_of(dt)) > MG_NOALLOC_SCRATCH_BYTES) return MG_ERR_SCRATCH_LIMIT;
    if (!h->scratch) return MG_ERR_INTERNAL;
    mg_status rc;
    if (dt == MG_F64) {
        if ((rc = potrf_impl<double>(h, n, (double*)A, lda, info))) return rc;
        return potrs_impl<double>(h, n, nrhs, (const double*)A, lda, (double*)B, ldb, (double*)h->scratch, info);
    }
    if ((rc = potrf_impl<float>(h, n, (float*)A, lda, info))) return rc;
    return potrs_impl<float>(h, n, nrhs, (const float*)A, lda, (float*)B, ldb, (float*)h->scratch, info);
}

mg_status mg_posv_mixed_buffer_size(mg_handle_t h, mg_prec lo, int64_t n, int64_t nrhs, int32_t fallback,
                                    size_t* bytes) {
    if (!h) return -1;
    if (lo != MG_PREC_F32 && lo != MG_PREC_BF16) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (!bytes) return -5;
    *bytes = mixed_work_bytes(n, nrhs, fallback ? 1 : 0, lo);
    return MG_OK;
}

mg_status mg_posv_mixed(mg_handle_t h, mg_prec lo, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double* X, int64_t ldx, const mg_ir_opts* opts, void* work,
                        size_t work_bytes, mg_ir_result* result, int32_t* info) {
    if (!h) return -1;
    if (lo != MG_PREC_F32 && lo != MG_PREC_BF16) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    const bool any = n > 0 && nrhs > 0;
    if (!A && n > 0) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (!B && any) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    if (!X && any) return -9;
    if (ldx < std::max<int64_t>(1, n)) return -10;
    mg_ir_opts o{1e-12, 30, 1};
    if (opts) {
        if (!(opts->tol >= 0.0) || opts->max_iter < 0) return -11;
        o = *opts;
    }
    const size_t need = mixed_work_bytes(n, nrhs, o.fallback ? 1 : 0, lo);
    if (!work && any) return -12;
    if (any && work_bytes < need) return -13;
    if (!result) return -14;
    if (!info) return -15;
    return posv_mixed_impl(h, (int)lo, n, nrhs, A, lda, B, ldb, X, ldx, &o, work, result, info);
}

mg_status mg_posv_backward(mg_handle_t h, int64_t n, int64_t nrhs, const double* L, int64_t lda, const double* X,
                           int64_t ldx, const double* gX, int64_t ldgx, double* gB, int64_t ldgb, double* gA,
                           int64_t ldga, mg_grad_mode mode, void* work, size_t work_bytes, int32_t* info) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    const int64_t ld1 = std::max<int64_t>(1, n);
    const bool any = n > 0 && nrhs > 0;
    if (!L && n > 0) return -4;
    if (lda < ld1) return -5;
    if (!X && any) return -6;
    if (ldx < ld1) return -7;
    if (!gX && any) return -8;
    if (ldgx < ld1) return -9;
    if (!gB && any) return -10;
    if (ldgb < ld1) return -11;
    if (!gA && n > 0) return -12;
    if (ldga < ld1) return -13;
    if (mode != MG_GRAD_SYM && mode != MG_GRAD_LOWER) return -14;
    const size_t need = potrs_work_bytes(n, nrhs, 8);
    if (need > 0 && !work) return -15;
    if (work_bytes < need) return -16;
    return posv_backward_impl(h, n, nrhs, L, lda, X, ldx, gX, ldgx, gB, ldgb, gA, ldga, (int)mode, work, info);
}

mg_status mg_potrf_backward_buffer_size(mg_handle_t h, int64_t n, size_t* bytes) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (!bytes) return -3;
    *bytes = potrf_backward_work_bytes(n);
    return MG_OK;
}

mg_status mg_potrf_backward(mg_handle_t h, int64_t n, const double* L, int64_t lda, const double* GL, int64_t ldgl,
                            double* GA, int64_t ldga, mg_grad_mode mode, void* work, size_t work_bytes,
                            int32_t* info) {
    if (!h) return -1;
    if (n < 0) return -2;
    const int64_t ld1 = std::max<int64_t>(1, n);
    if (!L && n > 0) return -3;
    if (lda < ld1) return -4;
    if (!GL && n > 0) return -5;
    if (ldgl < ld1) return -6;
    if (!GA && n > 0) return -7;
    if (ldga < ld1) return -8;
    if (mode != MG_GRAD_SYM && mode != MG_GRAD_LOWER) return -9;
    const size_t need = potrf_backward_work_bytes(n);
    if (need > 0 && !work) return -10;
    if (work_bytes < need) return -11;
    return potrf_backward_impl(h, n, L, lda, GL, ldgl, GA, ldga, (int)mode, work, info);
}

// ------------------------------------------------------- complex Hermitian

mg_status mg_zposv_buffer_size(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, size_t* bytes) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (!bytes) return -5;
    *bytes = zposv_work_bytes(n, nrhs, es_of(dt));
    return MG_OK;
}

static mg_status z_call(mg_handle_t h, mg_dtype dt, int op, int64_t n, int64_t nrhs, void* A, int64_t lda, void* B,
                        int64_t ldb, void* work, size_t work_bytes, int32_t* info) {
    if (dt == MG_F64)
        return zposv_impl<double>(h, op, n, nrhs, (double*)A, lda, (double*)B, ldb, work, info);
    return zposv_impl<float>(h, op, n, nrhs, (float*)A, lda, (float*)B, ldb, work, info);
}

mg_status mg_zpotrf(mg_handle_t h, mg_dtype dt, int64_t n, void* A, int64_t lda, void* work, size_t work_bytes,
                    int32_t* info) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (!A && n > 0) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    const size_t need = zposv_work_bytes(n, 0, es_of(dt));
    if (need > 0 && !work) return -6;
    if (work_bytes < need) return -7;
    if (!info) return -8;
    return z_call(h, dt, 0, n, 0, A, lda, nullptr, 1, work, work_bytes, info);
}

mg_status mg_zpotrs(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, const void* L, int64_t lda, void* B,
                    int64_t ldb, void* work, size_t work_bytes, int32_t* info) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (!L && n > 0) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    const size_t need = zposv_work_bytes(n, nrhs, es_of(dt));
    if (need > 0 && !work) return -9;
    if (work_bytes < need) return -10;
    if (n == 0 || nrhs == 0) return MG_OK;
    return z_call(h, dt, 1, n, nrhs, const_cast<void*>(L), lda, B, ldb, work, work_bytes, info);
}

mg_status mg_zposv(mg_handle_t h, mg_dtype dt, int64_t n, int64_t nrhs, void* A, int64_t lda, void* B, int64_t ldb,
                   void* work, size_t work_bytes, int32_t* info) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (nrhs < 0) return -4;
    if (!A && n > 0) return -5;
    if (lda < std::max<int64_t>(1, n)) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    const size_t need = zposv_work_bytes(n, nrhs, es_of(dt));
    if (need > 0 && !work) return -9;
    if (work_bytes < need) return -10;
    if (!info) return -11;
    return z_call(h, dt, 2, n, nrhs, A, lda, B, ldb, work, work_bytes, info);
}

// ------------------------------------------------------------ general solve

mg_status mg_getrf_buffer_size(mg_handle_t h, int64_t n, size_t* bytes) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (!bytes) return -3;
    *bytes = getrf_work_bytes(n);
    return MG_OK;
}

mg_status mg_getrf(mg_handle_t h, int64_t n, double* A, int64_t lda, int32_t* ipiv, void* work, size_t work_bytes,
                   int32_t* info) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (!A && n > 0) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (!ipiv && n > 0) return -5;
    const size_t need = getrf_work_bytes(n);
    if (need > 0 && !work) return -6;
    if (work_bytes < need) return -7;
    if (!info) return -8;
    return getrf_impl(h, n, A, lda, ipiv, work, info);
}

mg_status mg_getrs_buffer_size(mg_handle_t h, int64_t n, int64_t nrhs, size_t* bytes) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (!bytes) return -4;
    *bytes = getrs_work_bytes(n, nrhs);
    return MG_OK;
}

mg_status mg_getrs(mg_handle_t h, int64_t n, int64_t nrhs, const double* LU, int64_t lda, const int32_t* ipiv,
                   double* B, int64_t ldb, void* work, size_t work_bytes, int32_t* info) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (!LU && n > 0) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (!ipiv && n > 0) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    const size_t need = getrs_work_bytes(n, nrhs);
    if (need > 0 && !work) return -9;
    if (work_bytes < need) return -10;
    if (n > INT32_MAX - 1) return MG_ERR_UNSUPPORTED;
    return getrs_impl(h, n, nrhs, LU, lda, ipiv, B, ldb, work, info);
}

mg_status mg_gesv_buffer_size(mg_handle_t h, int64_t n, int64_t nrhs, size_t* bytes) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (!bytes) return -4;
    *bytes = std::max(getrf_work_bytes(n), getrs_work_bytes(n, nrhs));
    return MG_OK;
}

mg_status mg_gesv(mg_handle_t h, int64_t n, int64_t nrhs, double* A, int64_t lda, int32_t* ipiv, double* B,
                  int64_t ldb, void* work, size_t work_bytes, int32_t* info) {
    if (!h) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (!A && n > 0) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (!ipiv && n > 0) return -6;
    if (!B && n > 0 && nrhs > 0) return -7;
    if (ldb < std::max<int64_t>(1, n)) return -8;
    const size_t need = std::max(getrf_work_bytes(n), getrs_work_bytes(n, nrhs));
    if (need > 0 && !work) return -9;
    if (work_bytes < need) return -10;
    if (!info) return -11;
    mg_status rc;
    if ((rc = getrf_impl(h, n, A, lda, ipiv, work, info))) return rc;
    return getrs_impl(h, n, nrhs, A, lda, ipiv, B, ldb, work, info);
}

mg_status mg_logdet(mg_handle_t h, mg_dtype dt, int64_t n, const void* L, int64_t lda, double* out,
                    const int32_t* info) {
    if (!h) return -1;
    if (!dtype_ok(dt)) return -2;
    if (n < 0) return -3;
    if (!L && n > 0) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (!out) return -6;
    if (dt == MG_F64)
        hipLaunchKernelGGL((k_logdet<double>), dim3(1), dim3(256), 0, h->stream, (const double*)L, lda, n, out, info);
    else
        hipLaunchKernelGGL((k_logdet<float>), dim3(1), dim3(256), 0, h->stream, (const float*)L, lda, n, out, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

mg_status mg_set_profiling(mg_handle_t h, int32_t enable) {
    if (!h) return -1;
    h->profiling = enable ? (1u << MG_PROF_KINDS) - 1u : 0u;
    return MG_OK;
}

mg_status mg_set_profiling_kinds(mg_handle_t h, uint32_t kinds) {
    if (!h) return -1;
    if (kinds >> MG_PROF_KINDS) return -2;
    h->profiling = kinds;
    return MG_OK;
}

mg_status mg_profile_query(mg_handle_t h, int32_t kind, double* total_ms, int64_t* launches, double* flops,
                           double* bytes, int32_t reset) {
    if (!h) return -1;
    if (kind < 0 || kind >= MG_PROF_KINDS) return -2;
    if (!total_ms) return -3;
    if (!launches) return -4;
    if (!flops) return -5;
    if (!bytes) return -6;
    mg_prof_counter& pc = h->prof[kind];
    double ms = 0.0;
    if (pc.used > 0) {
        for (size_t k = 0; k < pc.used; ++k) {
            float t = 0.f;
            MG_HIP(hipEventSynchronize(pc.stop[k]));  // launches may sit on either stream
            MG_HIP(hipEventElapsedTime(&t, pc.start[k], pc.stop[k]));
            ms += (double)t;
        }
    }
    *total_ms = ms;
    *launches = (int64_t)pc.used;
    *flops = pc.flops;
    *bytes = pc.bytes;
    if (reset) {
        pc.used = 0;
        pc.flops = 0.0;
        pc.bytes = 0.0;
    }
    return MG_OK;
}

}  // extern "C"
