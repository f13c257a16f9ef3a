// potrs.hip -- X = A^{-1} B from the Cholesky factor: L Y = B, then L^T X = Y.
// Paper: JAXMg "Software design", potrs bullet (b is N x N_RHS).
//
// Each triangular sweep is ONE launch of a persistent kernel over blocks of
// JB = 64 rows.  A workgroup takes the next block from an atomic ticket (the
// forward sweep hands out blocks top-down, the backward sweep bottom-up), so a
// block only ever waits for blocks whose workgroups are already running, and
// blocks complete strictly in ticket order: block t can finish only after
// block t - 1.  One counter per sweep therefore says how many blocks are
// final; a workgroup polls it with acquire loads and publishes its own block
// with a release store.  Inside a workgroup:
//   * the four waves split the finished blocks j (j = w, w + 4, ...), each
//     streaming its rows of L straight from memory (one lane per row of the
//     block: L(i, j) for the forward sweep, read down a column of L for the
//     backward sweep, where L(j, i) is the transposed block) and applying
//     acc -= L_ij X_j with the block's solution broadcast by the scalar unit;
//   * the four partial sums are added in a fixed order through LDS;
//   * wave 0 solves the diagonal block by substitution in registers (a lane per
//     row, each step's pivot row broadcast by readlane), with L_ii staged in
//     LDS pre-scaled by its pivots (column c divided by L_cc for the forward
//     sweep, row c for the backward one, diagonal 0) so a step is one FMA per
//     value and the division by the pivot happens once at the end (integer
//     data with power-of-two pivots stays exact).
// Every wait is bounded: a counter that does not advance within the spin
// limit sets an error word in the workspace and the kernel drains.  Each sweep
// reads the lower triangle once (HBM-bound, nrhs/4 flop per byte in FP64); the
// chain of block solves is the latency floor.
#include <algorithm>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

constexpr int JB = 64;       // rows per block
constexpr int LDP = JB + 1;  // LDS leading dimension (bank spread)
constexpr int SWEEP_SPIN_LIMIT = 1 << 22;

// Per-sweep synchronisation words, kept in the workspace after Y.
struct SweepSync {
    int done;    // blocks final so far (in ticket order)
    int ticket;  // next block to hand out
    int err;     // set when a bounded wait gives up
    int pad;
};

static size_t y_bytes(int64_t n, int64_t nrhs, int es) { return align_up((size_t)n * (size_t)nrhs * es, 256); }

size_t potrs_work_bytes(int64_t n, int64_t nrhs, int es) {
    return (n == 0 || nrhs == 0) ? 0 : y_bytes(n, nrhs, es) + 256;
}

__global__ void k_sweep_init(SweepSync* s) {
    if (threadIdx.x < 2) s[threadIdx.x] = SweepSync{0, 0, 0, 0};
}

// L_jj (jb x jb lower, identity-padded to 64 x 64) into Ls[r*LDP + c] scaled
// by its pivots: by column (Ls(r,c) = L(r,c)/L(c,c)) when by_row is false,
// by row (Ls(r,c) = L(r,c)/L(r,r)) when it is true; the diagonal of Ls is 0
// and piv holds L(c,c).  All 256 threads take part.
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

// Cross-workgroup traffic of the sweeps (the counter and the solution blocks)
// uses device-coherent loads and stores, which bypass the per-XCD caches, so
// no cache invalidation or write-back fence is needed: a block's values are
// stored coherently, the storing wave waits for those stores to complete,
// and only then is the counter advanced.  A reader issues its loads of a
// block only after it has seen the counter pass that block.
__device__ __forceinline__ int load_coherent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T load_coherent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_coherent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Forward (FWD): Out = L^{-1} In.  Backward: Out = L^{-T} In.  In and Out are
// n x nrhs column-major; 16 RT right-hand sides per pass.
template <typename T, int RT, bool FWD>
__global__ __launch_bounds__(256) void k_sweep(const T* __restrict__ L, int64_t lda, int64_t n, int64_t nrhs,
                                               const T* __restrict__ In, int64_t ldi, T* Out, int64_t ldo,
                                               SweepSync* sy, const int32_t* info) {
    constexpr int NR = 16 * RT, XP = NR + 1, QW = NR / 4;
    __shared__ T Ls[JB * LDP];
    __shared__ T piv[JB];
    __shared__ T Xs[2][JB * XP];
    __shared__ T part[JB * XP];
    __shared__ int s_t;
    if (info && *info != 0) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
    if (tid == 0) s_t = atomicAdd(&sy->ticket, 1);
    __syncthreads();
    const int t = s_t;
    const int nblk = (int)((n + JB - 1) / JB);
    if (t >= nblk) return;
    const int bi = FWD ? t : nblk - 1 - t;
    const int64_t r0 = (int64_t)bi * JB;
    const int jb = (int)(n - r0 < JB ? n - r0 : JB);
    stage_diag<T, !FWD>(Ls, piv, L, lda, r0, jb);
    // MFMA phase: wave w owns rows 16 w .. 16 w + 15 of the block
    const int64_t rwc = (16 * w + i < jb) ? r0 + 16 * w + i : r0;  // clamped for loads
    // blocks this one depends on: j < bi (forward) or j > bi (backward); the
    // d-th of them in completion order is final once done > d
    const int ndep = FWD ? bi : nblk - 1 - bi;
    int ready = 0;
    bool abort = false;
    for (int64_t rc0 = 0; rc0 < nrhs; rc0 += NR) {
        V4<T> acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = V4<T>{0, 0, 0, 0};
        for (int d = 0; d < ndep; ++d) {
            if (ready <= d && !abort) {
                int spins = 0;
                while ((ready = load_coherent(&sy->done)) <= d) {
                    if (++spins > SWEEP_SPIN_LIMIT || load_coherent(&sy->err)) {
                        abort = true;
                        if (lane == 0) atomicExch(&sy->err, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            const int j = FWD ? d : nblk - 1 - d;
            const int64_t c0 = (int64_t)j * JB;
            const int jbj = (int)(n - c0 < JB ? n - c0 : JB);
            // the finished block X_j (jbj x NR) into LDS; consecutive threads
            // walk its rows, the contiguous direction
            T* xs = Xs[d & 1];
            for (int e = tid; e < JB * NR; e += 256) {
                const int c = e & (JB - 1), q = e >> 6;
                xs[c * XP + q] = (c < jbj && rc0 + q < nrhs) ? load_coherent(&Out[idx(c0 + c, rc0 + q, ldo)]) : (T)0;
            }
            __syncthreads();
            // acc += L_ij X_j (forward) or L_ji^T X_j (backward), 16 k-steps
#pragma unroll 4
            for (int ks = 0; ks < JB / 4; ++ks) {
                const int c = 4 * ks + g;
                const T x = (c < jbj) ? (FWD ? L[idx(rwc, c0 + c, lda)] : L[idx(c0 + c, rwc, lda)]) : (T)0;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) acc[rt] = mma_xzt(acc[rt], x, xs[c * XP + 16 * rt + i]);
            }
        }
        // partial products to LDS, one row per entry: lane (i, g) holds rows
        // 16 w + i, right-hand sides 16 rt + tcol(g, r)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[(16 * w + i) * XP + 16 * rt + tcol<T>(g, r)] = acc[rt][r];
        __syncthreads();
        // diagonal block by substitution: a lane per row, wave w takes the
        // right-hand sides q = w + 4 u
        {
            const T pl = piv[lane];
            T v[QW];
#pragma unroll
            for (int u = 0; u < QW; ++u) {
                const int q = w + 4 * u;
                v[u] = (lane < jb && rc0 + q < nrhs) ? In[idx(r0 + lane, rc0 + q, ldi)] - part[lane * XP + q] : (T)0;
            }
            if (FWD) {
#pragma unroll 8
                for (int c = 0; c < JB; ++c) {
                    const T lic = Ls[lane * LDP + c];  // L(lane,c)/L(c,c), 0 unless lane > c
#pragma unroll
                    for (int u = 0; u < QW; ++u) v[u] = v[u] - lic * readlane(v[u], c);
                }
            } else {
#pragma unroll 8
                for (int c = JB - 1; c >= 0; --c) {
                    const T lci = Ls[c * LDP + lane];  // L(c,lane)/L(c,c), 0 unless lane < c
#pragma unroll
                    for (int u = 0; u < QW; ++u) v[u] = v[u] - lci * readlane(v[u], c);
                }
            }
#pragma unroll
            for (int u = 0; u < QW; ++u) {
                const int q = w + 4 * u;
                if (lane < jb && rc0 + q < nrhs) store_coherent(&Out[idx(r0 + lane, rc0 + q, ldo)], v[u] / pl);
            }
        }
        __syncthreads();  // part is reused by the next pass
    }
    // every wave's coherent stores complete before the block is published
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) store_coherent(&sy->done, t + 1);
}

template <typename T, int RT>
static mg_status sweep(hipStream_t st, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B, int64_t ldb, T* Y,
                       SweepSync* sy, const int32_t* info) {
    const unsigned nblk = (unsigned)cdiv(n, JB);
    hipLaunchKernelGGL(k_sweep_init, dim3(1), dim3(64), 0, st, sy);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sweep<T, RT, true>), dim3(nblk), dim3(256), 0, st, L, lda, n, nrhs, (const T*)B, ldb, Y,
                       n, sy, info);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sweep<T, RT, false>), dim3(nblk), dim3(256), 0, st, L, lda, n, nrhs, (const T*)Y, n, B,
                       ldb, sy + 1, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

template <typename T>
mg_status potrs_impl(mg_handle_t h, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B, int64_t ldb, T* Y,
                     const int32_t* info) {
    if (n == 0 || nrhs == 0) return MG_OK;
    hipStream_t st = h->stream;
    mg_status rc;
    if ((rc = prof_begin(h, MG_PROF_SOLVE, st))) return rc;
    SweepSync* sy = (SweepSync*)((char*)Y + y_bytes(n, nrhs, (int)sizeof(T)));
    if (nrhs <= 16) rc = sweep<T, 1>(st, n, nrhs, L, lda, B, ldb, Y, sy, info);
    else if (nrhs <= 32) rc = sweep<T, 2>(st, n, nrhs, L, lda, B, ldb, Y, sy, info);
    else rc = sweep<T, 4>(st, n, nrhs, L, lda, B, ldb, Y, sy, info);
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
