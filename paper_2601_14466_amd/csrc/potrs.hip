// potrs.hip -- X = A^{-1} B from the Cholesky factor: L Y = B, then L^T X = Y.
// Paper: JAXMg "Software design", potrs bullet (b is N x N_RHS).
//
// Each triangular sweep is ONE launch of a persistent kernel over blocks of
// JB = 64 rows.  A workgroup takes the next block from an atomic ticket (the
// forward sweep hands out blocks top-down, the backward sweep bottom-up), so a
// block only ever waits for blocks whose workgroups are already running.
// Before a sweep its output array is filled with a signalling-NaN sentinel;
// a finished block simply stores its values (device-coherent stores), and a
// dependent block loads the values it needs (device-coherent loads) until
// none of them is the sentinel.  Arithmetic never produces a signalling NaN
// (IEEE operations quiet them), so a sentinel can only mean "not yet written",
// and the hand-over costs one store and one load, with no flag or fence.
// Inside a workgroup:
//   * each dependency block j is loaded into LDS once, then the four waves
//     (16 rows of the block each) apply acc += L_ij X_j with MFMAs (forward;
//     the backward sweep reads L down its columns for L_ji^T), L streamed
//     from memory;
//   * the diagonal block is then applied in one of two ways (a handle mode):
//     - inverse (default): when the workgroup starts, long before its last
//       dependency arrives, it forms Z = L_ii^{-1} in LDS (one lane per
//       column of Z); at the end v = b_i - sum goes through LDS and each
//       wave multiplies its 16 rows of Z (Z^T backward) by v on the matrix
//       pipe, so the chain after the last dependency is a few MFMAs;
//     - substitution: the products go through LDS to a row-per-lane layout
//       and wave w solves the right-hand sides w, w + 4, ... in registers
//       (each step's pivot row broadcast by readlane), with L_ii staged in LDS
//       pre-scaled by its pivots (column c divided by L_cc for the forward
//       sweep, row c for the backward one, diagonal 0) so a step is one FMA
//       per value and the division by the pivot happens once at the end
//       (integer data with power-of-two pivots stays exact).
// Every wait is bounded: a block that stays unwritten past the spin limit
// sets an error word in the workspace and the kernel drains; after the two
// sweeps a check kernel turns a set error word into a NaN-filled result and
// info = MG_INFO_SOLVE_ABORTED.  Each sweep reads the lower triangle once
// (HBM-bound, nrhs/4 flop per byte in FP64); the chain of block solves is
// the latency floor.
#include <algorithm>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

constexpr int JB = 64;       // rows per block
constexpr int LDP = JB + 1;  // LDS leading dimension (bank spread)
constexpr int SWEEP_SPIN_LIMIT = 1 << 22;  // default polls before a wait gives up

// Per-sweep words, kept in the workspace after Y.
struct SweepSync {
    int ticket;  // next block to hand out
    int err;     // set when a bounded wait gives up
    int pad[2];
};

static size_t y_bytes(int64_t n, int64_t nrhs, int es) { return align_up((size_t)n * (size_t)nrhs * es, 256); }

// right-hand sides are handled in passes of 16, all passes of a sweep in one
// launch (grid y), each with its own sweep words
constexpr int SW_NR = 16;
__host__ __device__ inline int64_t sweep_passes(int64_t nrhs) { return (nrhs + SW_NR - 1) / SW_NR; }

size_t potrs_work_bytes(int64_t n, int64_t nrhs, int es) {
    return (n == 0 || nrhs == 0) ? 0 : y_bytes(n, nrhs, es) + align_up(2 * sweep_passes(nrhs) * 16, 256);
}

// Signalling NaNs (quiet bit clear, non-zero payload): never produced by
// arithmetic, so they mark entries that have not been written yet.
__device__ __forceinline__ double sentinel(double*) { return __builtin_bit_cast(double, 0x7ff4d1e5a1f00d01ull); }
__device__ __forceinline__ float sentinel(float*) { return __builtin_bit_cast(float, 0x7fa1d1e5u); }
__device__ __forceinline__ bool is_sentinel(double v) {
    return __builtin_bit_cast(unsigned long long, v) == 0x7ff4d1e5a1f00d01ull;
}
__device__ __forceinline__ bool is_sentinel(float v) { return __builtin_bit_cast(unsigned, v) == 0x7fa1d1e5u; }

// Fill the sweep's output (n x nrhs, leading dimension ld) with the sentinel
// and reset its words.  Skipped when a preceding factorisation failed, so B
// is left as it was.
template <typename T>
__global__ __launch_bounds__(256) void k_sweep_init(T* Out, int64_t ld, int64_t n, int64_t nrhs, SweepSync* sy,
                                                    const int32_t* info) {
    if (info && *info != 0) return;
    if (blockIdx.x == 0)
        for (int64_t k = threadIdx.x; k < sweep_passes(nrhs); k += blockDim.x) sy[k] = SweepSync{0, 0, {0, 0}};
    const int64_t tot = n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256)
        Out[idx(e % n, e / n, ld)] = sentinel((T*)nullptr);
}

// The lower-triangular operator a sweep applies, entry (r, c) with r >= c:
// KIND 0, the Cholesky factor L (the lower triangle of the array); KIND 1,
// the unit lower factor of an LU factorisation (strict lower triangle of the
// array, 1 on the diagonal); KIND 2, U^T for the upper factor U of an LU
// factorisation (the upper triangle of the array read transposed), so that
// the backward sweep, which applies the operator's transpose, solves U x = y.
template <typename T, int KIND>
__device__ __forceinline__ T lop(const T* L, int64_t lda, int64_t r, int64_t c) {
    if constexpr (KIND == 2) return L[idx(c, r, lda)];
    if constexpr (KIND == 1)
        if (r == c) return (T)1;
    return L[idx(r, c, lda)];
}

// L_jj (jb x jb lower, identity-padded to 64 x 64) into Ls[r*LDP + c] scaled
// by its pivots: by column (Ls(r,c) = L(r,c)/L(c,c)) when by_row is false,
// by row (Ls(r,c) = L(r,c)/L(r,r)) when it is true; the diagonal of Ls is 0
// and piv holds L(c,c).  All 256 threads take part.
template <typename T, bool by_row, int KIND>
__device__ __forceinline__ void stage_diag(T* Ls, T* piv, const T* L, int64_t lda, int64_t j0, int jb) {
    const int tid = threadIdx.x;
    T v[JB * JB / 256];
#pragma unroll
    for (int q = 0; q < JB * JB / 256; ++q) {
        const int e = tid + 256 * q;
        const int rr = e & (JB - 1), cc = e >> 6;
        v[q] = (rr < jb && cc < jb && rr >= cc) ? lop<T, KIND>(L, lda, j0 + rr, j0 + cc) : (T)(rr == cc ? 1 : 0);
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

// Z = L_jj^{-1} (jb x jb lower, identity-padded to 64 x 64) into
// Ls[r*LDP + c] = Z(r, c).  L_jj is first staged column-major in the same
// buffer (Ls[c*LDP + r] = L(r, c) on and below the diagonal) with the
// reciprocals of its pivots in rpiv; wave 0 then forms Z a column per lane by
// right-looking substitution on the unit columns (z_c *= 1/L(c,c), then
// z_r -= L(r,c) z_c for r > c), z in registers and L read as LDS broadcasts
// (the same entry for every lane).  The wave reads all of Ls before it writes
// Z over it (LDS operations of one wave complete in program order).  All 256
// threads take part in the staging.
template <typename T, int KIND>
__device__ __forceinline__ void stage_inverse(T* Ls, T* rpiv, const T* L, int64_t lda, int64_t j0, int jb) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < JB * JB / 256; ++q) {
        const int e = tid + 256 * q;
        const int rr = e & (JB - 1), cc = e >> 6;
        const T v = (rr < jb && cc < jb && rr >= cc) ? lop<T, KIND>(L, lda, j0 + rr, j0 + cc) : (T)(rr == cc ? 1 : 0);
        Ls[cc * LDP + rr] = v;
        if (rr == cc) rpiv[rr] = (T)1 / v;
    }
    __syncthreads();
    if (tid < JB) {
        T z[JB];
#pragma unroll
        for (int r = 0; r < JB; ++r) z[r] = (r == tid) ? (T)1 : (T)0;
#pragma unroll
        for (int c = 0; c < JB; ++c) {
            const T zc = z[c] * rpiv[c];
            z[c] = zc;
#pragma unroll
            for (int r = c + 1; r < JB; ++r) z[r] = z[r] - Ls[c * LDP + r] * zc;
        }
#pragma unroll
        for (int r = 0; r < JB; ++r) Ls[r * LDP + tid] = z[r];
    }
    __syncthreads();
}

// Cross-workgroup traffic of the sweeps (the solution blocks and the error
// word) uses device-coherent loads and stores, which bypass the per-XCD
// caches, so a value stored by one workgroup is seen by the others without
// cache invalidation or write-back fences.
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
// spin_limit: polls before a wait gives up (0: give up at the first
// dependency without waiting, which exercises the give-up path).
// INV: the diagonal block is applied as its inverse (formed when the
// workgroup starts, off the chain of dependencies) by MFMA products;
// otherwise by substitution.  KIND selects the triangular operator (lop).
// rperm (forward sweep; may be null): row i of In is taken from row
// rperm[i], the row interchanges of an LU factorisation applied on the fly.
template <typename T, int RT, bool FWD, bool INV, int KIND = 0>
__global__ __launch_bounds__(256, 2) void k_sweep(const T* __restrict__ L, int64_t lda, int64_t n, int64_t nrhs,
                                               const T* __restrict__ In, int64_t ldi, T* Out, int64_t ldo,
                                               SweepSync* sy, const int32_t* info, int spin_limit,
                                               const int32_t* __restrict__ rperm) {
    constexpr int NR = 16 * RT, XP = NR + 1, QW = NR / 4;
    __shared__ T Ls[JB * LDP];
    __shared__ T piv[JB];
    __shared__ T Xs[2][JB * XP];
    __shared__ T part[JB * XP];
    __shared__ int s_t;
    if (info && *info != 0) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
    sy += blockIdx.y;  // this pass's words; it covers right-hand sides rc0 .. rc0 + NR - 1
    const int64_t rc0 = (int64_t)blockIdx.y * NR;
    if (tid == 0) s_t = atomicAdd(&sy->ticket, 1);
    __syncthreads();
    const int t = s_t;
    const int nblk = (int)((n + JB - 1) / JB);
    if (t >= nblk) return;
    const int bi = FWD ? t : nblk - 1 - t;
    const int64_t r0 = (int64_t)bi * JB;
    const int jb = (int)(n - r0 < JB ? n - r0 : JB);
    if constexpr (INV) stage_inverse<T, KIND>(Ls, piv, L, lda, r0, jb);
    else stage_diag<T, !FWD, KIND>(Ls, piv, L, lda, r0, jb);
    // MFMA phase: wave w owns rows 16 w .. 16 w + 15 of the block
    const int64_t rwc = (16 * w + i < jb) ? r0 + 16 * w + i : r0;  // clamped for loads
    // blocks this one depends on: j = 0 .. bi - 1 (forward) or j = nblk - 1
    // down to bi + 1 (backward), visited in the order they are handed out
    const int ndep = FWD ? bi : nblk - 1 - bi;
    bool abort = false;
    if (spin_limit == 0 && ndep > 0) {
        abort = true;
        if (tid == 0) atomicExch(&sy->err, 1);
    }
    constexpr int XPT = JB * NR / 256;  // solution values each thread moves per block
    // this block's right-hand sides (a lane per row, wave w takes q = w + 4 u),
    // requested now so that their latency is off the critical path
    // (substitution: a lane per row, wave w takes q = w + 4 u; inverse: the
    // accumulator layout, row 16 w + i, right-hand side 16 rt + tcol(g, r))
    T vin[INV ? 4 * RT : QW];
    if constexpr (INV) {
        const bool rok = 16 * w + i < jb;
        const int64_t rin = (rperm && rok) ? rperm[r0 + 16 * w + i] : r0 + 16 * w + i;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t q = rc0 + 16 * rt + tcol<T>(g, r);
                vin[4 * rt + r] = (rok && q < nrhs) ? In[idx(rin, q, ldi)] : (T)0;
            }
    } else {
        const int64_t rin = (rperm && lane < jb) ? rperm[r0 + lane] : r0 + lane;
#pragma unroll
        for (int u = 0; u < QW; ++u) {
            const int q = w + 4 * u;
            vin[u] = (lane < jb && rc0 + q < nrhs) ? In[idx(rin, rc0 + q, ldi)] : (T)0;
        }
    }
    {
        // two accumulators (even and odd k-steps) halve the chain of
        // dependent MFMAs after the last dependency arrives
        V4<T> acc[RT], acc2[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = acc2[rt] = V4<T>{0, 0, 0, 0};
        // Software pipeline over the dependency blocks: the L values (per
        // lane, one per k-step) stream through a ring of LR blocks, requested
        // LR - 1 blocks ahead (a workgroup's own stream of L is what limits a
        // sweep: one block of prefetch kept it at a fifth of HBM bandwidth);
        // the solution values of block d + 1 are requested before block d is
        // multiplied.
        constexpr int LR = 4;
        T lr[LR][JB / 4], xc[XPT], xn[XPT];
        auto load_l = [&](T* dst, int d) {
            const int j = FWD ? d : nblk - 1 - d;
            const int64_t c0 = (int64_t)j * JB;
            const int jbj = (int)(n - c0 < JB ? n - c0 : JB);
#pragma unroll
            for (int ks = 0; ks < JB / 4; ++ks) {
                const int c = 4 * ks + g;
                // forward: operator row rwc; backward: operator column rwc
                // (KIND 2 stores the operator transposed: both read along a row)
                dst[ks] = (c < jbj) ? ((FWD || KIND == 2) ? L[idx(rwc, c0 + c, lda)] : L[idx(c0 + c, rwc, lda)])
                                    : (T)0;
            }
        };
        auto load_x = [&](T* dst, int d) {
            const int j = FWD ? d : nblk - 1 - d;
            const int64_t c0 = (int64_t)j * JB;
            const int jbj = (int)(n - c0 < JB ? n - c0 : JB);
#pragma unroll
            for (int k = 0; k < XPT; ++k) {
                const int e = tid + 256 * k, c = e & (JB - 1), q = e >> 6;
                dst[k] = (c < jbj && rc0 + q < nrhs) ? load_coherent(&Out[idx(c0 + c, rc0 + q, ldo)]) : (T)0;
            }
        };
#pragma unroll
        for (int s = 0; s < LR - 1; ++s)
            if (s < ndep) load_l(lr[s], s);
        if (ndep > 0) load_x(xc, 0);
        for (int d0 = 0; d0 < ndep; d0 += LR)
#pragma unroll
        for (int sl = 0; sl < LR; ++sl) {
            const int d = d0 + sl;
            if (d >= ndep) break;  // uniform
            if (d + LR - 1 < ndep) load_l(lr[(sl + LR - 1) % LR], d + LR - 1);
            if (d + 1 < ndep) load_x(xn, d + 1);
            // block d's solution into LDS, reloaded until every value is
            // written (the barrier that checks this also publishes the LDS)
            T* xs = Xs[d & 1];
            for (int spins = 0;; ++spins) {
                bool ok = true;
#pragma unroll
                for (int k = 0; k < XPT; ++k) {
                    const int e = tid + 256 * k, c = e & (JB - 1), q = e >> 6;
                    xs[c * XP + q] = xc[k];
                    ok = ok && !is_sentinel(xc[k]);
                }
                if (__syncthreads_and(ok) || abort) break;
                // give up (uniformly across the workgroup) past the spin limit
                // or once another workgroup has given up; the error word is
                // read by one thread every 32 spins, so that a poll normally
                // costs one round trip (the reload below), not two
                if ((spins & 31) == 31) {
                    const int e = (tid == 0) ? load_coherent(&sy->err) : 0;
                    if (__syncthreads_or(spins > spin_limit || e != 0)) {
                        abort = true;
                        if (tid == 0) atomicExch(&sy->err, 1);
                        break;
                    }
                }
                // Every workgroup soon catches up with the block being
                // solved, so hundreds would poll the same few kilobytes:
                // those with more of their own dependencies still to go
                // after this one (and so with slack) poll less often, which
                // keeps the round trips of the next block's poll short.
                const int ahead = ndep - 1 - d;
                if (ahead == 0) {
                    __builtin_amdgcn_s_sleep(1);
                } else {
                    for (int z = 0; z < (ahead < 4 ? ahead : 4); ++z) __builtin_amdgcn_s_sleep(32);
                }
                load_x(xc, d);
            }
            // acc += L_ij X_j (forward) or L_ji^T X_j (backward), 16 k-steps
#pragma unroll
            for (int ks = 0; ks < JB / 4; ++ks) {
                const int c = 4 * ks + g;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (ks & 1) acc2[rt] = mma_xzt(acc2[rt], lr[sl][ks], xs[c * XP + 16 * rt + i]);
                    else acc[rt] = mma_xzt(acc[rt], lr[sl][ks], xs[c * XP + 16 * rt + i]);
                }
            }
#pragma unroll
            for (int k = 0; k < XPT; ++k) xc[k] = xn[k];
        }
        if constexpr (INV) {
            // v = In - sum over the dependencies, rows 16 w + i of this
            // wave, into LDS as v(row, rhs) (rows past jb are 0) ...
            const bool rok = 16 * w + i < jb;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    part[(16 * w + i) * XP + 16 * rt + tcol<T>(g, r)] =
                        rok ? vin[4 * rt + r] - (acc[rt][r] + acc2[rt][r]) : (T)0;
            __syncthreads();
            // ... then x = Z v (forward, Z = L_ii^{-1} lower: rows of wave w
            // need k < 16 (w + 1)) or x = Z^T v (backward: k >= 16 w), a
            // 16 x 16 tile per wave on the matrix pipe, two accumulators
            V4<T> xa[RT], xb[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) xa[rt] = xb[rt] = V4<T>{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < JB / 4; ++ks) {
                if (FWD ? (ks >= 4 * (w + 1)) : (ks < 4 * w)) continue;  // wave-uniform
                const int k = 4 * ks + g;
                const T zx = FWD ? Ls[(16 * w + i) * LDP + k] : Ls[k * LDP + 16 * w + i];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (ks & 1) xb[rt] = mma_xzt(xb[rt], zx, part[k * XP + 16 * rt + i]);
                    else xa[rt] = mma_xzt(xa[rt], zx, part[k * XP + 16 * rt + i]);
                }
            }
            if (16 * w + i < jb) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t q = rc0 + 16 * rt + tcol<T>(g, r);
                        if (q < nrhs) store_coherent(&Out[idx(r0 + 16 * w + i, q, ldo)], xa[rt][r] + xb[rt][r]);
                    }
            }
            return;
        }
        // partial products to LDS, one row per entry: lane (i, g) holds rows
        // 16 w + i, right-hand sides 16 rt + tcol(g, r)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[(16 * w + i) * XP + 16 * rt + tcol<T>(g, r)] = acc[rt][r] + acc2[rt][r];
        __syncthreads();
        // diagonal block by substitution: a lane per row, wave w takes the
        // right-hand sides q = w + 4 u
        {
            const T pl = piv[lane];
            T v[QW];
#pragma unroll
            for (int u = 0; u < QW; ++u) v[u] = vin[u] - part[lane * XP + w + 4 * u];
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

    }
}

// After both sweeps (one workgroup): when a wait of either sweep gave up (an
// error word is set), Out is filled with quiet NaNs and *info (when given)
// becomes MG_INFO_SOLVE_ABORTED.  Skipped when info was non-zero on entry
// (the sweeps did not run and their words are stale); every thread reads
// info before the barrier that precedes the one write.
template <typename T>
__global__ __launch_bounds__(256) void k_sweep_check(T* Out, int64_t ld, int64_t n, int64_t nrhs,
                                                     const SweepSync* sy, int nwords, int32_t* info) {
    if (info && *info != 0) return;
    bool bad = false;
    for (int k = 0; k < nwords; ++k) bad = bad || load_coherent(&sy[k].err) != 0;
    if (!bad) return;
    __syncthreads();
    if (info && threadIdx.x == 0) *info = MG_INFO_SOLVE_ABORTED;
    const int64_t tot = n * nrhs;
    for (int64_t e = threadIdx.x; e < tot; e += 256) Out[idx(e % n, e / n, ld)] = (T)NAN;
}

// ---------------------------------------------------------------------------
// Y L = C in place for a wide C (m x n, column-major) and L lower n x n,
// n % 64 == 0: blocked from the right in 64-column blocks.  With all the
// diagonal inverses Z_b = L_bb^{-1} formed first (one workgroup per block,
// stage_inverse), block b's columns become Y_b = C_b Z_b (k_right_mul, in
// place, a 64-row strip per workgroup on the FP64 matrix pipe) and the
// columns to its left receive C[:, 0:c0] -= Y_b L[c0:c0+64, 0:c0] on the
// general update kernel, by groups of eight blocks (rank 512).  The substitution chain of the
// sweeps becomes n / 64 steps of matrix products, for problems with as many
// right-hand sides as rows (the adjoint of the factorisation).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag_inverse(const double* __restrict__ L, int64_t lda, int64_t n,
                                                      double* __restrict__ Zw) {
    __shared__ double Ls[JB * LDP];
    __shared__ double rp[JB];
    const int64_t r0 = (int64_t)blockIdx.x * JB;
    const int jb = (int)(n - r0 < JB ? n - r0 : JB);
    stage_inverse<double, 0>(Ls, rp, L, lda, r0, jb);
    double* Z = Zw + (size_t)blockIdx.x * JB * JB;  // column-major, leading dimension 64
    for (int e = threadIdx.x; e < JB * JB; e += 256) {
        const int r = e & (JB - 1), c = e >> 6;
        Z[r + c * JB] = Ls[r * LDP + c];
    }
}

// Cb (m x 64, ldc) <- Cb Z for Z 64 x 64 (column-major, leading dimension
// 64): wave w of workgroup s takes rows 64 s + 16 w .. + 15, all 64 columns,
// reading its rows completely before it writes them.
__global__ __launch_bounds__(256) void k_right_mul(double* __restrict__ Cb, int64_t ldc, int64_t m,
                                                   const double* __restrict__ Z) {
    __shared__ double Zs[JB][LDP];  // Zs[k][j] = Z(k, j)
    for (int e = threadIdx.x; e < JB * JB; e += 256) {
        const int k = e & (JB - 1), j = e >> 6;
        Zs[k][j] = Z[k + j * JB];
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int64_t row = (int64_t)blockIdx.x * JB + 16 * w + i;
    const bool rok = row < m;
    double x[JB / 4];
#pragma unroll
    for (int ks = 0; ks < JB / 4; ++ks) x[ks] = rok ? Cb[idx(row, 4 * ks + g, ldc)] : 0.0;
    V4<double> acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = V4<double>{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < JB / 4; ++ks)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mma_xzt(acc[t], x[ks], Zs[4 * ks + g][16 * t + i]);
    if (!rok) return;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) Cb[idx(row, 16 * t + tcol<double>(g, r), ldc)] = acc[t][r];
}

constexpr int64_t RS_GROUP = 8;  // 64-column blocks per rank-512 update

bool right_solve_lower_ok(int64_t m, int64_t n, int64_t lda, int64_t ldc) {
    // the update kernel's 32-bit byte offsets (C, the group's Y columns and
    // the L block rows, from their bases)
    const int64_t ld = std::max(lda, ldc);
    return n > 0 && n % JB == 0 && (std::max(m, n) + (RS_GROUP + 1) * JB) * ld * 8 < ((int64_t)1 << 31);
}

size_t right_solve_lower_work_bytes(int64_t n) { return align_up((size_t)n * JB * 8, 256); }

mg_status right_solve_lower(hipStream_t st, int64_t m, int64_t n, const double* L, int64_t lda, double* C,
                            int64_t ldc, double* Zw) {
    if (m <= 0 || n <= 0) return MG_OK;
    if (!right_solve_lower_ok(m, n, lda, ldc)) return MG_ERR_UNSUPPORTED;
    const int64_t nblk = n / JB;
    hipLaunchKernelGGL(k_diag_inverse, dim3((unsigned)nblk), dim3(256), 0, st, L, lda, n, Zw);
    MG_LAUNCH_CHECK();
    mg_status rc;
    // groups of RS_GROUP blocks from the right: inside a group each block
    // updates the group's blocks to its left (rank 64); the finished group
    // then updates everything to its left at once (rank 512), which moves C
    // an eighth as many times as rank-64 updates would
    for (int64_t bh = nblk - 1; bh >= 0; bh -= RS_GROUP) {
        const int64_t bl = std::max<int64_t>(0, bh - RS_GROUP + 1), g0 = bl * JB;
        for (int64_t b = bh; b >= bl; --b) {
            const int64_t c0 = b * JB;
            hipLaunchKernelGGL(k_right_mul, dim3((unsigned)cdiv(m, JB)), dim3(256), 0, st, C + idx(0, c0, ldc), ldc,
                               m, (const double*)(Zw + (size_t)b * JB * JB));
            MG_LAUNCH_CHECK();
            if (c0 > g0 && (rc = gemm_sub_f64(st, C + idx(0, g0, ldc), ldc, C + idx(0, c0, ldc), ldc,
                                              L + idx(c0, g0, lda), lda, m, c0 - g0, JB)))
                return rc;
        }
        if (g0 > 0 && (rc = gemm_sub_f64(st, C, ldc, C + idx(0, g0, ldc), ldc, L + g0, lda, m, g0,
                                         (bh - bl + 1) * JB)))
            return rc;
    }
    return MG_OK;
}

// Many right-hand sides (an inverse, a gradient): passes of 64 instead of
// 16 (RT = 4; one workgroup per CU instead of two), so that the factor is
// streamed a quarter as many times.  Each right-hand side sees the same
// products in the same order either way.
constexpr int64_t SW_WIDE = 256;  // right-hand sides from which passes take 64
static int64_t wide_passes(int64_t nrhs) { return cdiv(nrhs, 4 * SW_NR); }

template <typename T, bool FWD, bool INV>
static void launch_sweep(hipStream_t st, bool wide, dim3 grid, const T* L, int64_t lda, int64_t n, int64_t nrhs,
                         const T* In, int64_t ldi, T* Out, int64_t ldo, SweepSync* sy, int32_t* info, int spin_limit) {
    if constexpr (sizeof(T) == 8) {
        if (wide) {
            hipLaunchKernelGGL((k_sweep<T, 4, FWD, INV>), grid, dim3(256), 0, st, L, lda, n, nrhs, In, ldi, Out, ldo,
                               sy, info, spin_limit, (const int32_t*)nullptr);
            return;
        }
    }
    hipLaunchKernelGGL((k_sweep<T, 1, FWD, INV>), grid, dim3(256), 0, st, L, lda, n, nrhs, In, ldi, Out, ldo, sy, info,
                       spin_limit, (const int32_t*)nullptr);
}

// the wide passes (binary64 only: binary32 at 64 right-hand sides per pass
// would spill under the kernel's two-workgroup register cap)
template <typename T>
static bool use_wide(int64_t nrhs) { return sizeof(T) == 8 && nrhs >= SW_WIDE; }

template <typename T, bool INV>
static mg_status sweep(hipStream_t st, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B, int64_t ldb, T* Y,
                       SweepSync* sy, int32_t* info, int spin_limit) {
    const bool wide = use_wide<T>(nrhs);
    const int64_t np = wide ? wide_passes(nrhs) : sweep_passes(nrhs);
    const dim3 grid((unsigned)cdiv(n, JB), (unsigned)np);
    const unsigned gfill = (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(n * nrhs, 256)), 2048);
    hipLaunchKernelGGL((k_sweep_init<T>), dim3(gfill), dim3(256), 0, st, Y, n, n, nrhs, sy, info);
    MG_LAUNCH_CHECK();
    launch_sweep<T, true, INV>(st, wide, grid, L, lda, n, nrhs, (const T*)B, ldb, Y, n, sy, info, spin_limit);
    MG_LAUNCH_CHECK();
    // B has been read; it now receives X
    hipLaunchKernelGGL((k_sweep_init<T>), dim3(gfill), dim3(256), 0, st, B, ldb, n, nrhs, sy + np, info);
    MG_LAUNCH_CHECK();
    launch_sweep<T, false, INV>(st, wide, grid, L, lda, n, nrhs, (const T*)Y, n, B, ldb, sy + np, info, spin_limit);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sweep_check<T>), dim3(1), dim3(256), 0, st, B, ldb, n, nrhs, (const SweepSync*)sy,
                       (int)(2 * np), info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

template <typename T>
mg_status potrs_impl(mg_handle_t h, int64_t n, int64_t nrhs, const T* L, int64_t lda, T* B, int64_t ldb, T* Y,
                     int32_t* info) {
    if (n == 0 || nrhs == 0) return MG_OK;
    hipStream_t st = h->stream;
    mg_status rc;
    if ((rc = prof_begin(h, MG_PROF_SOLVE, st))) return rc;
    SweepSync* sy = (SweepSync*)((char*)Y + y_bytes(n, nrhs, (int)sizeof(T)));
    const int lim = h->spin_limit < 0 ? SWEEP_SPIN_LIMIT : h->spin_limit;
    rc = h->solve_mode == MG_SOLVE_SUBSTITUTION ? sweep<T, false>(st, n, nrhs, L, lda, B, ldb, Y, sy, info, lim)
                                                 : sweep<T, true>(st, n, nrhs, L, lda, B, ldb, Y, sy, info, lim);
    if (rc) return rc;
    const double nd = (double)n;
    return prof_end(h, MG_PROF_SOLVE, 2.0 * nd * nd * (double)nrhs,
                    (nd * (nd + 1) + 4.0 * nd * (double)nrhs) * sizeof(T), st);
}

// Out = L^{-T} In alone (the backward sweep), In and Out distinct, nrhs
// columns in passes of 16; sy: the pass words (sweep_words_bytes(nrhs)).
// The sweep is followed by the give-up check (Out NaN and info =
// MG_INFO_SOLVE_ABORTED when a wait gave up); skipped when *info != 0.
size_t sweep_words_bytes(int64_t nrhs) { return align_up((size_t)sweep_passes(nrhs) * 16, 256); }

template <typename T>
mg_status trsm_lt_impl(mg_handle_t h, int64_t n, int64_t nrhs, const T* L, int64_t lda, const T* In, int64_t ldi,
                       T* Out, int64_t ldo, void* words, int32_t* info) {
    if (n == 0 || nrhs == 0) return MG_OK;
    hipStream_t st = h->stream;
    SweepSync* sy = (SweepSync*)words;
    const int lim = h->spin_limit < 0 ? SWEEP_SPIN_LIMIT : h->spin_limit;
    const bool wide = use_wide<T>(nrhs);
    const int64_t np = wide ? wide_passes(nrhs) : sweep_passes(nrhs);
    const dim3 grid((unsigned)cdiv(n, JB), (unsigned)np);
    const unsigned gfill = (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(n * nrhs, 256)), 2048);
    hipLaunchKernelGGL((k_sweep_init<T>), dim3(gfill), dim3(256), 0, st, Out, ldo, n, nrhs, sy, info);
    MG_LAUNCH_CHECK();
    if (h->solve_mode == MG_SOLVE_SUBSTITUTION)
        launch_sweep<T, false, false>(st, wide, grid, L, lda, n, nrhs, In, ldi, Out, ldo, sy, info, lim);
    else
        launch_sweep<T, false, true>(st, wide, grid, L, lda, n, nrhs, In, ldi, Out, ldo, sy, info, lim);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sweep_check<T>), dim3(1), dim3(256), 0, st, Out, ldo, n, nrhs, (const SweepSync*)sy,
                       (int)np, info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}
// The two sweeps of an LU solve: Y = L^{-1} (P B) with L the unit lower
// factor and row i of P B read from row rperm[i] of B, then B = U^{-1} Y,
// followed by the give-up check.  sy: two pass-word sets
// (2 * sweep_words_bytes(nrhs) bytes).  Skipped when *info != 0.
mg_status lu_sweeps(mg_handle_t h, int64_t n, int64_t nrhs, const double* LU, int64_t lda, const int32_t* rperm,
                    double* B, int64_t ldb, double* Y, void* words, int32_t* info) {
    if (n == 0 || nrhs == 0) return MG_OK;
    hipStream_t st = h->stream;
    const int64_t np = sweep_passes(nrhs);
    SweepSync* sy = (SweepSync*)words;
    const int lim = h->spin_limit < 0 ? SWEEP_SPIN_LIMIT : h->spin_limit;
    const dim3 grid((unsigned)cdiv(n, JB), (unsigned)np);
    const unsigned gfill = (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(n * nrhs, 256)), 2048);
    const bool sub = h->solve_mode == MG_SOLVE_SUBSTITUTION;
    hipLaunchKernelGGL((k_sweep_init<double>), dim3(gfill), dim3(256), 0, st, Y, n, n, nrhs, sy, info);
    MG_LAUNCH_CHECK();
    if (sub)
        hipLaunchKernelGGL((k_sweep<double, 1, true, false, 1>), grid, dim3(256), 0, st, LU, lda, n, nrhs,
                           (const double*)B, ldb, Y, n, sy, info, lim, rperm);
    else
        hipLaunchKernelGGL((k_sweep<double, 1, true, true, 1>), grid, dim3(256), 0, st, LU, lda, n, nrhs,
                           (const double*)B, ldb, Y, n, sy, info, lim, rperm);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sweep_init<double>), dim3(gfill), dim3(256), 0, st, B, ldb, n, nrhs, sy + np, info);
    MG_LAUNCH_CHECK();
    if (sub)
        hipLaunchKernelGGL((k_sweep<double, 1, false, false, 2>), grid, dim3(256), 0, st, LU, lda, n, nrhs,
                           (const double*)Y, n, B, ldb, sy + np, info, lim, (const int32_t*)nullptr);
    else
        hipLaunchKernelGGL((k_sweep<double, 1, false, true, 2>), grid, dim3(256), 0, st, LU, lda, n, nrhs,
                           (const double*)Y, n, B, ldb, sy + np, info, lim, (const int32_t*)nullptr);
    MG_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sweep_check<double>), dim3(1), dim3(256), 0, st, B, ldb, n, nrhs, (const SweepSync*)sy,
                       (int)(2 * np), info);
    MG_LAUNCH_CHECK();
    return MG_OK;
}

template mg_status trsm_lt_impl<double>(mg_handle_t, int64_t, int64_t, const double*, int64_t, const double*, int64_t,
                                        double*, int64_t, void*, int32_t*);

template mg_status potrs_impl<double>(mg_handle_t, int64_t, int64_t, const double*, int64_t, double*, int64_t,
                                      double*, int32_t*);
template mg_status potrs_impl<float>(mg_handle_t, int64_t, int64_t, const float*, int64_t, float*, int64_t,
                                     float*, int32_t*);

}  // namespace mg
