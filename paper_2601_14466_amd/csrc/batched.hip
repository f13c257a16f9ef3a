// batched.hip -- thousands of independent SPD solves of uneven size in one
// persistent launch.
//
// The paper's operation (JAXMg, "Software design", potrs bullet) applied to
// a batch; the paper has no batched form, so the schedule is ours:
//   - the host plan sorts the systems by decreasing order (longest
//     processing time first) and keeps that permutation on the device;
//   - a persistent grid of workgroups takes the next system from an atomic
//     counter until the batch is exhausted (every workgroup exits on its own;
//     nothing waits on another workgroup);
//   - one workgroup (four waves) factors a system in place with a
//     left-looking algorithm on 16-wide block columns: for block column j,
//     row block j of L (the MFMA z operand shared by every tile of the
//     column) is staged in LDS, each wave accumulates its tiles
//     A_Ij - sum_p L_Ip L_jp^T on the matrix pipe, the diagonal tile is
//     factored in registers (factor16) and the tiles below are solved
//     (solve16s); the forward substitution L y = b is fused into the same
//     sweep, then the backward substitution L^T x = y runs block by block.
// Per-system info: 0, or the first failing column (1-based); a failing system
// leaves its right-hand side untouched and does not affect the others.
#include <algorithm>
#include <cstring>
#include <vector>

#include "mg_internal.h"
#include "tile16.h"

namespace mg {

constexpr int BMAX = 512;           // largest order a workgroup handles
constexpr int BNT = BMAX / 16;      // tiles per side
constexpr int BTPW = BNT / 4;       // tiles of one block column per wave (4 waves)

template <typename T>
struct BatchArgs {
    const int32_t* order;   // systems, longest first
    const int32_t* nsz;     // order of each system
    T* const* A;            // device pointers
    const int64_t* lda;
    T* const* B;
    const int64_t* ldb;
    int32_t* info;
    unsigned* counter;
    int batch;
    int nrhs;
};

// Factor + solve one system: A (n x n, lda) in place, B (n x nrhs, ldb) overwritten
// by X.  Returns 0 or the failing column (1-based), uniform across the workgroup.
template <typename T>
__device__ __forceinline__ int solve_one(T* __restrict__ A, int64_t lda, int n, T* __restrict__ B, int64_t ldb, int nrhs,
                         T (*Zs)[BMAX + 1], T* Ls, T* Lsc, T* piv, T* bv, T (*xacc)[16], int* s_fail) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, g = l >> 4;
    const int nt = (n + 15) >> 4;
    for (int j = 0; j < nt; ++j) {
        // ---- stage row block j of L (columns 0..16j-1): the z operand of
        // every tile of block column j, and both operands of its diagonal tile
        for (int e = threadIdx.x; e < 16 * 16 * j; e += 256) {
            const int rr = e & 15, c = e >> 4;
            Zs[rr][c] = (16 * j + rr < n) ? A[idx(16 * j + rr, c, lda)] : (T)0;
        }
        __syncthreads();
        // ---- diagonal tile (wave 0): A_jj - sum_p L_jp L_jp^T from LDS, factor,
        // publish, forward substitution of block j
        if (w == 0) {
            V4<T> d;
            load_tile<T, T>(d, A, lda, 16 * j, 16 * j, n, n, true, true);
            for (int p = 0; p < j; ++p) {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int kk = 16 * p + 4 * ks + g;
                    d = mma_xzt(d, Zs[i][kk], -Zs[i][kk]);
                }
            }
            const int f = factor16<T, sizeof(T) == 8>(d);  // binary32: within the 168-register cap
            if (f) {
                if (l == 0) *s_fail = 16 * j + f;
            } else {
                tile_to_lds_lower<T, 17>(d, Ls);
                store_tile<T, T>(d, A, lda, 16 * j, 16 * j, n, n, true);
            }
        }
        __syncthreads();
        if (*s_fail) return *s_fail;
        scale_lower16<T, 17>(Ls, Lsc, piv, threadIdx.x);
        __syncthreads();
        if (w == 0 && l < 16) {
            for (int r = 0; r < nrhs; ++r) {
                T v = bv[r * BMAX + 16 * j + l];
                for (int c = 0; c < 16; ++c) {
                    const T vc = readlane(v, c);
                    v = v - Lsc[l * 17 + c] * vc;
                }
                bv[r * BMAX + 16 * j + l] = v / piv[l];
            }
        }
        __syncthreads();  // y_j in LDS
        // ---- tiles below the diagonal, two per wave at a time: left-looking
        // update (x operand streamed from memory one finished column ahead of
        // the MFMAs), solve against L_jj, store, and b_I -= L_Ij y_j
        for (int I0 = j + 1 + w; I0 < nt; I0 += 8) {
            V4<T> acc[2];
            int64_t rr_[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int I = I0 + 4 * u;
                const int64_t ri = 16 * I + i;
                rr_[u] = (I < nt && ri < n) ? ri : -1;
                if (I < nt) load_tile<T, T>(acc[u], A, lda, 16 * I, 16 * j, n, n, false, false);
                else acc[u] = V4<T>{0, 0, 0, 0};
            }
            T xa[2][4], xb[2][4];
#define MG_LDX(x, pp)                                                                            \
    _Pragma("unroll") for (int u = 0; u < 2; ++u)                                                \
        _Pragma("unroll") for (int ks = 0; ks < 4; ++ks)                                         \
            x[u][ks] = (rr_[u] >= 0) ? A[rr_[u] + (int64_t)(16 * (pp) + 4 * ks + g) * lda] : (T)0
#define MG_MMA(x, pp)                                                                            \
    do {                                                                                         \
        _Pragma("unroll") for (int ks = 0; ks < 4; ++ks) {                                       \
            const T z_ = -Zs[i][16 * (pp) + 4 * ks + g];                                         \
            _Pragma("unroll") for (int u = 0; u < 2; ++u) acc[u] = mma_xzt(acc[u], x[u][ks], z_); \
        }                                                                                        \
    } while (0)
            if (j > 0) { MG_LDX(xa, 0); }
            for (int p = 0; p < j; p += 2) {
                if (p + 1 < j) { MG_LDX(xb, p + 1); }
                MG_MMA(xa, p);
                if (p + 1 < j) {
                    if (p + 2 < j) { MG_LDX(xa, p + 2); }
                    MG_MMA(xb, p + 1);
                }
            }
#undef MG_LDX
#undef MG_MMA
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int I = I0 + 4 * u;
                if (I >= nt) continue;
                solve16s<T, 17, true>(acc[u], Lsc, piv);
                store_tile<T, T>(acc[u], A, lda, 16 * I, 16 * j, n, n, false);
                // b_I -= L_Ij y_j (each lane: its row, its 4 columns; reduce over groups)
                for (int r = 0; r < nrhs; ++r) {
                    T sm = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) sm = sm + acc[u][q] * bv[r * BMAX + 16 * j + tcol<T>(g, q)];
                    sm = sm + shfl(sm, l ^ 16);
                    sm = sm + shfl(sm, l ^ 32);
                    if (g == 0 && 16 * I + i < n) bv[r * BMAX + 16 * I + i] -= sm;
                }
            }
        }
        __syncthreads();
    }
    // ---- backward substitution L^T x = y, block by block from the bottom
    for (int j = nt - 1; j >= 0; --j) {
        for (int r = 0; r < nrhs; ++r) {
            // per-wave partial sums of L_Ij^T x_I over the wave's tiles I > j, in a fixed order
            T part[4] = {0, 0, 0, 0};
            for (int I = j + 1 + w; I < nt; I += 4) {
                V4<T> y;
                load_tile<T, T>(y, A, lda, 16 * I, 16 * j, n, n, false, false);
                const T xi = (16 * I + i < n) ? bv[r * BMAX + 16 * I + i] : (T)0;
#pragma unroll
                for (int q = 0; q < 4; ++q) part[q] = part[q] + y[q] * xi;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T v = part[q];  // reduce over the 16 rows of the lane group
                v = v + shfl(v, l ^ 1);
                v = v + shfl(v, l ^ 2);
                v = v + shfl(v, l ^ 4);
                v = v + shfl(v, l ^ 8);
                if (i == 0) xacc[w][tcol<T>(g, q)] = v;
            }
            __syncthreads();
            if (w == 0 && l < 16) {
                // diagonal block: L_jj^T x_j = y_j - sum by substitution from
                // the last row up; row c of L_jj^T is scaled by 1/L_cc (one
                // reciprocal per lane, broadcast by readlane)
                const T sum = ((xacc[0][l] + xacc[1][l]) + xacc[2][l]) + xacc[3][l];
                T v = bv[r * BMAX + 16 * j + l] - sum;
                const bool vl = 16 * j + l < n;
                const T lj = vl ? A[idx(16 * j + l, 16 * j + l, lda)] : (T)1;
                const T rl = (T)1 / lj;
                T lcl[16];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    lcl[c] = (l < c && 16 * j + c < n) ? A[idx(16 * j + c, 16 * j + l, lda)] : (T)0;
#pragma unroll
                for (int c = 15; c >= 0; --c) {
                    const T vc = readlane(v, c);
                    v = v - lcl[c] * (readlane(rl, c) * vc);
                }
                if (vl) bv[r * BMAX + 16 * j + l] = v * rl;
            }
            __syncthreads();
        }
    }
    // ---- write X
    for (int e = threadIdx.x; e < n * nrhs; e += 256) {
        const int row = e % n, r = e / n;
        B[idx(row, r, ldb)] = bv[r * BMAX + row];
    }
    return 0;
}

// Two workgroups per CU for binary64 (256 VGPRs and the 75 KB row block of L
// in LDS); three for binary32, whose smaller LDS footprint lets the register
// cap of 168 decide: the solve is bound by memory latency, and the third
// workgroup hides more of it than the few spilled registers cost.
template <typename T, int NRHS_MAX>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 3 : 2) void k_batched_posv(BatchArgs<T> a) {
    __shared__ T Zs[16][BMAX + 1];
    __shared__ T Ls[16 * 17], Lsc[16 * 17], piv[16];
    __shared__ T bv[NRHS_MAX * BMAX];
    __shared__ T xacc[4][16];
    __shared__ int s_q, s_fail;
    for (;;) {
        if (threadIdx.x == 0) {
            s_q = (int)atomicAdd(a.counter, 1u);
            s_fail = 0;
        }
        __syncthreads();
        const int q = s_q;
        if (q >= a.batch) break;
        const int sys = a.order[q];
        const int n = a.nsz[sys];
        T* A = a.A[sys];
        T* B = a.B[sys];
        const int64_t lda = a.lda[sys], ldb = a.ldb[sys];
        const int nrhs = a.nrhs;
        for (int e = threadIdx.x; e < NRHS_MAX * BMAX; e += 256) {
            const int row = e % BMAX, r = e / BMAX;
            bv[e] = (row < n && r < nrhs) ? B[idx(row, r, ldb)] : (T)0;
        }
        __syncthreads();
        int f = 0;
        if (n > 0) f = solve_one<T>(A, lda, n, B, ldb, nrhs, Zs, Ls, Lsc, piv, bv, xacc, &s_fail);
        if (threadIdx.x == 0) a.info[sys] = f;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Wide variant: eight waves per system.  The work of block column j -- the
// diagonal tile and the nt - j - 1 tiles below it, each a left-looking
// product over the j finished block columns -- is spread over the waves:
// with at least eight tiles, wave w takes tiles w, w + 8, ... whole; with
// fewer, each tile's range of earlier block columns is cut into 8 / (nt - j)
// chunks, one per wave, and the chunks' partial tiles are summed through LDS
// in a fixed order (results do not depend on timing).  The left-panel
// operands of every tile a wave holds are streamed from memory two block
// columns ahead of the MFMAs.  Each block column then costs a few barriers:
// the diagonal tile is factored (wave 0) while the tiles wait, wave 0
// substitutes b_j while the others solve their tiles against L_jj, and the
// owners apply b_I -= L_Ij y_j.
// ---------------------------------------------------------------------------
constexpr int NW8 = 8;                       // waves per workgroup
constexpr int TPW8 = (BNT + NW8 - 1) / NW8;  // tiles a wave holds at most

template <typename T>
__device__ __forceinline__ int solve_one_w8(T* __restrict__ A, int64_t lda, int n, T* __restrict__ B, int64_t ldb,
                                            int nrhs, T (*Zs)[BMAX + 1], T* Ls, T* Lsc, T* piv, T* bv,
                                            T (*xacc)[16], T (*dpart)[256], int* s_fail) {
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, i = l & 15, g = l >> 4;
    const int nt = (n + 15) >> 4;
    for (int j = 0; j < nt; ++j) {
        // ---- row block j of L (columns 0..16j-1): the z operand of every
        // tile of block column j, and the x operand of its diagonal tile
        for (int e = tid; e < 16 * 16 * j; e += 64 * NW8) {
            const int rr = e & 15, c = e >> 4;
            Zs[rr][c] = (16 * j + rr < n) ? A[idx(16 * j + rr, c, lda)] : (T)0;
        }
        __syncthreads();
        // ---- this wave's share: tiles u (tile row j + u; u = 0 is the
        // diagonal tile) and a range [p0, p1) of earlier block columns
        const int Tp = nt - j;
        const int nch = Tp >= NW8 ? 1 : NW8 / Tp;
        int ntw, h, u0;
        if (nch == 1) {
            u0 = w;
            h = 0;
            ntw = w < Tp ? (Tp - 1 - w) / NW8 + 1 : 0;
        } else {
            u0 = w % Tp;
            h = w / Tp;
            ntw = (w < Tp * nch) ? 1 : 0;
        }
        const int p0 = nch == 1 ? 0 : h * j / nch, p1 = nch == 1 ? j : (h + 1) * j / nch;
        V4<T> acc[TPW8];
        int64_t rowq[TPW8];  // operand row of each held tile (-1: past the order)
#pragma unroll
        for (int q = 0; q < TPW8; ++q) {
            const int I = j + u0 + NW8 * q;
            acc[q] = V4<T>{0, 0, 0, 0};
            rowq[q] = -1;
            if (q < ntw) {
                rowq[q] = (16 * I + i < n) ? 16 * I + i : -1;
                if (h == 0) load_tile<T, T>(acc[q], A, lda, 16 * I, 16 * j, n, n, I == j, I == j);
            }
        }
        // operands two block columns ahead: ring of three
        T xr[3][TPW8][4];
        auto ldx = [&](int slot, int p) {
#pragma unroll
            for (int q = 0; q < TPW8; ++q)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    xr[slot][q][ks] = (q < ntw && rowq[q] >= 0 && !(q == 0 && u0 == 0))
                                          ? A[rowq[q] + (int64_t)(16 * p + 4 * ks + g) * lda]
                                          : (T)0;
        };
        auto mma = [&](int slot, int p) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = 16 * p + 4 * ks + g;
                const T zv = Zs[i][kk];
#pragma unroll
                for (int q = 0; q < TPW8; ++q) {
                    if (q >= ntw) continue;  // wave-uniform
                    // the diagonal tile's x operand is row block j itself (LDS)
                    const T xv = (q == 0 && u0 == 0) ? zv : xr[slot][q][ks];
                    acc[q] = mma_xzt(acc[q], xv, -zv);
                }
            }
        };
        if (ntw > 0 && p0 < p1) {
            ldx(0, p0);
            if (p0 + 1 < p1) ldx(1, p0 + 1);
            for (int p = p0; p < p1; p += 3) {
                if (p + 2 < p1) ldx(2, p + 2);
                mma(0, p);
                if (p + 1 < p1) {
                    if (p + 3 < p1) ldx(0, p + 3);
                    mma(1, p + 1);
                }
                if (p + 2 < p1) {
                    if (p + 4 < p1) ldx(1, p + 4);
                    mma(2, p + 2);
                }
            }
        }
        // ---- chunked tiles: partial sums through LDS, added by the chunk-0
        // wave in chunk order
        if (nch > 1 && ntw == 1 && h > 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) dpart[w][4 * l + r] = acc[0][r];
        }
        __syncthreads();
        if (nch > 1 && ntw == 1 && h == 0) {
            for (int hh = 1; hh < nch; ++hh)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[0][r] += dpart[w + hh * Tp][4 * l + r];
        }
        // ---- diagonal tile (wave 0 holds it): factor, publish
        if (w == 0) {
            const int f = factor16<T, sizeof(T) == 8>(acc[0]);
            if (f) {
                if (l == 0) *s_fail = 16 * j + f;
            } else {
                tile_to_lds_lower<T, 17>(acc[0], Ls);
                store_tile<T, T>(acc[0], A, lda, 16 * j, 16 * j, n, n, true);
            }
        }
        __syncthreads();
        if (*s_fail) return *s_fail;
        scale_lower16<T, 17>(Ls, Lsc, piv, tid);
        __syncthreads();
        // ---- wave 0: forward substitution of block j; owners: solve the
        // tiles below against L_jj and store them
        if (w == 0 && l < 16) {
            for (int r = 0; r < nrhs; ++r) {
                T v = bv[r * BMAX + 16 * j + l];
                for (int c = 0; c < 16; ++c) {
                    const T vc = readlane(v, c);
                    v = v - Lsc[l * 17 + c] * vc;
                }
                bv[r * BMAX + 16 * j + l] = v / piv[l];
            }
        }
        if (h == 0) {
#pragma unroll
            for (int q = 0; q < TPW8; ++q) {
                const int I = j + u0 + NW8 * q;
                if (q >= ntw || I == j) continue;
                solve16s<T, 17, true>(acc[q], Lsc, piv);
                store_tile<T, T>(acc[q], A, lda, 16 * I, 16 * j, n, n, false);
            }
        }
        __syncthreads();  // y_j in LDS
        // ---- b_I -= L_Ij y_j (each lane: its row, its 4 columns; reduce over groups)
        if (h == 0) {
#pragma unroll
            for (int q = 0; q < TPW8; ++q) {
                const int I = j + u0 + NW8 * q;
                if (q >= ntw || I == j) continue;
                for (int r = 0; r < nrhs; ++r) {
                    T sm = 0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) sm = sm + acc[q][c] * bv[r * BMAX + 16 * j + tcol<T>(g, c)];
                    sm = sm + shfl(sm, l ^ 16);
                    sm = sm + shfl(sm, l ^ 32);
                    if (g == 0 && 16 * I + i < n) bv[r * BMAX + 16 * I + i] -= sm;
                }
            }
        }
        __syncthreads();
    }
    // ---- backward substitution L^T x = y, block by block from the bottom
    for (int j = nt - 1; j >= 0; --j) {
        for (int r = 0; r < nrhs; ++r) {
            // per-wave partial sums of L_Ij^T x_I over the wave's tiles I > j, in a fixed order
            T part[4] = {0, 0, 0, 0};
            for (int I = j + 1 + w; I < nt; I += NW8) {
                V4<T> y;
                load_tile<T, T>(y, A, lda, 16 * I, 16 * j, n, n, false, false);
                const T xi = (16 * I + i < n) ? bv[r * BMAX + 16 * I + i] : (T)0;
#pragma unroll
                for (int q = 0; q < 4; ++q) part[q] = part[q] + y[q] * xi;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T v = part[q];  // reduce over the 16 rows of the lane group
                v = v + shfl(v, l ^ 1);
                v = v + shfl(v, l ^ 2);
                v = v + shfl(v, l ^ 4);
                v = v + shfl(v, l ^ 8);
                if (i == 0) xacc[w][tcol<T>(g, q)] = v;
            }
            __syncthreads();
            if (w == 0 && l < 16) {
                T sum = xacc[0][l];
#pragma unroll
                for (int ww = 1; ww < NW8; ++ww) sum = sum + xacc[ww][l];
                T v = bv[r * BMAX + 16 * j + l] - sum;
                const bool vl = 16 * j + l < n;
                const T lj = vl ? A[idx(16 * j + l, 16 * j + l, lda)] : (T)1;
                const T rl = (T)1 / lj;
                T lcl[16];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    lcl[c] = (l < c && 16 * j + c < n) ? A[idx(16 * j + c, 16 * j + l, lda)] : (T)0;
#pragma unroll
                for (int c = 15; c >= 0; --c) {
                    const T vc = readlane(v, c);
                    v = v - lcl[c] * (readlane(rl, c) * vc);
                }
                if (vl) bv[r * BMAX + 16 * j + l] = v * rl;
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < n * nrhs; e += 64 * NW8) {
        const int row = e % n, r = e / n;
        B[idx(row, r, ldb)] = bv[r * BMAX + row];
    }
    return 0;
}

template <typename T, int NRHS_MAX>
__global__ __launch_bounds__(64 * NW8, 1) void k_batched_posv_w8(BatchArgs<T> a) {
    __shared__ T Zs[16][BMAX + 1];
    __shared__ T Ls[16 * 17], Lsc[16 * 17], piv[16];
    __shared__ T bv[NRHS_MAX * BMAX];
    __shared__ T xacc[NW8][16];
    __shared__ T dpart[NW8][256];
    __shared__ int s_q, s_fail;
    for (;;) {
        if (threadIdx.x == 0) {
            s_q = (int)atomicAdd(a.counter, 1u);
            s_fail = 0;
        }
        __syncthreads();
        const int q = s_q;
        if (q >= a.batch) break;
        const int sys = a.order[q];
        const int n = a.nsz[sys];
        T* A = a.A[sys];
        T* B = a.B[sys];
        const int64_t lda = a.lda[sys], ldb = a.ldb[sys];
        const int nrhs = a.nrhs;
        for (int e = threadIdx.x; e < NRHS_MAX * BMAX; e += 64 * NW8) {
            const int row = e % BMAX, r = e / BMAX;
            bv[e] = (row < n && r < nrhs) ? B[idx(row, r, ldb)] : (T)0;
        }
        __syncthreads();
        int f = 0;
        if (n > 0) f = solve_one_w8<T>(A, lda, n, B, ldb, nrhs, Zs, Ls, Lsc, piv, bv, xacc, dpart, &s_fail);
        if (threadIdx.x == 0) a.info[sys] = f;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Batched adjoint (reverse mode of the batched posv): for every system, from
// its stored factor L_k (left in A_k by the forward solve), its solution X_k
// and the upstream gradient gX_k:
//   gB_k = A_k^{-1} gX_k            (forward and back substitution with L_k)
//   gA_k = -1/2 (gB_k X_k^T + X_k gB_k^T)   (MG_GRAD_SYM, full n x n), or
//          the gradient with respect to the lower-triangle entries
//          (MG_GRAD_LOWER; strict upper triangle not written).
// Same persistent queue and order as the forward kernel (its own counter);
// one workgroup of four waves per system; gX, gB and X staged in LDS.  A
// system whose info is non-zero gets NaN in every entry the mode writes.
// ---------------------------------------------------------------------------
template <typename T>
struct BatchBwdArgs {
    const int32_t* order;
    const int32_t* nsz;
    const T* const* L;
    const int64_t* ldl;
    const T* const* X;
    const int64_t* ldx;
    const T* const* GX;
    const int64_t* ldgx;
    T* const* GB;
    const int64_t* ldgb;
    T* const* GA;
    const int64_t* ldga;
    const int32_t* info;
    unsigned* counter;
    int batch;
    int nrhs;
    int mode;
};

template <typename T, int NRHS_MAX>
__global__ __launch_bounds__(256) void k_batched_backward(BatchBwdArgs<T> a) {
    __shared__ T bv[NRHS_MAX * BMAX];  // gX, then gB
    __shared__ T xv[NRHS_MAX * BMAX];  // X
    __shared__ T xacc[4][16];
    __shared__ int s_q;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, i = l & 15, g = l >> 4;
    for (;;) {
        if (tid == 0) s_q = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int q = s_q;
        if (q >= a.batch) break;
        const int sys = a.order[q];
        const int n = a.nsz[sys], nrhs = a.nrhs;
        const T* Lm = a.L[sys];
        const int64_t lda = a.ldl[sys];
        const bool bad = a.info[sys] != 0;
        for (int e = tid; e < NRHS_MAX * BMAX; e += 256) {
            const int row = e % BMAX, r = e / BMAX;
            const bool in = row < n && r < nrhs;
            bv[e] = in ? a.GX[sys][idx(row, r, a.ldgx[sys])] : (T)0;
            xv[e] = in ? a.X[sys][idx(row, r, a.ldx[sys])] : (T)0;
        }
        __syncthreads();
        const int nt = (n + 15) >> 4;
        if (!bad) {
            // ---- forward substitution L y = gX, block by block
            for (int j = 0; j < nt; ++j) {
                if (w == 0 && l < 16) {
                    const bool vl = 16 * j + l < n;
                    const T lj = vl ? Lm[idx(16 * j + l, 16 * j + l, lda)] : (T)1;
                    T lrow[16];
#pragma unroll
                    for (int c = 0; c < 16; ++c)
                        lrow[c] = (c < l && vl) ? Lm[idx(16 * j + l, 16 * j + c, lda)] : (T)0;
                    for (int r = 0; r < nrhs; ++r) {
                        T v = bv[r * BMAX + 16 * j + l];
#pragma unroll
                        for (int c = 0; c < 16; ++c) {
                            v = (c == l) ? v / lj : v;      // row c is final: y_c
                            const T yc = readlane(v, c);
                            v = v - lrow[c] * yc;           // lrow[c] = 0 unless c < l
                        }
                        bv[r * BMAX + 16 * j + l] = v;
                    }
                }
                __syncthreads();  // y_j in LDS
                // b_I -= L_Ij y_j for the tiles below, four waves
                for (int I = j + 1 + w; I < nt; I += 4) {
                    V4<T> t;
                    load_tile<T, T>(t, Lm, lda, 16 * I, 16 * j, n, n, false, false);
                    for (int r = 0; r < nrhs; ++r) {
                        T sm = 0;
#pragma unroll
                        for (int c = 0; c < 4; ++c) sm = sm + t[c] * bv[r * BMAX + 16 * j + tcol<T>(g, c)];
                        sm = sm + shfl(sm, l ^ 16);
                        sm = sm + shfl(sm, l ^ 32);
                        if (g == 0 && 16 * I + i < n) bv[r * BMAX + 16 * I + i] -= sm;
                    }
                }
                __syncthreads();
            }
            // ---- back substitution L^T gB = y, block by block from the bottom
            for (int j = nt - 1; j >= 0; --j) {
                for (int r = 0; r < nrhs; ++r) {
                    T part[4] = {0, 0, 0, 0};
                    for (int I = j + 1 + w; I < nt; I += 4) {
                        V4<T> y;
                        load_tile<T, T>(y, Lm, lda, 16 * I, 16 * j, n, n, false, false);
                        const T xi = (16 * I + i < n) ? bv[r * BMAX + 16 * I + i] : (T)0;
#pragma unroll
                        for (int c = 0; c < 4; ++c) part[c] = part[c] + y[c] * xi;
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        T v = part[c];
                        v = v + shfl(v, l ^ 1);
                        v = v + shfl(v, l ^ 2);
                        v = v + shfl(v, l ^ 4);
                        v = v + shfl(v, l ^ 8);
                        if (i == 0) xacc[w][tcol<T>(g, c)] = v;
                    }
                    __syncthreads();
                    if (w == 0 && l < 16) {
                        const T sum = ((xacc[0][l] + xacc[1][l]) + xacc[2][l]) + xacc[3][l];
                        T v = bv[r * BMAX + 16 * j + l] - sum;
                        const bool vl = 16 * j + l < n;
                        const T lj = vl ? Lm[idx(16 * j + l, 16 * j + l, lda)] : (T)1;
                        T lcl[16];
#pragma unroll
                        for (int c = 0; c < 16; ++c)
                            lcl[c] = (l < c && 16 * j + c < n) ? Lm[idx(16 * j + c, 16 * j + l, lda)] : (T)0;
#pragma unroll
                        for (int c = 15; c >= 0; --c) {
                            v = (c == l) ? v / lj : v;      // row c is final: gB_c
                            const T vc = readlane(v, c);
                            v = v - lcl[c] * vc;            // lcl[c] = 0 unless l < c
                        }
                        if (vl) bv[r * BMAX + 16 * j + l] = v;
                    }
                    __syncthreads();
                }
            }
        }
        // ---- outputs: gB, then gA from the rank-2 nrhs product
        T* GBm = a.GB[sys];
        const int64_t ldgb = a.ldgb[sys];
        for (int e = tid; e < n * nrhs; e += 256) {
            const int row = e % n, r = e / n;
            GBm[idx(row, r, ldgb)] = bad ? (T)NAN : bv[r * BMAX + row];
        }
        T* GAm = a.GA[sys];
        const int64_t ldga = a.ldga[sys];
        for (int e = tid; e < n * n; e += 256) {
            const int ii = e % n, jj = e / n;
            if (a.mode == MG_GRAD_LOWER && ii < jj) continue;
            T s1 = 0, s2 = 0;
            for (int r = 0; r < nrhs; ++r) {
                s1 = s1 + bv[r * BMAX + ii] * xv[r * BMAX + jj];
                s2 = s2 + xv[r * BMAX + ii] * bv[r * BMAX + jj];
            }
            T v;
            if (a.mode == MG_GRAD_SYM) v = (T)-0.5 * (s1 + s2);
            else v = ii > jj ? -(s1 + s2) : -s1;
            GAm[idx(ii, jj, ldga)] = bad ? (T)NAN : v;
        }
        __syncthreads();
    }
}

__global__ void k_reset_counter(unsigned* c) {
    if (threadIdx.x == 0) *c = 0u;
}

}  // namespace mg

// ===========================================================================
// Host side: plan, graph, autotuner.
// ===========================================================================
namespace mg {

// Diagonally dominant symmetric matrices for tuning runs: entries in
// [-1, 1) from a counter hash, diagonal n + 1 (strictly dominant, so SPD).
template <typename T>
__global__ void k_fill_dd(T* const* A, const int64_t* lda, const int32_t* nsz, int batch) {
    const int sys = blockIdx.y;
    if (sys >= batch) return;
    const int n = nsz[sys];
    T* M = A[sys];
    const int64_t ld = lda[sys];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n, j = e / n;
        uint32_t hsh = (uint32_t)(i > j ? i * 2654435761u + j * 40503u : j * 2654435761u + i * 40503u) ^ (uint32_t)sys;
        hsh ^= hsh >> 13;
        hsh *= 0x5bd1e995u;
        hsh ^= hsh >> 15;
        const T v = (T)((double)(hsh & 0xffffu) / 32768.0 - 1.0);
        M[idx(i, j, ld)] = (i == j) ? (T)(n + 1) : v;
    }
}

struct PlanCfg {
    int variant = 0;  // 0: four waves per system, 1: eight waves (k_batched_posv_w8)
    int grid_per_cu = 2;
    int order = 0;  // 0: longest first, 1: input order
};

}  // namespace mg

struct mg_batch_plan_s {
    mg_dtype dt = MG_F64;
    int batch = 0;
    int nrhs = 1;
    int cu = 256;
    mg::PlanCfg cfg;
    double tuned_ms = -1.0;
    std::vector<int32_t> n_host;
    int32_t *d_order = nullptr, *d_n = nullptr, *d_info = nullptr;
    void** d_A = nullptr;
    void** d_B = nullptr;
    int64_t *d_lda = nullptr, *d_ldb = nullptr;
    unsigned* d_counter = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace mg {

static void order_for(const std::vector<int32_t>& n, int mode, std::vector<int32_t>& ord) {
    ord.resize(n.size());
    for (size_t k = 0; k < n.size(); ++k) ord[k] = (int32_t)k;
    if (mode == 0)
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
}

template <typename T, int NR>
static mg_status build_graph(mg_batch_plan_s* p) {
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    MG_HIP(hipGraphCreate(&p->graph, 0));
    hipGraphNode_t n1 = nullptr, n2 = nullptr;
    void* a1[] = {(void*)&p->d_counter};
    hipKernelNodeParams k1{};
    k1.func = (void*)k_reset_counter;
    k1.gridDim = dim3(1);
    k1.blockDim = dim3(64);
    k1.sharedMemBytes = 0;
    k1.kernelParams = a1;
    k1.extra = nullptr;
    MG_HIP(hipGraphAddKernelNode(&n1, p->graph, nullptr, 0, &k1));
    static thread_local BatchArgs<T> args;  // copied into the node at creation
    args.order = p->d_order;
    args.nsz = p->d_n;
    args.A = (T* const*)p->d_A;
    args.lda = p->d_lda;
    args.B = (T* const*)p->d_B;
    args.ldb = p->d_ldb;
    args.info = p->d_info;
    args.counter = p->d_counter;
    args.batch = p->batch;
    args.nrhs = p->nrhs;
    void* a2[] = {(void*)&args};
    hipKernelNodeParams k2{};
    k2.func = p->cfg.variant ? (void*)k_batched_posv_w8<T, NR> : (void*)k_batched_posv<T, NR>;
    k2.gridDim = dim3((unsigned)std::max(1, std::min(p->batch, p->cfg.grid_per_cu * p->cu)));
    k2.blockDim = dim3(p->cfg.variant ? 64 * NW8 : 256);
    k2.sharedMemBytes = 0;
    k2.kernelParams = a2;
    k2.extra = nullptr;
    MG_HIP(hipGraphAddKernelNode(&n2, p->graph, &n1, 1, &k2));
    MG_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return MG_OK;
}

static mg_status plan_graph(mg_batch_plan_s* p) {
    std::vector<int32_t> ord;
    order_for(p->n_host, p->cfg.order, ord);
    MG_HIP(hipMemcpy(p->d_order, ord.data(), sizeof(int32_t) * p->batch, hipMemcpyHostToDevice));
    if (p->dt == MG_F64) return p->nrhs == 1 ? build_graph<double, 1>(p) : build_graph<double, 8>(p);
    return p->nrhs == 1 ? build_graph<float, 1>(p) : build_graph<float, 8>(p);
}

static std::string tune_key(const mg_batch_plan_s* p, const char* arch) {
    // the size histogram (16-wide buckets) identifies the workload shape
    std::vector<int> hist(BNT + 1, 0);
    for (int32_t v : p->n_host) ++hist[(v + 15) / 16];
    uint64_t h = 1469598103934665603ull;
    for (int v : hist) {
        h ^= (uint64_t)v;
        h *= 1099511628211ull;
    }
    char buf[256];
    snprintf(buf, sizeof(buf), "v2/%s/%s/nrhs%d/batch%d/%016llx", arch, p->dt == MG_F64 ? "f64" : "f32", p->nrhs,
             p->batch, (unsigned long long)h);
    return std::string(buf);
}

static bool cache_lookup(const char* path, const std::string& key, PlanCfg& cfg, double& ms) {
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char k[256];
    int var = 0, gpc = 0, ord = 0;
    double t = 0;
    bool found = false;
    while (fscanf(f, "%255s %d %d %d %lf", k, &var, &gpc, &ord, &t) == 5) {
        if (key == k && (var == 0 || var == 1) && gpc >= 1 && gpc <= 8 && (ord == 0 || ord == 1)) {
            cfg.variant = var;
            cfg.grid_per_cu = gpc;
            cfg.order = ord;
            ms = t;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void cache_store(const char* path, const std::string& key, const PlanCfg& cfg, double ms) {
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %.17g\n", key.c_str(), cfg.variant, cfg.grid_per_cu, cfg.order, ms);
    fclose(f);
}

// Time the candidate launch shapes on synthetic systems of the plan's sizes.
static mg_status autotune(mg_batch_plan_s* p, hipStream_t st) {
    const size_t es = p->dt == MG_F64 ? 8 : 4;
    size_t tot = 0;
    std::vector<size_t> offA(p->batch), offB(p->batch);
    for (int k = 0; k < p->batch; ++k) {
        offA[k] = tot;
        tot += align_up((size_t)p->n_host[k] * p->n_host[k] * es, 256);
    }
    for (int k = 0; k < p->batch; ++k) {
        offB[k] = tot;
        tot += align_up((size_t)std::max(1, p->n_host[k]) * p->nrhs * es, 256);
    }
    char* buf = nullptr;
    MG_HIP(hipMalloc(&buf, std::max<size_t>(tot, 256)));
    std::vector<void*> pa(p->batch), pb(p->batch);
    std::vector<int64_t> la(p->batch), lb(p->batch);
    for (int k = 0; k < p->batch; ++k) {
        pa[k] = buf + offA[k];
        pb[k] = buf + offB[k];
        la[k] = lb[k] = std::max<int32_t>(1, p->n_host[k]);
    }
    mg_status rc = MG_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        if (hipMemcpy(p->d_A, pa.data(), sizeof(void*) * p->batch, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_B, pb.data(), sizeof(void*) * p->batch, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_lda, la.data(), sizeof(int64_t) * p->batch, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_ldb, lb.data(), sizeof(int64_t) * p->batch, hipMemcpyHostToDevice) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = MG_ERR_HIP;
            break;
        }
        double best = 1e300;
        PlanCfg bestc = p->cfg;
        // candidates: the kernel variant (four or eight waves per system),
        // workgroups per CU (what the variant's registers and LDS allow) and
        // the queue order
        for (int var = 0; var <= 1 && rc == MG_OK; ++var)
        for (int gpc = 1; gpc <= (var ? 2 : 3) && rc == MG_OK; ++gpc) {
            for (int ord = 0; ord <= 1 && rc == MG_OK; ++ord) {
                p->cfg.variant = var;
                p->cfg.grid_per_cu = gpc;
                p->cfg.order = ord;
                if ((rc = plan_graph(p))) break;
                float tmin = 1e30f;
                for (int rep = 0; rep < 3; ++rep) {
                    const dim3 fg(64, (unsigned)p->batch);
                    if (p->dt == MG_F64)
                        hipLaunchKernelGGL(k_fill_dd<double>, fg, dim3(256), 0, st, (double* const*)p->d_A, p->d_lda,
                                           p->d_n, p->batch);
                    else
                        hipLaunchKernelGGL(k_fill_dd<float>, fg, dim3(256), 0, st, (float* const*)p->d_A, p->d_lda,
                                           p->d_n, p->batch);
                    if (hipGetLastError() != hipSuccess || hipEventRecord(e0, st) != hipSuccess ||
                        hipGraphLaunch(p->exec, st) != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess) {
                        rc = MG_ERR_HIP;
                        break;
                    }
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (rep > 0) tmin = std::min(tmin, ms);
                }
                if (rc == MG_OK && tmin < best) {
                    best = tmin;
                    bestc = p->cfg;
                }
            }
        }
        p->cfg = bestc;
        p->tuned_ms = best;
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    return rc;
}

}  // namespace mg

using namespace mg;

extern "C" {

mg_status mg_batch_plan_create(mg_handle_t h, mg_dtype dt, int32_t batch, const int64_t* n_host, int32_t nrhs,
                               const mg_tune_opts* opts, mg_batch_plan_t* plan) {
    if (!h) return -1;
    if (dt != MG_F64 && dt != MG_F32) return -2;
    if (batch < 0) return -3;
    if (!n_host && batch > 0) return -4;
    for (int k = 0; k < batch; ++k)
        if (n_host[k] < 0 || n_host[k] > BMAX) return -4;
    if (nrhs < 1 || nrhs > 8) return -5;
    if (!plan) return -7;
    *plan = nullptr;
    mg_batch_plan_s* p = new mg_batch_plan_s();
    p->dt = dt;
    p->batch = batch;
    p->nrhs = nrhs;
    p->cu = h->cu_count;
    p->n_host.assign(n_host, n_host + batch);
    const size_t nb = (size_t)std::max(1, batch);
    bool ok = hipMalloc(&p->d_order, nb * 4) == hipSuccess && hipMalloc(&p->d_n, nb * 4) == hipSuccess &&
              hipMalloc(&p->d_info, nb * 4) == hipSuccess && hipMalloc(&p->d_A, nb * 8) == hipSuccess &&
              hipMalloc(&p->d_B, nb * 8) == hipSuccess && hipMalloc(&p->d_lda, nb * 8) == hipSuccess &&
              hipMalloc(&p->d_ldb, nb * 8) == hipSuccess && hipMalloc(&p->d_counter, 256) == hipSuccess;
    if (ok && batch > 0)
        ok = hipMemcpy(p->d_n, p->n_host.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice) == hipSuccess;
    mg_status rc = ok ? MG_OK : MG_ERR_HIP;
    const int tune = opts ? opts->autotune : 1;
    if (rc == MG_OK && opts && opts->grid_per_cu > 0) p->cfg.grid_per_cu = std::min(8, opts->grid_per_cu);
    if (rc == MG_OK && opts && opts->order >= 0) p->cfg.order = opts->order ? 1 : 0;
    if (rc == MG_OK && opts && opts->variant >= 0) p->cfg.variant = opts->variant ? 1 : 0;
    if (rc == MG_OK && tune && batch > 0) {
        hipDeviceProp_t prop;
        char arch[64] = "gfx";
        if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
            snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
            for (char* c = arch; *c; ++c)
                if (*c == ':' || *c == ' ') *c = '_';
        }
        const char* path = (opts && opts->cache_path) ? opts->cache_path : nullptr;
        const std::string key = tune_key(p, arch);
        PlanCfg c;
        double ms = 0;
        if (cache_lookup(path, key, c, ms)) {
            p->cfg = c;
            p->tuned_ms = ms;
        } else if ((rc = autotune(p, h->stream)) == MG_OK) {
            cache_store(path, key, p->cfg, p->tuned_ms);
        }
    }
    if (rc == MG_OK && batch > 0) rc = plan_graph(p);
    if (rc != MG_OK) {
        mg_batch_plan_destroy(p);
        return rc;
    }
    *plan = p;
    return MG_OK;
}

mg_status mg_batch_plan_info(mg_batch_plan_t p, int32_t* grid_per_cu, int32_t* order, double* tuned_ms,
                             int32_t* variant) {
    if (!p) return -1;
    if (variant) *variant = p->cfg.variant;
    if (grid_per_cu) *grid_per_cu = p->cfg.grid_per_cu;
    if (order) *order = p->cfg.order;
    if (tuned_ms) *tuned_ms = p->tuned_ms;
    return MG_OK;
}

mg_status mg_posv_batched(mg_handle_t h, mg_batch_plan_t p, void* const* A_dev, const int64_t* lda_dev,
                          void* const* B_dev, const int64_t* ldb_dev, int32_t* info_dev) {
    if (!h) return -1;
    if (!p) return -2;
    if (p->batch == 0) return MG_OK;
    if (!A_dev) return -3;
    if (!lda_dev) return -4;
    if (!B_dev) return -5;
    if (!ldb_dev) return -6;
    if (!info_dev) return -7;
    hipStream_t st = h->stream;
    const size_t nb = (size_t)p->batch;
    MG_HIP(hipMemcpyAsync(p->d_A, A_dev, nb * 8, hipMemcpyDeviceToDevice, st));
    MG_HIP(hipMemcpyAsync(p->d_lda, lda_dev, nb * 8, hipMemcpyDeviceToDevice, st));
    MG_HIP(hipMemcpyAsync(p->d_B, B_dev, nb * 8, hipMemcpyDeviceToDevice, st));
    MG_HIP(hipMemcpyAsync(p->d_ldb, ldb_dev, nb * 8, hipMemcpyDeviceToDevice, st));
    mg_status rc;
    if ((rc = prof_begin(h, MG_PROF_BATCHED, st))) return rc;
    MG_HIP(hipGraphLaunch(p->exec, st));
    double fl = 0.0;
    for (int32_t v : p->n_host) {
        const double n = v;
        fl += n * n * n / 3 + n * n / 2 + n / 6 + 2.0 * n * n * p->nrhs;
    }
    if ((rc = prof_end(h, MG_PROF_BATCHED, fl, 0.0, st))) return rc;
    MG_HIP(hipMemcpyAsync(info_dev, p->d_info, nb * 4, hipMemcpyDeviceToDevice, st));
    return MG_OK;
}

mg_status mg_posv_batched_backward(mg_handle_t h, mg_batch_plan_t p, const void* const* L_dev, const int64_t* ldl_dev,
                                   const void* const* X_dev, const int64_t* ldx_dev, const void* const* GX_dev,
                                   const int64_t* ldgx_dev, void* const* GB_dev, const int64_t* ldgb_dev,
                                   void* const* GA_dev, const int64_t* ldga_dev, mg_grad_mode mode,
                                   const int32_t* info_dev) {
    if (!h) return -1;
    if (!p) return -2;
    if (mode != MG_GRAD_SYM && mode != MG_GRAD_LOWER) return -15;
    if (p->batch == 0) return MG_OK;
    if (!L_dev) return -3;
    if (!ldl_dev) return -4;
    if (!X_dev) return -5;
    if (!ldx_dev) return -6;
    if (!GX_dev) return -7;
    if (!ldgx_dev) return -8;
    if (!GB_dev) return -9;
    if (!ldgb_dev) return -10;
    if (!GA_dev) return -11;
    if (!ldga_dev) return -12;
    if (!info_dev) return -16;
    hipStream_t st = h->stream;
    unsigned* ctr = p->d_counter + 16;  // the backward queue's own counter
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, ctr);
    MG_LAUNCH_CHECK();
    const unsigned grid = (unsigned)std::max(1, std::min(p->batch, 2 * p->cu));
    if (p->dt == MG_F64) {
        BatchBwdArgs<double> a{p->d_order, p->d_n, (const double* const*)L_dev, ldl_dev, (const double* const*)X_dev,
                               ldx_dev, (const double* const*)GX_dev, ldgx_dev, (double* const*)GB_dev, ldgb_dev,
                               (double* const*)GA_dev, ldga_dev, info_dev, ctr, p->batch, p->nrhs, (int)mode};
        if (p->nrhs == 1) hipLaunchKernelGGL((k_batched_backward<double, 1>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_batched_backward<double, 8>), dim3(grid), dim3(256), 0, st, a);
    } else {
        BatchBwdArgs<float> a{p->d_order, p->d_n, (const float* const*)L_dev, ldl_dev, (const float* const*)X_dev,
                              ldx_dev, (const float* const*)GX_dev, ldgx_dev, (float* const*)GB_dev, ldgb_dev,
                              (float* const*)GA_dev, ldga_dev, info_dev, ctr, p->batch, p->nrhs, (int)mode};
        if (p->nrhs == 1) hipLaunchKernelGGL((k_batched_backward<float, 1>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_batched_backward<float, 8>), dim3(grid), dim3(256), 0, st, a);
    }
    MG_LAUNCH_CHECK();
    return MG_OK;
}

mg_status mg_batch_plan_destroy(mg_batch_plan_t p) {
    if (!p) return MG_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->d_order);
    (void)hipFree(p->d_n);
    (void)hipFree(p->d_info);
    (void)hipFree(p->d_A);
    (void)hipFree(p->d_B);
    (void)hipFree(p->d_lda);
    (void)hipFree(p->d_ldb);
    (void)hipFree(p->d_counter);
    delete p;
    return MG_OK;
}

}  // extern "C"
