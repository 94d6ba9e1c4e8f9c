// Leaf kernels of the recursion: the unblocked Cholesky below the crossover
// size, the partial-pivoting LU panel with its pivot search, and the row
// interchanges (laswp) that the pivots induce on the rest of the matrix.
//
// The paper's recursion switches to LAPACK's unblocked kernels (dpotf2,
// dgetf2) once the problem is smaller than the crossover size c (Sec. 3,
// paragraph on the crossover size; Sec. 4). Here the crossover is set by
// on-chip capacity: a 64×64 FP64 diagonal block fits in one workgroup's LDS.
#include "common.hpp"

#include <climits>
#include <utility>
#include <type_traits>

namespace rl {

// ---------------------------------------------------------------------------
// potf2: unblocked Cholesky of an n×n diagonal block (n <= 64) in LDS.
// For uplo 'U' the block is read transposed (Uᵀ is lower) and written back
// transposed. On a pivot that is not > 0 (or NaN) the first failing global
// column off+k+1 is recorded in status->info, the block is written back as
// it stands (columns before k final, a_kk unchanged) and every later kernel
// of the call sees info != 0 and returns at once.
// ---------------------------------------------------------------------------
// One wave; lane i keeps row i of the block in registers. Column k: the
// diagonal comes from lane k (readlane), lanes below scale by its square root,
// and every lane subtracts l_ik·l_jk from its entries j > k, l_jk read from
// lane j. No LDS and no barrier: the wave runs the 64 steps in lockstep.
__device__ __forceinline__ double readlane_val(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_val(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

template <typename T>
__global__ __launch_bounds__(64) void potf2_k(int n, T *__restrict__ A, long long lda, int upper,
                                              long long off, DevStatus *st) {
    if (st->info) return;
    const int i = threadIdx.x;
    T a[64];
    // unconditional loads from clamped addresses, so all 64 are in flight together
    const int ic = i < n ? i : n - 1;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        const int jc = j < n ? j : n - 1;
        const T v = upper ? A[jc + (long long)ic * lda] : A[ic + (long long)jc * lda];
        a[j] = (i < n && j <= i) ? v : T(0);
    }
    int fail = 0;
#pragma unroll
    for (int k = 0; k < 64; ++k) {
        if (k < n && !fail) {
            const T akk = readlane_val(a[k], k);
            if (!(akk > T(0))) {
                fail = k + 1;
            } else {
                const T lkk = sqrt(akk);
                a[k] = (i == k) ? lkk : (i > k ? a[k] / lkk : a[k]);
#pragma unroll
                for (int j = k + 1; j < 64; ++j) {
                    const T ljk = readlane_val(a[k], j);
                    a[j] -= a[k] * ljk;   // entries j > i are never read or stored
                }
            }
        }
    }
    if (fail && i == 0) atomicCAS(&st->info, 0, (int)(off + fail));
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        if (i < n && j <= i) {
            if (upper) A[j + (long long)i * lda] = a[j];
            else A[i + (long long)j * lda] = a[j];
        }
    }
}

template <typename T>
void potf2(Ctx &c, char uplo, int n, T *A, long long lda, long long off) {
    if (plan_record(c, PK_POTF2, n, n, n)) return;
    if (n <= 0) return;
    trace_begin(c, PK_POTF2);
    hipLaunchKernelGGL((potf2_k<T>), dim3(1), dim3(64), 0, c.stream, n, A, lda,
                       (int)(uplo == 'U' || uplo == 'u'), off, c.dstat);
    RL_CHECK(hipGetLastError());
    trace_end(c, PK_POTF2, (double)n * n * n / 3.0, 8.0 * n * n);
}

template void potf2<double>(Ctx &, char, int, double *, long long, long long);
template void potf2<float>(Ctx &, char, int, float *, long long, long long);

// ---------------------------------------------------------------------------
// getf2 panel: partial-pivoting LU of the m_p × w panel A[c0:m, c0:c0+w]
// (w <= 32), rows distributed over G cooperating workgroups that each keep
// their R rows in LDS for the whole panel.
//
// Column j (diagonal row d = c0 + j):
//   1. each workgroup finds its largest |a_ij| over its rows i >= d (lowest
//      row index on ties; a NaN never wins);
//   2. if G > 1, workgroups publish (value, row, that row's w entries) and
//      the entries of row d, then meet at a counter barrier;
//   3. every workgroup reduces the G candidates to the pivot row p the same
//      way, so all agree; ipiv[d] = p + 1;
//   4. if the pivot is nonzero, rows d and p are exchanged across the panel
//      and the column below the diagonal is divided by it; otherwise info
//      records the first such column;
//   5. rank-1 update of the panel columns right of j.
// The source position of each row's content (before this panel's swaps) is
// tracked alongside the data and written to rowsrc, so that laswp can apply
// the panel's interchanges to the other columns with one gather.
// ---------------------------------------------------------------------------
constexpr int kPanelRows = 512;           // rows per workgroup
constexpr int kRecStride = kLuLeaf + 4;   // doubles per published record
constexpr int kPanelStageMax = 64;        // up to this many workgroups, records are staged in LDS

struct PanelArgs {
    long long m, c0;
    int w, G, R;
    long long lda;
    int *ipiv;
    int *rowsrc;
    DevStatus *st;
    double *rec;           // [2][G+1][kRecStride]
    unsigned int base;     // barrier counter value at entry
};

template <typename F, int... Js>
__device__ __forceinline__ void static_for(F &&f, std::integer_sequence<int, Js...>) {
    (f(std::integral_constant<int, Js>{}), ...);
}

__device__ __forceinline__ void cand_better(double v2, long long r2, double &v1, long long &r1) {
    if (v2 > v1 || (v2 == v1 && r2 < r1)) { v1 = v2; r1 = r2; }
}

__device__ __forceinline__ void pub(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double sub(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Rows live in registers: thread t owns panel rows t and t+256 of its
// workgroup's 512, all w <= 32 columns of each, so the scale and rank-1
// update of a column are register multiply-adds. The column loop is unrolled
// (register indices are compile-time); per-column LDS scratch is double
// buffered by column parity, so two workgroup barriers per column suffice
// when the panel fits one workgroup.
//
// Cross-workgroup exchange without cache-maintenance fences: records are
// written and read with device-coherent atomic accesses, every writer waits
// for its stores to complete (s_waitcnt) before the workgroup barrier, and
// only then is the arrival counter incremented. A reader that has seen the
// counter therefore reads complete records.
template <typename T>
__global__ __launch_bounds__(256) void getf2_panel_k(T *__restrict__ A, PanelArgs a) {
    constexpr int W = kLuLeaf;
    extern __shared__ unsigned char smem_raw[];
    double *recs = reinterpret_cast<double *>(smem_raw);  // [(G+1)][kRecStride] when staged
    __shared__ double red_v[2][4];
    __shared__ long long red_r[2][4];
    __shared__ T prow[2][W];   // pivot row entries
    __shared__ T drow[2][W];   // entries of row d before the interchange
    __shared__ int psrc_s[2], dsrc_s[2];
    __shared__ long long p_s[2];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = blockIdx.x, G = a.G, w = a.w;
    const long long c0 = a.c0, m = a.m;
    const long long rbeg = c0 + (long long)g * kPanelRows;
    DevStatus *st = a.st;

    T v[2][W];
    int src[2];
    long long grow[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        grow[k] = rbeg + tid + 256 * k;
        const bool in = grow[k] < m;
        const long long rc = in ? grow[k] : c0;
        src[k] = (int)grow[k];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const T x = A[rc + (c0 + (q < w ? q : 0)) * a.lda];
            v[k][q] = (in && q < w) ? x : T(0);
        }
    }

    // the column loop, unrolled at compile time so v[][] indices are constants
    auto column = [&](auto jc) __attribute__((always_inline)) {
        constexpr int j = decltype(jc)::value;
        if (j < w) {
            const int par = j & 1;
            const long long d = c0 + j;
            // 1. this workgroup's candidate: largest |a_ij|, rows i >= d, lowest row on ties
            double bv = -1.0;
            long long br = LLONG_MAX;
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if (grow[k] >= d && grow[k] < m) cand_better(fabs((double)v[k][j]), grow[k], bv, br);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const double v2 = __shfl_xor(bv, o);
                const long long r2 = __shfl_xor(br, o);
                cand_better(v2, r2, bv, br);
            }
            if (lane == 0) { red_v[par][wave] = bv; red_r[par][wave] = br; }
            __syncthreads();
            bv = red_v[par][0];
            br = red_r[par][0];
            for (int q = 1; q < 4; ++q) cand_better(red_v[par][q], red_r[par][q], bv, br);

            long long p;
            if (G == 1) {
                p = (br == LLONG_MAX) ? d : br;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (grow[k] == p) {
#pragma unroll
                        for (int q = 0; q < W; ++q) prow[par][q] = v[k][q];
                        psrc_s[par] = src[k];
                    }
                    if (grow[k] == d) {
#pragma unroll
                        for (int q = 0; q < W; ++q) drow[par][q] = v[k][q];
                        dsrc_s[par] = src[k];
                    }
                }
                if (tid == 0) p_s[par] = p;
            } else {
                // 2. publish this workgroup's candidate row (and row d), then meet
                double *slot = a.rec + ((size_t)(j & 1) * (G + 1)) * kRecStride;
                double *mine = slot + (size_t)g * kRecStride;
                if (br == LLONG_MAX && tid == 0) {
                    pub(&mine[0], -1.0);
                    pub(&mine[1], -1.0);
                }
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (br != LLONG_MAX && grow[k] == br) {
                        pub(&mine[0], bv);
                        pub(&mine[1], (double)br);   // row indices < 2^53 are exact
                        pub(&mine[2], (double)src[k]);
#pragma unroll
                        for (int q = 0; q < W; ++q) pub(&mine[4 + q], (double)v[k][q]);
                    }
                    if (grow[k] == d) {
                        double *dr = slot + (size_t)G * kRecStride;
                        pub(&dr[2], (double)src[k]);
#pragma unroll
                        for (int q = 0; q < W; ++q) pub(&dr[4 + q], (double)v[k][q]);
                    }
                }
                __builtin_amdgcn_s_waitcnt(0);   // this thread's stores have completed
                __syncthreads();
                if (tid == 0) {
                    __hip_atomic_fetch_add(&st->barrier, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned int target = a.base + (unsigned int)G * (unsigned int)(j + 1);
                    unsigned int spins = 0;
                    while (__hip_atomic_load(&st->barrier, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                        if (__hip_atomic_load(&st->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
                        if (++spins > (1u << 24)) {
                            atomicExch(&st->error, 1);
                            break;
                        }
                    }
                }
                __syncthreads();
                // 3. reduce the G candidates in every wave (all reach the same pivot)
                const bool staged = G <= kPanelStageMax;
                if (staged) {
                    // every record at once into LDS: a thread's loads are all issued
                    // before any is used, so they share one round trip
                    constexpr int kIt = ((kPanelStageMax + 1) * kRecStride + 255) / 256;
                    const int nrec = (G + 1) * kRecStride;
                    double tmp[kIt];
#pragma unroll
                    for (int u = 0; u < kIt; ++u) tmp[u] = sub(&slot[min(tid + u * 256, nrec - 1)]);
#pragma unroll
                    for (int u = 0; u < kIt; ++u) {
                        const int e = tid + u * 256;
                        if (e < nrec && e % kRecStride < 4 + w) recs[e] = tmp[u];
                    }
                    __syncthreads();
                }
                const double *base = staged ? recs : slot;
                double cv = -1.0;
                long long rr = LLONG_MAX;
                if (staged) {
                    for (int q = lane; q < G; q += 64) {
                        const double cr = base[q * kRecStride + 1];
                        if (cr >= 0.0) cand_better(base[q * kRecStride], (long long)cr, cv, rr);
                    }
                } else {
                    double vv[kPanelMaxWG / 64], rv[kPanelMaxWG / 64];
#pragma unroll
                    for (int u = 0; u < kPanelMaxWG / 64; ++u) {
                        const int q = min(lane + 64 * u, G - 1);
                        vv[u] = sub(&base[q * kRecStride]);
                        rv[u] = sub(&base[q * kRecStride + 1]);
                    }
#pragma unroll
                    for (int u = 0; u < kPanelMaxWG / 64; ++u)
                        if (lane + 64 * u < G && rv[u] >= 0.0) cand_better(vv[u], (long long)rv[u], cv, rr);
                }
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    const double v2 = __shfl_xor(cv, o);
                    const long long r2 = __shfl_xor(rr, o);
                    cand_better(v2, r2, cv, rr);
                }
                p = (rr == LLONG_MAX) ? d : rr;
                // row d's own record also serves when d is the pivot (or no row won)
                const double *dr = base + (size_t)G * kRecStride;
                const double *pr = (p == d) ? dr : base + (size_t)((p - c0) / kPanelRows) * kRecStride;
                if (tid < W) {
                    const double x1 = staged ? pr[4 + tid] : sub(&pr[4 + tid]);
                    const double x2 = staged ? dr[4 + tid] : sub(&dr[4 + tid]);
                    prow[par][tid] = (T)x1;
                    drow[par][tid] = (T)x2;
                }
                if (tid == 0) {
                    psrc_s[par] = (int)(staged ? pr[2] : sub(&pr[2]));
                    dsrc_s[par] = (int)(staged ? dr[2] : sub(&dr[2]));
                    p_s[par] = p;
                }
            }
            __syncthreads();
            p = p_s[par];
            if (g == 0 && tid == 0) a.ipiv[d] = (int)(p + 1);
            const T piv = prow[par][j];
            const bool nz = (piv != T(0));
            if (!nz && g == 0 && tid == 0) atomicCAS(&st->info, 0, (int)(d + 1));
            // 4+5. interchange, scale and rank-1 update, all in registers.
            // With a zero pivot nothing moves and row d supplies the U row.
            const T *urow = nz ? prow[par] : drow[par];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (nz && grow[k] == d) {
#pragma unroll
                    for (int q = 0; q < W; ++q) v[k][q] = prow[par][q];
                    src[k] = psrc_s[par];
                } else if (nz && p != d && grow[k] == p) {
#pragma unroll
                    for (int q = 0; q < W; ++q) v[k][q] = drow[par][q];
                    src[k] = dsrc_s[par];
                }
                if (grow[k] > d && grow[k] < m) {
                    T l = v[k][j];
                    if (nz) l = l / piv;
                    v[k][j] = l;
#pragma unroll
                    for (int q = j + 1; q < W; ++q) v[k][q] -= l * urow[q];
                }
            }
        }
    };
    static_for(column, std::make_integer_sequence<int, W>{});

#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (grow[k] < m) {
#pragma unroll
            for (int q = 0; q < W; ++q)
                if (q < w) A[grow[k] + (c0 + q) * a.lda] = v[k][q];
            a.rowsrc[grow[k]] = src[k];
        }
    }
}

template <typename T>
void getf2_panel(Ctx &c, long long m, int w, T *A, long long lda, long long c0, int *ipiv) {
    if (plan_record(c, PK_GETF2, m - c0, w, w)) return;
    const long long mp = m - c0;
    if (mp <= 0 || w <= 0) return;
    const int R = kPanelRows;   // two rows per thread, 256 threads
    const int G = (int)((mp + R - 1) / R);
    if (G > c.num_cu) { launch_error(hipErrorInvalidConfiguration); return; }
    PanelArgs a{};
    a.m = m; a.c0 = c0; a.w = w; a.G = G; a.R = R; a.lda = lda;
    a.ipiv = ipiv;
    a.rowsrc = c.rowsrc;
    a.st = c.dstat;
    a.rec = c.panel_rec;
    a.base = c.barrier_base;
    if (G > 1) c.barrier_base += (unsigned int)G * (unsigned int)w;
    const size_t shm =
        (G > 1 && G <= kPanelStageMax) ? (size_t)(G + 1) * kRecStride * sizeof(double) : 0;
    static size_t attr_bytes = 0;
    if (shm > attr_bytes) {
        RL_CHECK(hipFuncSetAttribute((const void *)getf2_panel_k<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        attr_bytes = shm;
    }
    trace_begin(c, PK_GETF2);
    hipLaunchKernelGGL((getf2_panel_k<T>), dim3(G), dim3(256), shm, c.stream, A, a);
    RL_CHECK(hipGetLastError());
    trace_end(c, PK_GETF2, (double)mp * w * w, 2.0 * sizeof(T) * mp * w);
}

template void getf2_panel<double>(Ctx &, long long, int, double *, long long, long long, int *);
template void getf2_panel<float>(Ctx &, long long, int, float *, long long, long long, int *);

// ---------------------------------------------------------------------------
// laswp after a panel: the panel's w interchanges, applied to every column
// outside the panel. The touched positions are the w diagonal rows and the w
// pivot rows; position i receives the content that sat at rowsrc[i] before
// the panel. Each workgroup gathers its columns' touched entries into
// registers, waits, then scatters them, so repeated pivot rows are harmless.
// Lanes run over the touched positions, so the w diagonal rows (contiguous
// in a column) are read and written coalesced.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void laswp_leaf_k(T *__restrict__ A, long long lda, long long c0, int w,
                                                    const int *__restrict__ ipiv,
                                                    const int *__restrict__ rowsrc, long long ncols,
                                                    const int *abort) {
    if (abort && *abort) return;
    constexpr int CPB = 32;  // columns per workgroup
    const int tid = threadIdx.x;
    const int slot = tid & 63, cq = tid >> 6;  // 64 slots × 4 column lanes
    long long pos = -1, srow = -1;
    if (slot < w) {
        pos = c0 + slot;
    } else if (slot < 2 * w) {
        const long long p = ipiv[c0 + slot - w] - 1;
        if (p >= c0 + w) pos = p;   // pivot rows inside the panel are covered above
    }
    if (pos >= 0) srow = rowsrc[pos];
    const long long lc0 = (long long)blockIdx.x * CPB;
    T vals[CPB / 4];
#pragma unroll
    for (int q = 0; q < CPB / 4; ++q) {
        const long long lc = lc0 + q * 4 + cq;
        const long long col = lc < c0 ? lc : lc + w;
        if (pos >= 0 && lc < ncols - w && srow != pos) vals[q] = A[srow + col * lda];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CPB / 4; ++q) {
        const long long lc = lc0 + q * 4 + cq;
        const long long col = lc < c0 ? lc : lc + w;
        if (pos >= 0 && lc < ncols - w && srow != pos) A[pos + col * lda] = vals[q];
    }
}

template <typename T>
void laswp_leaf(Ctx &c, long long ncols_total, T *A, long long lda, long long k0, int w, long long m,
                const int *ipiv, long long, long long) {
    if (plan_record(c, PK_LASWP, 2 * w, ncols_total - w, w)) return;
    const long long others = ncols_total - w;
    if (others <= 0 || w <= 0) return;
    (void)m;
    const int grid = (int)((others + 31) / 32);
    trace_begin(c, PK_LASWP);
    hipLaunchKernelGGL((laswp_leaf_k<T>), dim3(grid), dim3(256), 0, c.stream, A, lda, k0, w, ipiv,
                       c.rowsrc, ncols_total, (const int *)nullptr);
    RL_CHECK(hipGetLastError());
    trace_end(c, PK_LASWP, 0.0, 4.0 * sizeof(T) * w * others);
}

template void laswp_leaf<double>(Ctx &, long long, double *, long long, long long, int, long long,
                                 const int *, long long, long long);
template void laswp_leaf<float>(Ctx &, long long, float *, long long, long long, int, long long,
                                const int *, long long, long long);

// ---------------------------------------------------------------------------
// Row interchanges of a right-hand-side block (getrs): apply ipiv[k1..k2) in
// order (or in reverse) to the n columns of B. One thread per column walks the
// interchanges; right-hand sides are few, so this is a short kernel.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void laswp_rows_k(long long n, T *B, long long ldb, const int *ipiv, long long k1,
                             long long k2, int reverse) {
    const long long col = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= n) return;
    T *b = B + col * ldb;
    if (!reverse) {
        for (long long k = k1; k < k2; ++k) {
            const long long p = ipiv[k] - 1;
            if (p != k) { T t = b[k]; b[k] = b[p]; b[p] = t; }
        }
    } else {
        for (long long k = k2 - 1; k >= k1; --k) {
            const long long p = ipiv[k] - 1;
            if (p != k) { T t = b[k]; b[k] = b[p]; b[p] = t; }
        }
    }
}

// The same with the column held in LDS (one workgroup per column): the
// interchanges are a dependent chain, so each step should cost an LDS round
// trip rather than a memory one. rows: the rows the interchanges can touch.
template <typename T>
__global__ __launch_bounds__(256) void laswp_rows_lds_k(T *B, long long ldb, const int *ipiv, long long k1,
                                                        long long k2, long long rows, int reverse) {
    extern __shared__ unsigned char smem_raw[];
    T *v = reinterpret_cast<T *>(smem_raw);
    T *b = B + (long long)blockIdx.x * ldb;
    for (long long i = threadIdx.x; i < rows; i += 256) v[i] = b[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!reverse) {
            for (long long k = k1; k < k2; ++k) {
                const long long p = ipiv[k] - 1;
                const T t = v[k]; v[k] = v[p]; v[p] = t;
            }
        } else {
            for (long long k = k2 - 1; k >= k1; --k) {
                const long long p = ipiv[k] - 1;
                const T t = v[k]; v[k] = v[p]; v[p] = t;
            }
        }
    }
    __syncthreads();
    for (long long i = threadIdx.x; i < rows; i += 256) b[i] = v[i];
}

template <typename T>
void laswp_rows(Ctx &c, long long n, T *B, long long ldb, const int *ipiv, long long k1, long long k2,
                bool reverse) {
    if (plan_record(c, PK_LASWP, k2 - k1, n, 0)) return;
    if (n <= 0 || k2 <= k1) return;
    // square factorizations only: every pivot row lies in [k1, k2)
    const long long rows = k2;
    const size_t shm = (size_t)rows * sizeof(T);
    if (shm <= 150 * 1024) {
        static size_t attr = 0;
        if (shm > attr) {
            RL_CHECK(hipFuncSetAttribute((const void *)laswp_rows_lds_k<T>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
            attr = shm;
        }
        hipLaunchKernelGGL((laswp_rows_lds_k<T>), dim3((unsigned)n), dim3(256), shm, c.stream, B, ldb, ipiv, k1,
                           k2, rows, (int)reverse);
    } else {
        hipLaunchKernelGGL((laswp_rows_k<T>), dim3((unsigned)((n + 63) / 64)), dim3(64), 0, c.stream, n, B,
                           ldb, ipiv, k1, k2, (int)reverse);
    }
    RL_CHECK(hipGetLastError());
}

template void laswp_rows<double>(Ctx &, long long, double *, long long, const int *, long long,
                                 long long, bool);
template void laswp_rows<float>(Ctx &, long long, float *, long long, const int *, long long, long long,
                                bool);

}  // namespace rl
