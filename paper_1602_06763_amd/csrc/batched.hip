// Batched factorizations: many independent small matrices of uneven sizes in
// one launch, one workgroup per matrix, each matrix's recursion run on the
// device by that workgroup.
//
// The recursion is the one of the single-matrix routines (Sec. 3: split at
// n/2 rounded to the 64-wide matrix-core tile, leaves below the crossover;
// Sec. 5 keeps LAPACK's statement of xpotrf and xgetrf): Cholesky splits the
// matrix, LU splits the columns, and every off-leaf operation is a triangular
// solve or a product on the matrix cores. A matrix of at most 512 rows (SPD)
// or 256 rows (LU) stays in the L2 cache while its workgroup works on it, so
// the workgroup-level operations read their operands straight from memory:
//   - potf2 leaf: the unblocked Cholesky of a <= 64 block in LDS (potf2_block);
//   - LU leaf: a <= 32-column panel of all rows below the diagonal in LDS, one
//     row per thread, partial pivoting with the pivot rule of the single-matrix
//     panel (largest magnitude, lowest position on ties, a NaN never wins), the
//     rows interchanged in place, and the panel's interchanges applied to every
//     other column of the matrix before the recursion goes on (each interchange
//     reaches every column once, in order, as in LAPACK's dgetrf);
//   - triangular solves by 64-row blocks of the triangle (solve64 on 16 vectors
//     per wave) with the remaining rows updated on the matrix cores;
//   - products C -= A·B by 32×32 blocks per wave on the matrix cores, the lower
//     triangle only for the Cholesky update.
// The recursion depth is a template parameter, so the device code has no
// unbounded call stack.
#include "common.hpp"
#include "wg.hpp"

namespace rl {

constexpr int kBatchDepth = 6;   // deeper than any split chain of n <= 512

// Element (i, j) of a strided matrix view at p[i*r + j*c].
template <typename T>
struct WgMat {
    T *p;
    long long r, c;
    __device__ __forceinline__ T &operator()(long long i, long long j) const { return p[i * r + j * c]; }
};

template <typename T>
struct TrsmLds {
    T Nsh[64][65];
    T Xsh[4][64][17];
};

template <typename T>
struct PanelLdsB {
    T P[kBatchMaxGe][kLuLeaf + 1];
    unsigned long long rk[4];
    unsigned rp[4];
    int piv[kLuLeaf];   // panel row interchanged with row j at step j (j itself when none)
    int zfirst;         // first exactly zero pivot, global 1-based column; 0 = none
};

template <typename T>
union BatchLds {
    Potf2Lds<T> p2;
    TrsmLds<T> ts;
    PanelLdsB<T> pl;
};

extern __shared__ __attribute__((aligned(16))) unsigned char batch_smem[];

template <typename T>
__device__ __forceinline__ BatchLds<T> &blds() {
    return *reinterpret_cast<BatchLds<T> *>(batch_smem);
}

// C -= A·B by one workgroup on the matrix cores: C is M×N, A is M×K, B is
// K×N. Each wave takes 32×32 blocks of C in turn (four 16×16 accumulators,
// K in steps of 16); TRI computes and writes only the lower triangle of C.
// Operands are read with clamped indices (always inside the views) and
// zeroed outside them.
template <typename T, bool TRI>
__device__ __attribute__((noinline)) void wg_gemm(int M, int N, int K, WgMat<const T> A, WgMat<const T> B,
                                                  WgMat<T> C) {
    typedef LeafMfma<T> Op;
    typedef typename Op::acc_t acc_t;
    if (M <= 0 || N <= 0 || K <= 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int bm = (M + 31) / 32, bn = (N + 31) / 32;
    for (int blk = wave; blk < bm * bn; blk += 4) {
        const int bi = blk % bm, bj = blk / bm;
        if (TRI && bi < bj) continue;
        const int i0 = 32 * bi, j0 = 32 * bj;
        acc_t acc[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 2; ++t) acc[s][t] = acc_t{0, 0, 0, 0};
        for (int k0 = 0; k0 < K; k0 += 16) {
            T a[4][2], b[4][2];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = k0 + 4 * kk + lk;
                const int kc = min(k, K - 1);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int i = i0 + 16 * s + lr, j = j0 + 16 * s + lr;
                    const T av = A(min(i, M - 1), kc), bv = B(kc, min(j, N - 1));
                    a[kk][s] = (i < M && k < K) ? av : T(0);
                    b[kk][s] = (j < N && k < K) ? bv : T(0);
                }
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int t = 0; t < 2; ++t) acc[s][t] = Op::mma(a[kk][s], b[kk][t], acc[s][t]);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * s + Op::row(lane, v), j = j0 + 16 * t + lr;
                    if (i < M && j < N && (!TRI || i >= j)) C(i, j) -= acc[s][t][v];
                }
    }
}

// Solve N·x = b in place for nvec vectors by one workgroup: N is the t×t
// lower triangle N(i, j), i >= j (unit: its diagonal is taken as 1 and not
// read); element e of vector v is X(e, v). The triangle is taken in 64-row
// blocks in order: each block's diagonal part is staged in LDS (identity
// beyond the triangle) and solved for 64 vectors at a time (16 per wave),
// then the rows below it are updated on the matrix cores.
template <typename T>
__device__ __attribute__((noinline)) void wg_trsm(int t, int nvec, int unit, WgMat<const T> N, WgMat<T> X) {
    if (t <= 0 || nvec <= 0) return;
    TrsmLds<T> &L = blds<T>().ts;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T (*Xw)[17] = L.Xsh[wave];
    for (int J0 = 0; J0 < t; J0 += 64) {
        const int tb = min(64, t - J0);
        for (int idx = tid; idx < 64 * 64; idx += 256) {
            const int i = idx & 63, j = idx >> 6;
            T v = (i == j) ? T(1) : T(0);
            if (i < tb && j < tb) v = (j < i || (j == i && !unit)) ? N(J0 + i, J0 + j) : v;
            L.Nsh[i][j] = v;
        }
        __syncthreads();
        for (int v0 = 0; v0 < nvec; v0 += 64) {
            const int vb = v0 + 16 * wave;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = (lane >> 4) + 4 * u, q = lane & 15;
                Xw[e][q] = (e < tb && vb + q < nvec) ? X(J0 + e, vb + q) : T(0);
            }
            solve64<T, true>(L.Nsh, Xw, tb, unit, lane);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = (lane >> 4) + 4 * u, q = lane & 15;
                if (e < tb && vb + q < nvec) X(J0 + e, vb + q) = Xw[e][q];
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        if (J0 + tb < t)
            wg_gemm<T, false>(t - J0 - tb, nvec, tb,
                              WgMat<const T>{N.p + (J0 + tb) * N.r + J0 * N.c, N.r, N.c},
                              WgMat<const T>{X.p + J0 * X.r, X.r, X.c},
                              WgMat<T>{X.p + (J0 + tb) * X.r, X.r, X.c});
        __syncthreads();
    }
}

// Recursive Cholesky of the n×n block whose lower-factor element (i, j) is
// A[i*si + j*sj]: A11 = L11·L11ᵀ; A21 := A21·L11⁻ᵀ; A22 -= A21·A21ᵀ; A22 =
// L22·L22ᵀ. Returns 0 or the first failing column (1-based, as potf2_block).
template <typename T, int D>
__device__ __attribute__((noinline)) int potrf_b(int n, T *A, long long si, long long sj) {
    if (n <= kCholLeaf) {
        const int f = potf2_block(n, A, si, sj, blds<T>().p2);
        __syncthreads();
        return f;
    }
    if constexpr (D + 1 >= kBatchDepth) {
        return -1;
    } else {
        const int n1 = (int)split_size(n), n2 = n - n1;
        const int f = potrf_b<T, D + 1>(n1, A, si, sj);
        if (f) return f;
        // the rows of A21 are the vectors of the solve with the triangle L11
        wg_trsm<T>(n1, n2, 0, WgMat<const T>{A, si, sj}, WgMat<T>{A + n1 * si, sj, si});
        wg_gemm<T, true>(n2, n2, n1, WgMat<const T>{A + n1 * si, si, sj}, WgMat<const T>{A + n1 * si, sj, si},
                         WgMat<T>{A + n1 * si + n1 * sj, si, sj});
        __syncthreads();
        const int f2 = potrf_b<T, D + 1>(n2, A + n1 * si + n1 * sj, si, sj);
        return f2 > 0 ? n1 + f2 : f2;
    }
}

// LU panel of the columns c0..c0+w-1 (w <= 32) over the rows c0..n-1 of the
// n×n matrix A (leading dimension lda), one row per thread, in LDS. Per
// column j: the pivot among rows >= j, its row interchanged with row j when
// its value is nonzero, the column below divided by the pivot (left as it is
// for an exactly zero pivot), and the rank-1 update of the panel's remaining
// columns. ipiv gets the pivot rows (global, 1-based); afterwards the panel's
// interchanges are applied to every other column of the matrix. Returns the
// first exactly zero pivot column (global, 1-based) or 0.
template <typename T>
__device__ __attribute__((noinline)) int wg_getf2(int n, T *A, long long lda, int c0, int w, int *ipiv) {
    PanelLdsB<T> &P = blds<T>().pl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mp = n - c0;   // panel rows, <= kBatchMaxGe
    for (int q = 0; q < w; ++q)
        if (tid < mp) P.P[tid][q] = A[(c0 + tid) + (long long)(c0 + q) * lda];
    if (tid == 0) P.zfirst = 0;
    __syncthreads();
    for (int j = 0; j < w; ++j) {
        const int i = tid;
        const T xij = P.P[min(i, mp - 1)][j];
        const unsigned long long key = cand_key(fabs((double)xij), i >= j && i < mp);
        unsigned long long wk;
        unsigned wp;
        wave_winner(key, (unsigned)i, wk, wp);
        if (lane == 0) {
            P.rk[wave] = wk;
            P.rp[wave] = wp;
        }
        __syncthreads();
        unsigned long long bk = P.rk[0];
        unsigned bp = P.rp[0];
#pragma unroll
        for (int q = 1; q < 4; ++q)
            if (cand_wins(P.rk[q], P.rp[q], bk, bp)) { bk = P.rk[q]; bp = P.rp[q]; }
        const bool have = bk != 0;
        const bool useD = !have || bk == 1ull;   // no candidate, or an exact zero pivot
        const int p = have ? (int)bp : j;
        const bool nz = !have || bk != 1ull;     // NaN at the diagonal counts as nonzero
        const bool moved = !useD && p != j;
        if (tid == 0) {
            P.piv[j] = moved ? p : j;
            ipiv[c0 + j] = c0 + p + 1;
            if (!nz && P.zfirst == 0) P.zfirst = c0 + j + 1;
        }
        if (moved && tid < w) {
            const T t1 = P.P[j][tid];
            P.P[j][tid] = P.P[p][tid];
            P.P[p][tid] = t1;
        }
        __syncthreads();
        if (i > j && i < mp) {
            const T piv = P.P[j][j];
            const T x = P.P[i][j];
            const T l = nz ? x / piv : x;
            P.P[i][j] = l;
            for (int q = j + 1; q < w; ++q) P.P[i][q] -= l * P.P[j][q];
        }
        __syncthreads();
    }
    for (int q = 0; q < w; ++q)
        if (tid < mp) A[(c0 + tid) + (long long)(c0 + q) * lda] = P.P[tid][q];
    for (int col = tid; col < n; col += 256) {
        if (col >= c0 && col < c0 + w) continue;
        T *cp = A + (long long)col * lda + c0;
        for (int j = 0; j < w; ++j) {
            const int p = P.piv[j];
            if (p != j) {
                const T t1 = cp[j];
                cp[j] = cp[p];
                cp[p] = t1;
            }
        }
    }
    const int zf = P.zfirst;
    __syncthreads();
    return zf;
}

// Recursive LU with partial pivoting of the columns c0..c0+w-1 of the n×n
// matrix (rows c0..n-1): the left half, A12 := L11⁻¹·A12 (unit lower),
// A22 -= A21·A12, the right half. Returns the first exactly zero pivot column
// (global, 1-based) or 0; the factorization always completes.
template <typename T, int D>
__device__ __attribute__((noinline)) int getrf_b(int n, T *A, long long lda, int c0, int w, int *ipiv) {
    if (w <= kLuLeaf) return wg_getf2<T>(n, A, lda, c0, w, ipiv);
    if constexpr (D + 1 >= kBatchDepth) {
        return -1;
    } else {
        const int w1 = (int)split_size(w), w2 = w - w1;
        const int f1 = getrf_b<T, D + 1>(n, A, lda, c0, w1, ipiv);
        wg_trsm<T>(w1, w2, 1, WgMat<const T>{A + c0 + c0 * lda, 1, lda}, WgMat<T>{A + c0 + (c0 + w1) * lda, 1, lda});
        wg_gemm<T, false>(n - c0 - w1, w2, w1, WgMat<const T>{A + (c0 + w1) + c0 * lda, 1, lda},
                          WgMat<const T>{A + c0 + (c0 + w1) * lda, 1, lda},
                          WgMat<T>{A + (c0 + w1) + (c0 + w1) * lda, 1, lda});
        __syncthreads();
        const int f2 = getrf_b<T, D + 1>(n, A, lda, c0 + w1, w2, ipiv);
        return f1 ? f1 : f2;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void potrf_batched_k(int count, int upper, const int *__restrict__ nv,
                                                      T *const *__restrict__ Av, const int *__restrict__ ldav,
                                                      int *__restrict__ infov) {
    const int b = blockIdx.x;
    if (b >= count) return;
    const int n = nv[b], lda = ldav[b];
    int info = 0;
    if (n < 0 || n > kBatchMaxSpd) info = -2;
    else if (lda < max(1, n)) info = -4;
    else if (n > 0) {
        const long long si = upper ? lda : 1, sj = upper ? 1 : lda;
        info = potrf_b<T, 0>(n, Av[b], si, sj);
    }
    if (threadIdx.x == 0) infov[b] = info;
}

template <typename T>
__global__ __launch_bounds__(256) void getrf_batched_k(int count, const int *__restrict__ nv,
                                                      T *const *__restrict__ Av, const int *__restrict__ ldav,
                                                      int *const *__restrict__ ipivv, int *__restrict__ infov) {
    const int b = blockIdx.x;
    if (b >= count) return;
    const int n = nv[b], lda = ldav[b];
    int info = 0;
    if (n < 0 || n > kBatchMaxGe) info = -2;
    else if (lda < max(1, n)) info = -4;
    else if (n > 0) info = getrf_b<T, 0>(n, Av[b], lda, 0, n, ipivv[b]);
    if (threadIdx.x == 0) infov[b] = info;
}

template <typename T>
void potrf_batched(Ctx &c, bool upper, int count, const int *n, T *const *A, const int *lda, int *info) {
    if (count <= 0) return;
    const size_t shm = sizeof(BatchLds<T>);
    RL_CHECK(hipFuncSetAttribute((const void *)potrf_batched_k<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shm));
    rl_launch(c, potrf_batched_k<T>, dim3(count), dim3(256), (unsigned)shm, count, (int)upper, n, A, lda, info);
    RL_CHECK(hipGetLastError());
}

template <typename T>
void getrf_batched(Ctx &c, int count, const int *n, T *const *A, const int *lda, int *const *ipiv, int *info) {
    if (count <= 0) return;
    const size_t shm = sizeof(BatchLds<T>);
    RL_CHECK(hipFuncSetAttribute((const void *)getrf_batched_k<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shm));
    rl_launch(c, getrf_batched_k<T>, dim3(count), dim3(256), (unsigned)shm, count, n, A, lda, ipiv, info);
    RL_CHECK(hipGetLastError());
}

template void potrf_batched<double>(Ctx &, bool, int, const int *, double *const *, const int *, int *);
template void potrf_batched<float>(Ctx &, bool, int, const int *, float *const *, const int *, int *);
template void getrf_batched<double>(Ctx &, int, const int *, double *const *, const int *, int *const *, int *);
template void getrf_batched<float>(Ctx &, int, const int *, float *const *, const int *, int *const *, int *);

}  // namespace rl
