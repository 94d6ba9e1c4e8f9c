// Batched factorizations: many independent small matrices of uneven sizes in
// one persistent launch, each matrix's recursion run on the device by one
// workgroup. The workgroups (as many as the chip holds at once) take matrices
// from a device work queue in order of size, largest first; the leaf size and
// the matrix-core tile edge are chosen per size bucket from a table measured
// on the device (batched_tune.hpp); the launch sequence of a call (queue
// reset, size order, persistent kernel) is captured once into a HIP graph and
// replayed for later calls with the same arguments.
//
// The recursion is the one of the single-matrix routines (Sec. 3: split at
// n/2 rounded to the 64-wide matrix-core tile, leaves below the crossover;
// Sec. 5 keeps LAPACK's statement of xpotrf and xgetrf): Cholesky splits the
// matrix, LU splits the columns, and every off-leaf operation is a triangular
// solve or a product on the matrix cores. A matrix of at most 512 rows (SPD)
// or 256 rows (LU) stays in the L2 cache while its workgroup works on it; the
// workgroup-level operations are:
//   - potf2 leaf: the unblocked Cholesky of a <= 64 block in LDS (potf2_block);
//   - LU leaf: a <= 32-column panel of all rows below the diagonal, one row
//     per thread in registers, partial pivoting with the pivot rule of the
//     single-matrix panel (largest magnitude, lowest position on ties, a NaN
//     never wins), the pivot row and row j trading places through LDS, and the
//     panel's interchanges applied to every other column of the matrix before
//     the recursion goes on (each interchange reaches every column once, in
//     order, as in LAPACK's dgetrf);
//   - triangular solves by 64-row blocks of the triangle (solve64 on 16 vectors
//     per wave) with the remaining rows updated on the matrix cores;
//   - products C -= A·B by 64×64 tiles per workgroup on the matrix cores, K
//     staged through LDS, the lower triangle only for the Cholesky update.
// The recursion runs from an explicit stack of frames in LDS, so every
// operation is inlined once and the kernel makes no calls.
#include "common.hpp"
#include "wg.hpp"
#include "batched_tune.hpp"

#include <mutex>

namespace rl {


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
    T F[kBatchMaxGe][kLuLeaf + 1];   // finished entries: multipliers below, U rows on and above the diagonal
    T slotP[kLuLeaf], slotJ[kLuLeaf];   // the pivot row's window; row j's window when the two trade places
    unsigned long long rk[4];
    unsigned rp[4];
    int piv[kLuLeaf];        // panel row interchanged with row j at step j (j itself when none)
    int pos[kBatchMaxGe];    // after the panel: the panel row whose content sits at each position
    int zfirst;              // first exactly zero pivot, global 1-based column; 0 = none
};

template <typename T>
struct GemmLdsB {
    T As[2][32][65];   // [buffer][k][row]
    T Bs[2][32][65];   // [buffer][k][column]
};

template <typename T>
union BatchLds {
    Potf2Lds<T> p2;
    TrsmLds<T> ts;
    PanelLdsB<T> pl;
    GemmLdsB<T> gm;
};

extern __shared__ __attribute__((aligned(16))) unsigned char batch_smem[];

template <typename T>
__device__ __forceinline__ BatchLds<T> &blds() {
    return *reinterpret_cast<BatchLds<T> *>(batch_smem);
}

// C -= A·B by one workgroup on the matrix cores: C is M×N, A is M×K, B is
// K×N. The workgroup takes tile×tile tiles of C in turn (tile 64 or 32, a
// run-time choice so that one body serves both; each wave a quarter, 16×16
// accumulators); K goes in chunks of 32 staged in LDS, double buffered, the
// next chunk's loads in flight while the current one is multiplied. Threads
// run along whichever index of an operand has unit stride, so the loads are
// contiguous for every view the recursion passes. TRI computes and writes
// only the lower triangle of C. Operands are read with clamped indices
// (always inside the views) and zeroed outside them.
template <typename T, bool TRI>
__device__ __forceinline__ void wg_gemm_t(int tile, int M, int N, int K, WgMat<const T> A, WgMat<const T> B,
                                          WgMat<T> C) {
    typedef LeafMfma<T> Op;
    typedef typename Op::acc_t acc_t;
    if (M <= 0 || N <= 0 || K <= 0) return;
    GemmLdsB<T> &L = blds<T>().gm;
    const int TL = tile == 32 ? 32 : 64, sh = tile == 32 ? 5 : 6;   // tile edge and its log2
    const int WT = TL >> 1, sub = WT >> 4, ld = TL >> 3;             // wave tile, 16-blocks per edge, loads
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int wi = WT * (wave & 1), wj = WT * (wave >> 1);   // this wave's quarter of the tile
    const bool a_rows = A.r == 1, b_cols = B.c == 1;
    const int tm = (M + TL - 1) >> sh, tn = (N + TL - 1) >> sh;
    for (int t = 0; t < tm * tn; ++t) {
        const int bi = t % tm, bj = t / tm;
        if (TRI && bi < bj) continue;   // uniform across the workgroup
        const int i0 = TL * bi, j0 = TL * bj;
        T ra[8], rb[8];
        auto fetch = [&](int k0) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = tid + 256 * u;
                const int ia = a_rows ? (idx & (TL - 1)) : (idx >> 5), ka = a_rows ? (idx >> sh) : (idx & 31);
                const int jb = b_cols ? (idx & (TL - 1)) : (idx >> 5), kb = b_cols ? (idx >> sh) : (idx & 31);
                const int gi = i0 + ia, gka = k0 + ka, gj = j0 + jb, gkb = k0 + kb;
                const bool on = u < ld;
                const T av = A(min(gi, M - 1), min(gka, K - 1)), bv = B(min(gkb, K - 1), min(gj, N - 1));
                ra[u] = (on && gi < M && gka < K) ? av : T(0);
                rb[u] = (on && gj < N && gkb < K) ? bv : T(0);
            }
        };
        auto stage = [&](int buf) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (u < ld) {
                    const int idx = tid + 256 * u;
                    const int ia = a_rows ? (idx & (TL - 1)) : (idx >> 5), ka = a_rows ? (idx >> sh) : (idx & 31);
                    const int jb = b_cols ? (idx & (TL - 1)) : (idx >> 5), kb = b_cols ? (idx >> sh) : (idx & 31);
                    L.As[buf][ka][ia] = ra[u];
                    L.Bs[buf][kb][jb] = rb[u];
                }
            }
        };
        acc_t acc[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[s][q] = acc_t{0, 0, 0, 0};
        fetch(0);
        int buf = 0;
        for (int k0 = 0; k0 < K; k0 += 32) {
            stage(buf);
            __syncthreads();
            if (k0 + 32 < K) fetch(k0 + 32);
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = 4 * kk + lk;
                if (sub == 2) {
                    T a[2], b[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        a[s] = L.As[buf][k][wi + 16 * s + lr];
                        b[s] = L.Bs[buf][k][wj + 16 * s + lr];
                    }
#pragma unroll
                    for (int s = 0; s < 2; ++s)
#pragma unroll
                        for (int q = 0; q < 2; ++q) acc[s][q] = Op::mma(a[s], b[q], acc[s][q]);
                } else {
                    acc[0][0] = Op::mma(L.As[buf][k][wi + lr], L.Bs[buf][k][wj + lr], acc[0][0]);
                }
            }
            buf ^= 1;
        }
        __syncthreads();   // every wave is done with both buffers before the next tile stages
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + wi + 16 * s + Op::row(lane, v), j = j0 + wj + 16 * q + lr;
                    if (s < sub && q < sub && i < M && j < N && (!TRI || i >= j)) C(i, j) -= acc[s][q][v];
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
__device__ __forceinline__ void wg_trsm(int t, int nvec, int unit, WgMat<const T> N, WgMat<T> X, int tile) {
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
            wg_gemm_t<T, false>(tile, t - J0 - tb, nvec, tb,
                              WgMat<const T>{N.p + (J0 + tb) * N.r + J0 * N.c, N.r, N.c},
                              WgMat<const T>{X.p + J0 * X.r, X.r, X.c},
                              WgMat<T>{X.p + (J0 + tb) * X.r, X.r, X.c});
        __syncthreads();
    }
}

// Frames of the recursion, run by an explicit stack that every thread keeps
// identically in LDS: kind 0 = factor (off, n), kind 1 = the update between
// the halves (off, n, n1). A call pushes its right half, the update and its
// left half, so the left half is taken first, as in the recursive call.
struct BFrame {
    int kind, off, n, n1;
};
constexpr int kBatchStack = 3 * 8 + 1;   // three frames per level, 8 levels cover n <= 512

// Recursive Cholesky of the n×n matrix whose lower-factor element (i, j) is
// A[i*si + j*sj]: A11 = L11·L11ᵀ; A21 := A21·L11⁻ᵀ; A22 -= A21·A21ᵀ; A22 =
// L22·L22ᵀ. Returns 0 or the first failing column (1-based, as potf2_block);
// nothing after a failing leaf runs.
template <typename T>
__device__ __forceinline__ int potrf_b(int n, T *A, long long si, long long sj, BFrame *stk, int leaf, int tile) {
    int sp = 0;
    if (threadIdx.x == 0) stk[0] = BFrame{0, 0, n, 0};
    sp = 1;
    __syncthreads();
    while (sp > 0) {
        const BFrame f = stk[--sp];
        __syncthreads();   // every thread has read the frame before it is overwritten
        T *Ao = A + f.off * si + f.off * sj;
        if (f.kind == 0 && f.n <= leaf) {
            const int r = potf2_block(f.n, Ao, si, sj, blds<T>().p2);
            __syncthreads();
            if (r) return f.off + r;
        } else if (f.kind == 0) {
            const int n1 = (int)split_size(f.n);
            if (threadIdx.x == 0) {
                stk[sp] = BFrame{0, f.off + n1, f.n - n1, 0};
                stk[sp + 1] = BFrame{1, f.off, f.n, n1};
                stk[sp + 2] = BFrame{0, f.off, n1, 0};
            }
            sp += 3;
            __syncthreads();
        } else {
            const int n1 = f.n1, n2 = f.n - f.n1;
            // the rows of A21 are the vectors of the solve with the triangle L11
            wg_trsm<T>(n1, n2, 0, WgMat<const T>{Ao, si, sj}, WgMat<T>{Ao + n1 * si, sj, si}, tile);
            wg_gemm_t<T, true>(tile, n2, n2, n1, WgMat<const T>{Ao + n1 * si, si, sj},
                             WgMat<const T>{Ao + n1 * si, sj, si}, WgMat<T>{Ao + n1 * si + n1 * sj, si, sj});
            __syncthreads();
        }
    }
    return 0;
}

// LU panel of the columns c0..c0+w-1 (w <= 32) over the rows c0..n-1 of the
// n×n matrix A (leading dimension lda). Thread t owns the row at panel
// position t and keeps its not yet factored columns in registers as a sliding
// window (x[q] is column j+q at step j). Per column j: the pivot among rows
// >= j (largest magnitude, lowest position on ties, a NaN never wins); when
// its value is nonzero the pivot row and row j trade places (their windows
// through LDS, their finished multipliers in LDS); the column below is divided
// by the pivot (left as it is for an exactly zero pivot) and the rank-1 update
// is applied to the windows. ipiv gets the pivot rows (global, 1-based). The
// finished panel is written once at the end, and the panel's interchanges are
// then applied to every other column of the matrix as one gather of the
// touched rows (at most 2w per column). Returns the first exactly zero pivot
// column (global, 1-based) or 0.
template <typename T>
__device__ __forceinline__ int wg_getf2(int n, T *A, long long lda, int c0, int w, int *ipiv) {
    constexpr int W = kLuLeaf;
    PanelLdsB<T> &P = blds<T>().pl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mp = n - c0;   // panel rows, <= kBatchMaxGe
    T x[W];
    {
        const int r = min(tid, mp - 1);
#pragma unroll
        for (int q = 0; q < W; ++q) x[q] = A[(c0 + r) + (long long)(c0 + min(q, w - 1)) * lda];
    }
    if (tid == 0) P.zfirst = 0;
    for (int j = 0; j < w; ++j) {
        const unsigned long long key = cand_key(fabs((double)x[0]), tid >= j && tid < mp);
        unsigned long long wk;
        unsigned wp;
        wave_winner(key, (unsigned)tid, wk, wp);
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
        // the pivot row's window to slotP; row j's to slotJ when they trade places;
        // the finished multipliers of the two rows trade places as well
        if (tid == (moved ? p : j)) {
#pragma unroll
            for (int q = 0; q < W; ++q) P.slotP[q] = x[q];
        }
        if (moved && tid == j) {
#pragma unroll
            for (int q = 0; q < W; ++q) P.slotJ[q] = x[q];
        }
        if (moved && tid < j) {
            const T t1 = P.F[j][tid];
            P.F[j][tid] = P.F[p][tid];
            P.F[p][tid] = t1;
        }
        __syncthreads();
        if (moved && tid == p) {
#pragma unroll
            for (int q = 0; q < W; ++q) x[q] = P.slotJ[q];
        }
        // row j of U, and the multipliers and rank-1 update below it
        if (tid < w - j) P.F[j][j + tid] = P.slotP[tid];
        const T piv = P.slotP[0];
        const T l = nz ? x[0] / piv : x[0];
        const bool below = tid > j && tid < mp;
        if (below) P.F[tid][j] = l;
        const T lk = below ? l : T(0);
#pragma unroll
        for (int q = 0; q < W - 1; ++q) x[q] = x[q + 1] - lk * P.slotP[q + 1];
    }
    __syncthreads();
    if (tid < mp) {
        for (int q = 0; q < w; ++q) A[(c0 + tid) + (long long)(c0 + q) * lda] = P.F[tid][q];
        P.pos[tid] = tid;
    }
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j < w; ++j) {
            const int p = P.piv[j];
            if (p != j) {
                const int t1 = P.pos[j];
                P.pos[j] = P.pos[p];
                P.pos[p] = t1;
            }
        }
    }
    __syncthreads();
    // every other column: position e of the touched set takes the content of row pos[e]
    {
        const int e = tid & 63, cg = tid >> 6;
        const int te = e < w ? e : (e < 2 * w ? P.piv[e - w] : 0);
        const int se = P.pos[te];
        const bool act = e < 2 * w && se != te;
        for (int col0 = 0; col0 < n; col0 += 32) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int col = min(col0 + cg + 4 * u, n - 1);
                v[u] = A[(c0 + se) + (long long)col * lda];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int col = col0 + cg + 4 * u;
                if (act && col < n && (col < c0 || col >= c0 + w)) A[(c0 + te) + (long long)col * lda] = v[u];
            }
            __syncthreads();
        }
    }
    const int zf = P.zfirst;
    __syncthreads();
    return zf;
}

// Recursive LU with partial pivoting of the n×n matrix (columns split in
// halves, rows from the diagonal down): the left half, A12 := L11⁻¹·A12
// (unit lower), A22 -= A21·A12, the right half; frames as for the Cholesky
// (off = first column, n = columns, n1 = left half). Returns the first exactly
// zero pivot column (global, 1-based) or 0; the factorization always
// completes.
template <typename T>
__device__ __forceinline__ int getrf_b(int n, T *A, long long lda, int *ipiv, BFrame *stk, int leaf, int tile) {
    int sp = 0, info = 0;
    if (threadIdx.x == 0) stk[0] = BFrame{0, 0, n, 0};
    sp = 1;
    __syncthreads();
    while (sp > 0) {
        const BFrame f = stk[--sp];
        __syncthreads();
        const int c0 = f.off;
        if (f.kind == 0 && f.n <= leaf) {
            const int r = wg_getf2<T>(n, A, lda, c0, f.n, ipiv);
            if (info == 0) info = r;
        } else if (f.kind == 0) {
            const int w1 = (int)split_size(f.n);
            if (threadIdx.x == 0) {
                stk[sp] = BFrame{0, c0 + w1, f.n - w1, 0};
                stk[sp + 1] = BFrame{1, c0, f.n, w1};
                stk[sp + 2] = BFrame{0, c0, w1, 0};
            }
            sp += 3;
            __syncthreads();
        } else {
            const int w1 = f.n1, w2 = f.n - f.n1;
            wg_trsm<T>(w1, w2, 1, WgMat<const T>{A + c0 + c0 * lda, 1, lda},
                       WgMat<T>{A + c0 + (c0 + w1) * lda, 1, lda}, tile);
            wg_gemm_t<T, false>(tile, n - c0 - w1, w2, w1, WgMat<const T>{A + (c0 + w1) + c0 * lda, 1, lda},
                              WgMat<const T>{A + c0 + (c0 + w1) * lda, 1, lda},
                              WgMat<T>{A + (c0 + w1) + (c0 + w1) * lda, 1, lda});
            __syncthreads();
        }
    }
    return info;
}

// Order of the work queue: matrix indices sorted by size, largest first (one
// counting sort in one workgroup; sizes outside [0, KMAX] go last, where the
// factorization kernels reject them), so the longest factorizations start
// first and the short ones fill the tail. The order within one size is
// arbitrary; every matrix is factored by one workgroup either way, so results
// do not depend on it.
template <int KMAX>
__global__ __launch_bounds__(1024) void batch_order_k(int count, const int *__restrict__ nv,
                                                      int *__restrict__ perm) {
    __shared__ int start[KMAX + 2];
    const int tid = threadIdx.x;
    auto key = [&](int i) {
        const int n = nv[i];
        return (n < 0 || n > KMAX) ? KMAX + 1 : KMAX - n;
    };
    for (int k = tid; k < KMAX + 2; k += 1024) start[k] = 0;
    __syncthreads();
    for (int i = tid; i < count; i += 1024) atomicAdd(&start[key(i)], 1);
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int k = 0; k < KMAX + 2; ++k) {
            const int h = start[k];
            start[k] = s;
            s += h;
        }
    }
    __syncthreads();
    for (int i = tid; i < count; i += 1024) perm[atomicAdd(&start[key(i)], 1)] = i;
}

// Queue reset of a call (a kernel, so that the call's graph holds no memset).
__global__ void batch_queue_reset_k(unsigned *q) {
    if (threadIdx.x == 0) *q = 0u;
}

// Persistent batched Cholesky: each workgroup takes the next matrix of the
// size order from the queue until the queue is exhausted (every workgroup
// reaches that exit). Per matrix, the leaf size and tile edge of its size
// bucket.
template <typename T>
__global__ __launch_bounds__(256, 2) void potrf_batched_k(int count, int upper, const int *__restrict__ nv,
                                                      T *const *__restrict__ Av, const int *__restrict__ ldav,
                                                      int *__restrict__ infov, const int *__restrict__ perm,
                                                      unsigned *queue, BatchTune tune) {
    __shared__ BFrame stk[kBatchStack];
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int item = item_s;
        __syncthreads();   // read by every thread before the next matrix's fetch overwrites it
        if (item >= count) return;
        const int b = perm[item];
        const int n = nv[b], lda = ldav[b];
        int info = 0;
        if (n < 0 || n > kBatchMaxSpd) info = -2;
        else if (lda < max(1, n)) info = -4;
        else if (n > 0) {
            const long long si = upper ? lda : 1, sj = upper ? 1 : lda;
            const int bk = batch_bucket(n);
            info = potrf_b<T>(n, Av[b], si, sj, stk, tune.leaf[bk], tune.tile[bk]);
        }
        if (threadIdx.x == 0) infov[b] = info;
        __syncthreads();   // LDS of this matrix is free before the next one starts
    }
}

template <typename T>
__global__ __launch_bounds__(256, 2) void getrf_batched_k(int count, const int *__restrict__ nv,
                                                      T *const *__restrict__ Av, const int *__restrict__ ldav,
                                                      int *const *__restrict__ ipivv, int *__restrict__ infov,
                                                      const int *__restrict__ perm, unsigned *queue,
                                                      BatchTune tune) {
    __shared__ BFrame stk[kBatchStack];
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= count) return;
        const int b = perm[item];
        const int n = nv[b], lda = ldav[b];
        int info = 0;
        if (n < 0 || n > kBatchMaxGe) info = -2;
        else if (lda < max(1, n)) info = -4;
        else if (n > 0) {
            const int bk = batch_bucket(n);
            info = getrf_b<T>(n, Av[b], lda, ipivv[b], stk, tune.leaf[bk], tune.tile[bk]);
        }
        if (threadIdx.x == 0) infov[b] = info;
        __syncthreads();
    }
}

// ---- host side: tuning table, launch sequence, graph cache -------------------

namespace {

// routines: 0 dpotrf, 1 spotrf, 2 dgetrf, 3 sgetrf
BatchTune g_tune[4] = {kTuneDefault[0], kTuneDefault[1], kTuneDefault[2], kTuneDefault[3]};
bool g_graphs_on = true;

struct BatchGraph {
    bool used = false;
    int device = -1, routine = -1, count = 0, upper = 0, grid = 0;
    const void *n = nullptr, *A = nullptr, *lda = nullptr, *ipiv = nullptr, *info = nullptr;
    const void *ws = nullptr;
    BatchTune tune{};
    hipGraphExec_t exec = nullptr;
    unsigned long long stamp = 0;
};
constexpr int kGraphCache = 16;
BatchGraph g_cache[kGraphCache];
unsigned long long g_stamp = 0;
hipStream_t g_cap[16] = {};
std::mutex g_bmu;

bool same_tune(const BatchTune &a, const BatchTune &b) {
    for (int i = 0; i < kBatchBuckets; ++i)
        if (a.leaf[i] != b.leaf[i] || a.tile[i] != b.tile[i]) return false;
    return true;
}

template <typename K>
int batch_grid(Ctx &c, K kernel, size_t shm, int count) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, shm) != hipSuccess || per < 1) per = 1;
    const long long g = (long long)per * c.num_cu;
    return (int)(count < g ? count : g);
}

}  // namespace

bool batched_tune_set(int routine, int bucket, int leaf, int tile) {
    if (routine < 0 || routine > 3 || bucket < 0 || bucket >= kBatchBuckets) return false;
    const bool lu = routine >= 2;
    if (lu ? (leaf != 16 && leaf != 32) : (leaf != 32 && leaf != 64)) return false;
    if (tile != 32 && tile != 64) return false;
    std::lock_guard<std::mutex> lk(g_bmu);
    g_tune[routine].leaf[bucket] = (unsigned char)leaf;
    g_tune[routine].tile[bucket] = (unsigned char)tile;
    return true;
}

bool batched_tune_get(int routine, int bucket, int *leaf, int *tile) {
    if (routine < 0 || routine > 3 || bucket < 0 || bucket >= kBatchBuckets) return false;
    std::lock_guard<std::mutex> lk(g_bmu);
    if (leaf) *leaf = g_tune[routine].leaf[bucket];
    if (tile) *tile = g_tune[routine].tile[bucket];
    return true;
}

void batched_graphs(bool on) {
    std::lock_guard<std::mutex> lk(g_bmu);
    g_graphs_on = on;
}

void batched_release() {
    std::lock_guard<std::mutex> lk(g_bmu);
    for (auto &g : g_cache) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = BatchGraph();
    }
    for (auto &s : g_cap) {
        if (s) (void)hipStreamDestroy(s);
        s = nullptr;
    }
}

// The launch sequence of one batched call on stream s: queue reset, size
// order into the workspace, the persistent kernel.
template <typename T, bool LU>
static void batch_sequence(hipStream_t s, int grid, size_t shm, int count, int upper, const int *n, T *const *A,
                           const int *lda, int *const *ipiv, int *info, int *perm, unsigned *queue,
                           BatchTune tune) {
    constexpr int KMAX = LU ? kBatchMaxGe : kBatchMaxSpd;
    hipLaunchKernelGGL(batch_queue_reset_k, dim3(1), dim3(64), 0, s, queue);
    hipLaunchKernelGGL(batch_order_k<KMAX>, dim3(1), dim3(1024), 0, s, count, n, perm);
    if constexpr (LU)
        hipLaunchKernelGGL(getrf_batched_k<T>, dim3(grid), dim3(256), (unsigned)shm, s, count, n, A, lda, ipiv, info,
                           (const int *)perm, queue, tune);
    else
        hipLaunchKernelGGL(potrf_batched_k<T>, dim3(grid), dim3(256), (unsigned)shm, s, count, upper, n, A, lda,
                           info, (const int *)perm, queue, tune);
}

template <typename T, bool LU>
static void batched_call(Ctx &c, int routine, int count, int upper, const int *n, T *const *A, const int *lda,
                         int *const *ipiv, int *info) {
    if (count <= 0) return;
    // workspace: the size order (count ints), then the queue counter
    const size_t pbytes = ((size_t)count * sizeof(int) + 255) / 256 * 256;
    char *ws = (char *)workspace(c, kSlotBatchOrder, pbytes + 256);
    if (!ws) return;
    int *perm = (int *)ws;
    unsigned *queue = (unsigned *)(ws + pbytes);
    const size_t shm = sizeof(BatchLds<T>);
    const void *kfn = LU ? (const void *)getrf_batched_k<T> : (const void *)potrf_batched_k<T>;
    RL_CHECK(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    const int grid = LU ? batch_grid(c, getrf_batched_k<T>, shm, count) : batch_grid(c, potrf_batched_k<T>, shm, count);
    BatchTune tune;
    bool graphs;
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        tune = g_tune[routine];
        graphs = g_graphs_on;
    }
    if (!graphs || c.trace) {
        trace_begin(c, PK_OTHER);
        batch_sequence<T, LU>(c.stream, grid, shm, count, upper, n, A, lda, ipiv, info, perm, queue, tune);
        RL_CHECK(hipGetLastError());
        trace_end(c, PK_OTHER, 0.0, 0.0);
        return;
    }
    std::lock_guard<std::mutex> lk(g_bmu);
    BatchGraph *hit = nullptr, *slot = &g_cache[0];
    for (auto &g : g_cache) {
        if (g.used && g.device == c.device && g.routine == routine && g.count == count && g.upper == upper &&
            g.grid == grid && g.n == n && g.A == A && g.lda == lda && g.ipiv == ipiv && g.info == info &&
            g.ws == ws && same_tune(g.tune, tune)) {
            hit = &g;
            break;
        }
        if (!g.used || g.stamp < slot->stamp) slot = &g;
    }
    if (!hit) {
        // capture the sequence once on a private stream, keep the executable graph
        hipStream_t &cap = g_cap[c.device];
        if (!cap) RL_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        if (!cap) return;
        hipGraph_t graph = nullptr;
        RL_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        batch_sequence<T, LU>(cap, grid, shm, count, upper, n, A, lda, ipiv, info, perm, queue, tune);
        RL_CHECK(hipGetLastError());
        RL_CHECK(hipStreamEndCapture(cap, &graph));
        if (!graph) return;
        hipGraphExec_t exec = nullptr;
        RL_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
        if (!exec) return;
        if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
        *slot = BatchGraph();
        slot->used = true;
        slot->device = c.device; slot->routine = routine; slot->count = count; slot->upper = upper;
        slot->grid = grid;
        slot->n = n; slot->A = A; slot->lda = lda; slot->ipiv = ipiv; slot->info = info; slot->ws = ws;
        slot->tune = tune;
        slot->exec = exec;
        hit = slot;
    }
    hit->stamp = ++g_stamp;
    RL_CHECK(hipGraphLaunch(hit->exec, c.stream));
}

template <typename T>
void potrf_batched(Ctx &c, bool upper, int count, const int *n, T *const *A, const int *lda, int *info) {
    batched_call<T, false>(c, std::is_same<T, double>::value ? 0 : 1, count, (int)upper, n, A, lda,
                           (int *const *)nullptr, info);
}

template <typename T>
void getrf_batched(Ctx &c, int count, const int *n, T *const *A, const int *lda, int *const *ipiv, int *info) {
    batched_call<T, true>(c, std::is_same<T, double>::value ? 2 : 3, count, 0, n, A, lda, ipiv, info);
}

template void potrf_batched<double>(Ctx &, bool, int, const int *, double *const *, const int *, int *);
template void potrf_batched<float>(Ctx &, bool, int, const int *, float *const *, const int *, int *);
template void getrf_batched<double>(Ctx &, int, const int *, double *const *, const int *, int *const *, int *);
template void getrf_batched<float>(Ctx &, int, const int *, float *const *, const int *, int *const *, int *);

}  // namespace rl
