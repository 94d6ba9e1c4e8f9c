// Leaf kernels of the recursion: the unblocked Cholesky below the crossover
// size, the partial-pivoting LU panel with its pivot search, and the row
// interchanges (laswp) that the pivots induce on the rest of the matrix.
//
// The paper's recursion switches to LAPACK's unblocked kernels (dpotf2,
// dgetf2) once the problem is smaller than the crossover size c (Sec. 3,
// paragraph on the crossover size; Sec. 4). Here the crossover is set by
// on-chip capacity: a 64×64 FP64 diagonal block fits in one workgroup's LDS.
#include "common.hpp"
#include "wg.hpp"

#include <climits>
#include <utility>
#include <type_traits>

namespace rl {

// ---------------------------------------------------------------------------
// potf2: Cholesky of an n×n diagonal block (n <= 64) in one workgroup, the
// block held in LDS. For uplo 'U' the block is read transposed (Uᵀ is lower)
// and written back transposed. On a pivot that is not > 0 (or NaN) the first
// failing global column off+k+1 is recorded in status->info, the block is
// written back as it stands (columns before k final, column k holding its
// updated pivot) and every later kernel of the call sees info != 0 and
// returns at once. The factorization itself is potf2_block (wg.hpp).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void potf2_k(int n, T *__restrict__ A, long long lda, int upper,
                                               long long off, DevStatus *st) {
    if (st->info) return;
    __shared__ Potf2Lds<T> L;
    // element (i, j) of the lower factor lives at A[i + j*lda] ('L') or A[j + i*lda] ('U')
    const long long si = upper ? lda : 1, sj = upper ? 1 : lda;
    const int fail = potf2_block(n, A, si, sj, L);
    if (fail && threadIdx.x == 0) atomicCAS(&st->info, 0, (int)(off + fail));
}

// ---------------------------------------------------------------------------
// The bottom node of the recursion, 64 < n <= 128, in one launch: the same
// steps as the recursion takes there (split n1 = split_size(n), n2 = n - n1,
// both <= 64), each on LDS: potf2 of A11 (potf2_factor); A21 := A21·L11⁻ᵀ by
// the triangular-solve leaf's substitution (solve64, the rows of A21 as the
// right-hand sides, 16 per wave); A22 -= L21·L21ᵀ on the matrix cores over
// the whole K range in order, as the GEMM kernel sums it; potf2 of A22. A
// failing pivot in A11 leaves A21 and A22 untouched, as the recursion's later
// kernels do when they see info set.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void potf2x2_k(int n, T *__restrict__ A, long long lda, int upper,
                                                 long long off, DevStatus *st) {
    if (st->info) return;
    typedef LeafMfma<T> Op;
    typedef typename Op::acc_t acc_t;
    __shared__ Potf2Lds<T> L1, L2;
    __shared__ T X[4][64][17];   // A21: row n1 + 16w + q of the block, column e at X[w][e][q]
    const long long si = upper ? lda : 1, sj = upper ? 1 : lda;
    const int n1 = (int)split_size(n), n2 = n - n1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T *A21 = A + n1 * si, *A22 = A + n1 * si + n1 * sj;
    potf2_stage(n1, A, si, sj, L1.S);
    potf2_stage(n2, A22, si, sj, L2.S);
    {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            if (upper) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            const int r = 16 * wave + q;
            v[u] = A21[min(r, n2 - 1) * si + min(e, n1 - 1) * sj];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            if (upper) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            X[wave][e][q] = (16 * wave + q < n2 && e < n1) ? v[u] : T(0);
        }
    }
    if (tid == 0) { L1.fail_s = 0; L2.fail_s = 0; }
    __syncthreads();
    const int f1 = potf2_factor(n1, L1);
    if (f1) {
        potf2_store(n1, A, si, sj, L1.S);
        if (tid == 0) atomicCAS(&st->info, 0, (int)(off + f1));
        return;
    }
    solve64<T, true>(L1.S, X[wave], n1, 0, lane);
    __syncthreads();
    // A22 -= L21·L21ᵀ, lower 16×16 tiles (I, J), J <= I
    for (int tt = wave; tt < 10; tt += 4) {
        int I = 0, a0 = 0;
        while (a0 + I + 1 <= tt) { a0 += I + 1; ++I; }
        const int J = tt - a0;
        acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int k4 = 0; k4 < 16; ++k4) {
            const int k = 4 * k4 + (lane >> 4);
            acc = Op::mma(X[I][k][lane & 15], X[J][k][lane & 15], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) L2.S[16 * I + Op::row(lane, v)][16 * J + (lane & 15)] -= acc[v];
    }
    __syncthreads();
    const int f2 = potf2_factor(n2, L2);
    potf2_store(n1, A, si, sj, L1.S);
    potf2_store(n2, A22, si, sj, L2.S);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        int e, q;
        if (upper) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
        else { q = lane & 15; e = (lane >> 4) + 4 * u; }
        const int r = 16 * wave + q;
        if (r < n2 && e < n1) A21[r * si + e * sj] = X[wave][e][q];
    }
    if (f2 && tid == 0) atomicCAS(&st->info, 0, (int)(off + n1 + f2));
}

template <typename T>
void potf2x2(Ctx &c, char uplo, int n, T *A, long long lda, long long off) {
    if (plan_record(c, PK_POTF2, n, n, n)) return;
    trace_kernel_begin(c);
    rl_launch(c, potf2x2_k<T>, dim3(1), dim3(256), 0, n, A, lda, (int)(uplo == 'U' || uplo == 'u'), off, c.dstat);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_POTF2, (double)n * n * n / 3.0, 8.0 * n * n);
}

template void potf2x2<double>(Ctx &, char, int, double *, long long, long long);
template void potf2x2<float>(Ctx &, char, int, float *, long long, long long);

template <typename T>
void potf2(Ctx &c, char uplo, int n, T *A, long long lda, long long off) {
    if (plan_record(c, PK_POTF2, n, n, n)) return;
    if (n <= 0) return;
    trace_kernel_begin(c);
    rl_launch(c, potf2_k<T>, dim3(1), dim3(256), 0, n, A, lda, (int)(uplo == 'U' || uplo == 'u'), off, c.dstat);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_POTF2, (double)n * n * n / 3.0, 8.0 * n * n);
}

template void potf2<double>(Ctx &, char, int, double *, long long, long long);
template void potf2<float>(Ctx &, char, int, float *, long long, long long);

// ---------------------------------------------------------------------------
// getf2 panel: partial-pivoting LU of the m_p × w panel A[c0:m, c0:c0+w]
// (w <= 32; 16 for the complex types) with dgetf2's semantics (Sec. 5 keeps
// LAPACK's statement of the problem): for column j, with d = c0 + j,
//   - the pivot p is the first position i >= d with the largest |a_ij|
//     (|re| + |im| for complex entries, as izamax picks) (a NaN
//     never wins; with no candidate at all, p = d); ipiv[d] = p + 1;
//   - if a_pj != 0 (NaN counts as nonzero) rows d and p are interchanged and
//     the column below the diagonal is divided by the pivot; otherwise info
//     records the first such column and nothing moves;
//   - rank-1 update of the columns right of j with row d.
//
// Rows are spread over G cooperating workgroups of 256 threads; thread t owns
// the rows t and t+256 of its workgroup's 512-row chunk ("contents") for the
// whole panel and keeps the not yet factored columns of each in registers as
// a sliding window (x[q] is column j+q at step j), so every step addresses
// the same registers and the step loop stays a short runtime loop.
//
// Interchanges move no data: each content carries its current position. At
// step j the pivot content retires to position d as row j of U, the content
// that sat at d takes the pivot's old position, and every other live content
// is scaled and updated. Finished entries (multipliers, and U rows) collect
// in LDS and every content is written to its final position at the end; the
// source row of every position goes to rowsrc so that laswp can apply the
// panel's interchanges to the other columns with one gather.
//
// Workgroups exchange, per step, one record each: the key and position of
// their best candidate and that row's window. Every 64-bit word of a record
// carries the step's epoch in its upper half, so a reader polls exactly the
// words it needs until their epochs match: no counter, no fence, no reset.
// The winner is reduced identically in every workgroup, so all agree. Each
// step updates the next column alone first, searches it and publishes the
// next record, and only then updates the rest of the window, which thereby
// runs while the record crosses the grid (the arithmetic per entry is the
// same as updating the whole window at once).
// ---------------------------------------------------------------------------
struct PanelArgs {
    long long m, c0, lda;
    int w, G;
    int *ipiv;
    int *rowsrc;
    DevStatus *st;
    unsigned long long *rec;   // [kLuLeaf][kRecSlots][kRecWords]
    unsigned int epoch;        // step j publishes with epoch + j
};

constexpr unsigned int kPanelSpin = 1u << 22;   // poll bound per word group
constexpr int kPanelStageG = 12;                // up to this many workgroups, records are read whole
                                                // (one round trip); above, the headers and then
                                                // the winner's row (two round trips but far fewer
                                                // polled words: 3.73 against 3.94 us per column
                                                // at 32 workgroups, even at 16, slower at 8)

__device__ __forceinline__ void pubw(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long subw(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Scalar traits of the panel: window width W, the value's 32-bit chunks for
// the epoch-tagged words (NC of them), the pivot magnitude, the quotient and
// the update x - l·u, zero, and a broadcast from one lane. The complex
// instances (the c/z types) take 16 columns (their window then holds as many
// registers as the real one) and the magnitude |re| + |im|.
template <typename T> struct PanelT;
template <> struct PanelT<double> {
    static constexpr int W = kLuLeaf, NC = 2;
    static __device__ __forceinline__ unsigned get(double v, int h) {
        return h ? (unsigned)__double2hiint(v) : (unsigned)__double2loint(v);
    }
    static __device__ __forceinline__ double mag(double v) { return fabs(v); }
    static __device__ __forceinline__ double div(double a, double p) { return a / p; }
    static __device__ __forceinline__ double fms(double x, double l, double u) { return x - l * u; }
    static __device__ __forceinline__ double zero() { return 0.0; }
    static __device__ __forceinline__ double bcast(double v, int l) { return lane_bcast(v, l); }
};
template <> struct PanelT<float> {
    static constexpr int W = kLuLeaf, NC = 1;
    static __device__ __forceinline__ unsigned get(float v, int) { return __float_as_uint(v); }
    static __device__ __forceinline__ double mag(float v) { return fabs((double)v); }
    static __device__ __forceinline__ float div(float a, float p) { return a / p; }
    static __device__ __forceinline__ float fms(float x, float l, float u) { return x - l * u; }
    static __device__ __forceinline__ float zero() { return 0.f; }
    static __device__ __forceinline__ float bcast(float v, int l) { return lane_bcast(v, l); }
};
template <typename R> struct PanelT<cx<R>> {
    static constexpr int W = kZLuLeaf, NC = 2 * PanelT<R>::NC;
    static __device__ __forceinline__ unsigned get(cx<R> v, int h) {
        return h < PanelT<R>::NC ? PanelT<R>::get(v.re, h) : PanelT<R>::get(v.im, h - PanelT<R>::NC);
    }
    // |re| + |im| in the working precision, as the oracle and the one-workgroup
    // complex panel decide it
    static __device__ __forceinline__ double mag(cx<R> v) { return (double)cabs1(v); }
    static __device__ __forceinline__ cx<R> div(cx<R> a, cx<R> p) { return cdiv(a, p); }
    static __device__ __forceinline__ cx<R> fms(cx<R> x, cx<R> l, cx<R> u) { return csub(x, cmul(l, u)); }
    static __device__ __forceinline__ cx<R> zero() { return cx<R>{R(0), R(0)}; }
    static __device__ __forceinline__ cx<R> bcast(cx<R> v, int l) {
        return cx<R>{lane_bcast(v.re, l), lane_bcast(v.im, l)};
    }
};

// Per-step LDS of the panel, double buffered by step parity: a wave that has
// moved on to the next step never overwrites what a slower wave still reads.
template <typename T>
struct PanelStep {
    T cand[4][PanelT<T>::W];       // window of each wave's best candidate
    unsigned long long rk[2][4];   // [workgroup / grid reduction][wave]
    unsigned rp[2][4];
    int rc[2][4][2];
};

template <typename T>
__global__ __launch_bounds__(256) void getf2_panel_k(T *__restrict__ A, PanelArgs a) {
    typedef PanelT<T> P;
    constexpr int W = P::W;
    constexpr int R = kPanelRows;
    constexpr int NC = P::NC;
    constexpr int LDSW = W + 1;                // row stride of the finished-entry array
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T *F = reinterpret_cast<T *>(smem_raw);   // multipliers [R][LDSW]
    __shared__ PanelStep<T> ps[2];
    __shared__ T Urow[W][W + 1];               // row j of U, from the step that retired it
    __shared__ T dwin[W];                      // row d's window when it drives the update
    __shared__ __attribute__((aligned(16))) unsigned ub[W * NC];   // pivot window from a record
    __shared__ __attribute__((aligned(16))) unsigned stage[kPanelStageG * kRecWords];   // records, whole
    __shared__ int abort_s;
    __shared__ unsigned pvs[W];   // pivot position of every step
    __shared__ int zfirst;        // first step with an exact zero pivot

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = blockIdx.x, G = a.G, w = a.w;
    const long long c0 = a.c0;
    const long long rbeg = c0 + (long long)g * R;
    const int nr = (int)min((long long)R, a.m - rbeg);   // >= 1 for every launched workgroup
    DevStatus *st = a.st;
    if (tid == 0) { abort_s = 0; zfirst = -1; }

    T x[2][W];
    unsigned pos[2];
    int cid[2], rstep[2];
    bool act[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int r = tid + 256 * k;
        const long long rr = rbeg + min(r, nr - 1);
#pragma unroll
        for (int q = 0; q < W; ++q) x[k][q] = A[rr + (c0 + min(q, w - 1)) * a.lda];
        pos[k] = (unsigned)(rbeg + r);
        cid[k] = (int)(rbeg + r);
        act[k] = r < nr;
        rstep[k] = -1;
    }
    // all loads in flight before any is used
    asm volatile("" ::: "memory");

    // The workgroup's best candidate of one step, from the first live column's
    // values v[k] of the two contents: thread, wave (the winning lane writes the
    // candidate's window to LDS through put_window), then the workgroup (after
    // one barrier, every thread reduces the four waves' results itself).
    unsigned long long bk;
    unsigned bp;
    int bc, bwv;
    auto cand_step = [&](PanelStep<T> &S2, const T *v, auto put_window) {
        unsigned long long key = 0;
        unsigned kp = 0xFFFFFFFFu;
        int kc = -1, kb = 0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const unsigned long long kk = cand_key(P::mag(v[k]), act[k]);
            if (kk != 0 && cand_wins(kk, pos[k], key, kp)) { key = kk; kp = pos[k]; kc = cid[k]; kb = k; }
        }
        unsigned long long wk;
        unsigned wp;
        const int wl = wave_winner(key, kp, wk, wp);
        const int wc = __builtin_amdgcn_readlane(kc, wl < 0 ? 0 : wl);
        if (lane == wl && kb == 0) put_window(S2.cand[wave], 0);
        if (lane == wl && kb == 1) put_window(S2.cand[wave], 1);
        if (lane == 0) {
            S2.rk[0][wave] = wk;
            S2.rp[0][wave] = wp;
            S2.rc[0][wave][0] = wl < 0 ? -1 : wc;
            S2.rc[0][wave][1] = wave;
        }
        __syncthreads();
        bk = S2.rk[0][0];
        bp = S2.rp[0][0];
        bc = S2.rc[0][0][0];
        bwv = 0;
#pragma unroll
        for (int q = 1; q < 4; ++q)
            if (cand_wins(S2.rk[0][q], S2.rp[0][q], bk, bp)) { bk = S2.rk[0][q]; bp = S2.rp[0][q]; bc = S2.rc[0][q][0]; bwv = q; }
    };
    // publish this workgroup's candidate of step jj: one word per thread
    auto publish = [&](int jj, PanelStep<T> &S2) {
        const unsigned long long ETj = (unsigned long long)(a.epoch + (unsigned)jj) << 32;
        unsigned long long *mine = a.rec + ((size_t)jj * kRecSlots + g) * kRecWords;
        if (tid < 4 + NC * W) {
            unsigned v;
            if (tid == 0) v = (unsigned)bk;
            else if (tid == 1) v = (unsigned)(bk >> 32);
            else if (tid == 2) v = bp;
            else if (tid == 3) v = (unsigned)bc;
            else v = P::get(S2.cand[bwv][(tid - 4) / NC], (tid - 4) % NC);
            pubw(&mine[tid], ETj | v);
        }
    };

    // step 0's candidate, as loaded
    {
        T v0[2] = {x[0][0], x[1][0]};
        cand_step(ps[0], v0, [&](T *dst, int k) {
#pragma unroll
            for (int q = 0; q < W; ++q) dst[q] = k ? x[1][q] : x[0][q];
        });
        if (G > 1) publish(0, ps[0]);
    }

    for (int j = 0; j < w; ++j) {
        PanelStep<T> &S = ps[j & 1];
        const unsigned d = (unsigned)(c0 + j);
        const int nw = w - j;   // live window width
        const unsigned E = a.epoch + (unsigned)j;
        const unsigned long long ET = (unsigned long long)E << 32;

        int src_g = -1;   // workgroup whose record holds the pivot row (G > 1)
        T spiv = P::zero();   // the winner's first window entry, from the staged records
        if (G > 1) {
            if (G <= kPanelStageG) {
                // every record whole in one round trip: the headers, one word per
                // thread, and the windows, a wave per record and a lane per word
                const int nwin = NC * nw;
                constexpr int NQ = kPanelStageG / 4;
                const unsigned long long *hp =
                    &a.rec[((size_t)j * kRecSlots + min(tid >> 2, G - 1)) * kRecWords + (tid & 3)];
                const unsigned long long *wpq[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    wpq[q] = &a.rec[((size_t)j * kRecSlots + min(wave + 4 * q, G - 1)) * kRecWords + 4 +
                                    min(lane, nwin - 1)];
                // words of workgroups that do not exist are not loaded (they read as fresh)
                auto issue = [&](unsigned long long &h, unsigned long long *wv) {
                    h = ET;
                    if (tid < 4 * G) h = subw(hp);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        wv[q] = ET;
                        if (wave + 4 * q < G) wv[q] = subw(wpq[q]);
                    }
                };
                auto fresh = [&](unsigned long long h, const unsigned long long *wv) {
                    bool ok = tid >= 4 * G || (unsigned)(h >> 32) == E;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        ok = ok && (wave + 4 * q >= G || lane >= nwin || (unsigned)(wv[q] >> 32) == E);
                    return ok;
                };
                auto stage_in = [&](unsigned long long h, const unsigned long long *wv) {
                    if (tid < 4 * G) stage[(tid >> 2) * kRecWords + (tid & 3)] = (unsigned)h;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (wave + 4 * q < G && lane < nwin) stage[(wave + 4 * q) * kRecWords + 4 + lane] = (unsigned)wv[q];
                };
                unsigned long long ha, wa[NQ];
                unsigned spins = 0;
                while (true) {
                    issue(ha, wa);
                    if (fresh(ha, wa)) { stage_in(ha, wa); break; }
                    if (++spins > kPanelSpin) { atomicExch(&st->error, 1); abort_s = 1; break; }
                    if ((spins & 1023u) == 0 && __hip_atomic_load(&st->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        abort_s = 1;
                        break;
                    }
                }
                __syncthreads();
                if (abort_s) return;
                // every wave reduces the headers itself (lanes over workgroups)
                unsigned long long tk = 0;
                unsigned tp = 0xFFFFFFFFu;
                int tc = -1;
                T w0 = P::zero();
                if (lane < G) {
                    const unsigned *h = &stage[lane * kRecWords];
                    tk = ((unsigned long long)h[1] << 32) | h[0];
                    tp = h[2];
                    tc = (int)h[3];
                    w0 = reinterpret_cast<const T *>(&stage[lane * kRecWords + 4])[0];
                }
                unsigned long long gk2;
                unsigned gp2;
                const int gl = wave_winner(tk, tp, gk2, gp2);
                bk = gk2;
                bp = gp2;
                bc = __builtin_amdgcn_readlane(tc, gl < 0 ? 0 : gl);
                spiv = P::bcast(w0, gl < 0 ? 0 : gl);
                src_g = gl;
            } else {
            // every workgroup's header, one per thread
            unsigned long long tk = 0;
            unsigned tp = 0xFFFFFFFFu;
            int tc = -1;
            if (tid < G) {
                const unsigned long long *rr = a.rec + ((size_t)j * kRecSlots + tid) * kRecWords;
                unsigned long long h0, h1, h2, h3;
                unsigned spins = 0;
                while (true) {
                    h0 = subw(&rr[0]); h1 = subw(&rr[1]); h2 = subw(&rr[2]); h3 = subw(&rr[3]);
                    if ((unsigned)(h0 >> 32) == E && (unsigned)(h1 >> 32) == E && (unsigned)(h2 >> 32) == E &&
                        (unsigned)(h3 >> 32) == E)
                        break;
                    if (++spins > kPanelSpin) { atomicExch(&st->error, 1); abort_s = 1; break; }
                    if ((spins & 1023u) == 0 && __hip_atomic_load(&st->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        abort_s = 1;
                        break;
                    }
                }
                tk = ((unsigned long long)(unsigned)h1 << 32) | (unsigned)h0;
                tp = (unsigned)h2;
                tc = (int)(unsigned)h3;
            }
            // winner over the workgroups, with its content and workgroup index
            unsigned long long gk2;
            unsigned gp2;
            const int gl = wave_winner(tk, tp, gk2, gp2);
            const int gc2 = __builtin_amdgcn_readlane(tc, gl < 0 ? 0 : gl);
            if (lane == 0) {
                S.rk[1][wave] = gk2;
                S.rp[1][wave] = gp2;
                S.rc[1][wave][0] = gl < 0 ? -1 : gc2;
                S.rc[1][wave][1] = gl < 0 ? -1 : 64 * wave + gl;
            }
            __syncthreads();
            if (abort_s) return;
            bk = S.rk[1][0]; bp = S.rp[1][0]; bc = S.rc[1][0][0]; src_g = S.rc[1][0][1];
#pragma unroll
            for (int q = 1; q < 4; ++q)
                if (cand_wins(S.rk[1][q], S.rp[1][q], bk, bp)) {
                    bk = S.rk[1][q]; bp = S.rp[1][q]; bc = S.rc[1][q][0]; src_g = S.rc[1][q][1];
                }
            }
        }

        // -- the pivot decision (identical in every workgroup)
        const bool have = bk != 0;
        const bool useD = !have || bk == 1ull;   // no candidate, or an exact zero pivot
        const unsigned p = have ? bp : d;
        const bool nz = !have || bk != 1ull;      // NaN at d counts as nonzero

        // -- the window that drives the update: the pivot's, or row d's
        const T *u;
        if (G == 1) {
            u = S.cand[bwv];
            if (useD) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (act[k] && pos[k] == d) {
#pragma unroll
                        for (int q = 0; q < W; ++q) dwin[q] = x[k][q];
                    }
                }
                __syncthreads();
                u = dwin;
            }
        } else if (G <= kPanelStageG && !useD) {
            u = reinterpret_cast<const T *>(&stage[src_g * kRecWords + 4]);
        } else {
            unsigned long long *srcrec =
                a.rec + ((size_t)j * kRecSlots + (useD ? kPanelMaxWG : src_g)) * kRecWords;
            if (useD) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (act[k] && pos[k] == d) {
#pragma unroll
                        for (int q = 0; q < W; ++q)
#pragma unroll
                            for (int h = 0; h < NC; ++h) pubw(&srcrec[4 + NC * q + h], ET | P::get(x[k][q], h));
                    }
                }
            }
            if (tid < NC * nw) {
                unsigned long long v;
                unsigned spins = 0;
                while (true) {
                    v = subw(&srcrec[4 + tid]);
                    if ((unsigned)(v >> 32) == E) break;
                    if (++spins > kPanelSpin) { atomicExch(&st->error, 1); abort_s = 1; break; }
                    if ((spins & 1023u) == 0 && __hip_atomic_load(&st->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        abort_s = 1;
                        break;
                    }
                }
                ub[tid] = (unsigned)v;
            }
            __syncthreads();
            if (abort_s) return;
            u = reinterpret_cast<const T *>(ub);
        }
        if (tid == 0) {
            pvs[j] = p;
            if (!nz && zfirst < 0) zfirst = j;
        }
        // the rest of the pivot window is read while the multipliers are formed
        T uc[W - 1];
#pragma unroll
        for (int q = 0; q < W - 1; ++q) uc[q] = u[q + 1];
        const T piv = (G > 1 && G <= kPanelStageG && !useD) ? spiv : u[0];

        // -- scale the live rows, retire the pivot content, move row d's
        T lk[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = tid + 256 * k;
            const bool ret = act[k] && (useD ? pos[k] == d : cid[k] == bc);
            const bool sc = act[k] && !ret;
            const T l = nz ? P::div(x[k][0], piv) : x[k][0];
            lk[k] = sc ? l : P::zero();
            if (sc) {
                if (!useD && pos[k] == d) pos[k] = p;
                F[r * LDSW + j] = l;
            }
            if (ret) {
#pragma unroll
                for (int q = 0; q < W; ++q) Urow[j][q] = x[k][q];
                act[k] = false;
                pos[k] = d;
                rstep[k] = j;
            }
        }
        // -- the next step's candidate first: its column is updated alone, the
        // winning lane updates its whole window on the way to LDS, and the
        // record goes out before the rest of the window is updated, so that
        // update runs while the record crosses the grid
        if (j + 1 < w) {
            PanelStep<T> &S2 = ps[(j + 1) & 1];
            T v1[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) v1[k] = P::fms(x[k][1], lk[k], uc[0]);
            cand_step(S2, v1, [&](T *dst, int k) {
#pragma unroll
                for (int q = 0; q < W - 1; ++q) dst[q] = (k ? P::fms(x[1][q + 1], lk[1], uc[q]) : P::fms(x[0][q + 1], lk[0], uc[q]));
                dst[W - 1] = k ? x[1][W - 1] : x[0][W - 1];
            });
            if (G > 1) publish(j + 1, S2);
        }
        // x[q] <- x[q+1] - l·u[q+1] over the whole window: entries past the
        // live columns are never read, and a branch here would make the
        // compiler copy the window between registers at every step
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int q = 0; q < W - 1; ++q) x[k][q] = P::fms(x[k][q + 1], lk[k], uc[q]);
    }
    __syncthreads();
    if (g == 0) {
        if (tid < w) a.ipiv[c0 + tid] = (int)(pvs[tid] + 1);
        if (tid == 0 && zfirst >= 0) atomicCAS(&st->info, 0, (int)(c0 + zfirst + 1));
    }
    // every content to its final position; the source row of each position
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int r = tid + 256 * k;
        if (r < nr) {
            const long long fp = (long long)pos[k];
            const int rs = rstep[k] < 0 ? W : rstep[k];
            for (int q = 0; q < w; ++q) {
                const T lv = F[r * LDSW + q];
                const T uv = Urow[min(rs, W - 1)][max(q - rs, 0)];
                A[fp + (c0 + q) * a.lda] = q < rs ? lv : uv;
            }
            if (a.rowsrc) a.rowsrc[fp] = cid[k];
        }
    }
}

// Launch of the cooperative panel. Every workgroup waits on every other one,
// so all G must be resident: with strict, a launch the chip cannot hold is an
// error; otherwise nothing is launched and false returned.
template <typename T>
static bool panel_launch(Ctx &c, long long m, int w, T *A, long long lda, long long c0, int *ipiv, int *rowsrc,
                         int kind, double flops, bool strict) {
    const long long mp = m - c0;
    const int G = (int)((mp + kPanelRows - 1) / kPanelRows);
    if (G > c.num_cu || G > kPanelMaxWG) {
        if (strict) launch_error(hipErrorInvalidConfiguration);
        return false;
    }
    const size_t shm = (size_t)kPanelRows * (PanelT<T>::W + 1) * sizeof(T);
    static size_t attr_bytes = 0;
    static int per_cu = -1;   // workgroups of this kernel one CU can hold
    if (shm > attr_bytes) {
        RL_CHECK(hipFuncSetAttribute((const void *)getf2_panel_k<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        attr_bytes = shm;
        per_cu = -1;
    }
    if (per_cu < 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, getf2_panel_k<T>, 256, shm) != hipSuccess) nb = 0;
        per_cu = nb;
    }
    // refuse a launch the chip cannot hold at once instead of letting the
    // bounded waits expire
    if ((long long)per_cu * c.num_cu < G) {
        if (strict) launch_error(hipErrorCooperativeLaunchTooLarge);
        return false;
    }
    PanelArgs a{};
    a.m = m; a.c0 = c0; a.lda = lda; a.w = w; a.G = G;
    a.ipiv = ipiv;
    a.rowsrc = rowsrc;
    a.st = c.dstat;
    a.rec = panel_records(c, &a.epoch);
    if (!a.rec) return strict;
    trace_kernel_begin(c);
    rl_launch(c, getf2_panel_k<T>, dim3(G), dim3(256), (unsigned)shm, A, a);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, kind, flops, 2.0 * sizeof(T) * mp * w);
    return true;
}

template <typename T>
void getf2_panel(Ctx &c, long long m, int w, T *A, long long lda, long long c0, int *ipiv) {
    if (plan_record(c, PK_GETF2, m - c0, w, w)) return;
    if (m - c0 <= 0 || w <= 0) return;
    panel_launch<T>(c, m, w, A, lda, c0, ipiv, c.rowsrc, PK_GETF2, (double)(m - c0) * w * w, true);
}

template void getf2_panel<double>(Ctx &, long long, int, double *, long long, long long, int *);
template void getf2_panel<float>(Ctx &, long long, int, float *, long long, long long, int *);

template <typename T>
bool getf2_panel_cx(Ctx &c, long long m, int w, T *A, long long lda, long long c0, int *ipiv) {
    if (m - c0 <= 0 || w <= 0) return true;
    // the source row of every position goes to rowsrc, for laswp_leaf
    if (!c.rowsrc || c.rowsrc_elems < (size_t)m) return false;
    return panel_launch<T>(c, m, w, A, lda, c0, ipiv, c.rowsrc, PK_ZLEAF, 4.0 * (m - c0) * w * w, false);
}

template bool getf2_panel_cx<cx<double>>(Ctx &, long long, int, cx<double> *, long long, long long, int *);
template bool getf2_panel_cx<cx<float>>(Ctx &, long long, int, cx<float> *, long long, long long, int *);

// ---------------------------------------------------------------------------
// laswp after a panel: the panel's w interchanges, applied to the columns of
// the current block [blk0, blk1) outside the panel (every column of the
// matrix when the recursion applies no batches). The touched positions are
// the w diagonal rows and the w pivot rows; position i receives the content
// that sat at rowsrc[i] before the panel. Each workgroup gathers its columns'
// touched entries into registers, waits, then scatters them, so repeated
// pivot rows are harmless. Lanes run over the touched positions, so the w
// diagonal rows (contiguous in a column) are read and written coalesced.
//
// When the recursion applies interchanges in batches, the trailing
// workgroups also carry the row tracker forward: P[i] is the original row
// now at position i, so P_new[i] = P_old[rowsrc[i]] from the panel on
// (double-buffered, so no workgroup reads an entry another one rewrites).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void laswp_leaf_k(T *__restrict__ A, long long lda, long long c0, int w,
                                                    const int *__restrict__ ipiv,
                                                    const int *__restrict__ rowsrc, long long blk0,
                                                    long long nother, int colwg, const int *__restrict__ Pold,
                                                    int *__restrict__ Pnew, long long m) {
    constexpr int CPB = 32;  // columns per workgroup
    const int tid = threadIdx.x;
    if ((int)blockIdx.x >= colwg) {
        // row tracker: 4096 positions per workgroup
        const long long base = (long long)(blockIdx.x - colwg) * 4096;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const long long i = base + tid + 256 * u;
            if (i < m) Pnew[i] = Pold[i >= c0 ? rowsrc[i] : i];
        }
        return;
    }
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
        long long col = blk0 + lc;
        if (col >= c0) col += w;
        if (pos >= 0 && lc < nother && srow != pos) vals[q] = A[srow + col * lda];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CPB / 4; ++q) {
        const long long lc = lc0 + q * 4 + cq;
        long long col = blk0 + lc;
        if (col >= c0) col += w;
        if (pos >= 0 && lc < nother && srow != pos) A[pos + col * lda] = vals[q];
    }
}

template <typename T>
void laswp_leaf(Ctx &c, T *A, long long lda, long long k0, int w, long long m, const int *ipiv, long long blk0,
                long long blk1) {
    const long long nother = blk1 - blk0 - w;
    if (plan_record(c, PK_LASWP, 2 * w, nother, w)) return;
    if (w <= 0) return;
    const int colwg = (int)((max(nother, 0LL) + 31) / 32);
    const int pwg = c.lu_batch ? (int)((m + 4095) / 4096) : 0;
    if (colwg + pwg == 0) return;
    const int *Pold = c.lu_batch ? c.pv + (size_t)c.pcur * c.pv_m : nullptr;
    int *Pnew = c.lu_batch ? c.pv + (size_t)(c.pcur ^ 1) * c.pv_m : nullptr;
    trace_kernel_begin(c);
    rl_launch(c, laswp_leaf_k<T>, dim3(colwg + pwg), dim3(256), 0, A, lda, k0, w, ipiv, (const int *)c.rowsrc,
              blk0, max(nother, 0LL), colwg, Pold, Pnew, m);
    RL_CHECK(hipGetLastError());
    if (c.lu_batch) c.pcur ^= 1;
    trace_kernel_end(c, PK_LASWP, 0.0, 4.0 * sizeof(T) * w * max(nother, 0LL));
}

template void laswp_leaf<double>(Ctx &, double *, long long, long long, int, long long, const int *, long long,
                                 long long);
template void laswp_leaf<float>(Ctx &, float *, long long, long long, int, long long, const int *, long long,
                                long long);
template void laswp_leaf<cx<double>>(Ctx &, cx<double> *, long long, long long, int, long long, const int *,
                                     long long, long long);
template void laswp_leaf<cx<float>>(Ctx &, cx<float> *, long long, long long, int, long long, const int *,
                                    long long, long long);

// ---------------------------------------------------------------------------
// Batched interchanges (the recursion's own order: after one half is factored
// its pivots are applied to the other half's columns in one pass). With the
// row tracker P (original row at each position) and the inverse of the
// tracker taken when the batch's pivots began (inv: original row -> its
// position then), position i of a column must receive the entry that sat at
// src(i) = inv[P[i]]. A workgroup per column gathers every entry with
// src(i) != i into registers, waits, then writes them: the touched rows of a
// wide batch cover most of the column, so its lines are read and written
// about once each instead of once per interchange.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lu_iota_k(int *__restrict__ P, long long m) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < m) P[i] = (int)i;
}

__global__ __launch_bounds__(256) void lu_inverse_k(const int *__restrict__ P, int *__restrict__ inv, long long r0,
                                                    long long m) {
    const long long i = r0 + (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < m) inv[P[i]] = (int)i;
}

// the batch's source of every position, once for all of its columns
__global__ __launch_bounds__(256) void lu_src_k(const int *__restrict__ P, const int *__restrict__ inv,
                                                int *__restrict__ src, long long r0, long long m) {
    const long long i = r0 + (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < m) src[i] = inv[P[i]];
}

template <typename T, int R>
__global__ __launch_bounds__(1024) void laswp_batch_k(T *__restrict__ A, long long lda, long long j0, long long r0,
                                                      long long m, const int *__restrict__ srcp) {
    static_assert(R <= 32, "one bit per row in the mask");
    T *a = A + (j0 + (long long)blockIdx.x) * lda;
    const int tid = threadIdx.x;
    T v[R];
    unsigned moved = 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long i = r0 + tid + 1024LL * r;
        if (i < m) {
            const int s = srcp[i];
            if (s != i) { v[r] = a[s]; moved |= 1u << r; }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long i = r0 + tid + 1024LL * r;
        if (moved >> r & 1u) a[i] = v[r];
    }
}

void lu_track_begin(Ctx &c, long long m) {
    if (plan_record(c, PK_OTHER, m, 0, 0)) return;
    hipLaunchKernelGGL(lu_iota_k, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, c.stream,
                       c.pv + (size_t)c.pcur * c.pv_m, m);
    RL_CHECK(hipGetLastError());
}

int *lu_inverse(Ctx &c, int slot, long long r0, long long m) {
    if (plan_record(c, PK_OTHER, m - r0, 0, 0)) return nullptr;
    int *inv = c.pv + (size_t)(2 + slot) * c.pv_m;
    if (m > r0)
        hipLaunchKernelGGL(lu_inverse_k, dim3((unsigned)((m - r0 + 255) / 256)), dim3(256), 0, c.stream,
                           (const int *)(c.pv + (size_t)c.pcur * c.pv_m), inv, r0, m);
    RL_CHECK(hipGetLastError());
    return inv;
}

template <typename T>
void laswp_batch(Ctx &c, T *A, long long lda, long long j0, long long ncols, long long r0, long long m,
                 const int *inv, long long npiv) {
    if (plan_record(c, PK_LASWP, m - r0, ncols, npiv)) return;
    if (ncols <= 0 || m <= r0) return;
    const int *P = c.pv + (size_t)c.pcur * c.pv_m;
    int *src = c.pv + (size_t)(3 + 2 * kLaswpDepth) * c.pv_m;
    const long long rows = m - r0;
    hipLaunchKernelGGL(lu_src_k, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, c.stream, P, inv, src, r0, m);
    trace_kernel_begin(c);
    if (rows <= 8 * 1024)
        rl_launch(c, laswp_batch_k<T, 8>, dim3((unsigned)ncols), dim3(1024), 0, A, lda, j0, r0, m, (const int *)src);
    else if (rows <= 16 * 1024)
        rl_launch(c, laswp_batch_k<T, 16>, dim3((unsigned)ncols), dim3(1024), 0, A, lda, j0, r0, m, (const int *)src);
    else
        rl_launch(c, laswp_batch_k<T, 32>, dim3((unsigned)ncols), dim3(1024), 0, A, lda, j0, r0, m, (const int *)src);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_LASWP, 0.0, 4.0 * sizeof(T) * npiv * ncols);
}

template void laswp_batch<double>(Ctx &, double *, long long, long long, long long, long long, long long,
                                  const int *, long long);
template void laswp_batch<float>(Ctx &, float *, long long, long long, long long, long long, long long,
                                 const int *, long long);

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
