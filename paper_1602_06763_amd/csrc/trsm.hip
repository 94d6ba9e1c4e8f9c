// Triangular solves with many right-hand sides (BLAS-3 xtrsm), recursive.
//
// The recursion splits the triangle in two (the paper's block-size-n/2 rule,
// Sec. 3) so that every off-diagonal flop is a matrix-core GEMM; the leaf is a
// substitution kernel. Substitution (never an explicitly inverted diagonal
// block) keeps every step an exact operation on exactly representable data,
// which the integer test matrices rely on.
//
// Leaf: solve N·x = b for many vectors b, N a t×t triangle (t <= 64) held in
// LDS. Element (i, j) of N is T[i*ti + j*tj]; element e of vector r is
// B[e*se + r*sr]. Left-side solves use se = 1 (columns of B), right-side
// solves use sr = 1 (rows of B) with N = op(T)ᵀ.
#include "common.hpp"
#include "wg.hpp"

#include <type_traits>

namespace rl {

// INV = true: the right-hand sides are the columns of the identity (not read
// from B) and only the triangle of the solution is written back, so a single
// workgroup (nvec = t) writes N⁻¹ over N's own triangle in B = T; the whole
// triangle is staged in LDS before the first store.
template <typename TT, typename TB, typename TW, bool LOWER, bool INV = false>
__global__ __launch_bounds__(256) void trsm_leaf_mfma_k(int unit, int t, const TT *__restrict__ T, long long ti,
                                                        long long tj, long long nvec, TB *__restrict__ B,
                                                        long long se, long long sr, const int *abort) {
    if (abort && *abort) return;
    typedef LeafMfma<TW> Op;
    typedef typename Op::acc_t acc_t;
    __shared__ TW Nsh[64][65];
    __shared__ TW Xsh[4][64][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long v0 = (long long)blockIdx.x * 64 + wave * 16;   // this wave's 16 vectors
    TW (*X)[17] = Xsh[wave];
    // the triangle (16 elements per thread) and the vectors (16 per thread),
    // all loads in flight before any is used
    {
        TW tv[16], bv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            tv[u] = (TW)T[min(i, t - 1) * ti + min(j, t - 1) * tj];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            if (se == 1) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            bv[u] = INV ? TB(e == v0 + q) : (TB)B[min(e, t - 1) * se + min(v0 + q, nvec - 1) * sr];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            const bool in = i < t && j < t && (LOWER ? (j <= i) : (j >= i));
            // zero outside the triangle; the identity beyond t
            Nsh[i][j] = in ? tv[u] : ((i == j && i >= t) ? TW(1) : TW(0));
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            if (se == 1) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            X[e][q] = (e < t && v0 + q < nvec) ? (TW)bv[u] : TW(0);
        }
    }
    __syncthreads();
    solve64<TW, LOWER>(Nsh, X, t, unit, lane);

    // write the solved vectors back
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        int e, q;
        if (se == 1) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
        else { q = lane & 15; e = (lane >> 4) + 4 * u; }
        bool w = e < t && v0 + q < nvec;
        if (INV) w = w && (LOWER ? (unit ? e > v0 + q : e >= v0 + q) : (unit ? e < v0 + q : e <= v0 + q));
        if (w) B[e * se + (v0 + q) * sr] = (TB)X[e][q];
    }
}

// ---------------------------------------------------------------------------
// Two-block leaf for 64 < t <= 128: the bottom level of the recursion (two
// 64-leaves and the product between them) in one launch. The triangle is
// N = [D0 0; O D1] (lower) or [D0 O; 0 D1] (upper); the workgroup solves
// with the first diagonal block in the order of the solve, subtracts O times
// that part from the other rows on the matrix cores, then restages LDS with
// the second diagonal block (read into registers at the start) and solves
// with it. 64 vectors per workgroup, 16 per wave, as in the one-block leaf.
// ---------------------------------------------------------------------------
template <typename TT, typename TB, typename TW, bool LOWER>
__global__ __launch_bounds__(256) void trsm_leaf2_k(int unit, int t, const TT *__restrict__ T, long long ti,
                                                    long long tj, long long nvec, TB *__restrict__ B,
                                                    long long se, long long sr, const int *abort) {
    if (abort && *abort) return;
    typedef LeafMfma<TW> Op;
    typedef typename Op::acc_t acc_t;
    __shared__ TW Nsh[64][65];
    __shared__ TW Osh[64][65];
    __shared__ TW Xsh[4][128][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long v0 = (long long)blockIdx.x * 64 + wave * 16;
    TW (*X)[17] = Xsh[wave];
    const int t2 = t - 64;                                  // rows of the second block, 1..64
    const int first = LOWER ? 0 : 1, second = 1 - first;    // blocks in the order of the solve
    const int tf = first == 0 ? 64 : t2, ts = second == 0 ? 64 : t2;
    TW dsec[16];
    {
        TW df[16], ov[16], bv[32];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            const int fi = min(64 * first + i, t - 1), fj = min(64 * first + j, t - 1);
            const int si = min(64 * second + i, t - 1), sj = min(64 * second + j, t - 1);
            const int oi = min(LOWER ? 64 + i : i, t - 1), oj = min(LOWER ? j : 64 + j, t - 1);
            df[u] = (TW)T[fi * ti + fj * tj];
            dsec[u] = (TW)T[si * ti + sj * tj];
            ov[u] = (TW)T[oi * ti + oj * tj];
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            int e, q;
            if (se == 1) { e = (lane & 15) + 16 * (u & 7); q = (lane >> 4) + 4 * (u >> 3); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            bv[u] = (TW)B[min(e, t - 1) * se + min(v0 + q, nvec - 1) * sr];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            const bool tri = LOWER ? (j <= i) : (j >= i);
            Nsh[i][j] = (i < tf && j < tf && tri) ? df[u] : ((i == j && i >= tf) ? TW(1) : TW(0));
            Osh[i][j] = (LOWER ? i < t2 : j < t2) ? ov[u] : TW(0);
            dsec[u] = (i < ts && j < ts && tri) ? dsec[u] : ((i == j && i >= ts) ? TW(1) : TW(0));
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            int e, q;
            if (se == 1) { e = (lane & 15) + 16 * (u & 7); q = (lane >> 4) + 4 * (u >> 3); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            X[e][q] = (e < t && v0 + q < nvec) ? bv[u] : TW(0);
        }
    }
    __syncthreads();
    solve64<TW, LOWER>(Nsh, X + 64 * first, tf, unit, lane);
    // the other rows: X_second -= O·X_first (four independent 16-row blocks)
    {
        acc_t acc[4];
#pragma unroll
        for (int I = 0; I < 4; ++I) acc[I] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int k4 = 0; k4 < 16; ++k4) {
            const int k = 4 * k4 + (lane >> 4);
            const TW b = X[64 * first + k][lane & 15];
#pragma unroll
            for (int I = 0; I < 4; ++I) acc[I] = Op::mma(Osh[16 * I + (lane & 15)][k], b, acc[I]);
        }
#pragma unroll
        for (int I = 0; I < 4; ++I)
#pragma unroll
            for (int v = 0; v < 4; ++v) X[64 * second + 16 * I + Op::row(lane, v)][lane & 15] -= acc[I][v];
    }
    __syncthreads();   // every wave is done with the first diagonal block
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
        Nsh[i][j] = dsec[u];
    }
    __syncthreads();
    solve64<TW, LOWER>(Nsh, X + 64 * second, ts, unit, lane);
#pragma unroll
    for (int u = 0; u < 32; ++u) {
        int e, q;
        if (se == 1) { e = (lane & 15) + 16 * (u & 7); q = (lane >> 4) + 4 * (u >> 3); }
        else { q = lane & 15; e = (lane >> 4) + 4 * u; }
        if (e < t && v0 + q < nvec) B[e * se + (v0 + q) * sr] = (TB)X[e][q];
    }
}

template <typename TT, typename TB>
void trsm_leaf(Ctx &c, bool lower_eff, bool unit, int t, const TT *T, long long ti, long long tj,
               long long nvec, TB *B, long long se, long long sr) {
    if (plan_record(c, PK_TRSM_LEAF, t, nvec, t)) return;
    if (t <= 0 || nvec <= 0) return;
    const int grid = (int)((nvec + 255) / 256);
    const int *abort = c.abort_on_info ? &c.dstat->info : nullptr;
    trace_kernel_begin(c);
    typedef typename std::conditional<(sizeof(TB) == 8 || sizeof(TT) == 8), double, float>::type TW;
    const int grid64 = (int)((nvec + 63) / 64);
    if (t > 64) {
        if (lower_eff)
            rl_launch(c, trsm_leaf2_k<TT, TB, TW, true>, dim3(grid64), dim3(256), 0, (int)unit, t, T, ti, tj, nvec,
                      B, se, sr, abort);
        else
            rl_launch(c, trsm_leaf2_k<TT, TB, TW, false>, dim3(grid64), dim3(256), 0, (int)unit, t, T, ti, tj, nvec,
                      B, se, sr, abort);
    } else if (lower_eff)
        rl_launch(c, trsm_leaf_mfma_k<TT, TB, TW, true>, dim3(grid64), dim3(256), 0, (int)unit, t, T, ti, tj, nvec, B,
                  se, sr, abort);
    else
        rl_launch(c, trsm_leaf_mfma_k<TT, TB, TW, false>, dim3(grid64), dim3(256), 0, (int)unit, t, T, ti, tj, nvec,
                  B, se, sr, abort);
    (void)grid;
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_TRSM_LEAF, (double)t * t * nvec, 8.0 * (t * t + 2.0 * t * nvec));
}

// Unblocked inverse of a t×t triangle (t <= 64) in place: the leaf solve
// against the identity, one workgroup, only the triangle written back.
void trti2_leaf(Ctx &c, bool lower, bool unit, int t, double *A, long long lda) {
    if (plan_record(c, PK_TRTI2, t, t, t)) return;
    if (t <= 0) return;
    const int *abort = c.abort_on_info ? &c.dstat->info : nullptr;
    trace_kernel_begin(c);
    if (lower)
        rl_launch(c, trsm_leaf_mfma_k<double, double, double, true, true>, dim3(1), dim3(256), 0, (int)unit, t,
                  (const double *)A, 1LL, lda, (long long)t, A, 1LL, lda, abort);
    else
        rl_launch(c, trsm_leaf_mfma_k<double, double, double, false, true>, dim3(1), dim3(256), 0, (int)unit, t,
                  (const double *)A, 1LL, lda, (long long)t, A, 1LL, lda, abort);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_TRTI2, (double)t * t * t / 3.0, 8.0 * t * t);
}


// ---------------------------------------------------------------------------
// Blocked triangular solve for a few right-hand sides (nrhs <= 8 per launch):
// one launch for the whole triangle. Workgroups take 64-row blocks in the
// order they start (a ticket counter), so a workgroup only ever waits on
// blocks owned by workgroups that started before it.
//
// Wave 0 holds the block's rows of the diagonal block and the right-hand
// side in registers; waves 1..3 take every third earlier block: each loads
// its 64×64 tile of op(T) first (through LDS for the transposed case, so the
// loads stay coalesced), then waits for that block's solution and subtracts
// the product. After one barrier wave 0 solves the diagonal block by
// substitution (reciprocals of the diagonal formed up front, readlane
// broadcasts, the 64 steps unrolled so the row's entries stay in fixed
// registers) and publishes x. Published solutions are 64-bit words holding
// the launch's epoch in the upper half and one half of a value in the lower
// half, written and polled with device-coherent atomic accesses: a reader
// needs no flag, no fence and no reset. The triangle is read once, so the
// solve is bound by HBM bandwidth and by the chain of n/64 diagonal solves.
// ---------------------------------------------------------------------------
struct TrsvArgs {
    long long n;
    int nrhs, nb;
    long long ldt, ldb;
    int trans, lower_eff, unit;
    unsigned int epoch;
    unsigned long long *ticket;
    unsigned long long ticket_base;
    unsigned long long *xw;   // [n][8][2] epoch-tagged halves of x
    DevStatus *st;
    const double *dinv;       // DINV: inverses of the diagonal blocks of op(T), 64×64 column-major each
    int nch;                  // trsv16_k: chunks of 16 right-hand sides solved side by side
};

__device__ __forceinline__ double rl_readlane(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

template <typename TT, typename TB, int NR, bool DINV>
__global__ __launch_bounds__(256) void trsv_k(const TT *__restrict__ T, TB *__restrict__ B, TrsvArgs a) {
    __shared__ double tile[3][64][65];
    __shared__ double xs[3][64][NR];
    __shared__ double red[3][64][NR];
    __shared__ int bsh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) bsh = (int)(atomicAdd(a.ticket, 1ull) - a.ticket_base);
    __syncthreads();
    const int b = bsh, nb = a.nb;
    const bool fwd = a.lower_eff != 0;
    const long long n = a.n, ldt = a.ldt;
    const int pb = fwd ? b : nb - 1 - b;
    const long long r0 = (long long)pb * 64;
    const int nrow = (int)min(64LL, n - r0);
    const int nq = a.nrhs;
    const long long ri = r0 + min(lane, nrow - 1);   // clamped row of this lane
    const unsigned long long ET = (unsigned long long)a.epoch << 32;

    double d[64];      // wave 0: row `lane` of the diagonal block (strictly off-diagonal part)
    double r[NR];      // wave 0: right-hand side, then solution
    double rinv = 1.0;
    if (wave == 0 && DINV) {
        // row `lane` of the inverted diagonal block
        const double *Db = a.dinv + (size_t)pb * 4096;
#pragma unroll
        for (int k = 0; k < 64; ++k) d[k] = Db[lane + 64 * k];
#pragma unroll
        for (int q = 0; q < NR; ++q) r[q] = (double)B[ri + min(q, nq - 1) * a.ldb];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int q = 0; q < NR; ++q) r[q] = (lane < nrow && q < nq) ? r[q] : 0.0;
    } else if (wave == 0) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            const long long c = r0 + min(k, nrow - 1);
            d[k] = (double)(a.trans ? T[c + ri * ldt] : T[ri + c * ldt]);
        }
        const double dd = (double)T[ri + ri * ldt];
#pragma unroll
        for (int q = 0; q < NR; ++q) r[q] = (double)B[ri + min(q, nq - 1) * a.ldb];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            const bool off = fwd ? (k < lane) : (k > lane);
            d[k] = (lane < nrow && k < nrow && off) ? d[k] : 0.0;
        }
        rinv = (a.unit || lane >= nrow) ? 1.0 : 1.0 / dd;
#pragma unroll
        for (int q = 0; q < NR; ++q) r[q] = (lane < nrow && q < nq) ? r[q] : 0.0;
    } else {
        const int w = wave - 1;
        double acc[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] = 0.0;
        for (int jj = w; jj < b; jj += 3) {
            const int pj = fwd ? jj : nb - 1 - jj;
            const long long c0 = (long long)pj * 64;
            const int ncol = (int)min(64LL, n - c0);
            // the tile first, all its loads issued together and complete before
            // the wait for the block's solution (which arrives later), so no
            // memory latency sits between that solution and the product
            double mk[64];
            if (!a.trans) {
#pragma unroll
                for (int k = 0; k < 64; ++k) mk[k] = (double)T[ri + (c0 + min(k, ncol - 1)) * ldt];
                asm volatile("" ::: "memory");
#pragma unroll
                for (int k = 0; k < 64; ++k) asm volatile("" : "+v"(mk[k]));
            } else {
                // op(T)(r, c) = T[c + r*ldt]: lanes over c read contiguously,
                // then the tile is transposed through LDS
                const long long cl = c0 + min(lane, ncol - 1);
#pragma unroll
                for (int rr = 0; rr < 64; ++rr) mk[rr] = (double)T[cl + (r0 + min(rr, nrow - 1)) * ldt];
                asm volatile("" ::: "memory");
#pragma unroll
                for (int rr = 0; rr < 64; ++rr) tile[w][rr][lane] = mk[rr];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int k = 0; k < 64; ++k) mk[k] = tile[w][lane][k];
#pragma unroll
                for (int k = 0; k < 64; ++k) asm volatile("" : "+v"(mk[k]));
            }
            if (lane >= ncol) {
#pragma unroll
                for (int q = 0; q < NR; ++q) xs[w][lane][q] = 0.0;   // so the product needs no bounds
            } else {
                unsigned long long *src = a.xw + (size_t)(c0 + lane) * 16;
                // every word of the row's solutions in one round trip, polled
                // together until all carry this solve's epoch
                unsigned long long lo[NR], hi[NR];
                unsigned spins = 0;
                while (true) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        lo[q] = hi[q] = (unsigned long long)a.epoch << 32;
                        if (q < nq) {
                            lo[q] = __hip_atomic_load(&src[2 * q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            hi[q] = __hip_atomic_load(&src[2 * q + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                    bool fresh = true;
#pragma unroll
                    for (int q = 0; q < NR; ++q) fresh = fresh && (lo[q] >> 32) == a.epoch && (hi[q] >> 32) == a.epoch;
                    if (fresh) break;
                    if (++spins > (1u << 22)) { atomicExch(&a.st->error, 2); break; }
                }
#pragma unroll
                for (int q = 0; q < NR; ++q)
                    xs[w][lane][q] = q < nq ? __hiloint2double((int)(unsigned)hi[q], (int)(unsigned)lo[q]) : 0.0;
            }
            __builtin_amdgcn_wave_barrier();
            // the block's solution from LDS in one batch of reads, then the
            // products in four independent chains
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                double xv[64];
#pragma unroll
                for (int k = 0; k < 64; ++k) xv[k] = xs[w][k][q];
                asm volatile("" ::: "memory");
                double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
                for (int k = 0; k < 64; k += 4) {
                    p0 += mk[k] * xv[k];
                    p1 += mk[k + 1] * xv[k + 1];
                    p2 += mk[k + 2] * xv[k + 2];
                    p3 += mk[k + 3] * xv[k + 3];
                }
                acc[q] -= (p0 + p1) + (p2 + p3);
            }
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int q = 0; q < NR; ++q) red[w][lane][q] = acc[q];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int q = 0; q < NR; ++q)
            r[q] = lane < nrow ? r[q] + ((red[0][lane][q] + red[1][lane][q]) + red[2][lane][q]) : 0.0;
        if (DINV) {
            // x = D⁻¹·r: the block's right-hand side through LDS (each lane
            // overwrites only the row it has just read), four partial sums
#pragma unroll
            for (int q = 0; q < NR; ++q) red[0][lane][q] = r[q];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                double rv[64];
#pragma unroll
                for (int k = 0; k < 64; ++k) rv[k] = red[0][k][q];
                asm volatile("" ::: "memory");
                double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
                for (int k = 0; k < 64; k += 4) {
                    p0 += d[k] * rv[k];
                    p1 += d[k + 1] * rv[k + 1];
                    p2 += d[k + 2] * rv[k + 2];
                    p3 += d[k + 3] * rv[k + 3];
                }
                r[q] = lane < nrow ? (p0 + p1) + (p2 + p3) : 0.0;
            }
        } else {
            // substitution: x_k = r_k / t_kk, then r_i -= t_ik·x_k on the rows after k
#pragma unroll
            for (int s = 0; s < 64; ++s) {
                const int k = fwd ? s : 63 - s;
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const double xk = rl_readlane(r[q] * rinv, k);
                    r[q] = (lane == k) ? xk : r[q] - d[k] * xk;
                }
            }
        }
        if (lane < nrow) {
            unsigned long long *dst = a.xw + (size_t)(r0 + lane) * 16;
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                if (q < nq) {
                    B[ri + q * a.ldb] = (TB)r[q];
                    __hip_atomic_store(&dst[2 * q], ET | (unsigned)__double2loint(r[q]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&dst[2 * q + 1], ET | (unsigned)__double2hiint(r[q]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The same blocked solve for 2..64 right-hand sides, 16 per chain, all chains
// in one launch: ticket t takes block t / nch of chunk t % nch, so blocks of
// every chunk are dispatched in order and a workgroup only waits for blocks
// with smaller tickets. Waves 1-3 multiply the tiles of the earlier blocks
// with those blocks' solutions on the matrix cores (64 rows × 16 right-hand
// sides per tile, the solution words of a block polled in one round trip);
// wave 0 takes the block's right-hand sides, subtracts the three partial sums
// and solves with the diagonal block (staged in LDS by all waves) by
// substitution (solve64). Solutions are published as epoch-tagged words, 32
// per row and chunk.
// ---------------------------------------------------------------------------
template <typename TT, bool FWD>
__global__ __launch_bounds__(256) void trsv16_k(const TT *__restrict__ T, double *__restrict__ B, TrsvArgs a) {
    typedef LeafMfma<double> Op;
    typedef typename Op::acc_t acc_t;
    __shared__ double Nsh[64][65];
    __shared__ double Xs[64][17];
    __shared__ double red[3][64][17];
    __shared__ int bsh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) bsh = (int)(atomicAdd(a.ticket, 1ull) - a.ticket_base);
    __syncthreads();
    const int nch = a.nch, b = bsh / nch, ch = bsh % nch, nb = a.nb;
    const long long n = a.n, ldt = a.ldt, ldb = a.ldb;
    const int pb = FWD ? b : nb - 1 - b;
    const long long r0 = (long long)pb * 64;
    const int nrow = (int)min(64LL, n - r0);
    const int nq = min(16, a.nrhs - 16 * ch);
    double *Bc = B + (long long)(16 * ch) * ldb;
    unsigned long long *xw = a.xw + (size_t)ch * (size_t)n * 32;
    const unsigned long long ET = (unsigned long long)a.epoch << 32;
    auto opT = [&](long long r, long long c) { return (double)(a.trans ? T[c + r * ldt] : T[r + c * ldt]); };

    // the diagonal block, the identity beyond the triangle
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int i = idx & 63, j = idx >> 6;
        const bool in = i < nrow && j < nrow && (FWD ? j <= i : j >= i);
        const double v = opT(r0 + min(i, nrow - 1), r0 + min(j, nrow - 1));
        Nsh[i][j] = in ? v : (i == j ? 1.0 : 0.0);
    }
    if (wave == 0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = (lane >> 4) + 4 * u, q = lane & 15;
            const double v = Bc[r0 + min(e, nrow - 1) + (long long)min(q, nq - 1) * ldb];
            Xs[e][q] = (e < nrow && q < nq) ? v : 0.0;
        }
    } else {
        const int w = wave - 1, lr = lane & 15, lk = lane >> 4;
        acc_t acc[4];
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) acc[i4] = acc_t{0, 0, 0, 0};
        for (int jj = w; jj < b; jj += 3) {
            const int pj = FWD ? jj : nb - 1 - jj;
            const long long c0 = (long long)pj * 64;
            const int ncol = (int)min(64LL, n - c0);
            // the tile first, its loads in flight while the solution is polled
            double av[16][4];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int k = 4 * kk + lk;
#pragma unroll
                for (int i4 = 0; i4 < 4; ++i4) {
                    const int i = 16 * i4 + lr;
                    const double v = opT(r0 + min(i, nrow - 1), c0 + min(k, ncol - 1));
                    av[kk][i4] = (i < nrow && k < ncol) ? v : 0.0;
                }
            }
            asm volatile("" ::: "memory");
            unsigned long long lo[16], hi[16];
            unsigned spins = 0;
            while (true) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) {
                    const int k = 4 * kk + lk;
                    lo[kk] = hi[kk] = ET;
                    if (k < ncol && lr < nq) {
                        const unsigned long long *src = xw + (size_t)(c0 + k) * 32 + 2 * lr;
                        lo[kk] = __hip_atomic_load(&src[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        hi[kk] = __hip_atomic_load(&src[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                bool fresh = true;
#pragma unroll
                for (int kk = 0; kk < 16; ++kk)
                    fresh = fresh && (unsigned)(lo[kk] >> 32) == a.epoch && (unsigned)(hi[kk] >> 32) == a.epoch;
                if (fresh) break;
                if (++spins > (1u << 22)) { atomicExch(&a.st->error, 2); break; }
            }
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int k = 4 * kk + lk;
                const double bv = (k < ncol && lr < nq) ? __hiloint2double((int)(unsigned)hi[kk], (int)(unsigned)lo[kk])
                                                        : 0.0;
#pragma unroll
                for (int i4 = 0; i4 < 4; ++i4) acc[i4] = Op::mma(av[kk][i4], bv, acc[i4]);
            }
        }
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[w][16 * i4 + Op::row(lane, v)][lane & 15] = acc[i4][v];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = (lane >> 4) + 4 * u, q = lane & 15;
            Xs[e][q] -= (red[0][e][q] + red[1][e][q]) + red[2][e][q];
        }
        solve64<double, FWD>(Nsh, Xs, nrow, a.unit, lane);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = (lane >> 4) + 4 * u, q = lane & 15;
            if (e < nrow && q < nq) {
                const double x = Xs[e][q];
                Bc[r0 + e + (long long)q * ldb] = x;
                unsigned long long *dst = xw + (size_t)(r0 + e) * 32 + 2 * q;
                __hip_atomic_store(&dst[0], ET | (unsigned)__double2loint(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&dst[1], ET | (unsigned)__double2hiint(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Inverses of the 64×64 diagonal blocks of op(T) (rows/columns beyond m hold
// the identity), one workgroup per block: the leaf substitution against the
// identity, written out in full (zeros included), column-major per block.
// ---------------------------------------------------------------------------
template <typename TT, bool LOWER>
__global__ __launch_bounds__(256) void diag_inv_k(int unit, long long n, const TT *__restrict__ T, long long ti,
                                                  long long tj, double *__restrict__ dinv) {
    __shared__ double Nsh[64][65];
    __shared__ double Xsh[4][64][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long r0 = (long long)blockIdx.x * 64;
    const int t = (int)min(64LL, n - r0);
    const TT *Tb = T + r0 * ti + r0 * tj;
    double (*X)[17] = Xsh[wave];
    {
        double tv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            tv[u] = (double)Tb[min(i, t - 1) * ti + min(j, t - 1) * tj];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            const bool in = i < t && j < t && (LOWER ? (j <= i) : (j >= i));
            Nsh[i][j] = in ? tv[u] : ((i == j && i >= t) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = (lane & 15) + 16 * (u & 3), q = (lane >> 4) + 4 * (u >> 2);
            X[e][q] = (e == 16 * wave + q) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    solve64<double, LOWER>(Nsh, X, t, unit, lane);
    double *Db = dinv + (size_t)blockIdx.x * 4096;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = (lane & 15) + 16 * (u & 3), q = (lane >> 4) + 4 * (u >> 2);
        Db[e + 64 * (16 * wave + q)] = X[e][q];
    }
}

template <typename TT>
void trsv_diag_inverses(Ctx &c, bool lower_eff, bool trans, bool unit, long long m, const TT *T, long long ldt,
                        double *dinv) {
    if (plan_record(c, PK_OTHER, m, 64, 64)) return;
    const int nb = (int)((m + 63) / 64);
    if (nb <= 0) return;
    const long long ti = trans ? ldt : 1, tj = trans ? 1 : ldt;
    if (lower_eff)
        hipLaunchKernelGGL((diag_inv_k<TT, true>), dim3(nb), dim3(256), 0, c.stream, (int)unit, m, T, ti, tj, dinv);
    else
        hipLaunchKernelGGL((diag_inv_k<TT, false>), dim3(nb), dim3(256), 0, c.stream, (int)unit, m, T, ti, tj, dinv);
    RL_CHECK(hipGetLastError());
}

template void trsv_diag_inverses<float>(Ctx &, bool, bool, bool, long long, const float *, long long, double *);
template void trsv_diag_inverses<double>(Ctx &, bool, bool, bool, long long, const double *, long long, double *);

template <typename TT, typename TB>
void trsv(Ctx &c, bool lower_eff, bool trans, bool unit, long long m, long long nrhs, const TT *T,
          long long ldt, TB *B, long long ldb, const double *dinv) {
    const int nb = (int)((m + 63) / 64);
    if (nrhs > 1) {
        if constexpr (std::is_same<TB, double>::value) {
            const int nch = (int)((nrhs + 15) / 16);
            TrsvWork wk = trsv_work(c, m, nb, 1, 32LL * nch, nch);
            if (!wk.xw) return;
            trace_begin(c, PK_TRSM_LEAF);
            TrsvArgs a{};
            a.n = m; a.nrhs = (int)nrhs; a.nb = nb; a.nch = nch;
            a.ldt = ldt; a.ldb = ldb;
            a.trans = trans; a.lower_eff = lower_eff; a.unit = unit;
            a.epoch = wk.epoch;
            a.ticket = wk.ticket;
            a.ticket_base = wk.ticket_base;
            a.xw = wk.xw;
            a.st = c.dstat;
            if (lower_eff)
                hipLaunchKernelGGL((trsv16_k<TT, true>), dim3(nb * nch), dim3(256), 0, c.stream, T, B, a);
            else
                hipLaunchKernelGGL((trsv16_k<TT, false>), dim3(nb * nch), dim3(256), 0, c.stream, T, B, a);
            RL_CHECK(hipGetLastError());
            trace_end(c, PK_TRSM_LEAF, (double)m * m * nrhs, (double)sizeof(TT) * m * m / 2.0 + 16.0 * m * nrhs);
            return;
        }
    }
    TrsvWork wk = trsv_work(c, m, nb, (int)((nrhs + 7) / 8));
    if (!wk.xw) return;
    trace_begin(c, PK_TRSM_LEAF);
    for (long long q0 = 0; q0 < nrhs; q0 += 8) {
        TrsvArgs a{};
        a.n = m; a.nrhs = (int)min(8LL, nrhs - q0); a.nb = nb;
        a.ldt = ldt; a.ldb = ldb;
        a.trans = trans; a.lower_eff = lower_eff; a.unit = unit;
        a.epoch = wk.epoch + (unsigned)(q0 / 8);
        a.ticket = wk.ticket;
        a.ticket_base = wk.ticket_base + (unsigned long long)nb * (unsigned long long)(q0 / 8);
        a.xw = wk.xw;
        a.st = c.dstat;
        a.dinv = dinv;
        if (dinv && a.nrhs == 1) {
            // (the block products are used for one right-hand side at a time;
            // eight would not fit the registers next to the inverse's row)
            hipLaunchKernelGGL((trsv_k<TT, TB, 1, true>), dim3(nb), dim3(256), 0, c.stream, T, B + q0 * ldb, a);
        } else if (a.nrhs == 1) {
            hipLaunchKernelGGL((trsv_k<TT, TB, 1, false>), dim3(nb), dim3(256), 0, c.stream, T, B + q0 * ldb, a);
        } else {
            hipLaunchKernelGGL((trsv_k<TT, TB, 8, false>), dim3(nb), dim3(256), 0, c.stream, T, B + q0 * ldb, a);
        }
        RL_CHECK(hipGetLastError());
    }
    trace_end(c, PK_TRSM_LEAF, (double)m * m * nrhs, (double)sizeof(TT) * m * m / 2.0 + 16.0 * m * nrhs);
}

static inline bool is(char a, char b) { return a == b || a == (b + ('a' - 'A')); }

// Pointer to the block op(T)[r0:, c0:] and the op to use for it.
template <typename TT>
static inline const TT *opblock(const TT *T, long long ldt, bool trans, long long r0, long long c0) {
    return trans ? T + c0 + r0 * ldt : T + r0 + c0 * ldt;
}

template <typename TT, typename TB>
void trsm(Ctx &c, Mfma mode, char side, char uplo, char trans, char diag, long long m, long long n,
          const TT *T, long long ldt, TB *B, long long ldb) {
    if (m <= 0 || n <= 0) return;
    const bool tr = is(trans, 'T') || is(trans, 'C');
    const bool lowerM = is(uplo, 'L') != tr;  // op(T) is lower triangular
    const bool unit = is(diag, 'U');
    const char opc = tr ? 'T' : 'N';
    const int leaf = c.plan && c.plan_leaf > 0 ? c.plan_leaf : kTrsmLeaf;
    // the leaf kernels take up to two 64-blocks of the triangle
    const int top = leaf == kTrsmLeaf ? 2 * kTrsmLeaf : leaf;
    if (is(side, 'L')) {
        // op(T)·X = B, X m×n, triangle m×m
        if (!c.plan && !c.fixed && n <= kTrsvMaxRhs && m > top) {
            trsv<TT, TB>(c, lowerM, tr, unit, m, n, T, ldt, B, ldb, nullptr);
            return;
        }
        if (m <= top) {
            trsm_leaf<TT, TB>(c, lowerM, unit, (int)m, T, tr ? ldt : 1, tr ? 1 : ldt, n, B, 1, ldb);
            return;
        }
        const long long m1 = split_size(m), m2 = m - m1;
        const TT *T22 = T + m1 + m1 * ldt;
        if (lowerM) {
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m1, n, T, ldt, B, ldb);
            gemm<TT, TB, TB>(c, mode, opc, 'N', 0, m2, n, m1, -1.0, opblock(T, ldt, tr, m1, 0), ldt, B,
                             ldb, 1.0, B + m1, ldb);
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m2, n, T22, ldt, B + m1, ldb);
        } else {
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m2, n, T22, ldt, B + m1, ldb);
            gemm<TT, TB, TB>(c, mode, opc, 'N', 0, m1, n, m2, -1.0, opblock(T, ldt, tr, 0, m1), ldt,
                             B + m1, ldb, 1.0, B, ldb);
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m1, n, T, ldt, B, ldb);
        }
    } else {
        // X·op(T) = B, X m×n, triangle n×n. Row r of X solves op(T)ᵀ·xᵀ = bᵀ.
        if (n <= top) {
            // N = op(T)ᵀ: N(i,j) = op(T)(j,i) = tr ? T(i,j) : T(j,i)
            trsm_leaf<TT, TB>(c, !lowerM, unit, (int)n, T, tr ? 1 : ldt, tr ? ldt : 1, m, B, ldb, 1);
            return;
        }
        const long long n1 = split_size(n), n2 = n - n1;
        const TT *T22 = T + n1 + n1 * ldt;
        if (!lowerM) {
            // op(T) upper: X1 first, then B2 -= X1·op(T)12
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m, n1, T, ldt, B, ldb);
            gemm<TB, TT, TB>(c, mode, 'N', opc, 0, m, n2, n1, -1.0, B, ldb, opblock(T, ldt, tr, 0, n1),
                             ldt, 1.0, B + n1 * ldb, ldb);
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m, n2, T22, ldt, B + n1 * ldb, ldb);
        } else {
            // op(T) lower: X2 first, then B1 -= X2·op(T)21
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m, n2, T22, ldt, B + n1 * ldb, ldb);
            gemm<TB, TT, TB>(c, mode, 'N', opc, 0, m, n1, n2, -1.0, B + n1 * ldb, ldb,
                             opblock(T, ldt, tr, n1, 0), ldt, 1.0, B, ldb);
            trsm<TT, TB>(c, mode, side, uplo, trans, diag, m, n1, T, ldt, B, ldb);
        }
    }
}

template void trsv<float, double>(Ctx &, bool, bool, bool, long long, long long, const float *, long long,
                                  double *, long long, const double *);

template void trsm<double, double>(Ctx &, Mfma, char, char, char, char, long long, long long,
                                   const double *, long long, double *, long long);
template void trsm<float, float>(Ctx &, Mfma, char, char, char, char, long long, long long,
                                 const float *, long long, float *, long long);
template void trsm<float, double>(Ctx &, Mfma, char, char, char, char, long long, long long,
                                  const float *, long long, double *, long long);

}  // namespace rl
