// Complex instances (the c/z types of the collection, Sec. 5) of the
// recursive Cholesky and LU: zpotrf / cpotrf (A = L·Lᴴ or Uᴴ·U of a Hermitian
// positive definite matrix) and zgetrf / cgetrf (partial pivoting by
// |re| + |im|, LAPACK's izamax rule). Storage is LAPACK's: each element a
// (real, imaginary) pair, column-major.
//
// The recursion is the real one (Sec. 3: split at n/2 rounded to 64, a leaf
// kernel below the crossover): Cholesky potrf(A11); A21 := A21·L11⁻ᴴ;
// A22 -= A21·A21ᴴ; potrf(A22); LU getrf(left); A12 := L11⁻¹·A12;
// A22 -= A21·A12; getrf(right). Its pieces here:
//   - the complex product on the matrix cores: each complex multiply-add is
//     four real ones, re += ar·br − ai·bi and im += ar·bi + ai·br, each a
//     16×16×4 matrix-core step on the real and imaginary planes staged in LDS;
//   - the triangular-solve leaf: a triangle of at most 64 rows in LDS, 16
//     right-hand sides per wave, the products between its 16-row blocks on
//     the matrix cores and substitution within them;
//   - the Cholesky leaf: a block of at most 64 in LDS, 16-column panels by
//     one wave, the trailing updates on the matrix cores;
//   - the LU leaf: a panel of at most 16 columns over all rows below its
//     diagonal, one workgroup, the rows in global memory (the panel stays in
//     L2), and its interchanges applied at once to every other column.
// Quotients are a·conj(p) / |p|²; the pivot search keeps the first row of
// largest |re| + |im| (a NaN never wins).
#include "common.hpp"
#include "wg.hpp"

namespace rl {

constexpr int kZLeaf = 64;     // Cholesky and triangular-solve leaves

// ---------------------------------------------------------------------------
// C := beta·C + alpha·op(A)·op(B) on the matrix cores, alpha and beta real;
// op 0 = as stored, 1 = transposed, 2 = conjugate transposed. TRI 1 / 2:
// only the lower / upper triangle of a square C is computed and written
// (the Hermitian rank-k update of the Cholesky). A workgroup of four waves
// takes a 64×64 tile of C, each wave a 32×32 quarter as 2×2 blocks of
// 16×16 with a real and an imaginary accumulator; K goes in chunks of 16,
// staged in LDS as separate real and imaginary planes, the next chunk's loads
// in flight while the current one is multiplied.
// ---------------------------------------------------------------------------
template <typename R>
struct ZGemmArgs {
    long long m, n, k, lda, ldb, ldc;
    double alpha, beta;
    const cx<R> *A;
    const cx<R> *B;
    cx<R> *C;
    const DevStatus *st;
    int abort;
};

template <typename R, int OPA, int OPB, int TRI>
__global__ __launch_bounds__(256) void zgemm_k(ZGemmArgs<R> g) {
    if (g.abort && g.st->info) return;
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (TRI == 1 && bi < bj) return;
    if (TRI == 2 && bi > bj) return;
    typedef LeafMfma<R> Op;
    typedef typename Op::acc_t acc_t;
    constexpr int KC = 16;
    __shared__ R Ar[KC][65], Ai[KC][65], Br[KC][65], Bi[KC][65];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int wi = 32 * (wave & 1), wj = 32 * (wave >> 1);
    const long long i0 = 64LL * bi, j0 = 64LL * bj;
    const long long M = g.m, N = g.n, K = g.k;
    cx<R> ra[4], rb[4];
    // element u of this thread's share of the A tile: (row, k) within the tile
    auto a_idx = [&](int u, int &i, int &kk) {
        const int idx = tid + 256 * u;
        if (OPA == 0) { i = idx & 63; kk = idx >> 6; }
        else { kk = idx & 15; i = idx >> 4; }
    };
    auto b_idx = [&](int u, int &kk, int &j) {
        const int idx = tid + 256 * u;
        if (OPB == 0) { kk = idx & 15; j = idx >> 4; }
        else { j = idx & 63; kk = idx >> 6; }
    };
    auto fetch = [&](long long k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int i, kk;
            a_idx(u, i, kk);
            const long long gi = i0 + i, gk = k0 + kk;
            cx<R> v{R(0), R(0)};
            if (gi < M && gk < K) v = OPA == 0 ? g.A[gi + gk * g.lda] : g.A[gk + gi * g.lda];
            if (OPA == 2) v.im = -v.im;
            ra[u] = v;
            int j, kb;
            b_idx(u, kb, j);
            const long long gj = j0 + j, gkb = k0 + kb;
            cx<R> w{R(0), R(0)};
            if (gj < N && gkb < K) w = OPB == 0 ? g.B[gkb + gj * g.ldb] : g.B[gj + gkb * g.ldb];
            if (OPB == 2) w.im = -w.im;
            rb[u] = w;
        }
    };
    acc_t cr[2][2], ci[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) cr[s][t] = ci[s][t] = acc_t{0, 0, 0, 0};
    fetch(0);
    for (long long k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int i, kk, j;
            a_idx(u, i, kk);
            Ar[kk][i] = ra[u].re;
            Ai[kk][i] = ra[u].im;
            b_idx(u, kk, j);
            Br[kk][j] = rb[u].re;
            Bi[kk][j] = rb[u].im;
        }
        __syncthreads();
        if (k0 + KC < K) fetch(k0 + KC);
#pragma unroll
        for (int q = 0; q < KC / 4; ++q) {
            const int k = 4 * q + lk;
            R ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                ar[s] = Ar[k][wi + 16 * s + lr];
                ai[s] = Ai[k][wi + 16 * s + lr];
                br[s] = Br[k][wj + 16 * s + lr];
                bi[s] = Bi[k][wj + 16 * s + lr];
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    cr[s][t] = Op::mma(ar[s], br[t], cr[s][t]);
                    cr[s][t] = Op::mma(-ai[s], bi[t], cr[s][t]);
                    ci[s][t] = Op::mma(ar[s], bi[t], ci[s][t]);
                    ci[s][t] = Op::mma(ai[s], br[t], ci[s][t]);
                }
        }
        __syncthreads();
    }
    const R alpha = (R)g.alpha, beta = (R)g.beta;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long long i = i0 + wi + 16 * s + Op::row(lane, v), j = j0 + wj + 16 * t + lr;
                if (i >= M || j >= N) continue;
                if ((TRI == 1 && i < j) || (TRI == 2 && i > j)) continue;
                cx<R> &c = g.C[i + j * g.ldc];
                cx<R> r{alpha * cr[s][t][v], alpha * ci[s][t][v]};
                if (beta != R(0)) {
                    r.re += beta * c.re;
                    r.im += beta * c.im;
                }
                c = r;
            }
}

template <typename R>
static void zgemm(Ctx &c, int opa, int opb, int tri, long long m, long long n, long long k, double alpha,
                  const cx<R> *A, long long lda, const cx<R> *B, long long ldb, double beta, cx<R> *C, long long ldc) {
    if (plan_record(c, PK_ZGEMM, m, n, k)) return;
    if (m <= 0 || n <= 0) return;
    ZGemmArgs<R> a{m, n, k, lda, ldb, ldc, alpha, beta, A, B, C, c.dstat, c.abort_on_info ? 1 : 0};
    const dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
    trace_kernel_begin(c);
#define ZG(OA, OB, TR) rl_launch(c, zgemm_k<R, OA, OB, TR>, grid, dim3(256), 0, a)
    if (tri == 0) {
        if (opa == 0 && opb == 0) ZG(0, 0, 0);
        else if (opa == 0 && opb == 1) ZG(0, 1, 0);
        else if (opa == 0 && opb == 2) ZG(0, 2, 0);
        else if (opa == 1 && opb == 0) ZG(1, 0, 0);
        else if (opa == 2 && opb == 0) ZG(2, 0, 0);
        else if (opa == 1 && opb == 1) ZG(1, 1, 0);
        else if (opa == 2 && opb == 2) ZG(2, 2, 0);
        else if (opa == 1 && opb == 2) ZG(1, 2, 0);
        else ZG(2, 1, 0);
    } else if (tri == 1) {
        ZG(0, 2, 1);   // lower: C -= A·Aᴴ
    } else {
        ZG(2, 0, 2);   // upper: C -= Aᴴ·A
    }
#undef ZG
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_ZGEMM, 8.0 * m * n * k / (tri ? 2.0 : 1.0), 16.0 * (m * k + k * n + 2.0 * m * n));
}

// ---------------------------------------------------------------------------
// Triangular-solve leaf: N·x = b for nvec vectors, N the t×t (t <= 64)
// triangle with N(i, j) = T[i·ti + j·tj] (conjugated when conj), lower or
// upper, unit diagonal (taken as 1, not read) or not; element e of vector v
// at B[e·se + v·sr].
//
// 64 vectors per workgroup, 16 per wave; the triangle in LDS as real and
// imaginary planes (zeros outside it, the identity beyond t), each wave's
// vectors likewise. Blocks of 16 rows in the order of the solve: the product
// with the blocks already solved on the matrix cores (the complex product as
// four real 16×16×4 steps: re from ar·br and ai·bi, im from ar·bi + ai·br),
// then the 16×16 diagonal block by substitution with four lanes per vector
// (rows 4r..4r+3 of the block in lane r of the vector's quad), each solved
// entry the quotient x·conj(p)/|p|² by its diagonal entry and handed to the
// quad's other lanes by a broadcast.
// ---------------------------------------------------------------------------
template <typename R>
struct ZTrsmArgs {
    int t, unit, conj;
    long long ti, tj, nvec, se, sr;
    const cx<R> *T;
    cx<R> *B;
    const DevStatus *st;
    int abort;
};

// element (e, q) of a wave's vectors that lane and step u move: along e when
// it is contiguous (se = 1), along the vectors otherwise
__device__ __forceinline__ void ztrsm_eq(bool se1, int lane, int u, int &e, int &q) {
    if (se1) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
    else { q = lane & 15; e = (lane >> 4) + 4 * u; }
}

template <typename R, bool LOWER>
__global__ __launch_bounds__(256) void ztrsm_leaf_k(ZTrsmArgs<R> a) {
    if (a.abort && a.st->info) return;
    typedef LeafMfma<R> Op;
    typedef typename Op::acc_t acc_t;
    __shared__ R Nre[64][65], Nim[64][65];
    __shared__ R Xre[4][64][17], Xim[4][64][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, t = a.t;
    const long long v0 = (long long)blockIdx.x * 64 + wave * 16;   // this wave's 16 vectors
    R (*Xr)[17] = Xre[wave];
    R (*Xi)[17] = Xim[wave];
    const bool se1 = a.se == 1;
    {
        cx<R> tv[16], bv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            tv[u] = a.T[min(i, t - 1) * a.ti + min(j, t - 1) * a.tj];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            ztrsm_eq(se1, lane, u, e, q);
            bv[u] = a.B[min(e, t - 1) * a.se + min(v0 + q, a.nvec - 1) * a.sr];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            const bool in = i < t && j < t && (LOWER ? j < i : j > i);
            cx<R> v = tv[u];
            if (a.conj) v.im = -v.im;
            if (i == j) {
                if (i >= t || a.unit) v = cx<R>{R(1), R(0)};
            } else if (!in) {
                v = cx<R>{R(0), R(0)};
            }
            Nre[i][j] = v.re;
            Nim[i][j] = v.im;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            ztrsm_eq(se1, lane, u, e, q);
            const bool ok = e < t && v0 + q < a.nvec;
            Xr[e][q] = ok ? bv[u].re : R(0);
            Xi[e][q] = ok ? bv[u].im : R(0);
        }
    }
    __syncthreads();

    const int nblk = (t + 15) / 16;
    for (int s = 0; s < nblk; ++s) {
        const int I = LOWER ? s : nblk - 1 - s;
        if (s > 0) {
            // x_I -= Σ N_IJ·x_J over the blocks already solved
            acc_t arr = acc_t{0, 0, 0, 0}, aii = acc_t{0, 0, 0, 0}, aim = acc_t{0, 0, 0, 0};
            const int J0 = LOWER ? 0 : I + 1, J1 = LOWER ? I : nblk;
            for (int J = J0; J < J1; ++J) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 16 * J + 4 * kk + (lane >> 4), r = 16 * I + (lane & 15);
                    const R nr = Nre[r][k], ni = Nim[r][k], xr = Xr[k][lane & 15], xi = Xi[k][lane & 15];
                    arr = Op::mma(nr, xr, arr);
                    aii = Op::mma(ni, xi, aii);
                    aim = Op::mma(nr, xi, aim);
                    aim = Op::mma(ni, xr, aim);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * I + Op::row(lane, v);
                Xr[r][lane & 15] -= arr[v] - aii[v];
                Xi[r][lane & 15] -= aim[v];
            }
            __builtin_amdgcn_wave_barrier();
        }
        {
            const int v = lane >> 2, r4 = lane & 3, b0 = 16 * I;
            R xr[4], xi[4];
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                xr[t4] = Xr[b0 + 4 * r4 + t4][v];
                xi[t4] = Xi[b0 + 4 * r4 + t4][v];
            }
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) {
                const int j = LOWER ? s2 : 15 - s2, jb = j >> 2, jj = j & 3;
                const cx<R> p = cx<R>{Nre[b0 + j][b0 + j], Nim[b0 + j][b0 + j]};
                const cx<R> xj = cx<R>{xr[jj], xi[jj]};
                const cx<R> xs = a.unit ? xj : cdiv(xj, p);
                const cx<R> xb = cx<R>{quad_bcast_sel(xs.re, jb), quad_bcast_sel(xs.im, jb)};
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) {
                    const int r = b0 + 4 * r4 + t4;
                    const cx<R> f = csub(cx<R>{xr[t4], xi[t4]}, cmul(cx<R>{Nre[r][b0 + j], Nim[r][b0 + j]}, xb));
                    // rows after j in the order of the solve take the update,
                    // row j takes its solved value, the others stay
                    const bool after = LOWER ? (t4 > jj ? r4 >= jb : r4 > jb) : (t4 < jj ? r4 <= jb : r4 < jb);
                    const bool self = t4 == jj && r4 == jb;
                    xr[t4] = after ? f.re : (self ? xs.re : xr[t4]);
                    xi[t4] = after ? f.im : (self ? xs.im : xi[t4]);
                }
            }
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                Xr[b0 + 4 * r4 + t4][v] = xr[t4];
                Xi[b0 + 4 * r4 + t4][v] = xi[t4];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }

#pragma unroll
    for (int u = 0; u < 16; ++u) {
        int e, q;
        ztrsm_eq(se1, lane, u, e, q);
        if (e < t && v0 + q < a.nvec) a.B[e * a.se + (v0 + q) * a.sr] = cx<R>{Xr[e][q], Xi[e][q]};
    }
}

template <typename R>
static void ztrsm_leaf(Ctx &c, bool lower, bool unit, bool conj, int t, const cx<R> *T, long long ti, long long tj,
                       long long nvec, cx<R> *B, long long se, long long sr) {
    if (plan_record(c, PK_ZLEAF, t, nvec, t)) return;
    if (t <= 0 || nvec <= 0) return;
    ZTrsmArgs<R> a{t, unit ? 1 : 0, conj ? 1 : 0, ti, tj, nvec, se, sr, T, B, c.dstat, c.abort_on_info ? 1 : 0};
    trace_kernel_begin(c);
    const dim3 grid((unsigned)((nvec + 63) / 64));
    if (lower)
        rl_launch(c, ztrsm_leaf_k<R, true>, grid, dim3(256), 0, a);
    else
        rl_launch(c, ztrsm_leaf_k<R, false>, grid, dim3(256), 0, a);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_ZLEAF, 4.0 * t * t * nvec, 16.0 * (t * t / 2.0 + 2.0 * t * nvec));
}

// op(T)[r0:, c0:] and the op that goes with it (trans: 0 N, 1 T, 2 C)
template <typename R>
static inline const cx<R> *zblock(const cx<R> *T, long long ldt, int trans, long long r0, long long c0) {
    return trans ? T + c0 + r0 * ldt : T + r0 + c0 * ldt;
}

// Recursive triangular solve: side 'L': op(T)·X = B (X m×n); side 'R':
// X·op(T) = B; trans 0 N, 1 T, 2 C; X overwrites B.
template <typename R>
static void ztrsm(Ctx &c, char side, char uplo, int trans, bool unit, long long m, long long n, const cx<R> *T,
                  long long ldt, cx<R> *B, long long ldb) {
    if (m <= 0 || n <= 0) return;
    const bool lowerM = (uplo == 'L') != (trans != 0);   // op(T) is lower
    if (side == 'L') {
        if (m <= kZLeaf) {
            ztrsm_leaf<R>(c, lowerM, unit, trans == 2, (int)m, T, trans ? ldt : 1, trans ? 1 : ldt, n, B, 1, ldb);
            return;
        }
        const long long m1 = split_size(m), m2 = m - m1;
        const cx<R> *T22 = T + m1 + m1 * ldt;
        if (lowerM) {
            ztrsm<R>(c, side, uplo, trans, unit, m1, n, T, ldt, B, ldb);
            zgemm<R>(c, trans, 0, 0, m2, n, m1, -1.0, zblock(T, ldt, trans, m1, 0), ldt, B, ldb, 1.0, B + m1, ldb);
            ztrsm<R>(c, side, uplo, trans, unit, m2, n, T22, ldt, B + m1, ldb);
        } else {
            ztrsm<R>(c, side, uplo, trans, unit, m2, n, T22, ldt, B + m1, ldb);
            zgemm<R>(c, trans, 0, 0, m1, n, m2, -1.0, zblock(T, ldt, trans, 0, m1), ldt, B + m1, ldb, 1.0, B, ldb);
            ztrsm<R>(c, side, uplo, trans, unit, m1, n, T, ldt, B, ldb);
        }
    } else {
        if (n <= kZLeaf) {
            // row r of X solves N·x = b with N = op(T)ᵀ: N(i, j) = op(T)(j, i)
            ztrsm_leaf<R>(c, !lowerM, unit, trans == 2, (int)n, T, trans ? 1 : ldt, trans ? ldt : 1, m, B, ldb, 1);
            return;
        }
        const long long n1 = split_size(n), n2 = n - n1;
        const cx<R> *T22 = T + n1 + n1 * ldt;
        if (!lowerM) {
            ztrsm<R>(c, side, uplo, trans, unit, m, n1, T, ldt, B, ldb);
            zgemm<R>(c, 0, trans, 0, m, n2, n1, -1.0, B, ldb, zblock(T, ldt, trans, 0, n1), ldt, 1.0, B + n1 * ldb,
                     ldb);
            ztrsm<R>(c, side, uplo, trans, unit, m, n2, T22, ldt, B + n1 * ldb, ldb);
        } else {
            ztrsm<R>(c, side, uplo, trans, unit, m, n2, T22, ldt, B + n1 * ldb, ldb);
            zgemm<R>(c, 0, trans, 0, m, n1, n2, -1.0, B + n1 * ldb, ldb, zblock(T, ldt, trans, n1, 0), ldt, 1.0, B,
                     ldb);
            ztrsm<R>(c, side, uplo, trans, unit, m, n1, T, ldt, B, ldb);
        }
    }
}

// ---------------------------------------------------------------------------
// Cholesky leaf: a Hermitian block of n <= 64 in LDS (real and imaginary
// planes, the identity beyond n), one workgroup: l_kk = sqrt(re(a_kk)) (not
// > 0 or NaN: the first failing column off+k+1 into info, the block written
// back as it stands), the column divided by it, the trailing triangle
// updated by a_ij -= l_ik·conj(l_jk). For 'U' the block is read as L = Uᴴ and
// written back conjugate-transposed.
//
// The 64 columns go 16 at a time: one wave factors the 16-column panel (lane
// = row, the row's 16 entries in registers, the steps unrolled; each step's
// l_jk of the panel's own rows reach the other lanes by readlane), then all
// four waves subtract the panel's l_ik·conj(l_jk) from the trailing lower
// triangle on the matrix cores, the complex product as four real 16×16×4
// steps (re from lr·lr + li·li, im from li·lr − lr·li).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void zpotf2_k(int n, cx<R> *A, long long lda, int upper, long long off,
                                                DevStatus *st) {
    if (st->info) return;
    typedef LeafMfma<R> Op;
    typedef typename Op::acc_t acc_t;
    __shared__ R Sr[kZLeaf][kZLeaf + 1], Si[kZLeaf][kZLeaf + 1];
    __shared__ int fail_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        cx<R> v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = min(lane, n - 1), j = min(wave + 4 * u, n - 1);
            v[u] = upper ? A[j + (long long)i * lda] : A[i + (long long)j * lda];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = lane, j = wave + 4 * u;
            const bool in = i < n && j < n;
            const R im = upper ? -v[u].im : v[u].im;
            Sr[i][j] = in ? (j <= i ? v[u].re : R(0)) : (i == j ? R(1) : R(0));
            Si[i][j] = in && j <= i ? im : R(0);
        }
    }
    if (tid == 0) fail_s = 0;
    __syncthreads();
    const int nb = (n + 15) / 16;
    for (int J = 0; J < nb; ++J) {
        const int c0 = 16 * J;
        if (wave == 0) {
            const int r = lane;
            R xr[16], xi[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                xr[q] = Sr[r][c0 + q];
                xi[q] = Si[r][c0 + q];
            }
            int fail = 0;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int k = c0 + kk;
                if (fail == 0 && k < n) {
                    const R d = lane_bcast(xr[kk], k);
                    if (!(d > R(0))) {
                        fail = k + 1;
                    } else {
                        const R lkk = sqrt(d);
                        R lr = xr[kk] / lkk, li = xi[kk] / lkk;
                        if (r == k) { lr = lkk; li = R(0); }
                        if (r >= k) { xr[kk] = lr; xi[kk] = li; }
#pragma unroll
                        for (int q = kk + 1; q < 16; ++q) {
                            // a_rq -= l_rk·conj(l_qk), l_qk from lane c0 + q
                            const R cr = lane_bcast(lr, c0 + q), ci = lane_bcast(li, c0 + q);
                            xr[q] -= lr * cr + li * ci;
                            xi[q] -= li * cr - lr * ci;
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                Sr[r][c0 + q] = xr[q];
                Si[r][c0 + q] = xi[q];
            }
            if (r == 0) fail_s = fail;
        }
        __syncthreads();
        if (fail_s) break;
        // trailing lower triangle: tiles (I, Jt) with J < Jt <= I < nb
        const int m = nb - 1 - J;
        const int ntiles = m * (m + 1) / 2;
        for (int tt = wave; tt < ntiles; tt += 4) {
            int I = 0, acc0 = 0;
            while (acc0 + I + 1 <= tt) { acc0 += I + 1; ++I; }
            const int i0 = 16 * (J + 1 + I), j0 = 16 * (J + 1 + tt - acc0);
            acc_t are = acc_t{0, 0, 0, 0}, aim = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int c = c0 + 4 * kk + (lane >> 4);
                const R ar = Sr[i0 + (lane & 15)][c], ai = Si[i0 + (lane & 15)][c];
                const R br = Sr[j0 + (lane & 15)][c], bi = Si[j0 + (lane & 15)][c];
                are = Op::mma(ar, br, are);
                are = Op::mma(ai, bi, are);
                aim = Op::mma(ai, br, aim);
                aim = Op::mma(-ar, bi, aim);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + Op::row(lane, v), j = j0 + (lane & 15);
                Sr[i][j] -= are[v];
                Si[i][j] -= aim[v];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int i = lane, j = wave + 4 * u;
        if (i < n && j <= i) {
            if (upper) A[j + (long long)i * lda] = cx<R>{Sr[i][j], -Si[i][j]};
            else A[i + (long long)j * lda] = cx<R>{Sr[i][j], Si[i][j]};
        }
    }
    if (tid == 0 && fail_s) atomicCAS(&st->info, 0, (int)(off + fail_s));
}

template <typename R>
static void zpotrf_rec(Ctx &c, char uplo, long long n, cx<R> *A, long long lda, long long off) {
    if (n <= kZLeaf) {
        if (plan_record(c, PK_ZLEAF, n, n, n)) return;
        trace_kernel_begin(c);
        rl_launch(c, zpotf2_k<R>, dim3(1), dim3(256), 0, (int)n, A, lda, uplo == 'U' ? 1 : 0, off, c.dstat);
        RL_CHECK(hipGetLastError());
        trace_kernel_end(c, PK_ZLEAF, 4.0 * n * n * n / 3.0, 16.0 * n * n);
        return;
    }
    const long long n1 = split_size(n), n2 = n - n1;
    cx<R> *A22 = A + n1 + n1 * lda;
    c.level++;
    zpotrf_rec<R>(c, uplo, n1, A, lda, off);
    c.level--;
    if (uplo == 'L') {
        cx<R> *A21 = A + n1;
        ztrsm<R>(c, 'R', 'L', 2, false, n2, n1, A, lda, A21, lda);
        zgemm<R>(c, 0, 2, 1, n2, n2, n1, -1.0, A21, lda, A21, lda, 1.0, A22, lda);
    } else {
        cx<R> *A12 = A + n1 * lda;
        ztrsm<R>(c, 'L', 'U', 2, false, n1, n2, A, lda, A12, lda);
        zgemm<R>(c, 2, 0, 2, n2, n2, n1, -1.0, A12, lda, A12, lda, 1.0, A22, lda);
    }
    c.level++;
    zpotrf_rec<R>(c, uplo, n2, A22, lda, off + n1);
    c.level--;
}

// ---------------------------------------------------------------------------
// LU leaf: the panel A[c0:m, c0:c0+w] (w <= 16) by one workgroup of 1024
// threads, the rows in global memory. Per column: the first row of largest
// |re| + |im| (wave reduction, then across the waves in LDS), the two rows
// trade places within the panel (none for an exactly zero pivot, whose column
// then stays unscaled and which info records), the column below is divided
// by the pivot and the rank-1 update goes to the panel's later columns.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(1024) void zgetf2_k(long long m, int w, cx<R> *A, long long lda, long long c0, int *ipiv,
                                                 DevStatus *st) {
    __shared__ R kv[16];
    __shared__ long long ki[16];
    __shared__ cx<R> urow[kZLuLeaf];
    __shared__ long long piv_s;
    __shared__ int zero_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = 0; j < w; ++j) {
        const long long d = c0 + j, col = c0 + j;
        // candidate: the largest |re| + |im| in rows >= d, lowest row on ties
        R best = R(-1);
        long long bi = d;
        for (long long i = d + tid; i < m; i += 1024) {
            const R v = cabs1(A[i + col * lda]);
            if (v > best) { best = v; bi = i; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const R ov = __shfl_xor(best, off);
            const long long oi = __shfl_xor(bi, off);
            if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        if (lane == 0) { kv[wave] = best; ki[wave] = bi; }
        __syncthreads();
        if (tid == 0) {
            R b = kv[0];
            long long p = ki[0];
            for (int q = 1; q < 16; ++q)
                if (kv[q] > b || (kv[q] == b && ki[q] < p)) { b = kv[q]; p = ki[q]; }
            if (!(b >= R(0))) p = d;   // no candidate (all NaN): the diagonal row
            const cx<R> ap = A[p + col * lda];
            const int zero = ap.re == R(0) && ap.im == R(0);
            ipiv[d] = (int)(p + 1);
            if (zero) atomicCAS(&st->info, 0, (int)(d + 1));
            piv_s = zero ? d : p;
            zero_s = zero;
        }
        __syncthreads();
        const long long p = piv_s;
        const int zero = zero_s;
        if (p != d && tid < w) {
            const long long cc = c0 + tid;
            const cx<R> t = A[d + cc * lda];
            A[d + cc * lda] = A[p + cc * lda];
            A[p + cc * lda] = t;
        }
        __syncthreads();
        if (tid < w - j) urow[tid] = A[d + (col + tid) * lda];
        __syncthreads();
        const cx<R> piv = urow[0];
        for (long long i = d + 1 + tid; i < m; i += 1024) {
            cx<R> l = A[i + col * lda];
            if (!zero) {
                l = cdiv(l, piv);
                A[i + col * lda] = l;
            }
            for (int q = 1; q < w - j; ++q) {
                cx<R> &e = A[i + (col + q) * lda];
                e = csub(e, cmul(l, urow[q]));
            }
        }
        __syncthreads();
    }
}

// the interchanges ipiv[k1:k2) in order on every column outside [c0, c0 + w)
template <typename R>
__global__ void zlaswp_k(long long ncols, long long c0, int w, cx<R> *A, long long lda, const int *ipiv, long long k1,
                         long long k2) {
    const long long jj = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj >= ncols - w) return;
    const long long j = jj < c0 ? jj : jj + w;
    cx<R> *col = A + j * lda;
    for (long long k = k1; k < k2; ++k) {
        const long long p = ipiv[k] - 1;
        if (p != k) {
            const cx<R> t = col[k];
            col[k] = col[p];
            col[p] = t;
        }
    }
}

template <typename R>
static void zgetrf_rec(Ctx &c, long long m, long long ncols, cx<R> *A, long long lda, int *ipiv, long long c0,
                       long long w) {
    if (w <= kZLuLeaf) {
        if (plan_record(c, PK_ZLEAF, m - c0, w, w)) return;
        // the cooperative panel (row blocks across the CUs), its interchanges
        // gathered into the other columns through its source-row list; one
        // workgroup and the interchanges in order when the chip cannot hold
        // the panel's grid
        if (getf2_panel_cx<cx<R>>(c, m, (int)w, A, lda, c0, ipiv)) {
            if (ncols > w) laswp_leaf<cx<R>>(c, A, lda, c0, (int)w, m, ipiv, 0, ncols);
            return;
        }
        trace_kernel_begin(c);
        rl_launch(c, zgetf2_k<R>, dim3(1), dim3(1024), 0, m, (int)w, A, lda, c0, ipiv, c.dstat);
        RL_CHECK(hipGetLastError());
        trace_kernel_end(c, PK_ZLEAF, 8.0 * (m - c0) * w * w / 2.0, 32.0 * (m - c0) * w);
        if (ncols > w)
            hipLaunchKernelGGL(zlaswp_k<R>, dim3((unsigned)((ncols - w + 255) / 256)), dim3(256), 0, c.stream, ncols, c0,
                               (int)w, A, lda, (const int *)ipiv, c0, c0 + w);
        RL_CHECK(hipGetLastError());
        return;
    }
    const long long w1 = split_size(w), w2 = w - w1;
    c.level++;
    zgetrf_rec<R>(c, m, ncols, A, lda, ipiv, c0, w1);
    c.level--;
    cx<R> *A11 = A + c0 + c0 * lda, *A12 = A + c0 + (c0 + w1) * lda;
    cx<R> *A21 = A + (c0 + w1) + c0 * lda, *A22 = A + (c0 + w1) + (c0 + w1) * lda;
    ztrsm<R>(c, 'L', 'L', 0, true, w1, w2, A11, lda, A12, lda);
    zgemm<R>(c, 0, 0, 0, m - c0 - w1, w2, w1, -1.0, A21, lda, A12, lda, 1.0, A22, lda);
    c.level++;
    zgetrf_rec<R>(c, m, ncols, A, lda, ipiv, c0 + w1, w2);
    c.level--;
}

template <typename R>
void zpotrf_top(Ctx &c, char uplo, long long n, void *A, long long lda) {
    zpotrf_rec<R>(c, uplo, n, (cx<R> *)A, lda, 0);
}

template <typename R>
void zgetrf_top(Ctx &c, long long m, long long n, void *Av, long long lda, int *ipiv) {
    cx<R> *A = (cx<R> *)Av;
    const long long mn = m < n ? m : n;
    if (mn <= 0) return;
    c.lu_batch = false;   // interchanges go to the other columns after every panel
    zgetrf_rec<R>(c, m, n, A, lda, ipiv, 0, mn);
    if (n > m) ztrsm<R>(c, 'L', 'L', 0, true, m, n - m, A, lda, A + m * lda, lda);
}

template <typename R>
void zgemm_top(Ctx &c, int opa, int opb, long long m, long long n, long long k, double alpha, const void *A,
               long long lda, const void *B, long long ldb, double beta, void *C, long long ldc) {
    zgemm<R>(c, opa, opb, 0, m, n, k, alpha, (const cx<R> *)A, lda, (const cx<R> *)B, ldb, beta, (cx<R> *)C, ldc);
}

template void zpotrf_top<double>(Ctx &, char, long long, void *, long long);
template void zpotrf_top<float>(Ctx &, char, long long, void *, long long);
template void zgetrf_top<double>(Ctx &, long long, long long, void *, long long, int *);
template void zgetrf_top<float>(Ctx &, long long, long long, void *, long long, int *);
template void zgemm_top<double>(Ctx &, int, int, long long, long long, long long, double, const void *, long long,
                                const void *, long long, double, void *, long long);
template void zgemm_top<float>(Ctx &, int, int, long long, long long, long long, double, const void *, long long,
                               const void *, long long, double, void *, long long);

}  // namespace rl
