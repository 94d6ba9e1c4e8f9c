// Triangular inverse (xtrtri), triangular product with its own transpose
// (xlauum) and the triangular matrix product they are built from (BLAS-3
// xtrmm): the follow-on that turns a Cholesky factor into the inverse of the
// SPD matrix (Sec. 5: xtrtri and xlauum serve the SPD inversion xpotri).
//
// The inversion is the paper's worked example of a recursive algorithm
// (Sec. 3, Fig. recursive_alg): split the lower triangle into A_TL, A_BL, A_BR
// and apply
//   (1) A_TL := A_TL⁻¹                    (recursion)
//   (2) A_BL := A_BL·A_TL                 (triangular product, the inverted A_TL)
//   (3) A_BL := −A_BR⁻¹·A_BL              (triangular solve, the original A_BR)
//   (4) A_BR := A_BR⁻¹                    (recursion)
// with the unblocked inversion below the crossover size. The sign of (3) is
// carried by step (2) here (A_BL := −A_BL·A_TL), which gives the same matrix.
// The upper triangle is the mirror image.
//
// xlauum (lower: A := Lᵀ·L) follows the same split: Lᵀ·L has A_TL block
// L_TLᵀ·L_TL + L_BLᵀ·L_BL, A_BL block L_BRᵀ·L_BL and A_BR block L_BRᵀ·L_BR, so
//   lauum(A_TL); A_TL += A_BLᵀ·A_BL (SYRK); A_BL := A_BRᵀ·A_BL (TRMM);
//   lauum(A_BR).
//
// Device kernels (gfx950):
//  * trmm_leaf_k: y = α·N·x for 64 vectors per workgroup (16 per wave), N a
//    t×t triangle (t <= 64) staged in LDS with zeros outside it; the product
//    runs on the FP64 matrix cores (16×16×4 blocks, only the blocks inside
//    the triangle). Same operand addressing as the triangular-solve leaf.
//  * the unblocked inverse of a t×t triangle (t <= 64) is the triangular-solve
//    leaf run against the identity (trti2_leaf, next to that leaf).
//  * lauu2_k: Lᵀ·L (or U·Uᵀ) of a t×t triangle (t <= 64), 256 threads, 16
//    outputs each, straight from LDS.
//  * diag_zero_k: the first exact zero on the diagonal (LAPACK reports it
//    before inverting anything); every later kernel of the call then skips.
#include "common.hpp"
#include "wg.hpp"

#include <algorithm>

namespace rl {

static inline bool isc(char a, char b) { return a == b || a == (char)(b + ('a' - 'A')); }

// ---------------------------------------------------------------------------
// Leaf triangular product: y := α·N·x, N(i, j) = T[i*ti + j*tj] on the
// triangle (LOWER: j <= i), diagonal 1 if unit; element e of vector r is
// B[e*se + r*sr].
// ---------------------------------------------------------------------------
template <bool LOWER>
__global__ __launch_bounds__(256) void trmm_leaf_k(int unit, int t, const double *__restrict__ T, long long ti,
                                                   long long tj, long long nvec, double *__restrict__ B,
                                                   long long se, long long sr, double alpha, const int *abort) {
    if (abort && *abort) return;
    __shared__ double Nsh[64][65];
    __shared__ double Xsh[4][64][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long v0 = (long long)blockIdx.x * 64 + wave * 16;
    double (*X)[17] = Xsh[wave];
    {
        double tv[16], bv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            tv[u] = T[min(i, t - 1) * ti + min(j, t - 1) * tj];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            if (se == 1) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            bv[u] = B[min(e, t - 1) * se + min(v0 + q, nvec - 1) * sr];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            const bool in = i < t && j < t && (LOWER ? (j < i) : (j > i));
            const bool dg = i == j && i < t;
            Nsh[i][j] = in ? tv[u] : (dg ? (unit ? 1.0 : tv[u]) : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int e, q;
            if (se == 1) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
            else { q = lane & 15; e = (lane >> 4) + 4 * u; }
            X[e][q] = (e < t && v0 + q < nvec) ? bv[u] : 0.0;
        }
    }
    __syncthreads();

    const int nblk = (t + 15) / 16;
    d4 acc[4];
#pragma unroll
    for (int I = 0; I < 4; ++I) {
        acc[I] = d4{0, 0, 0, 0};
        if (I < nblk) {
            const int J0 = LOWER ? 0 : I, J1 = LOWER ? I : nblk - 1;
            for (int J = J0; J <= J1; ++J) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 16 * J + 4 * kk + (lane >> 4);
                    acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(Nsh[16 * I + (lane & 15)][k], X[k][lane & 15],
                                                                  acc[I], 0, 0, 0);
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    // FP64 16×16×4 result layout: element v of lane l is D[l/16 + 4v][l%16]
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) X[16 * I + (lane >> 4) + 4 * v][lane & 15] = alpha * acc[I][v];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        int e, q;
        if (se == 1) { e = (lane & 15) + 16 * (u & 3); q = (lane >> 4) + 4 * (u >> 2); }
        else { q = lane & 15; e = (lane >> 4) + 4 * u; }
        if (e < t && v0 + q < nvec) B[e * se + (v0 + q) * sr] = X[e][q];
    }
}

static void trmm_leaf(Ctx &c, bool lower_eff, bool unit, int t, const double *T, long long ti, long long tj,
                      long long nvec, double *B, long long se, long long sr, double alpha) {
    if (plan_record(c, PK_TRMM_LEAF, t, nvec, t)) return;
    if (t <= 0 || nvec <= 0) return;
    const int *abort = c.abort_on_info ? &c.dstat->info : nullptr;
    const int grid = (int)((nvec + 63) / 64);
    trace_kernel_begin(c);
    if (lower_eff)
        rl_launch(c, trmm_leaf_k<true>, dim3(grid), dim3(256), 0, (int)unit, t, T, ti, tj, nvec, B, se, sr,
                  alpha, abort);
    else
        rl_launch(c, trmm_leaf_k<false>, dim3(grid), dim3(256), 0, (int)unit, t, T, ti, tj, nvec, B, se, sr,
                  alpha, abort);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_TRMM_LEAF, (double)t * t * nvec, 8.0 * (t * t / 2.0 + 2.0 * t * nvec));
}

// ---------------------------------------------------------------------------
// Triangular product of a whole triangle in one launch (triangles of more
// than one leaf and at most kTrmmBlk rows): y := α·N·x for every vector, N
// the t×t triangle (LOWER: j <= i) as in trmm_leaf_k, x read from a copy of B
// in workspace (element e of vector r at X[e*xe + r*xr]) so that the output
// tiles of one launch are independent. A workgroup takes 64 rows × 64
// vectors, four waves of 32×32 on the FP64 matrix cores; K runs over the
// tile's part of the triangle only (k <= i for a lower N, k >= i for an
// upper one), 16 at a time, double-buffered through LDS. The K step that
// crosses the diagonal stages zeros outside the triangle (and 1 on a unit
// diagonal, which is not read). Heaviest tile rows are dealt first.
// ---------------------------------------------------------------------------
constexpr int kTrmmBlk = 1024;

struct TrmmBlkArgs {
    int unit, t, tiles_e;
    const double *T;
    long long ti, tj;
    const double *X;
    long long xe, xr;
    double *B;
    long long se, sr, nvec;
    double alpha;
    const int *abort;
};

template <bool LOWER, int TS>
__global__ __launch_bounds__(256) void trmm_blk_k(TrmmBlkArgs a) {
    constexpr int MI = TS / 32, EL = TS / 16;   // 16-blocks per wave and side, staged elements per thread
    if (a.abort && *a.abort) return;
    __shared__ double Ns[2][16][TS + 1];   // [k][row]
    __shared__ double Xs[2][16][TS + 1];   // [k][vector]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, t = a.t;
    const int rt = (int)(blockIdx.x % a.tiles_e);
    const int te = LOWER ? a.tiles_e - 1 - rt : rt;
    const long long v0 = (long long)(blockIdx.x / a.tiles_e) * TS;
    const int e0 = TS * te;
    const int kb = LOWER ? 0 : e0, ke = LOWER ? min(e0 + TS, t) : t;
    const int wm = (wave & 1) * (TS / 2), wn = (wave >> 1) * (TS / 2);
    const bool tcol = a.ti == 1, xcol = a.xe == 1;   // contiguous along the rows / along k
    double rn[EL], rx[EL];
    // staging coordinates (branch-free selects: reference outputs chosen by a
    // branch end up in scratch): row i / vector v and k of element u
    auto n_i = [&](int u) { return tcol ? tid % TS : (tid >> 4) + 16 * u; };
    auto n_k = [&](int u) { return tcol ? tid / TS + (256 / TS) * u : tid & 15; };
    auto x_k = [&](int u) { return xcol ? tid & 15 : tid / TS + (256 / TS) * u; };
    auto x_v = [&](int u) { return xcol ? (tid >> 4) + 16 * u : tid % TS; };
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < EL; ++u) {
            const int i = n_i(u), k = n_k(u);
            const int gi = e0 + i, gk = k0 + k;
            const bool in = gi < t && gk < t && (LOWER ? gk <= gi : gk >= gi);
            rn[u] = !in ? 0.0 : ((gk == gi && a.unit) ? 1.0 : a.T[gi * a.ti + gk * a.tj]);
        }
#pragma unroll
        for (int u = 0; u < EL; ++u) {
            const int k = x_k(u), v = x_v(u);
            const int gk = k0 + k;
            const long long gv = v0 + v;
            rx[u] = (gk < ke && gv < a.nvec) ? a.X[gk * a.xe + gv * a.xr] : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < EL; ++u) {
            Ns[buf][n_k(u)][n_i(u)] = rn[u];
        }
#pragma unroll
        for (int u = 0; u < EL; ++u) {
            Xs[buf][x_k(u)][x_v(u)] = rx[u];
        }
    };
    d4 acc[MI][MI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MI; ++j) acc[i][j] = d4{0, 0, 0, 0};
    const int KT = (ke - kb + 15) / 16;   // >= 1
    load(kb);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < KT) load(kb + 16 * (kt + 1));
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            double av[MI], bv[MI];
#pragma unroll
            for (int i = 0; i < MI; ++i) av[i] = Ns[buf][kr][wm + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < MI; ++j) bv[j] = Xs[buf][kr][wn + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < MI; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < KT) store(buf ^ 1);
        __syncthreads();
    }
    // FP64 16×16×4 result layout: element v of lane l is D[l/16 + 4v][l%16]
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MI; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = e0 + wm + 16 * i + (lane >> 4) + 4 * v;
                const long long r = v0 + wn + 16 * j + (lane & 15);
                if (e < t && r < a.nvec) a.B[e * a.se + r * a.sr] = a.alpha * acc[i][j][v];
            }
}

// X := B (t elements of nvec vectors), contiguous along whichever index B is
__global__ __launch_bounds__(256) void trmm_copy_k(const double *__restrict__ B, long long se, long long sr,
                                                   double *__restrict__ X, int t, long long nvec, const int *abort) {
    if (abort && *abort) return;
    const long long nel = (long long)t * nvec, stride = (long long)gridDim.x * 256;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < nel; idx += stride) {
        if (se == 1) {
            const long long e = idx % t, r = idx / t;
            X[idx] = B[e + r * sr];
        } else {
            const long long r = idx % nvec, e = idx / nvec;
            X[idx] = B[e * se + r];
        }
    }
}

static void trmm_blk(Ctx &c, bool lower_eff, bool unit, int t, const double *T, long long ti, long long tj,
                     long long nvec, double *B, long long se, long long sr, double alpha) {
    if (plan_record(c, PK_TRMM, t, nvec, t)) return;
    if (t <= 0 || nvec <= 0) return;
    double *X = (double *)workspace(c, kSlotTrmm, (size_t)t * (size_t)nvec * sizeof(double));
    if (!X) return;
    const int *abort = c.abort_on_info ? &c.dstat->info : nullptr;
    trace_begin(c, PK_TRMM);
    const long long nel = (long long)t * nvec;
    hipLaunchKernelGGL(trmm_copy_k, dim3((unsigned)std::min<long long>((nel + 255) / 256, 1LL << 20)), dim3(256), 0,
                       c.stream, B, se, sr, X, t, nvec, abort);
    RL_CHECK(hipGetLastError());
    // 64×64 output tiles, or 32×32 ones when the 64-tiles would not give every
    // CU two workgroups
    const bool small = (long long)((t + 63) / 64) * ((nvec + 63) / 64) < 2LL * c.num_cu;
    const int ts = small ? 32 : 64;
    TrmmBlkArgs a{unit ? 1 : 0, t, (t + ts - 1) / ts, T, ti, tj, X, se == 1 ? 1 : nvec, se == 1 ? (long long)t : 1,
                  B, se, sr, nvec, alpha, abort};
    const dim3 grid((unsigned)((long long)a.tiles_e * ((nvec + ts - 1) / ts)));
    if (small) {
        if (lower_eff) hipLaunchKernelGGL((trmm_blk_k<true, 32>), grid, dim3(256), 0, c.stream, a);
        else hipLaunchKernelGGL((trmm_blk_k<false, 32>), grid, dim3(256), 0, c.stream, a);
    } else {
        if (lower_eff) hipLaunchKernelGGL((trmm_blk_k<true, 64>), grid, dim3(256), 0, c.stream, a);
        else hipLaunchKernelGGL((trmm_blk_k<false, 64>), grid, dim3(256), 0, c.stream, a);
    }
    RL_CHECK(hipGetLastError());
    trace_end(c, PK_TRMM, (double)t * t * nvec, 8.0 * (t * t / 2.0 + 3.0 * t * nvec));
}

// Pointer to the block op(T)[r0:, c0:] in storage.
static inline const double *opblk(const double *T, long long ldt, bool trans, long long r0, long long c0) {
    return trans ? T + c0 + r0 * ldt : T + r0 + c0 * ldt;
}

// B := α·op(T)·B (side 'L', triangle m×m) or B := α·B·op(T) (side 'R',
// triangle n×n), recursive: the part of B that the off-diagonal product reads
// is transformed last, the other part first, so every block of B is read in
// its original state.
void trmm(Ctx &c, char side, char uplo, char trans, char diag, long long m, long long n, double alpha,
          const double *T, long long ldt, double *B, long long ldb) {
    if (m <= 0 || n <= 0) return;
    const bool tr = isc(trans, 'T') || isc(trans, 'C');
    const bool lowerM = isc(uplo, 'L') != tr;   // op(T) is lower triangular
    const bool unit = isc(diag, 'U');
    const char opc = tr ? 'T' : 'N';
    const int leaf = c.plan && c.plan_leaf > 0 ? c.plan_leaf : kTrsmLeaf;
    if (isc(side, 'L')) {
        if (m <= leaf) {
            trmm_leaf(c, lowerM, unit, (int)m, T, tr ? ldt : 1, tr ? 1 : ldt, n, B, 1, ldb, alpha);
            return;
        }
        if (m <= kTrmmBlk) {
            trmm_blk(c, lowerM, unit, (int)m, T, tr ? ldt : 1, tr ? 1 : ldt, n, B, 1, ldb, alpha);
            return;
        }
        const long long m1 = split_size(m), m2 = m - m1;
        const double *T22 = T + m1 + m1 * ldt;
        if (lowerM) {
            // [B1; B2] := α·[T11·B1; T21·B1 + T22·B2]
            trmm(c, side, uplo, trans, diag, m2, n, alpha, T22, ldt, B + m1, ldb);
            gemm<double, double, double>(c, Mfma::F64, opc, 'N', 0, m2, n, m1, alpha, opblk(T, ldt, tr, m1, 0), ldt,
                                         B, ldb, 1.0, B + m1, ldb);
            trmm(c, side, uplo, trans, diag, m1, n, alpha, T, ldt, B, ldb);
        } else {
            // [B1; B2] := α·[T11·B1 + T12·B2; T22·B2]
            trmm(c, side, uplo, trans, diag, m1, n, alpha, T, ldt, B, ldb);
            gemm<double, double, double>(c, Mfma::F64, opc, 'N', 0, m1, n, m2, alpha, opblk(T, ldt, tr, 0, m1), ldt,
                                         B + m1, ldb, 1.0, B, ldb);
            trmm(c, side, uplo, trans, diag, m2, n, alpha, T22, ldt, B + m1, ldb);
        }
    } else {
        if (n <= leaf) {
            // row r of B: b_r := α·b_r·op(T), i.e. y = α·op(T)ᵀ·x
            trmm_leaf(c, !lowerM, unit, (int)n, T, tr ? 1 : ldt, tr ? ldt : 1, m, B, ldb, 1, alpha);
            return;
        }
        if (n <= kTrmmBlk) {
            trmm_blk(c, !lowerM, unit, (int)n, T, tr ? 1 : ldt, tr ? ldt : 1, m, B, ldb, 1, alpha);
            return;
        }
        const long long n1 = split_size(n), n2 = n - n1;
        const double *T22 = T + n1 + n1 * ldt;
        if (lowerM) {
            // [B1 B2] := α·[B1·T11 + B2·T21, B2·T22]
            trmm(c, side, uplo, trans, diag, m, n1, alpha, T, ldt, B, ldb);
            gemm<double, double, double>(c, Mfma::F64, 'N', opc, 0, m, n1, n2, alpha, B + n1 * ldb, ldb,
                                         opblk(T, ldt, tr, n1, 0), ldt, 1.0, B, ldb);
            trmm(c, side, uplo, trans, diag, m, n2, alpha, T22, ldt, B + n1 * ldb, ldb);
        } else {
            // [B1 B2] := α·[B1·T11, B1·T12 + B2·T22]
            trmm(c, side, uplo, trans, diag, m, n2, alpha, T22, ldt, B + n1 * ldb, ldb);
            gemm<double, double, double>(c, Mfma::F64, 'N', opc, 0, m, n2, n1, alpha, B, ldb,
                                         opblk(T, ldt, tr, 0, n1), ldt, 1.0, B + n1 * ldb, ldb);
            trmm(c, side, uplo, trans, diag, m, n1, alpha, T, ldt, B, ldb);
        }
    }
}

// ---------------------------------------------------------------------------
// Unblocked Lᵀ·L (lower) or U·Uᵀ (upper) of a t×t triangle (t <= 64):
// thread (i = tid % 64, j = tid / 64 + 4u) forms entry (i, j) over all k with
// zeros outside the triangle; the result's triangle is written back.
// ---------------------------------------------------------------------------
template <bool LOWER>
__global__ __launch_bounds__(256) void lauu2_k(int t, double *__restrict__ A, long long lda, const int *abort) {
    if (abort && *abort) return;
    __shared__ double L[64][65];
    const int tid = threadIdx.x;
    {
        double tv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            tv[u] = A[min(i, t - 1) + min(j, t - 1) * lda];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, i = idx % 64, j = idx / 64;
            const bool in = i < t && j < t && (LOWER ? (j <= i) : (j >= i));
            L[i][j] = in ? tv[u] : 0.0;
        }
    }
    __syncthreads();
    const int i = tid & 63, j0 = tid >> 6;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int k = 0; k < 64; ++k) {
        // lower: (Lᵀ·L)_ij = Σ_k l_ki·l_kj; upper: (U·Uᵀ)_ij = Σ_k u_ik·u_jk
        const double a = LOWER ? L[k][i] : L[i][k];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int j = j0 + 4 * u;
            acc[u] += a * (LOWER ? L[k][j] : L[j][k]);
        }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int j = j0 + 4 * u;
        if (i < t && j < t && (LOWER ? i >= j : i <= j)) A[i + (long long)j * lda] = acc[u];
    }
}

static void lauu2(Ctx &c, bool lower, int t, double *A, long long lda) {
    if (plan_record(c, PK_LAUU2, t, t, t)) return;
    if (t <= 0) return;
    const int *abort = c.abort_on_info ? &c.dstat->info : nullptr;
    trace_kernel_begin(c);
    if (lower)
        rl_launch(c, lauu2_k<true>, dim3(1), dim3(256), 0, t, A, lda, abort);
    else
        rl_launch(c, lauu2_k<false>, dim3(1), dim3(256), 0, t, A, lda, abort);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_LAUU2, (double)t * t * t / 3.0, 8.0 * t * t);
}

// ---------------------------------------------------------------------------
// The inversion's bottom node (64 < n <= 128) in one launch: the four steps
// of Fig. recursive_alg on LDS, with n1 = split_size(n), n2 = n - n1 (both
// <= 64) and the triangle read as lower (an upper one as its transpose, whose
// inverse is the transpose of the inverse):
//   (1) A11 := A11⁻¹          the leaf solve against the identity (solve64);
//   (2) A21 := −A21·A11⁻¹     on the matrix cores;
//   (3) A21 := A22⁻¹·A21      the leaf solve with the original A22;
//   (4) A22 := A22⁻¹          the leaf solve against the identity.
// A unit diagonal is taken as 1 and neither read nor written.
// ---------------------------------------------------------------------------
template <bool LOWER>
__global__ __launch_bounds__(256) void trtri128_k(int n, int unit, double *__restrict__ A, long long lda,
                                                  const int *abort) {
    if (abort && *abort) return;
    __shared__ double N1[64][65], N2[64][65], S21[64][65];
    __shared__ double X[4][64][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n1 = (int)split_size(n), n2 = n - n1;
    // element (i, j) of the lower view: A[i·si + j·sj]
    const long long si = LOWER ? 1 : lda, sj = LOWER ? lda : 1;
    double *A21 = A + n1 * si, *A22 = A + n1 * si + n1 * sj;
    {
        double a[16], b[16], c[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, p = idx & 63, q = idx >> 6;
            const int i = LOWER ? p : q, j = LOWER ? q : p;   // the contiguous index across the threads
            a[u] = A[min(i, n1 - 1) * si + min(j, n1 - 1) * sj];
            b[u] = A22[min(i, n2 - 1) * si + min(j, n2 - 1) * sj];
            c[u] = A21[min(i, n2 - 1) * si + min(j, n1 - 1) * sj];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = tid + 256 * u, p = idx & 63, q = idx >> 6;
            const int i = LOWER ? p : q, j = LOWER ? q : p;
            // the triangles: zeros above, a unit diagonal as 1, the identity beyond the size
            N1[i][j] = (i < n1 && j < i) ? a[u] : (i == j ? ((i < n1 && !unit) ? a[u] : 1.0) : 0.0);
            N2[i][j] = (i < n2 && j < i) ? b[u] : (i == j ? ((i < n2 && !unit) ? b[u] : 1.0) : 0.0);
            S21[i][j] = (i < n2 && j < n1) ? c[u] : 0.0;
        }
        // (1): the identity's columns 16·wave .. 16·wave + 15 as this wave's vectors
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = (lane >> 4) + 4 * u, q = lane & 15;
            X[wave][e][q] = (e == 16 * wave + q && e < n1) ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    solve64<double, true>(N1, X[wave], n1, unit, lane);
    __syncthreads();
    // (2) row block `wave` of A21: −A21·A11⁻¹ (column j of A11⁻¹ is vector j % 16 of wave j / 16)
    {
        d4 acc[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) acc[jb] = d4{0, 0, 0, 0};
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 16 * kb + 4 * kk + (lane >> 4);
                const double av = S21[16 * wave + (lane & 15)][k];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, X[jb][k][lane & 15], acc[jb], 0, 0, 0);
            }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int v = 0; v < 4; ++v) S21[16 * wave + (lane >> 4) + 4 * v][16 * jb + (lane & 15)] = -acc[jb][v];
    }
    // A11⁻¹ out (its triangle; a unit diagonal stays as it is)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = (lane >> 4) + 4 * u, q = lane & 15, j = 16 * wave + q;
        if (e < n1 && j < n1 && (unit ? e > j : e >= j)) A[e * si + j * sj] = X[wave][e][q];
    }
    __syncthreads();
    // (3) the columns of A21 as vectors: X[w][e][q] = A21(e, 16w + q)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = (lane >> 4) + 4 * u, q = lane & 15;
        X[wave][e][q] = S21[e][16 * wave + q];
    }
    __builtin_amdgcn_wave_barrier();
    solve64<double, true>(N2, X[wave], n2, unit, lane);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = (lane >> 4) + 4 * u, q = lane & 15, j = 16 * wave + q;
        if (e < n2 && j < n1) A21[e * si + j * sj] = X[wave][e][q];
    }
    __builtin_amdgcn_wave_barrier();
    // (4)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = (lane >> 4) + 4 * u, q = lane & 15;
        X[wave][e][q] = (e == 16 * wave + q && e < n2) ? 1.0 : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    solve64<double, true>(N2, X[wave], n2, unit, lane);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = (lane >> 4) + 4 * u, q = lane & 15, j = 16 * wave + q;
        if (e < n2 && j < n2 && (unit ? e > j : e >= j)) A22[e * si + j * sj] = X[wave][e][q];
    }
}

static void trtri128(Ctx &c, bool lower, bool unit, int n, double *A, long long lda) {
    if (plan_record(c, PK_TRTI2, n, n, n)) return;
    const int *abort = c.abort_on_info ? &c.dstat->info : nullptr;
    trace_kernel_begin(c);
    if (lower)
        rl_launch(c, trtri128_k<true>, dim3(1), dim3(256), 0, n, (int)unit, A, lda, abort);
    else
        rl_launch(c, trtri128_k<false>, dim3(1), dim3(256), 0, n, (int)unit, A, lda, abort);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_TRTI2, (double)n * n * n / 3.0, 16.0 * n * n);
}

// ---------------------------------------------------------------------------
// lauum of a whole triangle of 64 < t <= 128 rows in one launch (the
// recursion's bottom node): entry (i, j), i >= j, of Lᵀ·L is the sum over
// k >= i of l_ki·l_kj (U·Uᵀ is the same with L = Uᵀ). The triangle is staged
// in LDS before anything is written, so the result overwrites it in place;
// 16×16 tiles of the result's lower triangle go to the four waves, each the
// sum on the FP64 matrix cores over k from its tile row on.
// ---------------------------------------------------------------------------
template <bool LOWER>
__global__ __launch_bounds__(256) void lauum128_k(int t, double *__restrict__ A, long long lda, const int *abort) {
    if (abort && *abort) return;
    __shared__ double L[128][129];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        // element (i, j) of L: A[i + j·lda] (lower) or A[j + i·lda] (L = Uᵀ);
        // the contiguous index runs fastest across the threads
        double v[64];
#pragma unroll
        for (int u = 0; u < 64; ++u) {
            const int idx = tid + 256 * u, a = idx & 127, b = idx >> 7;
            const int i = LOWER ? a : b, j = LOWER ? b : a;
            v[u] = A[LOWER ? min(i, t - 1) + (long long)min(j, t - 1) * lda
                           : min(j, t - 1) + (long long)min(i, t - 1) * lda];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < 64; ++u) {
            const int idx = tid + 256 * u, a = idx & 127, b = idx >> 7;
            const int i = LOWER ? a : b, j = LOWER ? b : a;
            L[i][j] = (i < t && j < t && j <= i) ? v[u] : 0.0;
        }
    }
    __syncthreads();
    const int nt = (t + 15) / 16, ntiles = nt * (nt + 1) / 2;
    for (int tt = wave; tt < ntiles; tt += 4) {
        int I = 0, a0 = 0;
        while (a0 + I + 1 <= tt) { a0 += I + 1; ++I; }
        const int J = tt - a0;
        d4 acc = d4{0, 0, 0, 0};
        for (int k0 = 16 * I; k0 < 16 * nt; k0 += 4) {
            const int k = k0 + (lane >> 4);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(L[k][16 * I + (lane & 15)], L[k][16 * J + (lane & 15)], acc,
                                                       0, 0, 0);
        }
        // FP64 16×16×4 result layout: element v of lane l is D[l/16 + 4v][l%16]
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + (lane >> 4) + 4 * v, j = 16 * J + (lane & 15);
            if (i < t && j <= i) {
                if (LOWER) A[i + (long long)j * lda] = acc[v];
                else A[j + (long long)i * lda] = acc[v];
            }
        }
    }
}

static void lauum128(Ctx &c, bool lower, int t, double *A, long long lda) {
    if (plan_record(c, PK_LAUU2, t, t, t)) return;
    const int *abort = c.abort_on_info ? &c.dstat->info : nullptr;
    trace_kernel_begin(c);
    if (lower)
        rl_launch(c, lauum128_k<true>, dim3(1), dim3(256), 0, t, A, lda, abort);
    else
        rl_launch(c, lauum128_k<false>, dim3(1), dim3(256), 0, t, A, lda, abort);
    RL_CHECK(hipGetLastError());
    trace_kernel_end(c, PK_LAUU2, (double)t * t * t / 3.0, 16.0 * t * t);
}

// ---------------------------------------------------------------------------
// First exact zero on the diagonal (1-based) into the call's info, 0 if none.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void diag_zero_k(long long n, const double *__restrict__ A, long long lda,
                                                   DevStatus *st) {
    __shared__ long long best[256];
    long long b = n;
    for (long long i = threadIdx.x; i < n; i += 256)
        if (A[i + i * lda] == 0.0) { b = i; break; }
    best[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) best[threadIdx.x] = min(best[threadIdx.x], best[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && best[0] < n) st->info = (int)(best[0] + 1);
}

void diag_zero(Ctx &c, long long n, const double *A, long long lda) {
    if (plan_record(c, PK_OTHER, n, 0, 0)) return;
    hipLaunchKernelGGL(diag_zero_k, dim3(1), dim3(256), 0, c.stream, n, A, lda, c.dstat);
    RL_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Recursions (Fig. recursive_alg for the inverse; the same split for lauum).
// ---------------------------------------------------------------------------
void trtri_rec(Ctx &c, char uplo, char diag, long long n, double *A, long long lda) {
    const int leaf = c.plan && c.plan_leaf > 0 ? c.plan_leaf : kTrsmLeaf;
    const bool lower = isc(uplo, 'L');
    if (n <= leaf) {
        trti2_leaf(c, lower, isc(diag, 'U'), (int)n, A, lda);
        return;
    }
    if (n <= 2 * kTrsmLeaf && !(c.plan && c.plan_leaf > 0)) {
        trtri128(c, lower, isc(diag, 'U'), (int)n, A, lda);   // the bottom node in one launch
        return;
    }
    const long long n1 = split_size(n), n2 = n - n1;
    double *A22 = A + n1 + n1 * lda;
    c.level++;
    trtri_rec(c, uplo, diag, n1, A, lda);                                   // (1) A_TL := A_TL⁻¹
    c.level--;
    if (lower) {
        double *A21 = A + n1;
        trmm(c, 'R', 'L', 'N', diag, n2, n1, -1.0, A, lda, A21, lda);        // (2) A_BL := −A_BL·A_TL
        trsm<double, double>(c, Mfma::F64, 'L', 'L', 'N', diag, n2, n1, A22, lda, A21, lda);  // (3) A_BR⁻¹·A_BL
    } else {
        double *A12 = A + n1 * lda;
        trmm(c, 'L', 'U', 'N', diag, n1, n2, -1.0, A, lda, A12, lda);        // (2) A_TR := −A_TL·A_TR
        trsm<double, double>(c, Mfma::F64, 'R', 'U', 'N', diag, n1, n2, A22, lda, A12, lda);  // (3) A_TR·A_BR⁻¹
    }
    c.level++;
    trtri_rec(c, uplo, diag, n2, A22, lda);                                 // (4) A_BR := A_BR⁻¹
    c.level--;
}

void lauum_rec(Ctx &c, char uplo, long long n, double *A, long long lda) {
    const int leaf = c.plan && c.plan_leaf > 0 ? c.plan_leaf : kTrsmLeaf;
    const bool lower = isc(uplo, 'L');
    if (n <= leaf) {
        lauu2(c, lower, (int)n, A, lda);
        return;
    }
    if (n <= 2 * kTrsmLeaf && !(c.plan && c.plan_leaf > 0)) {
        lauum128(c, lower, (int)n, A, lda);   // the bottom node in one launch
        return;
    }
    const long long n1 = split_size(n), n2 = n - n1;
    double *A22 = A + n1 + n1 * lda;
    c.level++;
    lauum_rec(c, uplo, n1, A, lda);
    c.level--;
    if (lower) {
        double *A21 = A + n1;
        // A_TL += A_BLᵀ·A_BL (lower tiles), then A_BL := A_BRᵀ·A_BL
        gemm<double, double, double>(c, Mfma::F64, 'T', 'N', 'L', n1, n1, n2, 1.0, A21, lda, A21, lda, 1.0, A, lda);
        trmm(c, 'L', 'L', 'T', 'N', n2, n1, 1.0, A22, lda, A21, lda);
    } else {
        double *A12 = A + n1 * lda;
        // A_TL += A_TR·A_TRᵀ (upper tiles), then A_TR := A_TR·A_BRᵀ
        gemm<double, double, double>(c, Mfma::F64, 'N', 'T', 'U', n1, n1, n2, 1.0, A12, lda, A12, lda, 1.0, A, lda);
        trmm(c, 'R', 'U', 'T', 'N', n1, n2, 1.0, A22, lda, A12, lda);
    }
    c.level++;
    lauum_rec(c, uplo, n2, A22, lda);
    c.level--;
}

}  // namespace rl
