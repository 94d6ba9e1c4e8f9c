// Matrix-core GEMM / SYRK for the trailing updates of the recursion.
//
// C := beta*C + alpha*op(A)*op(B). These carry almost all of the flops of a
// recursive factorization: the paper's analysis (Sec. 3, Fig.
// recursive_breakdown and the flop-share equation beside it) shows that the
// BLAS-3 calls of the top recursion level alone hold 3/4 of the work and the
// BLAS-3 calls of all levels more than 99.6 % of it. Cholesky's trailing update
// A22 -= A21*A21ᵀ is the triangular ("tri") instance of the same kernel: only
// the tiles of one triangle are launched and the diagonal tiles are masked.
//
// Design (gfx950):
//  * 128×128 tiles: 512 threads = 8 waves in a 4×2 arrangement, each wave
//    owning 32×64 of the tile; 64×64 and 32×32 tiles: 256 threads = 4 waves
//    in a 2×2 arrangement. Each wave's part is a grid of 16×16 matrix-core
//    blocks; BK = 16 is staged through LDS, double-buffered, one barrier per
//    K step. Operands are stored in LDS k-major ([k][m]) so that the 16 lanes
//    of a matrix-core row group read 16 consecutive elements. (Four waves of
//    64×64 on the 128-tile need 332 registers per lane, one wave per SIMD,
//    and leave the matrix cores idle whenever that wave waits; eight waves of
//    32×64 fit in 128, so a SIMD holds several.)
//  * The K loop prefetches the next tile from HBM into registers while the
//    matrix cores work on the current one.
//  * XCD-aware launch: workgroup b runs on XCD b % 8; logical tiles are dealt
//    out so that each XCD gets a contiguous run of them, and tiles are ordered
//    in groups of 8 tile-rows (triangles: bands of 8 tile rows, column by
//    column) so that neighbours share operand panels in that XCD's L2.
//  * FP64 (v_mfma_f64_16x16x4f64) and FP32 (v_mfma_f32_16x16x4f32) operands;
//    the operand type in LDS (TL) may differ from the storage types, e.g. FP32
//    factors multiplied in FP64 during iterative refinement.
#include "common.hpp"

#include <type_traits>

namespace rl {

template <typename TL>
struct MfmaK1;

template <>
struct MfmaK1<double> {
    typedef d4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // FP64 16×16×4: element v of lane l is D[l/16 + 4v][l%16]
    static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};

template <>
struct MfmaK1<float> {
    typedef f4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // FP32 16×16×4: element v of lane l is D[4*(l/16) + v][l%16]
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

template <typename TA, typename TB, typename TC>
struct GemmArgs {
    long long m, n, k;
    double alpha, beta;
    const TA *A;
    long long lda;
    const TB *B;
    long long ldb;
    TC *C;
    long long ldc;
    int tiles_m, tiles_n, ntiles;
    const int *abort;  // non-null: skip all work when *abort != 0
    int *ovf;          // half-precision operands: set to 1 when one rounds to infinity
    // Triangular tail: when tail_T > 0 the launch covers, with tiles of half
    // the edge, the parent tiles tail_first.. of the band enumeration of a
    // tail_T-tile triangle (four quarters per parent, consecutive).
    int tail_T, tail_first;
};

// Map the hardware workgroup id to a logical tile id, giving each of the 8 XCDs
// a contiguous range of logical tiles (the grid is padded to a multiple of 8).
__device__ __forceinline__ int xcd_logical(int bid, int grid) {
    const int per = grid >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Logical tile -> (t, u), t >= u, of a T×T lower tile triangle: bands of 8
// tile rows, each band column by column (first its full 8-row part, then its
// own lower triangle), so that consecutive tiles, which the launch keeps on
// one XCD, form 8×8 blocks as in the full grid and share operand panels in
// that XCD's L2.
__device__ __forceinline__ void tri_band_tile(int tile, int T, int &t, int &u) {
    int b = 0, start = 0, h = 0;
    while (true) {
        h = min(8, T - 8 * b);
        const int sz = h * 8 * b + h * (h + 1) / 2;
        if (tile < start + sz) break;
        start += sz;
        ++b;
    }
    int r = tile - start;
    if (r < h * 8 * b) {
        u = r / h;
        t = 8 * b + r % h;
    } else {
        r -= h * 8 * b;
        int c = 0;
        while (r >= h - c) { r -= h - c; ++c; }
        u = 8 * b + c;
        t = u + r;
    }
}

// Threads of a workgroup for a tile edge: 8 waves on 128-tiles, 4 otherwise.
constexpr int k1_threads(int bm) { return bm == 128 ? 512 : 256; }

template <typename TL, typename TA, typename TB, typename TC, bool TRA, bool TRB, int TRI, int BM,
          int BN, bool VEC>
__global__ __launch_bounds__(k1_threads(BM)) void gemm_k1(GemmArgs<TA, TB, TC> g) {
    constexpr int BK = 16;
    constexpr int NT = k1_threads(BM);
    constexpr int WM = NT / 128, WN = 2;   // waves along the tile's rows and columns
    // VEC: each thread moves pairs of elements that are adjacent in memory
    // (one 2-wide load per pair on full tiles; the host selects this only when
    // both operands' base and leading dimension keep every pair aligned); the
    // even pad keeps the pairs aligned in LDS as well.
    constexpr int PAD = VEC ? 2 : 1;
    constexpr int MI = BM / WM / 16, NI = BN / WN / 16;
    constexpr int EA = BM * BK / NT, EB = BN * BK / NT;
    typedef MfmaK1<TL> Op;
    typedef typename Op::acc_t acc_t;

    if (g.abort && *g.abort) return;
    const int tile = xcd_logical(blockIdx.x, gridDim.x);
    if (tile >= g.ntiles) return;

    int tm, tn;
    if (TRI == 0) {
        constexpr int GROUP = 8;
        const int gsize = GROUP * g.tiles_n;
        const int grp = tile / gsize;
        const int first = grp * GROUP;
        const int gm = min(g.tiles_m - first, GROUP);
        const int r = tile - grp * gsize;
        tm = first + r % gm;
        tn = r / gm;
    } else {
        int t, u;
        if (g.tail_T > 0) {
            const int q = tile & 3;
            tri_band_tile(g.tail_first + (tile >> 2), g.tail_T, t, u);
            t = 2 * t + (q >> 1);
            u = 2 * u + (q & 1);
            if (u > t) return;   // the quarter above the diagonal of a diagonal parent
        } else {
            tri_band_tile(tile, g.tiles_m, t, u);
        }
        if (TRI == 1) { tm = t; tn = u; }   // lower: tm >= tn
        else { tm = u; tn = t; }            // upper: tm <= tn
    }

    const long long m0 = (long long)tm * BM, n0 = (long long)tn * BN;
    const long long M = g.m, N = g.n, K = g.k;
    const TA *__restrict__ A = g.A;
    const TB *__restrict__ B = g.B;

    __shared__ TL As[2][BK][BM + PAD];
    __shared__ TL Bs[2][BK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave % WM) * (BM / WM), wn = (wave / WM) * (BN / WN);

    // K tiles staged in registers on their way to LDS: one set on 128-tiles
    // (stored a quarter step after its loads were issued when they are paired,
    // after the whole step otherwise; more sets cost the 128-tiles their
    // second workgroup per CU), PF sets on the smaller tiles, whose short K
    // steps cannot cover a global round trip with one tile in flight (a 64×64
    // tile's K step is about 1000 matrix-core cycles per wave)
    constexpr bool EARLY = VEC && BM == 128;
    constexpr int PF = BM == 128 ? 1 : 4;
    TA ra[PF][EA];
    TB rb[PF][EB];

    // element coordinates of this thread's share of a K tile; with VEC,
    // elements 2p and 2p+1 are neighbours along the operand's contiguous index
    auto a_coord = [&](int i, int &r, int &kk) {
        if (VEC) {
            const int p = i >> 1, h = i & 1;
            if (!TRA) { r = 2 * (tid % (BM / 2)) + h; kk = tid / (BM / 2) + p * (2 * NT / BM); }
            else { kk = 2 * (tid % (BK / 2)) + h; r = tid / (BK / 2) + p * (2 * NT / BK); }
        } else {
            if (!TRA) { r = tid % BM; kk = tid / BM + i * (NT / BM); }
            else { kk = tid % BK; r = tid / BK + i * (NT / BK); }
        }
    };
    auto b_coord = [&](int i, int &c, int &kk) {
        if (VEC) {
            const int p = i >> 1, h = i & 1;
            if (TRB) { c = 2 * (tid % (BN / 2)) + h; kk = tid / (BN / 2) + p * (2 * NT / BN); }
            else { kk = 2 * (tid % (BK / 2)) + h; c = tid / (BK / 2) + p * (2 * NT / BK); }
        } else {
            if (TRB) { c = tid % BN; kk = tid / BN + i * (NT / BN); }
            else { kk = tid % BK; c = tid / BK + i * (NT / BK); }
        }
    };
    typedef TA TA2 __attribute__((ext_vector_type(2)));
    typedef TB TB2 __attribute__((ext_vector_type(2)));

    // IN (compile time): the tile lies inside C and K is a multiple of BK, so
    // no load needs a guard. Interior tiles run a copy of the K loop and of
    // the epilogue without the edge checks (the checks inside the K loop cost
    // the 128-tiles about a tenth of their rate); edge tiles take the guarded
    // copy.
    auto load_tiles = [&](long long k0, auto in_tag, TA (&ra)[EA], TB (&rb)[EB]) {
        constexpr bool IN = decltype(in_tag)::value;
        const bool afull = IN || ((m0 + BM <= M) && (k0 + BK <= K));
        const bool bfull = IN || ((n0 + BN <= N) && (k0 + BK <= K));
        if (afull && VEC) {
#pragma unroll
            for (int i = 0; i < EA; i += 2) {
                int r, kk;
                a_coord(i, r, kk);
                const long long gr = m0 + r, gk = k0 + kk;
                const TA2 v = *(const TA2 *)(A + (TRA ? gk + gr * g.lda : gr + gk * g.lda));
                ra[i] = v.x;
                ra[i + 1] = v.y;
            }
        } else if (afull) {
#pragma unroll
            for (int i = 0; i < EA; ++i) {
                int r, kk;
                a_coord(i, r, kk);
                const long long gr = m0 + r, gk = k0 + kk;
                ra[i] = A[TRA ? gk + gr * g.lda : gr + gk * g.lda];
            }
        } else if (!IN) {
            // edge tile: guarded loads keep register pressure at the fast
            // path's level
#pragma unroll
            for (int i = 0; i < EA; ++i) {
                int r, kk;
                a_coord(i, r, kk);
                const long long gr = m0 + r, gk = k0 + kk;
                ra[i] = (gr < M && gk < K) ? A[TRA ? gk + gr * g.lda : gr + gk * g.lda] : TA(0);
            }
        }
        if (bfull && VEC) {
#pragma unroll
            for (int i = 0; i < EB; i += 2) {
                int c, kk;
                b_coord(i, c, kk);
                const long long gc = n0 + c, gk = k0 + kk;
                const TB2 v = *(const TB2 *)(B + (TRB ? gc + gk * g.ldb : gk + gc * g.ldb));
                rb[i] = v.x;
                rb[i + 1] = v.y;
            }
        } else if (bfull) {
#pragma unroll
            for (int i = 0; i < EB; ++i) {
                int c, kk;
                b_coord(i, c, kk);
                const long long gc = n0 + c, gk = k0 + kk;
                rb[i] = B[TRB ? gc + gk * g.ldb : gk + gc * g.ldb];
            }
        } else if (!IN) {
#pragma unroll
            for (int i = 0; i < EB; ++i) {
                int c, kk;
                b_coord(i, c, kk);
                const long long gc = n0 + c, gk = k0 + kk;
                rb[i] = (gc < N && gk < K) ? B[TRB ? gc + gk * g.ldb : gk + gc * g.ldb] : TB(0);
            }
        }
    };
    auto store_tiles = [&](int buf, const TA (&ra)[EA], const TB (&rb)[EB]) {
#pragma unroll
        for (int i = 0; i < EA; ++i) {
            int r, kk;
            a_coord(i, r, kk);
            As[buf][kk][r] = (TL)ra[i];
        }
#pragma unroll
        for (int i = 0; i < EB; ++i) {
            int c, kk;
            b_coord(i, c, kk);
            Bs[buf][kk][c] = (TL)rb[i];
        }
    };

    acc_t acc[MI][NI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const long long KT = (K + BK - 1) / BK;
    // EARLY (paired loads on 128-tiles): the next K tile goes to LDS right
    // after the first quarter of the products (the other buffer was last read
    // before the previous barrier), and the waves raise their issue priority
    // while they feed the matrix cores. Measured at n = 4096 and 8192 against
    // storing after the last quarter at normal priority with element-wise
    // loads: from on par to 7 % faster, depending on the run. On 64-tiles
    // (four products per quarter and wave) it measured slower at n = 1024, so
    // they take the paired loads alone (n = 1024 / 2048: 7 % faster).
    // the products of one K tile from LDS buffer buf; stage_next runs after
    // the first quarter of them on paired 128-tiles (the early store of the
    // next tile) and after the last quarter otherwise
    constexpr int STORE_AFTER = EARLY ? 0 : BK / 4 - 1;
    auto k_step = [&](int buf, auto stage_next) {
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            TL a[MI], b[NI];
#pragma unroll
            for (int i = 0; i < MI; ++i) a[i] = As[buf][kr][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NI; ++j) b[j] = Bs[buf][kr][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NI; ++j) acc[i][j] = Op::mma(a[i], b[j], acc[i][j]);
            if (ks == STORE_AFTER) stage_next();
        }
    };
    auto k_loop = [&](auto in_tag) {
        if (PF == 1) {
            if (KT > 0) {
                load_tiles(0, in_tag, ra[0], rb[0]);
                store_tiles(0, ra[0], rb[0]);
                __syncthreads();
            }
            for (long long kt = 0; kt < KT; ++kt) {
                const int buf = (int)(kt & 1);
                if (kt + 1 < KT) load_tiles((kt + 1) * BK, in_tag, ra[0], rb[0]);
                if (EARLY) __builtin_amdgcn_s_setprio(1);
                k_step(buf, [&] {
                    if (kt + 1 < KT) store_tiles(buf ^ 1, ra[0], rb[0]);
                });
                if (EARLY) __builtin_amdgcn_s_setprio(0);
                __syncthreads();
            }
        } else {
            // PF tiles in flight: step kt computes from LDS buffer kt & 1,
            // moves tile kt + 1 (loaded PF - 1 steps earlier) into the other
            // buffer and reuses tile kt's registers for tile kt + PF; the loop
            // is unrolled by PF (even) so every register set index is static
#pragma unroll
            for (int p = 0; p < PF; ++p)
                if (p < KT) load_tiles((long long)p * BK, in_tag, ra[p], rb[p]);
            if (KT > 0) {
                store_tiles(0, ra[0], rb[0]);
                __syncthreads();
            }
            for (long long kt0 = 0; kt0 < KT; kt0 += PF) {
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const long long kt = kt0 + u;
                    if (kt < KT) {
                        k_step(u & 1, [] {});   // (PF > 1: stores below)
                        if (kt + 1 < KT) store_tiles((u & 1) ^ 1, ra[(u + 1) % PF], rb[(u + 1) % PF]);
                        if (kt + PF < KT) load_tiles((kt + PF) * BK, in_tag, ra[u], rb[u]);
                        __syncthreads();
                    }
                }
            }
        }
    };

    const double alpha = g.alpha, beta = g.beta;
    TC *__restrict__ C = g.C;
    // C := alpha·acc + beta·C on this wave's part (BZ: beta = 0, C not read)
    auto epilogue = [&](auto in_tag, auto bz_tag) {
        constexpr bool IN = decltype(in_tag)::value, BZ = decltype(bz_tag)::value;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const long long r = m0 + wm + i * 16 + Op::row(lane, v);
                    const long long cc = n0 + wn + j * 16 + (lane & 15);
                    if (!IN && (r >= M || cc >= N)) continue;
                    if (TRI == 1 && r < cc) continue;
                    if (TRI == 2 && r > cc) continue;
                    TC *p = C + r + cc * g.ldc;
                    const double val = (double)acc[i][j][v];
                    if (BZ) *p = (TC)(alpha * val);
                    else *p = (TC)(alpha * val + beta * (double)(*p));
                }
    };
    typedef std::integral_constant<bool, true> yes;
    typedef std::integral_constant<bool, false> no;
    const bool inner = (m0 + BM <= M) && (n0 + BN <= N) && (K % BK == 0);
    if (inner) k_loop(yes{});
    else k_loop(no{});
    if (inner) {
        if (beta == 0.0) epilogue(yes{}, yes{});
        else epilogue(yes{}, no{});
    } else {
        if (beta == 0.0) epilogue(no{}, yes{});
        else epilogue(no{}, no{});
    }
}

template <typename TL, typename TA, typename TB, typename TC, bool TRA, bool TRB, int TRI, int BM,
          bool VEC = false>
static void launch_k1(Ctx &c, const GemmArgs<TA, TB, TC> &args0, int ntiles = -1) {
    GemmArgs<TA, TB, TC> a = args0;
    a.tiles_m = (int)((a.m + BM - 1) / BM);
    a.tiles_n = (int)((a.n + BM - 1) / BM);
    a.ntiles = ntiles >= 0 ? ntiles : (TRI ? a.tiles_m * (a.tiles_m + 1) / 2 : a.tiles_m * a.tiles_n);
    if (a.ntiles <= 0) return;
    const int grid = (a.ntiles + 7) / 8 * 8;
    rl_launch(c, gemm_k1<TL, TA, TB, TC, TRA, TRB, TRI, BM, BM, VEC>, dim3(grid), dim3(k1_threads(BM)), 0, a);
    RL_CHECK(hipGetLastError());
}

// Tiles of the last, partly filled round of a triangular launch on 128-tiles
// (two workgroups per CU), when that round is at most half full: they are run
// afterwards as 64-tiles, four per parent tile, so the round's work is spread
// over more CUs instead of leaving most of them idle. 0 = no split.
static int tri_tail_tiles(const Ctx &c, long long m) {
    const long long T = (m + 127) / 128, tiles = T * (T + 1) / 2, slots = 2LL * c.num_cu;
    const long long r = tiles % slots;
    return (tiles > slots && r > 0 && 2 * r <= slots) ? (int)r : 0;
}

// Pairs of adjacent elements of an operand can be read as one 2-wide load
// when its base and every column start are aligned to the pair size.
template <typename T>
static bool pairs_aligned(const T *p, long long ld) {
    return ((uintptr_t)p % (2 * sizeof(T))) == 0 && ld % 2 == 0;
}

template <typename TL, typename TA, typename TB, typename TC, bool TRA, bool TRB, int TRI>
static void dispatch_tile(Ctx &c, const GemmArgs<TA, TB, TC> &a) {
    const bool pairs = pairs_aligned(a.A, a.lda) && pairs_aligned(a.B, a.ldb);
    auto tile64 = [&](const GemmArgs<TA, TB, TC> &g, int ntiles) {
        if (pairs) launch_k1<TL, TA, TB, TC, TRA, TRB, TRI, 64, true>(c, g, ntiles);
        else launch_k1<TL, TA, TB, TC, TRA, TRB, TRI, 64, false>(c, g, ntiles);
    };
    const long long big = ((a.m + 127) / 128) * ((a.n + 127) / 128) / (TRI ? 2 : 1);
    if (big >= 2LL * c.num_cu) {
        const int r = TRI ? tri_tail_tiles(c, a.m) : 0;
        const int T = (int)((a.m + 127) / 128), tiles = T * (T + 1) / 2;
        if (pairs)
            launch_k1<TL, TA, TB, TC, TRA, TRB, TRI, 128, true>(c, a, r > 0 ? tiles - r : -1);
        else
            launch_k1<TL, TA, TB, TC, TRA, TRB, TRI, 128, false>(c, a, r > 0 ? tiles - r : -1);
        if (r > 0) {
            GemmArgs<TA, TB, TC> t = a;
            t.tail_T = T;
            t.tail_first = tiles - r;
            tile64(t, 4 * r);
        }
    } else if (TRI && ((a.m + 63) / 64) * ((a.m + 63) / 64 + 1) / 2 <= 4LL * c.num_cu) {
        // small triangular updates: 32-tiles give the chip four times the
        // workgroups (SYRK n = k = 1024: 88 -> 70 us; 512: 53 -> 35 us)
        launch_k1<TL, TA, TB, TC, TRA, TRB, TRI, 32>(c, a);
    } else {
        tile64(a, -1);
    }
}

template <typename TL, typename TA, typename TB, typename TC>
static void dispatch(Ctx &c, char ta, char tb, char tri, const GemmArgs<TA, TB, TC> &a) {
    const bool TA_ = (ta == 'T' || ta == 't'), TB_ = (tb == 'T' || tb == 't');
    const int T = (tri == 'L' || tri == 'l') ? 1 : (tri == 'U' || tri == 'u') ? 2 : 0;
#define RL_G(x, y, z)                                                         \
    if (TA_ == x && TB_ == y && T == z) {                                     \
        dispatch_tile<TL, TA, TB, TC, x, y, z>(c, a);                         \
        return;                                                               \
    }
    RL_G(false, false, 0) RL_G(false, true, 0) RL_G(true, false, 0) RL_G(true, true, 0)
    RL_G(false, true, 1) RL_G(true, false, 1) RL_G(false, true, 2) RL_G(true, false, 2)
#undef RL_G
    launch_error(hipErrorInvalidValue);
}


// ---------------------------------------------------------------------------
// Half-precision operands (FP16 or BF16) with FP32 accumulation, for the
// low-precision factorization of the mixed solvers. Storage stays FP32 (the
// Schur complements accumulate in FP32); operands are rounded to 16 bits as
// they are staged into LDS. v_mfma_f32_16x16x32_{f16,bf16}: each lane feeds 8
// consecutive k of one row/column, so LDS holds tiles k-contiguous
// ([m][k], padded) and a lane's operand is one 16-byte LDS read. The output
// layout is D[4*(l/16) + v][l%16].
// ---------------------------------------------------------------------------
template <typename H>
struct MfmaK8;

template <>
struct MfmaK8<_Float16> {
    typedef h8 vec_t;
    static __device__ __forceinline__ f4 mma(vec_t a, vec_t b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct MfmaK8<__bf16> {
    typedef bh8 vec_t;
    static __device__ __forceinline__ f4 mma(vec_t a, vec_t b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <typename H, bool TRA, bool TRB, int TRI, int BM>
__global__ __launch_bounds__(256) void gemm_k8(GemmArgs<float, float, float> g) {
    constexpr int BN = BM;
    constexpr int BK = 32;
    constexpr int LDK = BK + 8;  // halves per LDS row (16-byte aligned rows, skewed banks)
    constexpr int MI = BM / 32, NI = BN / 32;
    constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
    typedef MfmaK8<H> Op;
    typedef typename Op::vec_t vec_t;

    if (g.abort && *g.abort) return;
    const int tile = xcd_logical(blockIdx.x, gridDim.x);
    if (tile >= g.ntiles) return;
    int tm, tn;
    if (TRI == 0) {
        constexpr int GROUP = 8;
        const int gsize = GROUP * g.tiles_n;
        const int grp = tile / gsize;
        const int first = grp * GROUP;
        const int gm = min(g.tiles_m - first, GROUP);
        const int r = tile - grp * gsize;
        tm = first + r % gm;
        tn = r / gm;
    } else {
        int t, u;
        tri_band_tile(tile, g.tiles_m, t, u);
        if (TRI == 1) { tm = t; tn = u; }
        else { tm = u; tn = t; }
    }
    const long long m0 = (long long)tm * BM, n0 = (long long)tn * BN;
    const long long M = g.m, N = g.n, K = g.k;
    const float *__restrict__ A = g.A;
    const float *__restrict__ B = g.B;

    __shared__ __attribute__((aligned(16))) H As[2][BM][LDK];
    __shared__ __attribute__((aligned(16))) H Bs[2][BN][LDK];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * (BM / 2), wn = (wave >> 1) * (BN / 2);
    float ra[EA], rb[EB];

    auto a_coord = [&](int i, int &r, int &kk) {
        if (!TRA) { r = tid % BM; kk = tid / BM + i * (256 / BM); }
        else { kk = tid % BK; r = tid / BK + i * (256 / BK); }
    };
    auto b_coord = [&](int i, int &c, int &kk) {
        if (TRB) { c = tid % BN; kk = tid / BN + i * (256 / BN); }
        else { kk = tid % BK; c = tid / BK + i * (256 / BK); }
    };
    auto load_tiles = [&](long long k0) {
        const bool afull = (m0 + BM <= M) && (k0 + BK <= K);
        const bool bfull = (n0 + BN <= N) && (k0 + BK <= K);
#pragma unroll
        for (int i = 0; i < EA; ++i) {
            int r, kk;
            a_coord(i, r, kk);
            const long long gr = m0 + r, gk = k0 + kk;
            const long long off = TRA ? gk + gr * g.lda : gr + gk * g.lda;
            const bool in = afull || (gr < M && gk < K);
            const float v = A[in ? off : 0];
            ra[i] = in ? v : 0.f;
        }
#pragma unroll
        for (int i = 0; i < EB; ++i) {
            int c, kk;
            b_coord(i, c, kk);
            const long long gc = n0 + c, gk = k0 + kk;
            const long long off = TRB ? gc + gk * g.ldb : gk + gc * g.ldb;
            const bool in = bfull || (gc < N && gk < K);
            const float v = B[in ? off : 0];
            rb[i] = in ? v : 0.f;
        }
    };
    // an operand too large for the 16-bit format rounds to infinity: noted
    // once per thread and reported at the end (the solve falls back to FP64)
    bool inf_seen = false;
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int i = 0; i < EA; ++i) {
            int r, kk;
            a_coord(i, r, kk);
            const H h = (H)ra[i];
            inf_seen |= __builtin_isinf((float)h);
            As[buf][r][kk] = h;
        }
#pragma unroll
        for (int i = 0; i < EB; ++i) {
            int c, kk;
            b_coord(i, c, kk);
            const H h = (H)rb[i];
            inf_seen |= __builtin_isinf((float)h);
            Bs[buf][c][kk] = h;
        }
    };

    f4 acc[MI][NI];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) acc[i][j] = f4{0, 0, 0, 0};

    const long long KT = (K + BK - 1) / BK;
    if (KT > 0) {
        load_tiles(0);
        store_tiles(0);
        __syncthreads();
    }
    for (long long kt = 0; kt < KT; ++kt) {
        const int buf = (int)(kt & 1);
        if (kt + 1 < KT) load_tiles((kt + 1) * BK);
        const int kq = 8 * (lane >> 4);
        vec_t a[MI], b[NI];
#pragma unroll
        for (int i = 0; i < MI; ++i) a[i] = *reinterpret_cast<const vec_t *>(&As[buf][wm + i * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int j = 0; j < NI; ++j) b[j] = *reinterpret_cast<const vec_t *>(&Bs[buf][wn + j * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j) acc[i][j] = Op::mma(a[i], b[j], acc[i][j]);
        if (kt + 1 < KT) store_tiles(buf ^ 1);
        __syncthreads();
    }

    if (inf_seen && g.ovf) __hip_atomic_store(g.ovf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float alpha = (float)g.alpha, beta = (float)g.beta;
    float *__restrict__ C = g.C;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long long r = m0 + wm + i * 16 + 4 * (lane >> 4) + v;
                const long long cc = n0 + wn + j * 16 + (lane & 15);
                if (r >= M || cc >= N) continue;
                if (TRI == 1 && r < cc) continue;
                if (TRI == 2 && r > cc) continue;
                float *p = C + r + cc * g.ldc;
                *p = beta == 0.f ? alpha * acc[i][j][v] : alpha * acc[i][j][v] + beta * (*p);
            }
}

template <typename H, bool TRA, bool TRB, int TRI, int BM>
static void launch_k8(Ctx &c, const GemmArgs<float, float, float> &args0) {
    GemmArgs<float, float, float> a = args0;
    a.tiles_m = (int)((a.m + BM - 1) / BM);
    a.tiles_n = (int)((a.n + BM - 1) / BM);
    a.ntiles = TRI ? a.tiles_m * (a.tiles_m + 1) / 2 : a.tiles_m * a.tiles_n;
    if (a.ntiles <= 0) return;
    const int grid = (a.ntiles + 7) / 8 * 8;
    rl_launch(c, gemm_k8<H, TRA, TRB, TRI, BM>, dim3(grid), dim3(256), 0, a);
    RL_CHECK(hipGetLastError());
}

template <typename H>
static void dispatch8(Ctx &c, char ta, char tb, char tri, const GemmArgs<float, float, float> &a) {
    const bool TA_ = (ta == 'T' || ta == 't'), TB_ = (tb == 'T' || tb == 't');
    const int T = (tri == 'L' || tri == 'l') ? 1 : (tri == 'U' || tri == 'u') ? 2 : 0;
    const long long big = ((a.m + 127) / 128) * ((a.n + 127) / 128) / (T ? 2 : 1);
    const bool b128 = big >= 2LL * c.num_cu;
#define RL_G8(x, y, z)                                                                      \
    if (TA_ == x && TB_ == y && T == z) {                                                   \
        if (b128) launch_k8<H, x, y, z, 128>(c, a); else launch_k8<H, x, y, z, 64>(c, a);   \
        return;                                                                             \
    }
    RL_G8(false, false, 0) RL_G8(false, true, 0) RL_G8(true, false, 0) RL_G8(true, true, 0)
    RL_G8(false, true, 1) RL_G8(true, false, 1) RL_G8(false, true, 2) RL_G8(true, false, 2)
#undef RL_G8
    launch_error(hipErrorInvalidValue);
}

template <typename TA, typename TB, typename TC>
static inline void dispatch_half(Ctx &, Mfma, char, char, char, const GemmArgs<TA, TB, TC> &) {
    launch_error(hipErrorInvalidValue);  // half-precision operands need FP32 storage throughout
}

static inline void dispatch_half(Ctx &c, Mfma mode, char ta, char tb, char tri,
                                 const GemmArgs<float, float, float> &a) {
    if (mode == Mfma::F16) dispatch8<_Float16>(c, ta, tb, tri, a);
    else dispatch8<__bf16>(c, ta, tb, tri, a);
}

template <typename TA, typename TB, typename TC>
void gemm(Ctx &c, Mfma mode, char ta, char tb, char tri, long long m, long long n, long long k,
          double alpha, const TA *A, long long lda, const TB *B, long long ldb, double beta, TC *C,
          long long ldc) {
    const double flops = tri ? (double)m * (double)(m + 1) * (double)k : 2.0 * m * n * k;
    if (plan_record(c, tri ? PK_SYRK : PK_GEMM, m, n, k)) return;
    if (m <= 0 || n <= 0) return;
    GemmArgs<TA, TB, TC> a{};
    a.m = m; a.n = n; a.k = k;
    a.alpha = alpha; a.beta = beta;
    a.A = A; a.lda = lda; a.B = B; a.ldb = ldb; a.C = C; a.ldc = ldc;
    a.abort = c.dstat ? &c.dstat->info : nullptr;
    if (!c.abort_on_info) a.abort = nullptr;
    a.ovf = c.dstat ? &c.dstat->ovf : nullptr;
    // the launch below picks 128×128 tiles exactly when this holds
    const bool big = ((m + 127) / 128) * ((n + 127) / 128) / (tri ? 2 : 1) >= 2LL * c.num_cu;
    const int kind = mode == Mfma::F64 ? (tri ? PK_SYRK : (big ? PK_GEMM_BIG : PK_GEMM))
                                       : (tri ? PK_SYRK_LP : PK_GEMM_LP);
    // a triangular update with a split-off tail is two launches: timed as a region
    const bool two = tri && big && (mode == Mfma::F64 || mode == Mfma::F32) && tri_tail_tiles(c, m) > 0;
    if (two) trace_begin(c, kind);
    else trace_kernel_begin(c);
    if (mode == Mfma::F64) dispatch<double>(c, ta, tb, tri, a);
    else if (mode == Mfma::F32) dispatch<float>(c, ta, tb, tri, a);
    else dispatch_half(c, mode, ta, tb, tri, a);
    const double bytes = (double)sizeof(TA) * m * k + (double)sizeof(TB) * k * n +
                         2.0 * sizeof(TC) * m * n / (tri ? 2.0 : 1.0);
    if (two) trace_end(c, kind, flops, bytes);
    else trace_kernel_end(c, kind, flops, bytes);
}

template void gemm<double, double, double>(Ctx &, Mfma, char, char, char, long long, long long,
                                           long long, double, const double *, long long,
                                           const double *, long long, double, double *, long long);
template void gemm<float, float, float>(Ctx &, Mfma, char, char, char, long long, long long,
                                        long long, double, const float *, long long,
                                        const float *, long long, double, float *, long long);
template void gemm<double, float, double>(Ctx &, Mfma, char, char, char, long long, long long,
                                          long long, double, const double *, long long,
                                          const float *, long long, double, double *, long long);
template void gemm<float, double, double>(Ctx &, Mfma, char, char, char, long long, long long,
                                          long long, double, const float *, long long,
                                          const double *, long long, double, double *, long long);

}  // namespace rl
