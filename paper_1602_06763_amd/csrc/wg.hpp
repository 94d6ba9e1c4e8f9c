// Workgroup-level building blocks shared by the leaf kernels of the
// recursion and by the batched factorizations (one workgroup per matrix):
// lane broadcasts, the matrix-core triangular-solve block, and the unblocked
// Cholesky of a block held in LDS.
#pragma once

#include "common.hpp"

namespace rl {

// ---------------------------------------------------------------------------
// Matrix-core leaf: a workgroup solves N·x = b for 64 vectors (16 per wave),
// triangle t <= 64 in LDS, blocked by 16: block I of x is
//     x_I = N_II⁻¹ (b_I - Σ_{J before I} N_IJ·x_J),
// the sum on the matrix cores (16×16×4 steps, vectors as columns), the 16×16
// diagonal solve by substitution with four lanes per vector. The reciprocals
// of the diagonal are formed once after the triangle is staged, and rows
// beyond t are padded with the identity, so the substitution is straight-line
// code with a multiply, a quad broadcast and an FMA on its dependency chain
// per step. Each wave works on its own 16 vectors, so waves never wait for
// each other after the triangle is staged.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_bcast(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_bcast(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// The value of lane S of each group of four lanes, in all four (DPP quad_perm).
template <int S>
__device__ __forceinline__ float quad_bcast(float x) {
    constexpr int ctrl = S | (S << 2) | (S << 4) | (S << 6);
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xF, 0xF, false));
}
template <int S>
__device__ __forceinline__ double quad_bcast(double x) {
    constexpr int ctrl = S | (S << 2) | (S << 4) | (S << 6);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// quad_bcast with the source lane chosen at run time; fully unrolled callers
// pass a constant, so the switch folds away.
template <typename T>
__device__ __forceinline__ T quad_bcast_sel(T x, int s) {
    switch (s & 3) {
    case 0: return quad_bcast<0>(x);
    case 1: return quad_bcast<1>(x);
    case 2: return quad_bcast<2>(x);
    default: return quad_bcast<3>(x);
    }
}

template <typename TW>
struct LeafMfma;
template <>
struct LeafMfma<double> {
    typedef d4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct LeafMfma<float> {
    typedef f4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// One wave solves N·x = b for its 16 vectors, N the 64×64 triangle in Nsh
// (rows and columns beyond t padded with the identity), x in the wave's X
// (64 rows × 16 vectors): 16-row blocks in the order of the solve, each first
// updated on the matrix cores with the blocks already solved, then finished
// by substitution.
template <typename TW, bool LOWER>
__device__ __forceinline__ void solve64(TW (*Nsh)[65], TW (*X)[17], int t, int unit, int lane) {
    typedef LeafMfma<TW> Op;
    typedef typename Op::acc_t acc_t;
    // reciprocal of diagonal element `lane`, formed in every wave off the
    // substitution's dependency chain (read back with readlane)
    TW rdl = (unit || lane >= t) ? TW(1) : TW(1) / Nsh[lane][lane];
    asm volatile("" : "+v"(rdl));

    const int nblk = (t + 15) / 16;
    for (int s = 0; s < nblk; ++s) {
        const int I = LOWER ? s : nblk - 1 - s;
        // X_I -= Σ N_IJ·X_J over the blocks already solved
        if (s > 0) {
            acc_t acc = acc_t{0, 0, 0, 0};
            const int J0 = LOWER ? 0 : I + 1, J1 = LOWER ? I : nblk;
            for (int J = J0; J < J1; ++J) {
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 16 * J + 4 * kk + (lane >> 4);
                    acc = Op::mma(Nsh[16 * I + (lane & 15)][k], X[k][lane & 15], acc);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) X[16 * I + Op::row(lane, v)][lane & 15] -= acc[v];
            __builtin_amdgcn_wave_barrier();
        }
        // diagonal 16×16 block: four lanes per vector (lane = 4·vector + r,
        // rows 4r..4r+3 of the block), so all 64 lanes work and each step's
        // x_j reaches the vector's other lanes by a quad broadcast; the
        // block's reciprocals come from readlane in uniform control flow and
        // the next column's entries are read ahead of the current updates
        TW rds[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) rds[j] = lane_bcast(rdl, 16 * I + j);
        {
            const int v = lane >> 2, r4 = lane & 3;
            TW x[4], nc[4], nn[4];
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) x[t4] = X[16 * I + 4 * r4 + t4][v];
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) nc[t4] = Nsh[16 * I + 4 * r4 + t4][16 * I + (LOWER ? 0 : 15)];
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2) {
                const int j = LOWER ? s2 : 15 - s2, jb = j >> 2, jj = j & 3;
                if (s2 + 1 < 16) {
#pragma unroll
                    for (int t4 = 0; t4 < 4; ++t4) nn[t4] = Nsh[16 * I + 4 * r4 + t4][16 * I + (LOWER ? j + 1 : j - 1)];
                }
                // the column read one step ago is complete here; the empty asm
                // also keeps the compiler from turning the selects below into
                // branches around the loads
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) asm volatile("" : "+v"(nc[t4]));
                const TW xs = x[jj] * rds[j];
                const TW xb = quad_bcast_sel(xs, jb);
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) {
                    const TW f = x[t4] - nc[t4] * xb;
                    // rows after j in the order of the solve take the update,
                    // row j takes its solved value, the others stay
                    const bool after = LOWER ? (t4 > jj ? r4 >= jb : r4 > jb) : (t4 < jj ? r4 <= jb : r4 < jb);
                    const TW keep = (t4 == jj && r4 == jb) ? xs : x[t4];
                    x[t4] = after ? f : keep;
                }
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) nc[t4] = nn[t4];
            }
#pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) X[16 * I + 4 * r4 + t4][v] = x[t4];
        }
        __builtin_amdgcn_wave_barrier();
    }

}

// C(16×16 tile at rows i0, columns j0) -= P(i0.., 16 columns from c0)·P(j0.., same)ᵀ
// on the matrix cores; S is row-major with row stride 65.
template <typename T>
__device__ __forceinline__ void potf2_tile_update(T (*S)[65], int i0, int j0, int c0, int lane);
template <>
__device__ __forceinline__ void potf2_tile_update<double>(double (*S)[65], int i0, int j0, int c0, int lane) {
    d4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int c = c0 + 4 * kk + (lane >> 4);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(S[i0 + (lane & 15)][c], S[j0 + (lane & 15)][c], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) S[i0 + (lane >> 4) + 4 * v][j0 + (lane & 15)] -= acc[v];
}
template <>
__device__ __forceinline__ void potf2_tile_update<float>(float (*S)[65], int i0, int j0, int c0, int lane) {
    f4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int c = c0 + 4 * kk + (lane >> 4);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(S[i0 + (lane & 15)][c], S[j0 + (lane & 15)][c], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) S[i0 + 4 * (lane >> 4) + v][j0 + (lane & 15)] -= acc[v];
}

// LDS of the unblocked Cholesky below.
template <typename T>
struct Potf2Lds {
    T S[64][65];
    T cb[2][16];
    T dd[16];   // pivots a_kk of the current panel
    int fail_s;
};

// ---------------------------------------------------------------------------
// Unblocked Cholesky of an n×n block (n <= 64) by one workgroup of 256
// threads, the block held in LDS; element (i, j) of the lower factor is
// A[i*si + j*sj] (si = 1, sj = lda for 'L'; transposed for 'U'). Returns 0,
// or the first column whose pivot is not > 0 (or NaN) plus one; the block is
// written back as it stands (columns before that one final, that column
// holding its updated pivot).
//
// The 64 columns are taken 16 at a time, right-looking: one wave factors the
// 16-column panel (lane = row, the panel's 16 entries of the row in
// registers, the 16 steps unrolled so every register index is fixed), then
// all four waves subtract the panel's contribution from the trailing lower
// triangle on the FP64 matrix cores. A step subtracts (a_rk / a_kk)·a_jk
// from a_rj, which equals l_rk·l_jk and keeps the square root and the column
// scaling off the step-to-step dependency chain; the panel's columns are
// scaled to l_rk = a_rk / sqrt(a_kk) by all waves once the panel is done.
// ---------------------------------------------------------------------------
// Stage the n×n block (element (i, j) of the lower factor at A[i*si + j*sj])
// into S: its lower triangle, zeros above, the identity beyond n.
template <typename T>
__device__ __forceinline__ void potf2_stage(int n, const T *__restrict__ A, long long si, long long sj,
                                            T (*S)[65]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int i = lane, j = wave + 4 * u;
        v[u] = A[min(i, n - 1) * si + min(j, n - 1) * sj];
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int i = lane, j = wave + 4 * u;
        // lower triangle; rows and columns past n are the identity
        S[i][j] = (i < n && j < n) ? (j <= i ? v[u] : T(0)) : (i == j ? T(1) : T(0));
    }
}

// Write back the lower triangle of the n×n block from S.
template <typename T>
__device__ __forceinline__ void potf2_store(int n, T *__restrict__ A, long long si, long long sj, T (*S)[65]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int i = lane, j = wave + 4 * u;
        if (i < n && j <= i) A[i * si + j * sj] = S[i][j];
    }
}

// The factorization of a block staged in L.S (L.fail_s = 0 and a barrier
// before the call); every thread of the workgroup returns the same value
// after a final barrier.
template <typename T>
__device__ __forceinline__ int potf2_factor(int n, Potf2Lds<T> &L) {
    T (*S)[65] = L.S;
    T (&cb)[2][16] = L.cb;
    T (&dd)[16] = L.dd;
    int &fail_s = L.fail_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = (n + 15) / 16;
    for (int J = 0; J < nb; ++J) {
        if (wave == 0) {
            const int r = lane;
            T x[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) x[q] = S[r][16 * J + q];
            int fail = 0;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int k = 16 * J + kk;
                if (fail == 0 && k < n) {
                    if ((r >> 4) == J) cb[kk & 1][r & 15] = x[kk];
                    const T d = lane_bcast(x[kk], k);
                    if (!(d > T(0))) {
                        fail = k + 1;
                    } else {
                        // column kk of the panel's diagonal rows, as broadcasts
                        T cv[16];
#pragma unroll
                        for (int q = kk + 1; q < 16; ++q) cv[q] = cb[kk & 1][q];
                        const T t = x[kk] * (T(1) / d);
                        S[r][k] = x[kk];   // a_rk; scaled by 1/sqrt(a_kk) after the panel
                        if (r == 0) dd[kk] = d;
#pragma unroll
                        for (int q = kk + 1; q < 16; ++q) x[q] -= t * cv[q];
                    }
                }
            }
            if (fail) {
                // the panel's columns from the failing one on, as they stand
                const int k = fail - 1;
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (16 * J + q >= k && r >= 16 * J + q) S[r][16 * J + q] = x[q];
                if (r == 0) fail_s = fail;
            }
        }
        __syncthreads();
        // l_rc = a_rc / sqrt(a_cc) for the panel's finished columns
        {
            const int fk = fail_s ? fail_s - 1 : n;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = lane, c = 16 * J + wave + 4 * u;
                if (c < fk && r >= c) {
                    const T lkk = sqrt(dd[c - 16 * J]);
                    S[r][c] = (r == c) ? lkk : S[r][c] / lkk;
                }
            }
        }
        __syncthreads();
        if (fail_s) break;
        // trailing lower triangle: tiles (I, Jt) with J < Jt <= I < nb
        const int m = nb - 1 - J;   // trailing tile rows
        const int ntiles = m * (m + 1) / 2;
        for (int tt = wave; tt < ntiles; tt += 4) {
            // tt -> (I, Jt) in the trailing triangle
            int I = 0, acc = 0;
            while (acc + I + 1 <= tt) { acc += I + 1; ++I; }
            const int Jt = tt - acc;
            potf2_tile_update<T>(S, 16 * (J + 1 + I), 16 * (J + 1 + Jt), 16 * J, lane);
        }
        __syncthreads();
    }
    return fail_s;
}

template <typename T>
__device__ __forceinline__ int potf2_block(int n, T *__restrict__ A, long long si, long long sj, Potf2Lds<T> &L) {
    potf2_stage(n, A, si, sj, L.S);
    if (threadIdx.x == 0) L.fail_s = 0;
    __syncthreads();
    const int fail = potf2_factor(n, L);
    potf2_store(n, A, si, sj, L.S);
    return fail;
}

// ---- wave-level reductions (DPP, no LDS crossbar) --------------------------
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned x) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ unsigned rlane(unsigned x, int l) { return (unsigned)__builtin_amdgcn_readlane((int)x, l); }
// Maximum / minimum over the wave, in every lane: quad swaps, then the
// half-row and row mirrors give each 16-lane row its extreme; the 4 rows are
// combined from one lane of each.
__device__ __forceinline__ unsigned wave_max_u32(unsigned x) {
    x = max(x, dpp_u32<0xB1>(x));   // quad_perm [1,0,3,2]
    x = max(x, dpp_u32<0x4E>(x));   // quad_perm [2,3,0,1]
    x = max(x, dpp_u32<0x141>(x));  // row_half_mirror
    x = max(x, dpp_u32<0x140>(x));  // row_mirror
    return max(max(rlane(x, 0), rlane(x, 16)), max(rlane(x, 32), rlane(x, 48)));
}
__device__ __forceinline__ unsigned wave_min_u32(unsigned x) {
    x = min(x, dpp_u32<0xB1>(x));
    x = min(x, dpp_u32<0x4E>(x));
    x = min(x, dpp_u32<0x141>(x));
    x = min(x, dpp_u32<0x140>(x));
    return min(min(rlane(x, 0), rlane(x, 16)), min(rlane(x, 32), rlane(x, 48)));
}
// Candidate key: 0 for "no candidate" (retired, out of range or NaN), else
// the bit pattern of the non-negative magnitude plus one, so keys order like
// magnitudes and key 1 is an exact zero.
__device__ __forceinline__ unsigned long long cand_key(double mag, bool valid) {
    return (valid && mag == mag) ? (unsigned long long)__double_as_longlong(mag) + 1ull : 0ull;
}
// (key, position) order of the pivot search: larger key, then lower position.
__device__ __forceinline__ bool cand_wins(unsigned long long k2, unsigned p2, unsigned long long k1, unsigned p1) {
    return k2 > k1 || (k2 == k1 && p2 < p1);
}
// The wave's winning lane (-1 if no lane has a candidate) with its key and
// position. Positions are only compared when keys tie exactly. Uniform
// control flow throughout (readlane). The 64-bit maximum takes the high
// halves first; a unique largest high half (the usual case for data that are
// not exact ties) already names the winner, else the low halves of the lanes
// that share it decide.
__device__ __forceinline__ int wave_winner(unsigned long long key, unsigned pos, unsigned long long &wk, unsigned &wp) {
    const unsigned khi = (unsigned)(key >> 32);
    const unsigned hi = wave_max_u32(khi);
    const unsigned long long bh = __ballot(khi == hi);
    if (__builtin_popcountll(bh) == 1) {
        // hi exceeds every other lane's high half, so it is nonzero: a candidate
        const int wl = (int)__builtin_ctzll(bh);
        wk = ((unsigned long long)hi << 32) | rlane((unsigned)key, wl);
        wp = rlane(pos, wl);
        return wl;
    }
    wk = ((unsigned long long)hi << 32) | wave_max_u32(khi == hi ? (unsigned)key : 0u);
    const bool mine = key == wk && key != 0;
    const unsigned long long ball = __ballot(mine);
    if (ball == 0) { wp = 0xFFFFFFFFu; return -1; }
    if (__builtin_popcountll(ball) == 1) {
        const int wl = (int)__builtin_ctzll(ball);
        wp = rlane(pos, wl);
        return wl;
    }
    wp = wave_min_u32(mine ? pos : 0xFFFFFFFFu);
    return (int)__builtin_ctzll(__ballot(mine && pos == wp));
}

}  // namespace rl
