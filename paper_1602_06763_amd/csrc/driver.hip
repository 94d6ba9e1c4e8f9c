// Recursion driver: the recursive Cholesky and LU of the ReLAPACK collection,
// expressed as a size-based split with no block-size tuning.
//
// The recursive algorithm is the blocked algorithm with block size n/2, the
// unblocked kernel call replaced by a recursive call (Sec. 3, first paragraph
// and footnote); halves are multiples of a fixed quantum where possible (the
// footnote on alignment in Sec. 3); below the crossover size the unblocked
// kernel runs (Sec. 3, paragraph on c). Cholesky and LU are the routines
// xpotrf and xgetrf of Sec. 5.
#include "common.hpp"

namespace rl {

// ---------------------------------------------------------------------------
// Cholesky, lower: A = L·Lᵀ.  potrf(A11); A21 := A21·L11⁻ᵀ; A22 -= A21·A21ᵀ;
// potrf(A22).  Upper: A = Uᵀ·U.  potrf(A11); A12 := U11⁻ᵀ·A12;
// A22 -= A12ᵀ·A12; potrf(A22).
// ---------------------------------------------------------------------------
template <typename T>
void potrf_rec(Ctx &c, Mfma mode, char uplo, long long n, T *A, long long lda, long long off) {
    const int leaf = c.plan && c.plan_leaf > 0 ? c.plan_leaf : kCholLeaf;
    if (n <= leaf) {
        potf2<T>(c, uplo, (int)n, A, lda, off);
        return;
    }
    // the bottom node in one launch, unless a plan asks for another leaf size
    // (a plan with an explicit crossover records the plain recursion at that
    // crossover); its update runs in the storage precision, also under the
    // mixed solver's FP16/BF16 operands (one 64×64×64 product per node, on a
    // factor that only preconditions the refinement)
    const bool native = mode == (sizeof(T) == 8 ? Mfma::F64 : Mfma::F32);
    if ((native || sizeof(T) == 4) && !(c.plan && c.plan_leaf > 0) && n <= 2 * kCholLeaf) {
        potf2x2<T>(c, uplo, (int)n, A, lda, off);
        return;
    }
    const long long n1 = split_size(n), n2 = n - n1;
    const bool lower = (uplo == 'L' || uplo == 'l');
    T *A11 = A, *A22 = A + n1 + n1 * lda;
    c.level++;
    potrf_rec<T>(c, mode, uplo, n1, A11, lda, off);
    c.level--;
    if (lower) {
        T *A21 = A + n1;
        trsm<T, T>(c, mode, 'R', 'L', 'T', 'N', n2, n1, A11, lda, A21, lda);
        gemm<T, T, T>(c, mode, 'N', 'T', 'L', n2, n2, n1, -1.0, A21, lda, A21, lda, 1.0, A22, lda);
    } else {
        T *A12 = A + n1 * lda;
        trsm<T, T>(c, mode, 'L', 'U', 'T', 'N', n1, n2, A11, lda, A12, lda);
        gemm<T, T, T>(c, mode, 'T', 'N', 'U', n2, n2, n1, -1.0, A12, lda, A12, lda, 1.0, A22, lda);
    }
    c.level++;
    potrf_rec<T>(c, mode, uplo, n2, A22, lda, off + n1);
    c.level--;
}

template void potrf_rec<double>(Ctx &, Mfma, char, long long, double *, long long, long long);
template void potrf_rec<float>(Ctx &, Mfma, char, long long, float *, long long, long long);

// ---------------------------------------------------------------------------
// LU with partial pivoting on the columns [c0, c0+w) of an m×ncols matrix,
// rows [c0, m).  getrf(left half); A12 := L11⁻¹·A12; A22 -= A21·A12;
// getrf(right half).  Row interchanges reach every other column once, at the
// latest before anything reads that column again:
//  * nodes wider than kLaswpBlock follow the recursion's own order: after
//    the left half is factored its pivots are applied to the right half's
//    columns in one batch, and after the right half its pivots go to the left
//    half's columns in one batch;
//  * below that, each leaf panel applies its interchanges at once to the
//    other columns of its block (the topmost node of at most kLaswpBlock
//    columns, or the whole matrix when there are no batches).
// Every column receives exactly the interchanges it would have received, in
// the same order, so the result is the same as with the recursion's order
// at every level.
// ---------------------------------------------------------------------------
// Look-ahead (a batch node whose right half's update is not too large): the
// right half's leftmost block of at most kLaswpBlock columns, B1, is updated
// first, and B1 is factored on a stream restricted to a small CU set while
// the rest of the right half's update runs on the other CUs; the call returns
// to its own stream once B1 is done (la_join). B1's kernels touch only B1's
// columns (its interchanges stay inside its block until its parent's batch),
// and the rest of the update reads only the left half and writes only the
// other columns, so the two are independent. Above kLaMaxFlops the update
// alone would outlast B1 on the reduced CU set, and splitting it only slows it.
constexpr double kLaMaxFlops = 2.5e11;

static void la_join(Ctx &c, long long c0, long long w) {
    if (c.la_c0 != c0 || c.la_w != w) return;
    RL_CHECK(hipEventRecord(c.la_ev_small, c.stream));
    c.stream = c.la_main;
    c.num_cu = c.la_main_cu;
    RL_CHECK(hipStreamWaitEvent(c.stream, c.la_ev_small, 0));
    RL_CHECK(hipStreamWaitEvent(c.stream, c.la_ev_big, 0));
    c.la_c0 = -1;
    c.la_w = 0;
}

template <typename T>
static void getrf_rec(Ctx &c, Mfma mode, long long m, long long ncols, T *A, long long lda, int *ipiv,
                      long long c0, long long w, long long blk0, long long blk1, int depth) {
    const int leaf = c.plan && c.plan_leaf > 0 ? c.plan_leaf : kLuLeaf;
    if (w <= leaf) {
        getf2_panel<T>(c, m, (int)w, A, lda, c0, ipiv);
        laswp_leaf<T>(c, A, lda, c0, (int)w, m, ipiv, blk0, blk1);
        la_join(c, c0, w);
        return;
    }
    const long long w1 = split_size(w), w2 = w - w1;
    const bool batch = c.lu_batch && w > kLaswpBlock && depth < kLaswpDepth;
    // a child that is no batch node under a batch node starts its own block
    const long long lb0 = batch ? c0 : blk0, lb1 = batch ? c0 + w1 : blk1;
    const long long rb0 = batch ? c0 + w1 : blk0, rb1 = batch ? c0 + w : blk1;
    const int *inv = batch ? lu_inverse(c, 2 * depth, c0, m) : nullptr;
    c.level++;
    getrf_rec<T>(c, mode, m, ncols, A, lda, ipiv, c0, w1, lb0, lb1, depth + 1);
    c.level--;
    if (batch) laswp_batch<T>(c, A, lda, c0 + w1, w2, c0, m, inv, w1);
    T *A11 = A + c0 + c0 * lda;
    T *A12 = A + c0 + (c0 + w1) * lda;
    T *A21 = A + (c0 + w1) + c0 * lda;
    T *A22 = A + (c0 + w1) + (c0 + w1) * lda;
    long long b1w = w2;   // the right half's leftmost block of at most kLaswpBlock columns
    while (b1w > kLaswpBlock) b1w = split_size(b1w);
    const long long rw = w2 - b1w;
    LaStreams las;
    const bool la = batch && c.lu_batch && !c.plan && !c.fixed && c.la_c0 < 0 && rw > 0 && lookahead_enabled() &&
                    2.0 * (double)(m - c0 - w1) * (double)rw * (double)w1 <= kLaMaxFlops &&
                    (m - c0 - w1 + kPanelRows - 1) / kPanelRows <= 64 && lookahead_streams(c, &las);
    if (!la) {
        trsm<T, T>(c, mode, 'L', 'L', 'N', 'U', w1, w2, A11, lda, A12, lda);
        gemm<T, T, T>(c, mode, 'N', 'N', 0, m - c0 - w1, w2, w1, -1.0, A21, lda, A12, lda, 1.0, A22, lda);
    } else {
        // B1's columns on the calling stream
        trsm<T, T>(c, mode, 'L', 'L', 'N', 'U', w1, b1w, A11, lda, A12, lda);
        gemm<T, T, T>(c, mode, 'N', 'N', 0, m - c0 - w1, b1w, w1, -1.0, A21, lda, A12, lda, 1.0, A22, lda);
    }
    const int *inv2 = batch ? lu_inverse(c, 2 * depth + 1, c0 + w1, m) : nullptr;
    if (la) {
        // fork: the rest of the update on the large CU set, B1 on the small one
        const hipStream_t main = c.stream;
        const int main_cu = c.num_cu;
        RL_CHECK(hipEventRecord(las.ev[0], main));
        RL_CHECK(hipStreamWaitEvent(las.big, las.ev[0], 0));
        RL_CHECK(hipStreamWaitEvent(las.small, las.ev[0], 0));
        c.stream = las.big;
        c.num_cu = las.big_cu;
        trsm<T, T>(c, mode, 'L', 'L', 'N', 'U', w1, rw, A11, lda, A12 + b1w * lda, lda);
        gemm<T, T, T>(c, mode, 'N', 'N', 0, m - c0 - w1, rw, w1, -1.0, A21, lda, A12 + b1w * lda, lda, 1.0,
                      A22 + b1w * lda, lda);
        RL_CHECK(hipEventRecord(las.ev[1], las.big));
        c.stream = las.small;
        c.num_cu = las.small_cu;
        c.la_c0 = c0 + w1;
        c.la_w = b1w;
        c.la_main = main;
        c.la_main_cu = main_cu;
        c.la_ev_big = las.ev[1];
        c.la_ev_small = las.ev[2];
    }
    c.level++;
    getrf_rec<T>(c, mode, m, ncols, A, lda, ipiv, c0 + w1, w2, rb0, rb1, depth + 1);
    c.level--;
    if (batch) laswp_batch<T>(c, A, lda, c0, w1, c0 + w1, m, inv2, w2);
    la_join(c, c0, w);
}

template <typename T>
void getrf_top(Ctx &c, Mfma mode, long long m, long long n, T *A, long long lda, int *ipiv) {
    const long long mn = m < n ? m : n;
    c.lu_tracked = false;
    if (mn <= 0) return;
    // batches when the top node is wide and a column's rows fit the batch kernel
    c.lu_batch = mn > kLaswpBlock && m <= kLaswpBatchRows;
    if (c.lu_batch && !c.plan) {
        c.pv_m = m;
        c.pv = (int *)workspace(c, 7, (size_t)(4 + 2 * kLaswpDepth) * (size_t)m * sizeof(int));
        c.pcur = 0;
        if (!c.pv) { c.lu_batch = false; return; }
    }
    int *inv0 = nullptr;
    if (c.lu_batch) {
        lu_track_begin(c, m);
        if (n > mn) inv0 = lu_inverse(c, 2 * kLaswpDepth, 0, m);   // of the identity
    }
    c.la_c0 = -1;
    getrf_rec<T>(c, mode, m, n, A, lda, ipiv, 0, mn, 0, n, 0);
    if (c.la_c0 >= 0) {   // never left pending; restore the calling stream regardless
        c.stream = c.la_main;
        c.num_cu = c.la_main_cu;
        c.la_c0 = -1;
    }
    if (c.lu_batch && n > mn) laswp_batch<T>(c, A, lda, mn, n - mn, 0, m, inv0, mn);
    c.lu_tracked = c.lu_batch && !c.plan;
    c.lu_batch = false;
    if (n > m) {
        // U12 = L11⁻¹·(P·A12) for the columns beyond the square part
        trsm<T, T>(c, mode, 'L', 'L', 'N', 'U', m, n - m, A, lda, A + m * lda, lda);
    }
}

template void getrf_top<double>(Ctx &, Mfma, long long, long long, double *, long long, int *);
template void getrf_top<float>(Ctx &, Mfma, long long, long long, float *, long long, int *);

}  // namespace rl
