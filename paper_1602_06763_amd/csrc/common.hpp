// Shared declarations of the recursive-factorization library (gfx950 only).
//
// Layout conventions used everywhere: column-major storage with a leading
// dimension (LAPACK), 64-bit index arithmetic, 1-based pivot indices.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "cx.hpp"

namespace rl {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bh8 __attribute__((ext_vector_type(8)));

// Arithmetic used by the matrix cores in the low-precision factorization.
enum class Mfma : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3 };

// Compile-time recursion constants. The leaf sizes are fixed by on-chip
// capacity (a 64×64 FP64 block is 32 KiB of LDS), not tuned per size.
constexpr int kSplitQuantum = 64;   // halves are multiples of this where possible
constexpr int kCholLeaf = 64;       // potf2 leaf: n <= kCholLeaf
constexpr int kTrsmLeaf = 64;       // triangular solve leaf: triangle <= kTrsmLeaf
constexpr int kLuLeaf = 32;         // getf2 panel width
constexpr int kPanelMaxWG = 256;    // cooperative panel: at most one workgroup per CU
constexpr int kBatchMaxSpd = 512;   // batched Cholesky: largest matrix (one workgroup per matrix)
constexpr int kBatchMaxGe = 256;    // batched LU: largest matrix
constexpr int kPanelRows = 512;     // panel rows per workgroup (two per thread)
constexpr int kRecWords = 72;       // 64-bit words per panel exchange record
constexpr int kRecSlots = kPanelMaxWG + 1;   // per step: one per workgroup, one for row d
constexpr int kTrsvMaxRhs = 64;    // left-side solves with at most this many right-hand sides use TRSV
                                    // take the single-launch blocked solve
constexpr int kLaswpBlock = 512;    // LU nodes wider than this apply interchanges in batches
constexpr long long kLaswpBatchRows = 32768;   // batches need m <= this (a column's rows in registers)
constexpr int kLaswpDepth = 12;     // batch-node depths with their own tracker inverses

// Per-call status record shared by every kernel of one library call.
struct DevStatus {
    int info;       // LAPACK info (first failing column, 1-based), 0 = fine
    int error;      // internal failure (e.g. a bounded wait that expired)
    unsigned int barrier;  // reserved
    int ovf;        // a value overflowed when rounded to a lower precision (mixed solves)
};

// One recorded kernel call (plan mode and the per-family timers).
struct PlanRec {
    int kind;   // see PlanKind
    int level;  // recursion depth (0 = top)
    long long m, n, k;
};

enum PlanKind : int {
    PK_POTF2 = 1, PK_TRSM_LEAF = 2, PK_GEMM = 3, PK_SYRK = 4, PK_GETF2 = 5, PK_LASWP = 6,
    PK_CONVERT = 7, PK_RESID = 8, PK_OTHER = 9, PK_GEMM_LP = 10, PK_SYRK_LP = 11,
    PK_GEMM_BIG = 12,  // FP64 GEMM launches on 128×128 tiles (traced separately from PK_GEMM)
    PK_TRTI2 = 13, PK_TRMM_LEAF = 14, PK_LAUU2 = 15,
    PK_ZGEMM = 16,   // complex products on the matrix cores
    PK_ZLEAF = 17,   // complex leaves (Cholesky block, triangular-solve leaf, LU panel)
    PK_TRMM = 18     // triangular product of a whole triangle in one launch
};

// Workspace that a caller-free entry point brings in from a fixed device
// array instead of the library's grow-only allocations: the LU row tracker
// (what workspace slot 7 holds otherwise) and the panel exchange records with
// their own epoch counter. Nothing is allocated while it is set.
struct FixedWs {
    int *tracker = nullptr;
    size_t tracker_bytes = 0;
    unsigned long long *rec = nullptr;
    unsigned int *epoch = nullptr;   // next free epoch of rec (host side, per device)
};

// Per-thread library state: stream, plan recording, tracing.
struct Ctx {
    hipStream_t stream = nullptr;
    int device = -1;
    DevStatus *dstat = nullptr;      // device status block (per device)
    DevStatus *hstat = nullptr;      // pinned host mirror
    int *rowsrc = nullptr;
    size_t rowsrc_elems = 0;
    // LU with batched interchanges: row tracker (two buffers, current = pcur),
    // 2·kLaswpDepth + 1 inverse slots and one batch source map, each pv_m ints
    bool lu_batch = false;
    bool lu_tracked = false;         // the last getrf left its final row tracker at pv + pcur·pv_m
    int *pv = nullptr;
    long long pv_m = 0;
    int pcur = 0;
    // plan mode: record instead of launch
    bool plan = false;
    std::vector<PlanRec> *plan_out = nullptr;
    int level = 0;
    int plan_leaf = 0;               // override of leaf sizes in plan mode (0 = defaults)
    // potrf: every kernel returns at once after a leaf has reported info != 0
    bool abort_on_info = false;
    // tracing: per-kernel-family event timing on the library stream
    bool trace = false;
    hipEvent_t tev0 = nullptr, tev1 = nullptr;   // armed pair for the next launch
    bool tev_armed = false, tev_used = false;
    int num_cu = 256;
    // set only during a caller-free call: workspace comes from here, and the
    // left-side solves avoid the single-launch TRSV (which needs its own buffers)
    FixedWs *fixed = nullptr;
    // LU look-ahead in progress: the block [la_c0, la_c0 + la_w) is being
    // factored on the small CU-masked stream; when it is done, the call
    // returns to la_main after waiting for la_ev_big (the rest of the update)
    long long la_c0 = -1, la_w = 0;
    hipStream_t la_main = nullptr;
    hipEvent_t la_ev_big = nullptr, la_ev_small = nullptr;
    int la_main_cu = 0;
};

// Two streams of one device restricted to disjoint CU sets (default
// priority) for the LU look-ahead, with the events that order them.
struct LaStreams {
    hipStream_t small = nullptr, big = nullptr;
    int small_cu = 0, big_cu = 0;
    hipEvent_t ev[3] = {};
};
bool lookahead_streams(Ctx &c, LaStreams *out);   // false: not available on this device
bool lookahead_enabled();
void lookahead_enable(bool on);

Ctx &ctx();
void ensure_device(Ctx &c);
void *workspace(Ctx &c, int slot, size_t bytes);   // grow-only per-device workspace
constexpr int kSlotBatchOrder = 9;                 // workspace slot: launch order of a batch
constexpr int kSlotTrmm = 11;                      // workspace slot: copy of a triangular product's B
// Exchange records of the cooperative LU panel ([kLuLeaf][kRecSlots][kRecWords]
// words) and the first of kLuLeaf consecutive epochs reserved for one panel.
unsigned long long *panel_records(Ctx &c, unsigned int *epoch);

// Tracing hooks. A region of several launches is bracketed by events recorded
// on the stream (trace_begin / trace_end); a single launch through rl_launch
// between trace_kernel_begin / trace_kernel_end is timed by the launch itself
// (the kernel's own start and end timestamps).
void trace_begin(Ctx &c, int kind);
void trace_end(Ctx &c, int kind, double flops, double bytes);
void trace_kernel_begin(Ctx &c);
void trace_kernel_end(Ctx &c, int kind, double flops, double bytes);

template <typename F, typename... Args>
inline void rl_launch(Ctx &c, F kernel, dim3 grid, dim3 block, unsigned shm, Args... args) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c.tev_armed) {
        e0 = c.tev0;
        e1 = c.tev1;
        c.tev_armed = false;
        c.tev_used = true;
    }
    hipExtLaunchKernelGGL(kernel, grid, block, shm, c.stream, e0, e1, 0u, args...);
}

inline bool plan_record(Ctx &c, int kind, long long m, long long n, long long k) {
    if (!c.plan) return false;
    if (c.plan_out) c.plan_out->push_back(PlanRec{kind, c.level, m, n, k});
    return true;
}

// ---- building blocks (host launchers) --------------------------------------

// C := beta*C + alpha*op(A)*op(B), with op = identity ('N') or transpose ('T').
// TA/TB/TC: storage types in HBM; mode: matrix-core arithmetic. tri = 0: full
// C; 'L'/'U': only the lower/upper triangle of a square C is read or written.
template <typename TA, typename TB, typename TC>
void gemm(Ctx &c, Mfma mode, char ta, char tb, char tri, long long m, long long n, long long k,
          double alpha, const TA *A, long long lda, const TB *B, long long ldb, double beta, TC *C,
          long long ldc);

// Triangular solve with many right-hand sides, recursive down to the leaf:
// side 'L': op(T)·X = B, side 'R': X·op(T) = B; X overwrites B (m×n).
// TT: triangle storage type, TB: right-hand-side storage type.
template <typename TT, typename TB>
void trsm(Ctx &c, Mfma mode, char side, char uplo, char trans, char diag, long long m, long long n,
          const TT *T, long long ldt, TB *B, long long ldb);

// Single-launch blocked solve op(T)·X = B for a few right-hand sides; with
// dinv (the inverses of op(T)'s 64×64 diagonal blocks, from
// trsv_diag_inverses) each diagonal block is applied as a product instead of
// a substitution (the refinement's correction solves).
template <typename TT, typename TB>
void trsv(Ctx &c, bool lower_eff, bool trans, bool unit, long long m, long long nrhs, const TT *T, long long ldt,
          TB *B, long long ldb, const double *dinv);
template <typename TT>
void trsv_diag_inverses(Ctx &c, bool lower_eff, bool trans, bool unit, long long m, const TT *T, long long ldt,
                        double *dinv);

// Cholesky / LU recursion (typed over the storage type of the matrix).
template <typename T>
void potrf_rec(Ctx &c, Mfma mode, char uplo, long long n, T *A, long long lda, long long off);
template <typename T>
void getrf_top(Ctx &c, Mfma mode, long long m, long long n, T *A, long long lda, int *ipiv);

// Leaf kernels.
template <typename T>
void potf2(Ctx &c, char uplo, int n, T *A, long long lda, long long off);
// The recursion's bottom node (64 < n <= 128: potf2, solve, update, potf2)
// in one launch.
template <typename T>
void potf2x2(Ctx &c, char uplo, int n, T *A, long long lda, long long off);
template <typename TT, typename TB>
void trsm_leaf(Ctx &c, bool lower_eff, bool unit, int t, const TT *T, long long ti, long long tj,
               long long nvec, TB *B, long long se, long long sr);
template <typename T>
void getf2_panel(Ctx &c, long long m, int w, T *A, long long lda, long long off, int *ipiv);
// The same cooperative panel for the complex instances (T = cx<double> or
// cx<float>, at most kZLuLeaf columns), the source row of every position
// into c.rowsrc; returns false, launching nothing, when the chip cannot hold
// all its workgroups at once or no source-row list of m entries is set up.
template <typename T>
bool getf2_panel_cx(Ctx &c, long long m, int w, T *A, long long lda, long long off, int *ipiv);
template <typename T>
void laswp_leaf(Ctx &c, T *A, long long lda, long long k0, int w, long long m, const int *ipiv, long long blk0,
                long long blk1);
// Row tracker of the batched interchanges: start (identity), inverse of the
// current tracker over positions [r0, m) into inverse slot `slot`, and one
// batch: columns [j0, j0+ncols), rows [r0, m), npiv pivots (for the records).
void lu_track_begin(Ctx &c, long long m);
int *lu_inverse(Ctx &c, int slot, long long r0, long long m);
template <typename T>
void laswp_batch(Ctx &c, T *A, long long lda, long long j0, long long ncols, long long r0, long long m,
                 const int *inv, long long npiv);
template <typename T>
void laswp_rows(Ctx &c, long long n, T *B, long long ldb, const int *ipiv, long long k1, long long k2,
                bool reverse);

// Triangular product, inverse and Lᵀ·L / U·Uᵀ (FP64): B := α·op(T)·B (side
// 'L') or α·B·op(T) (side 'R'); the recursive xtrtri and xlauum; the first
// zero on the diagonal into the call's info.
void trmm(Ctx &c, char side, char uplo, char trans, char diag, long long m, long long n, double alpha,
          const double *T, long long ldt, double *B, long long ldb);
void trtri_rec(Ctx &c, char uplo, char diag, long long n, double *A, long long lda);
void lauum_rec(Ctx &c, char uplo, long long n, double *A, long long lda);
void diag_zero(Ctx &c, long long n, const double *A, long long lda);
// Batched factorizations (batched.hip): one workgroup per matrix; the per-matrix
// arrays (n, A, lda, ipiv, info) are device arrays of `count` entries.
template <typename T>
void potrf_batched(Ctx &c, bool upper, int count, const int *n, T *const *A, const int *lda, int *info);
template <typename T>
void getrf_batched(Ctx &c, int count, const int *n, T *const *A, const int *lda, int *const *ipiv, int *info);
void trti2_leaf(Ctx &c, bool lower, bool unit, int t, double *A, long long lda);
// Complex instances (complex.hip): A and C point to interleaved (re, im)
// pairs of R; ops 0 = N, 1 = T, 2 = C.
template <typename R>
void zpotrf_top(Ctx &c, char uplo, long long n, void *A, long long lda);
template <typename R>
void zgetrf_top(Ctx &c, long long m, long long n, void *A, long long lda, int *ipiv);
template <typename R>
void zgemm_top(Ctx &c, int opa, int opb, long long m, long long n, long long k, double alpha, const void *A,
               long long lda, const void *B, long long ldb, double beta, void *C, long long ldc);
// Per-bucket leaf / tile choices of the batched routines (0 dpotrf, 1 spotrf,
// 2 dgetrf, 3 sgetrf), graph capture on or off, and release of the captured
// graphs.
bool batched_tune_set(int routine, int bucket, int leaf, int tile);
bool batched_tune_get(int routine, int bucket, int *leaf, int *tile);
void batched_graphs(bool on);
void batched_release();

// Mixed precision helpers.
void scale_spd_f32(Ctx &c, char uplo, long long n, const double *A, long long lda, double *d,
                   float *S, long long lds);
void scale_ge_f32(Ctx &c, long long n, const double *A, long long lda, double *r, double *cs,
                  float *S, long long lds);

// What the last mixed solve of the calling thread did: refinement sweeps in
// all, the sweep from which GMRES-IR ran (0: plain refinement throughout), the
// GMRES-IR sweeps and their Arnoldi steps, the final status (1 converged, -2,
// -3, -31 as iter).
struct MixedStats {
    int sweeps = 0, switched_at = 0, gmres_sweeps = 0, gmres_steps = 0, status = 0;
};
MixedStats mixed_last_stats();
int mixed_solve(Ctx &c, bool spd, char uplo, long long n, long long nrhs, const double *A, long long lda,
                int *ipiv_out, const double *B, long long ldb, double *X, long long ldx, int prec, int *iter,
                double *berr);

// Split rule: halves are multiples of kSplitQuantum where possible.
__host__ __device__ inline long long split_size(long long n, long long quantum = kSplitQuantum) {
    if (n >= 2 * quantum) {
        long long n1 = ((n / 2 + quantum / 2) / quantum) * quantum;
        if (n1 < quantum) n1 = quantum;
        if (n1 >= n) n1 = n - quantum;
        return n1;
    }
    return n / 2;
}

int launch_error(hipError_t e);

// Workspace of the single-launch triangular solve: ticket counter and the
// published solutions as epoch-tagged 64-bit words ([m][8][2]; a fresh buffer
// is zeroed and epochs start at 1).
struct TrsvWork {
    unsigned long long *xw = nullptr;
    unsigned long long *ticket = nullptr;
    unsigned long long ticket_base = 0;
    unsigned int epoch = 0;
};
// Reserves ticket and epoch ranges for ceil(nrhs/8) launches of nb blocks.
TrsvWork trsv_work(Ctx &c, long long m, int nb, int launches = 4, long long row_words = 16,
                   int tickets_per_block = 1);  // records a HIP failure in the calling thread's state

}  // namespace rl

#define RL_CHECK(expr)                                        \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) { rl::launch_error(_e); }       \
    } while (0)
