/*
 * relapack.h -- C ABI of librelapack_mi355x.so, recursive dense factorizations
 * for AMD MI355X (gfx950).
 *
 * The operations are those of the ReLAPACK collection (Peise & Bientinesi,
 * "Recursive Algorithms for Dense Linear Algebra: The ReLAPACK Collection"):
 * recursive Cholesky (xpotrf, Sec. 5) and recursive LU with partial pivoting
 * (xgetrf, Sec. 5), built as the paper prescribes (Sec. 3): the blocked
 * algorithm with block size n/2 and the unblocked kernel replaced by a
 * recursive call, halves aligned to a fixed quantum where possible, an
 * unblocked kernel below a fixed crossover size, no block-size tuning. Almost
 * every flop lands in the BLAS-3 updates of the top recursion levels (Sec. 3,
 * flop-share analysis next to Fig. recursive_breakdown), which here run on the
 * FP64 matrix cores. The argument conventions are LAPACK's, whose interface
 * the paper keeps (Sec. 5, first paragraph).
 *
 * Conventions common to every entry point
 *   - Matrices and pivot vectors (A, B, X, C, ipiv, d, r, c, S) are DEVICE
 *     pointers (hipMalloc or a torch CUDA tensor's data_ptr()), column-major
 *     with the given leading dimension. The caller owns them.
 *   - Scalar outputs (info, iter, berr) are HOST pointers. A NULL info makes
 *     the call a no-op.
 *   - Every call is stream-ordered on the calling thread's library stream
 *     (relapack_set_stream) and returns after the work has completed, so info
 *     is valid on return. Calls from several threads on one device run one
 *     at a time (the per-device workspace is shared); each holds the device
 *     until its work has completed.
 *   - info = 0: success. info = -k: argument k (counted in the C signature
 *     order below) is illegal; nothing was launched. info in (-2000, -1000]:
 *     a HIP runtime error e was reported (info = -1000 - e). info <= -2000:
 *     an internal wait of the LU panel timed out (the result is unusable).
 *   - The library keeps a grow-only device workspace per device (status
 *     block, pivot bookkeeping, low-precision copies, the launch order of a
 *     batch); relapack_finalize() releases it.
 *   - Integer arguments are 32-bit as in LAPACK; index arithmetic inside is
 *     64-bit.
 */
#ifndef RELAPACK_MI355X_H
#define RELAPACK_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

/* Library version (1). */
int relapack_version(void);

/* Set the calling thread's stream (a hipStream_t; NULL = the null stream).
 * Returns 0. */
int relapack_set_stream(void *hip_stream);

/* The calling thread's stream. */
void *relapack_get_stream(void);

/* Free the per-device workspace of every device the library has touched. */
void relapack_finalize(void);

/*
 * Cholesky factorization (xpotrf; Sec. 5 and Fig. bvsr_others):
 *   uplo = 'L': A = L·Lᵀ, L overwrites the lower triangle;
 *   uplo = 'U': A = Uᵀ·U, U overwrites the upper triangle.
 * The strict other triangle is neither read nor written.
 * A: n×n, lda >= max(1, n).
 * info = k > 0: the leading minor of order k is not positive definite (its
 * pivot is <= 0 or NaN); every kernel after the failing leaf returns at once,
 * so columns before k hold the factor and column k holds its updated pivot.
 * The recursion's leaves are 64 columns; its bottom node (64 < n <= 128:
 * two leaves, the solve and the update between them) runs as one launch.
 * Errors: uplo -1, n -2, lda -4.
 */
void relapack_dpotrf(char uplo, int n, double *A, int lda, int *info);

/*
 * LU factorization with partial (row) pivoting (xgetrf; Sec. 5): A = P·L·U,
 * L unit lower trapezoidal (m×min(m,n)), U upper trapezoidal; both overwrite
 * A. ipiv (device, min(m,n) ints, 1-based): row i was interchanged with row
 * ipiv[i], in order. The pivot is the first row holding the largest |a_ik|
 * (a NaN never wins).
 * info = k > 0: U(k,k) is exactly zero (the first such k); the factorization
 * is completed.
 * Limits: every leaf panel (at most 32 columns over all rows below its
 * diagonal) runs as ceil(rows / 512) cooperating workgroups, one per CU, that
 * wait on each other, so m <= 512·(number of CUs) = 131072 on MI355X. Before
 * each panel the library checks that the kernel's occupancy lets the chip
 * hold all of them at once (else info = -1000 - hipErrorCooperativeLaunchTooLarge
 * and that panel is not launched). Every wait is bounded: if other work on the
 * GPU keeps some of them from starting for about a second, the call returns
 * info <= -2000 and A and ipiv are unusable.
 * Errors: m -1, n -2, lda -4.
 */
void relapack_dgetrf(int m, int n, double *A, int lda, int *ipiv, int *info);

/*
 * Look-ahead of the LU recursion (relapack_dgetrf, relapack_sgetrf and the
 * mixed solves' LU; off by default, on = 1 enables it): at a node whose right
 * half's update is at most 2.5e11 flops, the right half's leftmost block of
 * at most 512 columns is updated first and factored on a second stream while
 * the rest of the update runs on a stream restricted to all but 64 CUs (both
 * of default priority, created on first use, ordered against the calling
 * stream by events). Results are bit-identical with it on or off. Measured
 * on MI355X it is slower (dgetrf n = 16384: 142.0 ms off, 153.3 ms on;
 * n = 32768: 602.4 against 626.9 ms): the streams overlap, but the split
 * update on fewer CUs loses as much as the overlap hides, because the block's
 * factorization, bound by its 16 panels' latency, outlasts the rest of the
 * update at every node where the update is short enough to split.
 */
void relapack_lookahead(int on);

/*
 * relapack_dgetrf without any allocation, for callers that cannot allocate
 * device memory while they run (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same operation, arguments, results
 * and kernels as relapack_dgetrf; the caller still passes A and ipiv. Its
 * workspace (status block, row bookkeeping, panel exchange records; about
 * 8.6 MB) is a fixed device array of the library, one per GPU, held until the
 * process ends; the call makes no hipMalloc, hipFree or other allocating call.
 * Limit: m <= 32768 (else info = -1 and nothing is launched). Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (from
 * several processes, or from threads that bypass the per-device call lock
 * by using different library instances) race. Within one process the
 * per-device call lock serializes them.
 * Errors: m -1 (negative or above 32768), n -2, lda -4.
 */
void relapack_dgetrf_noalloc(int m, int n, double *A, int lda, int *ipiv, int *info);

/*
 * Solve A·X = B with the factor from relapack_dpotrf (xpotrs). A: the n×n
 * factor; B: n×nrhs, overwritten by X.
 * Errors: uplo -1, n -2, nrhs -3, lda -5, ldb -7.
 */
void relapack_dpotrs(char uplo, int n, int nrhs, const double *A, int lda, double *B, int ldb,
                     int *info);

/*
 * Solve A·X = B (trans 'N') or Aᵀ·X = B (trans 'T'/'C') with the factors and
 * pivots from relapack_dgetrf of a square A (xgetrs). B: n×nrhs, overwritten.
 * Errors: trans -1, n -2, nrhs -3, lda -5, ldb -8.
 */
void relapack_dgetrs(char trans, int n, int nrhs, const double *A, int lda, const int *ipiv,
                     double *B, int ldb, int *info);

/*
 * Mixed-precision solve of an SPD system with FP64 iterative refinement.
 * A (n×n, only the uplo triangle is read, never modified), B (n×nrhs, read),
 * X (n×nrhs, written). The factorization runs on a power-of-two scaled copy
 * D·A·D held in FP32 with its matrix-core updates in the arithmetic prec:
 * 32 (FP32), 16 (FP16 operands, FP32 accumulation) or 'b' (BF16 operands,
 * FP32 accumulation). FP64 is used for the residual r = b - A·x, the update
 * and the correction solve. Stops when every column's normwise backward error
 * eta = ||r||inf / (||A||inf·||x||inf + ||b||inf) <= 1e-14.
 * Sweeps: plain refinement (x += M⁻¹r, M the scaled low-precision factors,
 * applied in FP64) while each sweep at least halves eta; after that
 * GMRES-IR: each sweep solves A·d = r by FP64 GMRES left-preconditioned by
 * M⁻¹ (restart 40, inner tolerance 1e-6, at most 40 Arnoldi steps per
 * solve, one restart cycle: a longer refinement costs more than the FP64
 * solve it replaces; Carson and Higham's GMRES-based refinement).
 * Refinement stops after 30 sweeps, when eta fails twice to halve under
 * GMRES-IR, or when a GMRES sweep's average residual reduction per step,
 * checked from its 12th step on, would not reach 1e-6 within the remaining
 * Arnoldi budget (the preconditioned matrix then has too many scattered
 * eigenvalues, as when kappa times the factorization's unit roundoff is well
 * above 1).
 * iter (host): > 0 refinement sweeps used; < 0 the FP64 path was used
 * instead: -2 a value overflowed when rounded to the low precision (a scaled
 * entry beyond the FP32 range, or a matrix-core operand beyond the FP16/BF16
 * range during the factorization), -3 the low-precision factorization failed,
 * -31 no convergence.
 * berr (host): the final max_j eta_j, computed in FP64.
 * Errors: uplo -1, n -2, nrhs -3, lda -5, ldb -7, ldx -9, prec -10.
 */
void relapack_dposv_mixed(char uplo, int n, int nrhs, const double *A, int lda, const double *B,
                          int ldb, double *X, int ldx, int prec, int *iter, double *berr,
                          int *info);

/*
 * Mixed-precision solve of a general system with FP64 iterative refinement;
 * as relapack_dposv_mixed with a partial-pivoting LU of the two-sided
 * power-of-two scaled copy R·A·C in FP32. ipiv (device, n ints) receives the
 * low-precision factorization's pivots (or the FP64 ones after a fallback).
 * Errors: n -1, nrhs -2, lda -4, ldb -7, ldx -9, prec -10.
 */
void relapack_dgesv_mixed(int n, int nrhs, const double *A, int lda, int *ipiv, const double *B,
                          int ldb, double *X, int ldx, int prec, int *iter, double *berr,
                          int *info);

/*
 * What the calling thread's last mixed solve did: refinement sweeps in all,
 * the sweep from which GMRES-IR ran (0: plain refinement throughout), the
 * GMRES-IR sweeps and their Arnoldi steps. NULL pointers are skipped.
 */
void relapack_mixed_last(int *sweeps, int *gmres_from, int *gmres_sweeps, int *gmres_steps);

/* ---- complex instances (the c/z types of Sec. 5) ------------------------- */

/*
 * Complex Cholesky (xpotrf for complex types; Sec. 5 lists every routine of
 * the collection in the four types s, d, c, z): A Hermitian positive
 * definite, uplo 'L': A = L·Lᴴ; 'U': A = Uᴴ·U; the factor overwrites that
 * triangle, the strict other triangle is neither read nor written. A points
 * to LAPACK's complex storage: n×n (re, im) pairs of doubles (z) or floats
 * (c), column-major, lda >= max(1, n) elements. Only the real part of a
 * diagonal entry is read; the factor's diagonal is real (its imaginary parts
 * written as 0). info = k > 0: re(a_kk) not > 0 (or NaN) at step k, the
 * factorization stops there (as relapack_dpotrf). Same recursion as the real
 * routine, its products C -= A·Bᴴ on the matrix cores as four real
 * products each, leaves of at most 64.
 * Errors: uplo -1, n -2, lda -4.
 */
void relapack_zpotrf(char uplo, int n, void *A, int lda, int *info);
void relapack_cpotrf(char uplo, int n, void *A, int lda, int *info);

/*
 * Complex LU with partial pivoting (xgetrf for complex types): A = P·L·U,
 * the pivot of column k the first row with the largest |re| + |im| (LAPACK's
 * izamax; a NaN never wins), ipiv (device, min(m, n) ints, 1-based) as
 * relapack_dgetrf. A: m×n complex (z: pairs of doubles, c: pairs of floats),
 * column-major. info = k > 0: U(k, k) is exactly zero (both parts), the first
 * such k; the factorization completes. Leaves are panels of at most 16
 * columns, factored as relapack_dgetrf's (ceil(rows / 512) cooperating
 * workgroups with bounded waits: info <= -2000 if other GPU work keeps some
 * from starting for about a second), or, where the chip cannot hold that
 * grid at once, by one workgroup (no limit on m); their interchanges are
 * applied at once to every other column.
 * Errors: m -1, n -2, lda -4.
 */
void relapack_zgetrf(int m, int n, void *A, int lda, int *ipiv, int *info);
void relapack_cgetrf(int m, int n, void *A, int lda, int *ipiv, int *info);

/*
 * C := beta·C + alpha·op(A)·op(B), complex double (pairs of doubles), op 'N',
 * 'T' or 'C' (conjugate transpose), alpha and beta real: the complex product
 * the recursion uses, exported for testing. C: m×n.
 * Errors: transa -1, transb -2, m -3, n -4, k -5, lda -8, ldb -10, ldc -13.
 */
void relapack_zgemm(char transa, char transb, int m, int n, int k, double alpha, const void *A, int lda,
                    const void *B, int ldb, double beta, void *C, int ldc, int *info);

/* ---- building blocks on the recursion's path (FP64 matrix cores) -------- */

/*
 * C := beta·C + alpha·op(A)·op(B), op = 'N' or 'T' (xgemm; the Schur-complement
 * updates of the recursion, Sec. 3). C: m×n.
 * Errors: transa -1, transb -2, m -3, n -4, k -5, lda -8, ldb -10, ldc -13.
 */
void relapack_dgemm(char transa, char transb, int m, int n, int k, double alpha, const double *A,
                    int lda, const double *B, int ldb, double beta, double *C, int ldc, int *info);

/*
 * C := beta·C + alpha·op(A)·op(A)ᵀ on the uplo triangle of C only (xsyrk;
 * Cholesky's trailing update). trans 'N': op(A) = A (n×k); 'T': op(A) = Aᵀ.
 * Errors: uplo -1, trans -2, n -3, k -4, lda -7, ldc -10.
 */
void relapack_dsyrk(char uplo, char trans, int n, int k, double alpha, const double *A, int lda,
                    double beta, double *C, int ldc, int *info);

/*
 * Triangular solve with many right-hand sides, B := op(A)⁻¹·B (side 'L') or
 * B := B·op(A)⁻¹ (side 'R') (xtrsm with alpha = 1), recursive down to a
 * substitution leaf. A: triangular (uplo), unit diagonal if diag = 'U'.
 * Errors: side -1, uplo -2, transa -3, diag -4, m -5, n -6, lda -8, ldb -10.
 */
void relapack_dtrsm(char side, char uplo, char transa, char diag, int m, int n, const double *A,
                    int lda, double *B, int ldb, int *info);

/*
 * Triangular matrix product (xtrmm; step (2) of the recursive inversion in
 * Sec. 3, Fig. recursive_alg): B := alpha·op(A)·B (side 'L', A m×m) or
 * B := alpha·B·op(A) (side 'R', A n×n); A triangular (uplo), unit diagonal if
 * diag = 'U' (then its diagonal is not read). B: m×n, overwritten. Recursive
 * down to triangles of at most 1024 rows, each then one launch over a copy
 * of its part of B (library workspace, grown on demand, kept until
 * relapack_finalize), or a 64×64 matrix-core leaf for triangles of at most
 * 64 rows.
 * Errors: side -1, uplo -2, transa -3, diag -4, m -5, n -6, lda -9, ldb -11.
 */
void relapack_dtrmm(char side, char uplo, char transa, char diag, int m, int n, double alpha,
                    const double *A, int lda, double *B, int ldb, int *info);

/* ---- SPD inverse (xtrtri, xlauum; Sec. 5) ------------------------------ */

/*
 * Inverse of a triangular matrix in place (xtrtri, Sec. 5; the recursive
 * algorithm of Sec. 3, Fig. recursive_alg: invert A_TL, A_BL := A_BL·A_TL,
 * A_BL := −A_BR⁻¹·A_BL, invert A_BR; unblocked below 64, the bottom node
 * of at most 128 rows in one launch). uplo selects the
 * triangle; diag = 'U': unit diagonal, not read and not written. The strict
 * other triangle is neither read nor written.
 * info = i > 0: A(i,i) is exactly zero (diag = 'N'); this is checked before
 * anything is written, and A is then left unchanged.
 * Errors: uplo -1, diag -2, n -3, lda -5.
 */
void relapack_dtrtri(char uplo, char diag, int n, double *A, int lda, int *info);

/*
 * Product of a triangle with its own transpose in place (xlauum, Sec. 5):
 * uplo = 'L': the lower triangle of A becomes that of Lᵀ·L; uplo = 'U': the
 * upper triangle becomes that of U·Uᵀ. Recursive: lauum(A_TL), A_TL +=
 * A_BLᵀ·A_BL (matrix-core SYRK), A_BL := A_BRᵀ·A_BL (trmm), lauum(A_BR);
 * a triangle of at most 128 rows in one launch. The strict other triangle is
 * neither read nor written.
 * Errors: uplo -1, n -2, lda -4.
 */
void relapack_dlauum(char uplo, int n, double *A, int lda, int *info);

/*
 * Inverse of an SPD matrix from its Cholesky factor (xpotri, the user of
 * xtrtri and xlauum named in Sec. 5): on entry the factor from
 * relapack_dpotrf(uplo, ...); on exit the uplo triangle of A⁻¹ = L⁻ᵀ·L⁻¹
 * (uplo 'L') or U⁻¹·U⁻ᵀ (uplo 'U'), i.e. dtrtri(uplo, 'N') then dlauum(uplo).
 * info = i > 0: the factor's (i,i) entry is exactly zero; A is unchanged.
 * Errors: uplo -1, n -2, lda -4.
 */
void relapack_dpotri(char uplo, int n, double *A, int lda, int *info);

/* ---- pieces of the mixed-precision path -------------------------------- */

/*
 * Power-of-two symmetric scaling and conversion: d_i = 2^-t_i with
 * 4^t_i <= a_ii < 4^(t_i+1) (d_i = 1 if a_ii is not positive and finite);
 * S = D·A·D rounded to FP32 (round to nearest even) in the uplo triangle.
 * d: n doubles; S: n×n floats, lds >= max(1, n). Errors: uplo -1, n -2, lda -4, lds -7.
 */
void relapack_scale_spd_f32(char uplo, int n, const double *A, int lda, double *d, float *S, int lds,
                            int *info);

/*
 * Two-sided power-of-two scaling and conversion: r_i = 2^-t with
 * 2^t <= max_j |a_ij| < 2^(t+1), then c_j the same for the columns of R·A
 * (1 for an all-zero row or column); S = R·A·C rounded to FP32.
 * Errors: n -1, lda -3, lds -7.
 */
void relapack_scale_ge_f32(int n, const double *A, int lda, double *r, double *c, float *S, int lds,
                           int *info);

/*
 * Recursive Cholesky / partial-pivoting LU of an FP32 matrix whose
 * matrix-core updates use the arithmetic prec (32, 16 or 'b'; FP32
 * accumulation). Same argument and info conventions as the FP64 routines;
 * prec is argument -5 (potrf) / -6 (getrf).
 */
void relapack_spotrf_lp(char uplo, int n, float *A, int lda, int prec, int *info);
void relapack_sgetrf_lp(int m, int n, float *A, int lda, int *ipiv, int prec, int *info);

/* ---- single precision (the paper's x = s instances, Sec. 5) ------------ */

/*
 * FP32 Cholesky / partial-pivoting LU (xpotrf / xgetrf with x = s, Sec. 5):
 * FP32 storage and FP32 matrix-core updates, otherwise exactly the FP64
 * routines' recursion, arguments and info (relapack_dpotrf, relapack_dgetrf).
 * Errors: as relapack_dpotrf / relapack_dgetrf.
 */
void relapack_spotrf(char uplo, int n, float *A, int lda, int *info);
void relapack_sgetrf(int m, int n, float *A, int lda, int *ipiv, int *info);

/* ---- batched factorizations ---------------------------------------------- */

/*
 * Cholesky of `count` independent SPD matrices of uneven sizes in one launch
 * (the recursive xpotrf of Sec. 3 and Sec. 5 per matrix, run on the device,
 * one workgroup per matrix). Matrix b is n[b]×n[b] at A[b] with leading
 * dimension lda[b], column-major; uplo as in relapack_dpotrf (only that
 * triangle is read and written).
 *   n, A, lda, info: DEVICE arrays of `count` entries (A: device pointers to
 *   the caller's device matrices); the caller owns all of them.
 *   info[b] (device): 0, k > 0 (leading minor k not positive definite; that
 *   matrix's factorization stopped there), -2 (n[b] < 0 or n[b] > 512),
 *   -4 (lda[b] < max(1, n[b])).
 *   One persistent launch: as many workgroups as the chip holds at once take
 *   the matrices from a device work queue in order of size, largest first
 *   (the order, count ints, and the queue counter live in the library's
 *   workspace). Each matrix's recursion uses the leaf size and product tile
 *   edge of its size bucket (relapack_batched_tune). The launch sequence is
 *   captured into a HIP graph the first time a (routine, count, arrays,
 *   tuning) combination is seen and replayed afterwards (at most 16 graphs
 *   are kept; relapack_batched_graphs(0) launches directly instead).
 * Returns 0, -1 (uplo), -2 (count < 0), -3 (a null array with count > 0),
 * or -1000 - hipError_t. Stream-ordered; returns after completion.
 */
int relapack_dpotrf_batched(char uplo, int count, const int *n, double *const *A, const int *lda, int *info);
int relapack_spotrf_batched(char uplo, int count, const int *n, float *const *A, const int *lda, int *info);

/*
 * LU with partial pivoting of `count` independent square matrices of uneven
 * sizes in one launch (the recursive xgetrf of Sec. 3 and Sec. 5 per matrix,
 * on the device, one workgroup per matrix): P·A = L·U with LAPACK's ipiv.
 *   n, A, lda, ipiv, info: DEVICE arrays of `count` entries; ipiv[b] points
 *   to the caller's device array of n[b] ints (1-based pivot rows).
 *   info[b] (device): 0, k > 0 (U(k,k) exactly zero, the first such k; the
 *   factorization completes), -2 (n[b] < 0 or n[b] > 256), -4 (lda[b] <
 *   max(1, n[b])). Persistent launch, work queue in order of size, tuning
 *   and graph capture as in relapack_dpotrf_batched.
 * Returns 0, -1 (count < 0), -2 (a null array with count > 0), or
 * -1000 - hipError_t. Stream-ordered; returns after completion.
 */
int relapack_dgetrf_batched(int count, const int *n, double *const *A, const int *lda, int *const *ipiv,
                            int *info);
int relapack_sgetrf_batched(int count, const int *n, float *const *A, const int *lda, int *const *ipiv,
                            int *info);

/*
 * Per-size-bucket choices of the batched routines (routine: 0 dpotrf,
 * 1 spotrf, 2 dgetrf, 3 sgetrf; bucket: 0 n <= 64, 1 n <= 128, 2 n <= 256,
 * 3 above): leaf = the crossover of each matrix's recursion (Cholesky 32 or
 * 64, LU panel width 16 or 32), tile = the edge of the matrix-core product
 * tiles (32 or 64). The defaults are the table measured by
 * paper_1602_06763_amd/autotune.py on MI355X. Returns 0, -1 (routine),
 * -2 (bucket), -3 (a value not offered). Not thread-safe against running
 * batched calls of other threads (their next call picks the new values up).
 */
int relapack_batched_tune(int routine, int bucket, int leaf, int tile);
int relapack_batched_tune_get(int routine, int bucket, int *leaf, int *tile);

/* Batched calls through captured HIP graphs (on = 1, the default) or by
 * direct launches (on = 0). Tracing always launches directly. */
void relapack_batched_graphs(int on);

/* ---- measurement and inspection ------------------------------------------ */

/* Bracket every kernel launch of this thread with HIP events (on = 1) and
 * clear the collected records. */
void relapack_trace_enable(int on);

/* Per kernel family k in [0, cap): out[4k .. 4k+3] = {launches, total ms,
 * algorithmic flops, algorithmic bytes}; families: 1 potf2, 2 trsm leaf,
 * 3 gemm on 64×64 tiles and 12 gemm on 128×128 tiles, 4 syrk (FP64 matrix
 * cores), 5 getf2 panel, 6 laswp, 7 convert, 8 residual, 10 gemm and 11 syrk
 * with FP32/FP16/BF16 operands, 13 triangular-inverse leaf, 14 trmm leaf,
 * 15 lauum leaf, 16 complex products, 17 complex leaves, 18 trmm of a whole
 * triangle in one launch (with its copy of B). Single-kernel families are
 * timed by the
 * kernel's own start/end timestamps, the others by events around them.
 * Synchronizes the stream and clears the records. Returns cap, or -1 on a
 * HIP error. */
int relapack_trace_collect(double *out, int cap);

/* The kernel-call sequence of one factorization without launching anything
 * (no GPU needed): routine "potrf_L", "potrf_U", "getrf", "trtri_L",
 * "trtri_U", "lauum_L" or "lauum_U"; leaf > 0 overrides every crossover
 * size and records the plain recursion at it (leaf = 0: the library's own
 * sizes, with the one-launch bottom nodes as one record each of kind 1, 13
 * or 15). Writes up to cap records of 5 int64
 * {kind, depth, m, n, k} to rec; returns the total number of calls. */
long long relapack_plan(const char *routine, long long m, long long n, int leaf, long long *rec,
                        long long cap);

/* Size of the first half when the recursion splits n (host rule, no GPU). */
long long relapack_split(long long n);

#ifdef __cplusplus
}
#endif

#endif /* RELAPACK_MI355X_H */
