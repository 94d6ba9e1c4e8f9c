/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the recursive
 * factorizations compute, used to check the HIP library. Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it; the library
 * never does, and this file shares no code, header or constant with it.
 *
 * Conventions: column-major storage with leading dimension lda (LAPACK),
 * 0-based loops, 1-based ipiv and info as LAPACK defines them. Built with
 * -O2 -ffp-contract=off and no fast-math: every update is one rounded multiply
 * followed by one rounded subtract, in increasing elimination step k.
 *
 * Definitions followed (Peise & Bientinesi, "Recursive Algorithms for Dense
 * Linear Algebra: The ReLAPACK Collection"):
 *   - Cholesky: L·Lᵀ := A for symmetric positive definite A (Sec. 5, routine
 *     xpotrf; Sec. 4, Fig. bvsr_others). The factor is unique, so the oracle is
 *     the textbook right-looking elimination that produces it.
 *   - LU with partial pivoting: P·L·U := A (Sec. 5, routine xgetrf). The
 *     recursive algorithm is the blocked algorithm with block size n/2
 *     (Sec. 3, first paragraph and its footnote), and all blocked variants of
 *     one traversal yield the same recursive algorithm, so in exact arithmetic
 *     it selects the same pivots as unblocked right-looking Gaussian elimination
 *     with partial pivoting, which is what this file implements.
 *   - Status codes and argument semantics follow LAPACK, whose interface the
 *     paper preserves (Sec. 5, first paragraph).
 *
 * OpenMP splits only the independent columns j of each rank-1 update, so the
 * result is bitwise identical for every thread count.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(A, lda, i, j) ((A)[(size_t)(j) * (size_t)(lda) + (size_t)(i)])

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int oracle_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int is_lower(char uplo) { return uplo == 'L' || uplo == 'l'; }

/*
 * Cholesky (xpotrf). uplo = 'L': A = L·Lᵀ, L overwrites the lower triangle.
 * uplo = 'U': A = Uᵀ·U, U overwrites the upper triangle. The strict other
 * triangle is never read or written.
 *
 * Step k: if a_kk is not > 0 (this includes NaN) the leading minor of order
 * k+1 is not positive definite; return k+1 with a_kk left as it was.
 * Otherwise a_kk := sqrt(a_kk), scale the rest of column (row) k by it, and
 * subtract the rank-1 term from the trailing triangle.
 */
int oracle_dpotrf(char uplo, int n, double *A, int lda)
{
    if (is_lower(uplo)) {
        for (int k = 0; k < n; ++k) {
            double akk = AT(A, lda, k, k);
            if (!(akk > 0.0)) return k + 1;
            akk = sqrt(akk);
            AT(A, lda, k, k) = akk;
            for (int i = k + 1; i < n; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / akk;
#pragma omp parallel for schedule(static)
            for (int j = k + 1; j < n; ++j) {
                const double ljk = AT(A, lda, j, k);
                for (int i = j; i < n; ++i) {
                    const double prod = AT(A, lda, i, k) * ljk;
                    AT(A, lda, i, j) = AT(A, lda, i, j) - prod;
                }
            }
        }
    } else {
        for (int k = 0; k < n; ++k) {
            double akk = AT(A, lda, k, k);
            if (!(akk > 0.0)) return k + 1;
            akk = sqrt(akk);
            AT(A, lda, k, k) = akk;
            for (int j = k + 1; j < n; ++j) AT(A, lda, k, j) = AT(A, lda, k, j) / akk;
#pragma omp parallel for schedule(static)
            for (int j = k + 1; j < n; ++j) {
                const double ukj = AT(A, lda, k, j);
                for (int i = k + 1; i <= j; ++i) {
                    const double prod = AT(A, lda, k, i) * ukj;
                    AT(A, lda, i, j) = AT(A, lda, i, j) - prod;
                }
            }
        }
    }
    return 0;
}

/*
 * LU with partial (row) pivoting (xgetrf) of an m×n matrix: A = P·L·U with L
 * unit lower trapezoidal (m×min(m,n)) and U upper trapezoidal (min(m,n)×n).
 *
 * Step k, for k < min(m, n):
 *   1. p = the smallest row index i >= k that maximizes |a_ik|. The scan keeps
 *      the first strict maximum, so a NaN never becomes the pivot; if every
 *      candidate is NaN, p = k.
 *   2. ipiv[k] = p + 1.
 *   3. If a_pk != 0: swap rows k and p across all n columns, then divide the
 *      entries below the diagonal of column k by the pivot. Otherwise record
 *      info = k + 1 if no earlier zero pivot was seen, and neither swap nor
 *      scale (the factorization still runs to completion).
 *   4. a_ij -= a_ik·a_kj for every i > k, j > k.
 */
static int gepp(int m, int n, double *A, int lda, int *ipiv, double *margin)
{
    int info = 0;
    const int mn = m < n ? m : n;
    for (int k = 0; k < mn; ++k) {
        int p = k;
        double best = -1.0, second = -1.0;
        for (int i = k; i < m; ++i) {
            const double v = fabs(AT(A, lda, i, k));
            if (v > best) {
                second = best;
                best = v;
                p = i;
            } else if (v > second) {
                second = v;
            }
        }
        ipiv[k] = p + 1;
        /* diagnostic only: how far the winner is ahead of the runner-up */
        if (margin) margin[k] = best > 0.0 ? (best - (second > 0.0 ? second : 0.0)) / best : 0.0;
        if (AT(A, lda, p, k) != 0.0) {
            if (p != k) {
                for (int j = 0; j < n; ++j) {
                    const double t = AT(A, lda, k, j);
                    AT(A, lda, k, j) = AT(A, lda, p, j);
                    AT(A, lda, p, j) = t;
                }
            }
            const double piv = AT(A, lda, k, k);
            for (int i = k + 1; i < m; ++i) AT(A, lda, i, k) = AT(A, lda, i, k) / piv;
        } else if (info == 0) {
            info = k + 1;
        }
#pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {
            const double ukj = AT(A, lda, k, j);
            for (int i = k + 1; i < m; ++i) {
                const double prod = AT(A, lda, i, k) * ukj;
                AT(A, lda, i, j) = AT(A, lda, i, j) - prod;
            }
        }
    }
    return info;
}

int oracle_dgetrf(int m, int n, double *A, int lda, int *ipiv)
{
    return gepp(m, n, A, lda, ipiv, NULL);
}

/*
 * The same elimination, also reporting for every step k the pivot's relative
 * lead over the runner-up, margin[k] = (|a_pk| - max_{i != p} |a_ik|) / |a_pk|
 * (0 when the column is all zero). A floating-point implementation that
 * rounds differently can legitimately choose another row only where this
 * lead is within rounding of zero (a near-tie), so a pivot mismatch at a step
 * with a clear lead is an error and one at a near-tie is not.
 */
int oracle_dgetrf_margin(int m, int n, double *A, int lda, int *ipiv, double *margin)
{
    return gepp(m, n, A, lda, ipiv, margin);
}

/*
 * Solve A·X = B with the Cholesky factor from oracle_dpotrf (xpotrs): for
 * uplo = 'L', forward substitution with L then back substitution with Lᵀ;
 * for uplo = 'U', forward with Uᵀ then back with U. B (n×nrhs) is overwritten.
 */
void oracle_dpotrs(char uplo, int n, int nrhs, const double *A, int lda, double *B, int ldb)
{
    const int lower = is_lower(uplo);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nrhs; ++c) {
        double *b = B + (size_t)c * (size_t)ldb;
        /* forward: M·y = b with M = L (lower) or Uᵀ (upper); M(i,k) for k < i */
        for (int i = 0; i < n; ++i) {
            double s = b[i];
            for (int k = 0; k < i; ++k) {
                const double mik = lower ? AT(A, lda, i, k) : AT(A, lda, k, i);
                s = s - mik * b[k];
            }
            b[i] = s / AT(A, lda, i, i);
        }
        /* backward: Mᵀ·x = y; Mᵀ(i,k) for k > i is M(k,i) */
        for (int i = n - 1; i >= 0; --i) {
            double s = b[i];
            for (int k = i + 1; k < n; ++k) {
                const double mki = lower ? AT(A, lda, k, i) : AT(A, lda, i, k);
                s = s - mki * b[k];
            }
            b[i] = s / AT(A, lda, i, i);
        }
    }
}

/*
 * Solve A·X = B (trans = 'N') or Aᵀ·X = B (trans = 'T') with the factors from
 * oracle_dgetrf of a square n×n A (xgetrs).
 *   'N': apply the interchanges k = 0..n-1 to B, solve L·y = b (unit), U·x = y.
 *   'T': solve Uᵀ·y = b, Lᵀ·z = y (unit), then apply the interchanges in
 *        reverse order k = n-1..0.
 */
void oracle_dgetrs(char trans, int n, int nrhs, const double *A, int lda, const int *ipiv,
                   double *B, int ldb)
{
    const int notrans = (trans == 'N' || trans == 'n');
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nrhs; ++c) {
        double *b = B + (size_t)c * (size_t)ldb;
        if (notrans) {
            for (int k = 0; k < n; ++k) {
                const int p = ipiv[k] - 1;
                if (p != k) {
                    const double t = b[k];
                    b[k] = b[p];
                    b[p] = t;
                }
            }
            for (int i = 0; i < n; ++i) {
                double s = b[i];
                for (int k = 0; k < i; ++k) s = s - AT(A, lda, i, k) * b[k];
                b[i] = s;
            }
            for (int i = n - 1; i >= 0; --i) {
                double s = b[i];
                for (int k = i + 1; k < n; ++k) s = s - AT(A, lda, i, k) * b[k];
                b[i] = s / AT(A, lda, i, i);
            }
        } else {
            for (int i = 0; i < n; ++i) {
                double s = b[i];
                for (int k = 0; k < i; ++k) s = s - AT(A, lda, k, i) * b[k];
                b[i] = s / AT(A, lda, i, i);
            }
            for (int i = n - 1; i >= 0; --i) {
                double s = b[i];
                for (int k = i + 1; k < n; ++k) s = s - AT(A, lda, k, i) * b[k];
                b[i] = s;
            }
            for (int k = n - 1; k >= 0; --k) {
                const int p = ipiv[k] - 1;
                if (p != k) {
                    const double t = b[k];
                    b[k] = b[p];
                    b[p] = t;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Triangular inverse and triangular product (the SPD-inverse follow-on).     */
/* ------------------------------------------------------------------------ */

/*
 * Inverse of a triangular matrix (xtrtri, Sec. 5; the worked example of
 * Sec. 3, Fig. blocked_alg and Fig. recursive_alg: A := A^-1 in place).
 * Definition used: column j of X = T^-1 solves T·x = e_j, by substitution in
 * the order of the triangle (forward for lower, backward for upper):
 *   lower: x_i = (delta_ij - sum_{k=j}^{i-1} t_ik·x_k) / t_ii,  i = j..n-1,
 *   upper: x_i = (delta_ij - sum_{k=i+1}^{j} t_ik·x_k) / t_ii,  i = j..0,
 * each sum taken in increasing k, one rounded multiply and one rounded
 * subtract per term. diag = 'U': t_ii is taken as 1 and never read, and the
 * diagonal of A is left as it is. As in LAPACK, a non-unit triangle with an
 * exact zero on the diagonal is reported (info = first such index, 1-based)
 * before anything is written. The strict other triangle is never touched.
 */
int oracle_dtrtri(char uplo, char diag, int n, double *A, int lda)
{
    const int lower = is_lower(uplo);
    const int unit = (diag == 'U' || diag == 'u');
    if (!unit)
        for (int i = 0; i < n; ++i)
            if (AT(A, lda, i, i) == 0.0) return i + 1;
    double *X = (double *)calloc((size_t)n * (size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        double *x = X + (size_t)j * (size_t)n;
        if (lower) {
            for (int i = j; i < n; ++i) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) s = s - AT(A, lda, i, k) * x[k];
                x[i] = unit ? s : s / AT(A, lda, i, i);
            }
        } else {
            for (int i = j; i >= 0; --i) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int k = i + 1; k <= j; ++k) s = s - AT(A, lda, i, k) * x[k];
                x[i] = unit ? s : s / AT(A, lda, i, i);
            }
        }
    }
    for (int j = 0; j < n; ++j) {
        const double *x = X + (size_t)j * (size_t)n;
        if (lower) {
            for (int i = unit ? j + 1 : j; i < n; ++i) AT(A, lda, i, j) = x[i];
        } else {
            for (int i = 0; i <= (unit ? j - 1 : j); ++i) AT(A, lda, i, j) = x[i];
        }
    }
    free(X);
    return 0;
}

/*
 * Product of a triangular matrix with its transpose (xlauum, Sec. 5):
 *   uplo = 'L': A := Lᵀ·L,  (Lᵀ·L)_ij = sum_{k=max(i,j)}^{n-1} l_ki·l_kj,
 *   uplo = 'U': A := U·Uᵀ,  (U·Uᵀ)_ij = sum_{k=max(i,j)}^{n-1} u_ik·u_jk,
 * each sum in increasing k; the result's own triangle (the one the factor
 * came in) is written, the strict other triangle is never touched.
 */
void oracle_dlauum(char uplo, int n, double *A, int lda)
{
    const int lower = is_lower(uplo);
    double *C = (double *)calloc((size_t)n * (size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        if (lower) {
            for (int i = j; i < n; ++i) {
                double s = 0.0;
                for (int k = i; k < n; ++k) s = s + AT(A, lda, k, i) * AT(A, lda, k, j);
                C[(size_t)j * n + i] = s;
            }
        } else {
            for (int i = 0; i <= j; ++i) {
                double s = 0.0;
                for (int k = j; k < n; ++k) s = s + AT(A, lda, i, k) * AT(A, lda, j, k);
                C[(size_t)j * n + i] = s;
            }
        }
    }
    for (int j = 0; j < n; ++j) {
        if (lower)
            for (int i = j; i < n; ++i) AT(A, lda, i, j) = C[(size_t)j * n + i];
        else
            for (int i = 0; i <= j; ++i) AT(A, lda, i, j) = C[(size_t)j * n + i];
    }
    free(C);
}

/* ------------------------------------------------------------------------ */
/* Mixed-precision preprocessing and the FP64 backward error.                */
/* ------------------------------------------------------------------------ */

/*
 * Power-of-two exponent t with 4^t <= x < 4^(t+1) for finite x > 0, i.e. the
 * d = 2^-t that maps x into [1, 4) as d²·x. frexp gives x = f·2^e, f in
 * [0.5, 1), so log2(x) lies in [e-1, e) and t = floor((e-1)/2).
 */
static int quarter_exponent(double x)
{
    int e;
    (void)frexp(x, &e);
    const int em1 = e - 1;
    return em1 >= 0 ? em1 / 2 : -((-em1 + 1) / 2);
}

/* Exponent t with 2^t <= x < 2^(t+1) for finite x > 0. */
static int half_exponent(double x)
{
    int e;
    (void)frexp(x, &e);
    return e - 1;
}

/*
 * Symmetric diagonal scaling for the SPD mixed solve: d_i = 2^-t_i with
 * 4^t_i <= a_ii < 4^(t_i+1), so (D·A·D)_ii lies in [1, 4) and every scaled
 * entry is bounded by 4 in magnitude. Non-positive or non-finite a_ii get
 * d_i = 1. Writes S = D·A·D (the uplo triangle only, exact in binary64 away
 * from underflow) rounded to binary32 into S32 (column-major, lds).
 */
void oracle_scale_spd_f32(char uplo, int n, const double *A, int lda, double *d, float *S32,
                          int lds)
{
    for (int i = 0; i < n; ++i) {
        const double aii = AT(A, lda, i, i);
        d[i] = (aii > 0.0 && isfinite(aii)) ? ldexp(1.0, -quarter_exponent(aii)) : 1.0;
    }
    const int lower = is_lower(uplo);
    for (int j = 0; j < n; ++j) {
        const int i0 = lower ? j : 0, i1 = lower ? n : j + 1;
        for (int i = i0; i < i1; ++i) {
            const double s = (d[i] * AT(A, lda, i, j)) * d[j];
            S32[(size_t)j * lds + i] = (float)s;
        }
    }
}

/*
 * Two-sided power-of-two scaling for the general mixed solve: first
 * r_i = 2^-t_i with 2^t_i <= max_j |a_ij| < 2^(t_i+1), then c_j the same
 * for the columns of R·A (rows or columns that are entirely zero keep a
 * factor of 1). S = R·A·C, rounded to binary32.
 */
void oracle_scale_ge_f32(int n, const double *A, int lda, double *r, double *c, float *S32,
                         int lds)
{
    for (int i = 0; i < n; ++i) {
        double mx = 0.0;
        for (int j = 0; j < n; ++j) {
            const double v = fabs(AT(A, lda, i, j));
            if (v > mx) mx = v;
        }
        r[i] = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -half_exponent(mx)) : 1.0;
    }
    for (int j = 0; j < n; ++j) {
        double mx = 0.0;
        for (int i = 0; i < n; ++i) {
            const double v = fabs(r[i] * AT(A, lda, i, j));
            if (v > mx) mx = v;
        }
        c[j] = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -half_exponent(mx)) : 1.0;
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            S32[(size_t)j * lds + i] = (float)((r[i] * AT(A, lda, i, j)) * c[j]);
}

/*
 * Normwise backward error of each column of a computed solution X of
 * A·X = B (Rigal–Gaches):  eta_j = ||b_j - A·x_j||_inf /
 *                                   (||A||_inf·||x_j||_inf + ||b_j||_inf).
 * For a symmetric A stored in one triangle pass sym = 'L' or 'U'; else 'N'.
 * Returns max_j eta_j and writes each column's value to eta (may be NULL).
 */
double oracle_backward_error(char sym, int n, int nrhs, const double *A, int lda,
                             const double *X, int ldx, const double *B, int ldb, double *eta)
{
    double *rowsum = (double *)calloc((size_t)n, sizeof(double));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double aij;
            if (sym == 'L' || sym == 'l')
                aij = i >= j ? AT(A, lda, i, j) : AT(A, lda, j, i);
            else if (sym == 'U' || sym == 'u')
                aij = i <= j ? AT(A, lda, i, j) : AT(A, lda, j, i);
            else
                aij = AT(A, lda, i, j);
            rowsum[i] += fabs(aij);
        }
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        if (rowsum[i] > anorm) anorm = rowsum[i];
    free(rowsum);

    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        const double *x = X + (size_t)c * ldx;
        const double *b = B + (size_t)c * ldb;
        double rmax = 0.0, xmax = 0.0, bmax = 0.0;
        for (int i = 0; i < n; ++i) {
            double s = b[i];
            for (int j = 0; j < n; ++j) {
                double aij;
                if (sym == 'L' || sym == 'l')
                    aij = i >= j ? AT(A, lda, i, j) : AT(A, lda, j, i);
                else if (sym == 'U' || sym == 'u')
                    aij = i <= j ? AT(A, lda, i, j) : AT(A, lda, j, i);
                else
                    aij = AT(A, lda, i, j);
                s = s - aij * x[j];
            }
            if (fabs(s) > rmax) rmax = fabs(s);
            if (fabs(x[i]) > xmax) xmax = fabs(x[i]);
            if (fabs(b[i]) > bmax) bmax = fabs(b[i]);
        }
        const double den = anorm * xmax + bmax;
        const double e = den > 0.0 ? rmax / den : (rmax > 0.0 ? INFINITY : 0.0);
        if (eta) eta[c] = e;
        if (e > worst || isnan(e)) worst = e;
    }
    return worst;
}

/* ---------------------------------------------------------------------------
 * Complex instances (the c/z types of the collection, Sec. 5): storage is
 * LAPACK's, each element a (real, imaginary) pair of doubles, column-major.
 * The arithmetic is written out in real operations so that its order is
 * visible:
 *   product   (a·b) = (a.re·b.re − a.im·b.im, a.re·b.im + a.im·b.re)
 *   quotient  a / p = (a·conj(p)) / (p.re² + p.im²), each part divided
 *   pivot size cabs1(z) = |z.re| + |z.im| (LAPACK's izamax rule)
 * --------------------------------------------------------------------------- */
typedef struct { double re, im; } zel;

#define ZAT(A, lda, i, j) ((A)[(size_t)(j) * (size_t)(lda) + (size_t)(i)])

static zel zmul(zel a, zel b)
{
    zel r;
    const double p1 = a.re * b.re, p2 = a.im * b.im, p3 = a.re * b.im, p4 = a.im * b.re;
    r.re = p1 - p2;
    r.im = p3 + p4;
    return r;
}

static zel zconj(zel a) { a.im = -a.im; return a; }

static zel zsub(zel a, zel b) { zel r; r.re = a.re - b.re; r.im = a.im - b.im; return r; }

static zel zdiv(zel a, zel p)
{
    const double d1 = p.re * p.re, d2 = p.im * p.im;
    const double den = d1 + d2;
    const zel q = zmul(a, zconj(p));
    zel r;
    r.re = q.re / den;
    r.im = q.im / den;
    return r;
}

static double cabs1(zel z) { return fabs(z.re) + fabs(z.im); }

/*
 * Cholesky of a Hermitian positive definite matrix (xpotrf, complex):
 * uplo = 'L': A = L·Lᴴ, L overwrites the lower triangle; uplo = 'U':
 * A = Uᴴ·U, U overwrites the upper triangle. Only the real part of a
 * diagonal entry is read; the diagonal of the factor is real (imaginary part
 * written as 0). Step k: if re(a_kk) is not > 0 (NaN included) return k+1
 * with a_kk left as it was; else l_kk = sqrt(re(a_kk)), the rest of column
 * (row) k is divided by it, and the trailing triangle takes
 * a_ij −= l_ik·conj(l_jk) (lower) or a_ij −= conj(u_ki)·u_kj (upper).
 */
int oracle_zpotrf(char uplo, int n, double *Ad, int lda)
{
    zel *A = (zel *)Ad;
    const int lower = is_lower(uplo);
    for (int k = 0; k < n; ++k) {
        const double akk = ZAT(A, lda, k, k).re;
        if (!(akk > 0.0)) return k + 1;
        const double lkk = sqrt(akk);
        ZAT(A, lda, k, k).re = lkk;
        ZAT(A, lda, k, k).im = 0.0;
        for (int i = k + 1; i < n; ++i) {
            zel *e = lower ? &ZAT(A, lda, i, k) : &ZAT(A, lda, k, i);
            e->re = e->re / lkk;
            e->im = e->im / lkk;
        }
#pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {
            if (lower) {
                const zel cjk = zconj(ZAT(A, lda, j, k));
                for (int i = j; i < n; ++i) ZAT(A, lda, i, j) = zsub(ZAT(A, lda, i, j), zmul(ZAT(A, lda, i, k), cjk));
            } else {
                const zel ukj = ZAT(A, lda, k, j);
                for (int i = k + 1; i <= j; ++i)
                    ZAT(A, lda, i, j) = zsub(ZAT(A, lda, i, j), zmul(zconj(ZAT(A, lda, k, i)), ukj));
            }
        }
    }
    return 0;
}

/*
 * LU with partial pivoting of a complex m×n matrix (xgetrf, complex): as
 * oracle_dgetrf with the pivot the first row maximizing cabs1(a_ik) (a NaN
 * never wins), the column below divided by the pivot, and the rank-1 update
 * a_ij −= a_ik·a_kj. A pivot with both parts zero is exactly zero: no swap,
 * no division, info records the first such column.
 */
int oracle_zgetrf(int m, int n, double *Ad, int lda, int *ipiv)
{
    zel *A = (zel *)Ad;
    int info = 0;
    const int mn = m < n ? m : n;
    for (int k = 0; k < mn; ++k) {
        int p = k;
        double best = -1.0;
        for (int i = k; i < m; ++i) {
            const double v = cabs1(ZAT(A, lda, i, k));
            if (v > best) { best = v; p = i; }
        }
        ipiv[k] = p + 1;
        const zel ap = ZAT(A, lda, p, k);
        if (ap.re != 0.0 || ap.im != 0.0) {
            if (p != k) {
                for (int j = 0; j < n; ++j) {
                    const zel t = ZAT(A, lda, k, j);
                    ZAT(A, lda, k, j) = ZAT(A, lda, p, j);
                    ZAT(A, lda, p, j) = t;
                }
            }
            const zel piv = ZAT(A, lda, k, k);
            for (int i = k + 1; i < m; ++i) ZAT(A, lda, i, k) = zdiv(ZAT(A, lda, i, k), piv);
        } else if (info == 0) {
            info = k + 1;
        }
#pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {
            const zel ukj = ZAT(A, lda, k, j);
            for (int i = k + 1; i < m; ++i) ZAT(A, lda, i, j) = zsub(ZAT(A, lda, i, j), zmul(ZAT(A, lda, i, k), ukj));
        }
    }
    return info;
}
