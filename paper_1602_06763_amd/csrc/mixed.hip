// Mixed-precision solves with FP64 iterative refinement.
//
// The factorization is the same recursion as the FP64 one, run on a
// power-of-two scaled FP32 copy of A whose matrix-core updates use FP32, FP16
// or BF16 operands with FP32 accumulation. FP64 is kept for the residual
// r = b - A·x, the solution update and the correction solve, which reads the
// low-precision factors and computes in FP64. The loop stops once the
// normwise backward error eta = ||r||inf / (||A||inf·||x||inf + ||b||inf) of
// every right-hand side is at most 1e-14, and falls back to the FP64
// factorization when the low-precision one fails or refinement stalls.
#include "common.hpp"

#include <cmath>
#include <cstring>

namespace rl {

enum ScratchSlot { SL_LP = 0, SL_FULL = 1, SL_VEC = 2, SL_RED = 3, SL_FB = 4, SL_PIV = 5, SL_PERM = 6, SL_DINV = 8,
                  SL_GM = 10 };

__global__ void reset_info_k(DevStatus *s) {
    if (threadIdx.x == 0) { s->info = 0; s->error = 0; s->barrier = 0u; s->ovf = 0; }
}

__global__ void zero_u64_k(long long n, unsigned long long *p) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---- power-of-two scaling ----------------------------------------------------

// t with 4^t <= x < 4^(t+1): frexp gives x = f·2^e, f in [0.5, 1)
__device__ __forceinline__ double quarter_scale(double x) {
    if (!(x > 0.0) || !isfinite(x)) return 1.0;
    int e;
    (void)frexp(x, &e);
    const int em1 = e - 1;
    const int t = em1 >= 0 ? em1 / 2 : -((-em1 + 1) / 2);
    return ldexp(1.0, -t);
}

// 2^-t with 2^t <= x < 2^(t+1)
__device__ __forceinline__ double half_scale(double x) {
    if (!(x > 0.0) || !isfinite(x)) return 1.0;
    int e;
    (void)frexp(x, &e);
    return ldexp(1.0, -(e - 1));
}

__global__ void spd_diag_scale_k(long long n, const double *A, long long lda, double *d) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = quarter_scale(A[i + i * lda]);
}

// A scaled entry that rounds to an infinite float (the FP32 range is
// exceeded) marks the status block: the solve then falls back to FP64.
__device__ __forceinline__ float to_f32_flag(double v, DevStatus *st) {
    const float f = (float)v;
    if (__builtin_isinf(f) && st) __hip_atomic_store(&st->ovf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return f;
}

__global__ void spd_convert_k(long long n, const double *__restrict__ A, long long lda,
                              const double *__restrict__ d, float *__restrict__ S, long long lds,
                              int lower, DevStatus *st) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long j = blockIdx.y;
    if (i >= n) return;
    if (lower ? (i < j) : (i > j)) return;
    S[i + j * lds] = to_f32_flag((d[i] * A[i + j * lda]) * d[j], st);
}

// max |a_ij| over each row, 2-D tiles combined with an atomic max on the
// (non-negative, hence order-preserving) bit pattern.
__global__ void row_absmax_k(long long n, const double *__restrict__ A, long long lda,
                             const double *__restrict__ scale, unsigned long long *rmax) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long j0 = (long long)blockIdx.y * 256, j1 = min(n, j0 + 256);
    double mx = 0.0;
    for (long long j = j0; j < j1; ++j) {
        double v = fabs(A[i + j * lda]);
        if (scale) v = fabs(scale[i] * A[i + j * lda]);
        if (v > mx) mx = v;
    }
    atomicMax(&rmax[i], (unsigned long long)__double_as_longlong(mx));
}

// max over each column of |r_i·a_ij|, one workgroup per column
__global__ __launch_bounds__(256) void col_absmax_k(long long n, const double *__restrict__ A, long long lda,
                                                    const double *__restrict__ r, double *cmax) {
    const long long j = blockIdx.x;
    __shared__ double red[256];
    double mx = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) {
        const double v = fabs(r[i] * A[i + j * lda]);
        if (v > mx) mx = v;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) cmax[j] = red[0];
}

__global__ void bits_to_half_scale_k(long long n, const unsigned long long *bits, double *s) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = half_scale(__longlong_as_double((long long)bits[i]));
}

__global__ void to_half_scale_k(long long n, const double *mx, double *s) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = half_scale(mx[i]);
}

__global__ void ge_convert_k(long long n, const double *__restrict__ A, long long lda,
                             const double *__restrict__ r, const double *__restrict__ c,
                             float *__restrict__ S, long long lds, DevStatus *st) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long j = blockIdx.y;
    if (i >= n) return;
    S[i + j * lds] = to_f32_flag((r[i] * A[i + j * lda]) * c[j], st);
}

static inline unsigned blocks(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

void scale_spd_f32(Ctx &c, char uplo, long long n, const double *A, long long lda, double *d, float *S,
                   long long lds) {
    if (plan_record(c, PK_CONVERT, n, n, 0)) return;
    trace_begin(c, PK_CONVERT);
    hipLaunchKernelGGL(spd_diag_scale_k, dim3(blocks(n)), dim3(256), 0, c.stream, n, A, lda, d);
    hipLaunchKernelGGL(spd_convert_k, dim3(blocks(n), (unsigned)n), dim3(256), 0, c.stream, n, A, lda, d, S,
                       lds, (int)(uplo == 'L' || uplo == 'l'), c.dstat);
    RL_CHECK(hipGetLastError());
    trace_end(c, PK_CONVERT, 0.0, 6.0 * n * n);
}

void scale_ge_f32(Ctx &c, long long n, const double *A, long long lda, double *r, double *cs, float *S,
                  long long lds) {
    if (plan_record(c, PK_CONVERT, n, n, 0)) return;
    unsigned long long *bits = (unsigned long long *)workspace(c, SL_RED, (size_t)n * 8);
    if (!bits) return;
    trace_begin(c, PK_CONVERT);
    hipLaunchKernelGGL(zero_u64_k, dim3(blocks(n)), dim3(256), 0, c.stream, n, bits);
    hipLaunchKernelGGL(row_absmax_k, dim3(blocks(n), blocks(n)), dim3(256), 0, c.stream, n, A, lda,
                       (const double *)nullptr, bits);
    hipLaunchKernelGGL(bits_to_half_scale_k, dim3(blocks(n)), dim3(256), 0, c.stream, n, bits, r);
    hipLaunchKernelGGL(col_absmax_k, dim3((unsigned)n), dim3(256), 0, c.stream, n, A, lda, r,
                       (double *)bits);
    hipLaunchKernelGGL(to_half_scale_k, dim3(blocks(n)), dim3(256), 0, c.stream, n, (const double *)bits, cs);
    hipLaunchKernelGGL(ge_convert_k, dim3(blocks(n), (unsigned)n), dim3(256), 0, c.stream, n, A, lda, r, cs, S,
                       lds, c.dstat);
    RL_CHECK(hipGetLastError());
    trace_end(c, PK_CONVERT, 0.0, 14.0 * n * n);
}

// ---- FP64 residual and backward error ---------------------------------------

// Full symmetric copy of a triangle-stored SPD matrix (for the FP64 residual),
// by 64×64 tiles of the stored triangle: each tile is read once (coalesced),
// written in place and, transposed through LDS, into its mirror position.
__global__ __launch_bounds__(256) void symmetrize_k(long long n, const double *__restrict__ A, long long lda,
                                                    double *__restrict__ F, int lower) {
    const long long I = blockIdx.x, J = blockIdx.y;
    if (lower ? I < J : I > J) return;   // tiles of the stored triangle only
    __shared__ double S[64][65];
    const int tid = threadIdx.x, r = tid & 63, c4 = tid >> 6;
    const long long i0 = I * 64, j0 = J * 64;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int cc = c4 + 4 * u;
        const long long i = i0 + r, j = j0 + cc;
        S[r][cc] = (i < n && j < n) ? A[i + j * lda] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int cc = c4 + 4 * u;
        const long long i = i0 + r, j = j0 + cc;
        if (i < n && j < n) {
            if (I != J) F[i + j * n] = S[r][cc];
            else F[i + j * n] = (lower ? r >= cc : r <= cc) ? S[r][cc] : S[cc][r];
        }
        // the mirror tile (J, I): element (j0 + r, i0 + cc) = A(i0 + cc, j0 + r)
        const long long mi = j0 + r, mj = i0 + cc;
        if (I != J && mi < n && mj < n) F[mi + mj * n] = S[cc][r];
    }
}

__global__ void copy_cols_k(long long n, long long ncol, const double *S, long long lds, double *D,
                            long long ldd) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long j = blockIdx.y;
    if (i < n && j < ncol) D[i + j * ldd] = S[i + j * lds];
}

// ||A||inf partial row sums over 256-column chunks (deterministic two-pass)
__global__ void row_abssum_part_k(long long n, const double *__restrict__ A, long long lda, double *part) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long j0 = (long long)blockIdx.y * 256, j1 = min(n, j0 + 256);
    double s = 0.0;
    for (long long j = j0; j < j1; ++j) s += fabs(A[i + j * lda]);
    part[(long long)blockIdx.y * n + i] = s;
}

// row sums from the partials (a thread per row), then the largest per workgroup
__global__ __launch_bounds__(256) void inf_norm_rows_k(long long n, long long nchunk, const double *part,
                                                       double *bmax) {
    __shared__ double red[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (i < n)
        for (long long q = 0; q < nchunk; ++q) s += part[q * n + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k && (red[threadIdx.x + k] > red[threadIdx.x] || red[threadIdx.x + k] != red[threadIdx.x + k]))
            red[threadIdx.x] = red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) bmax[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void inf_norm_finish_k(long long nb, const double *bmax, double *out) {
    __shared__ double red[256];
    double mx = 0.0;
    for (long long i = threadIdx.x; i < nb; i += 256) {
        const double s = bmax[i];
        if (s > mx || s != s) mx = s;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s && (red[threadIdx.x + s] > red[threadIdx.x] || red[threadIdx.x + s] != red[threadIdx.x + s]))
            red[threadIdx.x] = red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// eta_j for every column j (one workgroup per column); out[j] = eta_j
__global__ __launch_bounds__(256) void col_eta_k(long long n, const double *R, long long ldr, const double *X,
                                                 long long ldx, const double *B, long long ldb,
                                                 const double *anorm, double *out) {
    const long long j = blockIdx.x;
    __shared__ double rr[256], xx[256], bb[256];
    double r = 0, x = 0, b = 0;
    for (long long i = threadIdx.x; i < n; i += 256) {
        const double rv = fabs(R[i + j * ldr]), xv = fabs(X[i + j * ldx]), bv = fabs(B[i + j * ldb]);
        if (rv > r || rv != rv) r = rv;
        if (xv > x || xv != xv) x = xv;
        if (bv > b) b = bv;
    }
    rr[threadIdx.x] = r; xx[threadIdx.x] = x; bb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const int t = threadIdx.x;
            if (rr[t + s] > rr[t] || rr[t + s] != rr[t + s]) rr[t] = rr[t + s];
            if (xx[t + s] > xx[t] || xx[t + s] != xx[t + s]) xx[t] = xx[t + s];
            if (bb[t + s] > bb[t]) bb[t] = bb[t + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double den = (*anorm) * xx[0] + bb[0];
        out[j] = den > 0.0 ? rr[0] / den : (rr[0] > 0.0 ? INFINITY : 0.0);
    }
}

__global__ void max_of_k(long long n, const double *v, double *out) {
    __shared__ double red[256];
    double mx = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256)
        if (v[i] > mx || v[i] != v[i]) mx = v[i];
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s && (red[threadIdx.x + s] > red[threadIdx.x] || red[threadIdx.x + s] != red[threadIdx.x + s]))
            red[threadIdx.x] = red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Y[i,j] = s[i] * X[i,j] (s may be null: plain copy)
__global__ void scale_rows_k(long long n, long long ncol, const double *s, const double *X, long long ldx,
                             double *Y, long long ldy) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long j = blockIdx.y;
    if (i >= n) return;
    const double v = X[i + j * ldx];
    Y[i + j * ldy] = s ? s[i] * v : v;
}

// X[i,j] += s[i] * D[i,j]
__global__ void axpy_rows_k(long long n, long long ncol, const double *s, const double *D, long long ldd,
                            double *X, long long ldx) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long j = blockIdx.y;
    if (i >= n) return;
    X[i + j * ldx] += s[i] * D[i + j * ldd];
}

// ---- the refinement driver -----------------------------------------------------

struct MixedWork {
    float *S = nullptr;        // n×n low-precision factors
    double *Af = nullptr;      // full FP64 matrix for the residual (SPD: symmetrized copy)
    long long ldaf = 0;
    double *s1 = nullptr, *s2 = nullptr;   // scalings (d, or r and c)
    double *R = nullptr, *D = nullptr;     // residual, correction (n×nrhs)
    double *eta = nullptr;                 // nrhs column backward errors
    double *scal = nullptr;                // [0] ||A||inf, [1] max eta
    double *part = nullptr;                // row-sum partials
    int *ipiv = nullptr;
    int *perm = nullptr;                   // general: the pivots as a gather map
    double *dinv1 = nullptr, *dinv2 = nullptr;   // inverted 64×64 diagonal blocks of the two
                                                 // triangular factors (first and second solve)
};

static double fetch_scalar(Ctx &c, const double *dptr) {
    double h = 0.0;
    RL_CHECK(hipMemcpyAsync(&h, dptr, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    RL_CHECK(hipStreamSynchronize(c.stream));
    return h;
}

static int fetch_info(Ctx &c) {
    RL_CHECK(hipMemcpyAsync(c.hstat, c.dstat, sizeof(DevStatus), hipMemcpyDeviceToHost, c.stream));
    RL_CHECK(hipStreamSynchronize(c.stream));
    return c.hstat->error ? -2000 - c.hstat->error : c.hstat->info;
}

static Mfma prec_mode(int prec) {
    if (prec == 16) return Mfma::F16;
    if (prec == 'b' || prec == 'B') return Mfma::BF16;
    return Mfma::F32;
}

// R = B - Af·X, eta per column, returns max eta (one 8-byte read-back)
// R = B - A·X in FP64 for a few right-hand sides (the residual of an IR
// sweep is a matrix-vector product, bound by reading A once from HBM): a
// workgroup per 64 rows, its four waves splitting the columns, lane = row so
// every load of A is a coalesced 512-byte column segment; 16 columns are in
// flight per wave.
constexpr int kResidMaxRhs = 4;
template <int NR, bool MV = false>
__global__ __launch_bounds__(256) void resid_k(long long n, const double *__restrict__ A, long long lda,
                                               const double *__restrict__ X, long long ldx,
                                               const double *__restrict__ B, long long ldb, double *__restrict__ R,
                                               long long ldr) {
    __shared__ double part[4][NR][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long row = (long long)blockIdx.x * 64 + lane;
    const long long rc = row < n ? row : n - 1;
    const long long per = (n + 3) / 4;
    const long long j0 = wave * per, j1 = min(n, j0 + per);
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    long long j = j0;
    for (; j + 16 <= j1; j += 16) {
        double a[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = A[rc + (j + u) * lda];
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] = fma(a[u], X[(j + u) + r * ldx], acc[r]);
    }
    for (; j < j1; ++j) {
        const double a = A[rc + j * lda];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = fma(a, X[j + r * ldx], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) part[wave][r][lane] = acc[r];
    __syncthreads();
    if (wave == 0 && row < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
        {
            const double ax = (part[0][r][lane] + part[1][r][lane]) + (part[2][r][lane] + part[3][r][lane]);
            R[row + r * ldr] = MV ? ax : B[row + r * ldb] - ax;
        }
    }
}

static double residual_eta(Ctx &c, long long n, long long nrhs, MixedWork &w, const double *B, long long ldb,
                           const double *X, long long ldx) {
    if (nrhs <= kResidMaxRhs) {
        trace_begin(c, PK_RESID);
        const dim3 g((unsigned)((n + 63) / 64));
        if (nrhs == 1)
            hipLaunchKernelGGL(resid_k<1>, g, dim3(256), 0, c.stream, n, w.Af, w.ldaf, X, ldx, B, ldb, w.R, n);
        else if (nrhs == 2)
            hipLaunchKernelGGL(resid_k<2>, g, dim3(256), 0, c.stream, n, w.Af, w.ldaf, X, ldx, B, ldb, w.R, n);
        else
            for (long long r0 = 0; r0 < nrhs; r0 += 1)
                hipLaunchKernelGGL(resid_k<1>, g, dim3(256), 0, c.stream, n, w.Af, w.ldaf, X + r0 * ldx, ldx,
                                   B + r0 * ldb, ldb, w.R + r0 * n, n);
        trace_end(c, PK_RESID, 2.0 * n * n * nrhs, 8.0 * n * n + 24.0 * n * nrhs);
    } else {
        trace_begin(c, PK_RESID);
        hipLaunchKernelGGL(copy_cols_k, dim3(blocks(n), (unsigned)nrhs), dim3(256), 0, c.stream, n, nrhs, B, ldb,
                           w.R, n);
        trace_end(c, PK_RESID, 0.0, 16.0 * n * nrhs);
        gemm<double, double, double>(c, Mfma::F64, 'N', 'N', 0, n, nrhs, n, -1.0, w.Af, w.ldaf, X, ldx, 1.0, w.R, n);
    }
    hipLaunchKernelGGL(col_eta_k, dim3((unsigned)nrhs), dim3(256), 0, c.stream, n, w.R, n, X, ldx, B, ldb,
                       w.scal, w.eta);
    hipLaunchKernelGGL(max_of_k, dim3(1), dim3(256), 0, c.stream, nrhs, w.eta, w.scal + 1);
    RL_CHECK(hipGetLastError());
    return fetch_scalar(c, w.scal + 1);
}

static void inf_norm(Ctx &c, long long n, const double *A, long long lda, MixedWork &w) {
    const long long nchunk = (n + 255) / 256;
    hipLaunchKernelGGL(row_abssum_part_k, dim3(blocks(n), (unsigned)nchunk), dim3(256), 0, c.stream, n, A, lda,
                       w.part);
    double *bmax = w.part + nchunk * n;
    hipLaunchKernelGGL(inf_norm_rows_k, dim3(blocks(n)), dim3(256), 0, c.stream, n, nchunk, (const double *)w.part,
                       bmax);
    hipLaunchKernelGGL(inf_norm_finish_k, dim3(1), dim3(256), 0, c.stream, (long long)blocks(n),
                       (const double *)bmax, w.scal);
    RL_CHECK(hipGetLastError());
}

// The row permutation of a partial-pivoting factorization as a gather map:
// perm[i] is the row of the original matrix that ends up in row i after the
// interchanges ipiv[0..n) are applied in order. One workgroup; the sequential
// interchanges run on LDS copies when they fit, else on the output array.
__global__ __launch_bounds__(256) void ipiv_to_perm_k(long long n, const int *__restrict__ ipiv, int *perm) {
    extern __shared__ int pl[];   // [2n] perm, ipiv (when they fit)
    const bool lds = n <= 16384;
    int *P = lds ? pl : perm;
    for (long long i = threadIdx.x; i < n; i += 256) {
        P[i] = (int)i;
        if (lds) pl[n + i] = ipiv[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (long long k = 0; k < n; ++k) {
            const long long p = (lds ? pl[n + k] : ipiv[k]) - 1;
            if (p != k) {
                const int t = P[k];
                P[k] = P[p];
                P[p] = t;
            }
        }
    }
    __syncthreads();
    if (lds)
        for (long long i = threadIdx.x; i < n; i += 256) perm[i] = pl[i];
}

// D(i, :) = s(perm[i]) · R(perm[i], :): the row scaling and the interchanges
// of the general correction solve in one gather.
__global__ void perm_scale_rows_k(long long n, long long ncol, const int *__restrict__ perm, const double *s,
                                  const double *R, long long ldr, double *D, long long ldd) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long c = blockIdx.y;
    if (i < n) {
        const long long p = perm[i];
        D[i + c * ldd] = s[p] * R[p + c * ldr];
    }
}

// D = A_lp⁻¹·R through the scaled low-precision factors, in FP64 arithmetic
static void correction(Ctx &c, bool spd, char uplo, long long n, long long nrhs, MixedWork &w) {
    const dim3 g(blocks(n), (unsigned)nrhs);
    // D = s1 ∘ R (SPD: D·r), or P·(s1 ∘ R) (general: P·R·r) in one gather
    if (spd)
        hipLaunchKernelGGL(scale_rows_k, g, dim3(256), 0, c.stream, n, nrhs, (const double *)w.s1, w.R, n, w.D, n);
    else
        hipLaunchKernelGGL(perm_scale_rows_k, g, dim3(256), 0, c.stream, n, nrhs, (const int *)w.perm,
                           (const double *)w.s1, (const double *)w.R, n, w.D, n);
    if (w.dinv1) {
        // one right-hand side: single-launch blocked solves with the factors'
        // inverted diagonal blocks (formed once per factorization)
        if (spd && uplo == 'L') {
            trsv<float, double>(c, true, false, false, n, nrhs, w.S, n, w.D, n, w.dinv1);
            trsv<float, double>(c, false, true, false, n, nrhs, w.S, n, w.D, n, w.dinv2);
        } else if (spd) {
            trsv<float, double>(c, true, true, false, n, nrhs, w.S, n, w.D, n, w.dinv1);
            trsv<float, double>(c, false, false, false, n, nrhs, w.S, n, w.D, n, w.dinv2);
        } else {
            trsv<float, double>(c, true, false, true, n, nrhs, w.S, n, w.D, n, w.dinv1);
            trsv<float, double>(c, false, false, false, n, nrhs, w.S, n, w.D, n, w.dinv2);
        }
        return;
    }
    if (spd) {
        if (uplo == 'L') {
            trsm<float, double>(c, Mfma::F64, 'L', 'L', 'N', 'N', n, nrhs, w.S, n, w.D, n);
            trsm<float, double>(c, Mfma::F64, 'L', 'L', 'T', 'N', n, nrhs, w.S, n, w.D, n);
        } else {
            trsm<float, double>(c, Mfma::F64, 'L', 'U', 'T', 'N', n, nrhs, w.S, n, w.D, n);
            trsm<float, double>(c, Mfma::F64, 'L', 'U', 'N', 'N', n, nrhs, w.S, n, w.D, n);
        }
    } else {
        trsm<float, double>(c, Mfma::F64, 'L', 'L', 'N', 'U', n, nrhs, w.S, n, w.D, n);
        trsm<float, double>(c, Mfma::F64, 'L', 'U', 'N', 'N', n, nrhs, w.S, n, w.D, n);
    }
}

// The inverted diagonal blocks of both factors, for the single-launch solves
// of the corrections (same effective triangles as the solves above).
static void prepare_correction(Ctx &c, bool spd, char uplo, long long n, long long nrhs, MixedWork &w) {
    if (nrhs != 1 || n <= 2 * kTrsmLeaf) return;   // one right-hand side: the single-launch solve
    const long long nb = (n + 63) / 64;
    double *d = (double *)workspace(c, SL_DINV, (size_t)2 * nb * 4096 * sizeof(double));
    if (!d) return;
    w.dinv1 = d;
    w.dinv2 = d + nb * 4096;
    if (spd && uplo == 'L') {
        trsv_diag_inverses<float>(c, true, false, false, n, w.S, n, w.dinv1);
        trsv_diag_inverses<float>(c, false, true, false, n, w.S, n, w.dinv2);
    } else if (spd) {
        trsv_diag_inverses<float>(c, true, true, false, n, w.S, n, w.dinv1);
        trsv_diag_inverses<float>(c, false, false, false, n, w.S, n, w.dinv2);
    } else {
        trsv_diag_inverses<float>(c, true, false, true, n, w.S, n, w.dinv1);
        trsv_diag_inverses<float>(c, false, false, false, n, w.S, n, w.dinv2);
    }
}

// ---- GMRES-IR ----------------------------------------------------------------
// When plain refinement contracts slowly (kappa·u_f near or above 1), each
// sweep instead solves the correction equation A·d = r with FP64 GMRES, left
// preconditioned by the low-precision factors: the Krylov space of M⁻¹A is
// built from M⁻¹r, where M⁻¹ = C·(L·U)⁻¹·P·R is the correction solve above
// (scalings and interchanges included), orthogonalized by classical
// Gram-Schmidt applied twice, and the small least-squares problem is updated
// by Givens rotations (Carson and Higham's GMRES-based refinement). All
// right-hand sides run together, each with its own basis and rotations; a
// column stops once its preconditioned residual has dropped by kGmTol.
constexpr int kGmMax = 40;        // Arnoldi steps per sweep (restart length)
constexpr int kGmTotal = 40;      // Arnoldi steps per solve before giving up. A step costs one
                                  // low-precision correction solve and one FP64 product with A;
                                  // at n = 16384 the FP64 LU costs about 85 such steps and the
                                  // low-precision LU already two thirds of the FP64 one, so a
                                  // refinement much longer than one restart cycle cannot beat
                                  // the FP64 solve and only adds to the fallback's cost
constexpr double kGmTol = 1e-6;   // relative reduction of the preconditioned residual
constexpr int kGmProbe = 12;      // from this many steps of a sweep on, its rate so far must reach
                                  // kGmTol within the solve's remaining Arnoldi budget, else
                                  // the solve is abandoned: M⁻¹A then has too many scattered
                                  // eigenvalues for a short Krylov space (kappa·u_f well above 1)
constexpr int kGmH = kGmMax + 1;  // rows of each column's Hessenberg matrix

struct GmWork {
    double *V = nullptr;      // kGmH blocks of n×nrhs: V_j(r, c) = V[(j·nrhs + c)·n + r]
    double *H = nullptr;      // per column kGmH × kGmMax, column-major
    double *hv = nullptr;     // per column kGmH: second projection pass, new norm
    double *cs = nullptr, *sn = nullptr;   // per column kGmMax rotations
    double *g = nullptr;      // per column kGmH: rotated right-hand side
    double *y = nullptr;      // per column kGmMax: least-squares solution
    double *beta = nullptr;   // per column: ||M⁻¹r||
    double *flag = nullptr;   // [0]: largest residual ratio of unfinished columns
    int *kk = nullptr;        // per column: Arnoldi steps that count
    int *done = nullptr;      // per column: finished
};

// hout[c·ldh + i] = V_i(:, c)ᵀ·W(:, c), i < cnt (a workgroup per (i, c))
__global__ __launch_bounds__(256) void gm_dot_k(long long n, long long nrhs, const double *__restrict__ V,
                                                const double *__restrict__ W, double *hout, long long ldh) {
    const long long i = blockIdx.x, c = blockIdx.y;
    const double *v = V + (i * nrhs + c) * n, *w = W + c * n;
    __shared__ double red[256];
    double s = 0.0;
    for (long long r = threadIdx.x; r < n; r += 256) s = fma(v[r], w[r], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) hout[c * ldh + i] = red[0];
}

// W(:, c) -= Σ_{i<cnt} h[c·ldh + i]·V_i(:, c)
__global__ void gm_orth_k(long long n, long long nrhs, const double *__restrict__ V, int cnt,
                          const double *__restrict__ h, long long ldh, double *W) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long c = blockIdx.y;
    if (r >= n) return;
    double acc = 0.0;
    for (int i = 0; i < cnt; ++i) acc = fma(h[c * ldh + i], V[((long long)i * nrhs + c) * n + r], acc);
    W[c * n + r] -= acc;
}

// nrm[c·ld] = ||W(:, c)||, then W(:, c) /= nrm (left at zero when nrm is 0)
__global__ __launch_bounds__(256) void gm_norm_scale_k(long long n, double *W, double *nrm, long long ld) {
    const long long c = blockIdx.x;
    double *w = W + c * n;
    __shared__ double red[256];
    double s = 0.0;
    for (long long r = threadIdx.x; r < n; r += 256) s = fma(w[r], w[r], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double nv = sqrt(red[0]);
    if (threadIdx.x == 0) nrm[c * ld] = nv;
    if (nv > 0.0) {
        const double inv = 1.0 / nv;
        for (long long r = threadIdx.x; r < n; r += 256) w[r] *= inv;
    }
}

// start of a sweep: beta = ||M⁻¹r|| per column (from gm_norm_scale_k into hv[c·kGmH])
__global__ void gm_init_k(long long nrhs, GmWork gw) {
    for (long long c = threadIdx.x; c < nrhs; c += blockDim.x) {
        const double b = gw.hv[c * kGmH];
        gw.beta[c] = b;
        gw.g[c * kGmH] = b;
        gw.kk[c] = 0;
        gw.done[c] = !(b > 0.0) || !isfinite(b);
    }
}

// Arnoldi step j of every unfinished column: add the second projection pass,
// apply the earlier rotations to the new Hessenberg column, form the rotation
// that zeroes its subdiagonal, update g; flag[0] = the largest
// |g_{j+1}| / beta of the columns still running (0 when all have finished).
__global__ __launch_bounds__(256) void gm_givens_k(long long nrhs, int j, GmWork gw) {
    __shared__ double red[256];
    double mx = 0.0;
    for (long long c = threadIdx.x; c < nrhs; c += 256) {
        if (gw.done[c]) continue;
        double *h = gw.H + c * kGmH * kGmMax + (long long)j * kGmH;
        const double *h2 = gw.hv + c * kGmH;
        for (int i = 0; i <= j; ++i) h[i] += h2[i];
        h[j + 1] = h2[j + 1];
        double *cs = gw.cs + c * kGmMax, *sn = gw.sn + c * kGmMax, *g = gw.g + c * kGmH;
        for (int i = 0; i < j; ++i) {
            const double t = cs[i] * h[i] + sn[i] * h[i + 1];
            h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
            h[i] = t;
        }
        const double a = h[j], b = h[j + 1];
        const double r = hypot(a, b);
        if (!(r > 0.0) || !isfinite(r)) {   // singular step: the least squares stop before it
            gw.done[c] = 1;
            continue;
        }
        cs[j] = a / r;
        sn[j] = b / r;
        h[j] = r;
        h[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        gw.kk[c] = j + 1;
        const double res = fabs(g[j + 1]) / gw.beta[c];
        if (res <= kGmTol || !(h2[j + 1] > 0.0)) gw.done[c] = 1;
        else if (res > mx || res != res) mx = res;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k && (red[threadIdx.x + k] > red[threadIdx.x] || red[threadIdx.x + k] != red[threadIdx.x + k]))
            red[threadIdx.x] = red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) gw.flag[0] = red[0];
}

// y = R⁻¹·g over each column's kk steps (upper triangular back substitution)
__global__ void gm_backsolve_k(long long nrhs, GmWork gw) {
    for (long long c = threadIdx.x; c < nrhs; c += blockDim.x) {
        const int k = gw.kk[c];
        const double *H = gw.H + c * kGmH * kGmMax, *g = gw.g + c * kGmH;
        double *y = gw.y + c * kGmMax;
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(long long)l * kGmH + i] * y[l];
            y[i] = s / H[(long long)i * kGmH + i];
        }
    }
}

// X(:, c) += Σ_{l<kk} y_l·V_l(:, c)
__global__ void gm_update_k(long long n, long long nrhs, GmWork gw, double *X, long long ldx) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long c = blockIdx.y;
    if (r >= n) return;
    const int k = gw.kk[c];
    const double *y = gw.y + c * kGmMax;
    double acc = 0.0;
    for (int l = 0; l < k; ++l) acc = fma(y[l], gw.V[((long long)l * nrhs + c) * n + r], acc);
    X[r + c * ldx] += acc;
}

static GmWork gmres_work(Ctx &c, long long n, long long nrhs) {
    GmWork gw;
    const size_t per = (size_t)nrhs * (size_t)(kGmH * kGmMax + 2 * kGmH + 3 * kGmMax + 1);
    const size_t dbl = (size_t)kGmH * n * nrhs + per + 1;
    const size_t bytes = dbl * sizeof(double) + 2 * (size_t)nrhs * sizeof(int);
    char *p = (char *)workspace(c, SL_GM, bytes);
    if (!p) return gw;
    double *d = (double *)p;
    gw.V = d; d += (size_t)kGmH * n * nrhs;
    gw.H = d; d += (size_t)nrhs * kGmH * kGmMax;
    gw.hv = d; d += (size_t)nrhs * kGmH;
    gw.g = d; d += (size_t)nrhs * kGmH;
    gw.cs = d; d += (size_t)nrhs * kGmMax;
    gw.sn = d; d += (size_t)nrhs * kGmMax;
    gw.y = d; d += (size_t)nrhs * kGmMax;
    gw.beta = d; d += (size_t)nrhs;
    gw.flag = d; d += 1;
    gw.kk = (int *)d;
    gw.done = gw.kk + nrhs;
    return gw;
}

// W = A·X in FP64 (the residual kernel without b, or the GEMM for many columns)
static void matvec(Ctx &c, long long n, long long nrhs, MixedWork &w, const double *X, long long ldx, double *W) {
    if (nrhs <= kResidMaxRhs) {
        trace_begin(c, PK_RESID);
        const dim3 g((unsigned)((n + 63) / 64));
        for (long long r0 = 0; r0 < nrhs; r0 += 2) {
            if (nrhs - r0 >= 2)
                hipLaunchKernelGGL((resid_k<2, true>), g, dim3(256), 0, c.stream, n, w.Af, w.ldaf, X + r0 * ldx, ldx,
                                   (const double *)nullptr, 0LL, W + r0 * n, n);
            else
                hipLaunchKernelGGL((resid_k<1, true>), g, dim3(256), 0, c.stream, n, w.Af, w.ldaf, X + r0 * ldx, ldx,
                                   (const double *)nullptr, 0LL, W + r0 * n, n);
        }
        RL_CHECK(hipGetLastError());
        trace_end(c, PK_RESID, 2.0 * n * n * nrhs, 8.0 * n * n + 16.0 * n * nrhs);
    } else {
        gemm<double, double, double>(c, Mfma::F64, 'N', 'N', 0, n, nrhs, n, 1.0, w.Af, w.ldaf, X, ldx, 0.0, W, n);
    }
}

// One GMRES-IR sweep: w.R holds r = b − A·x; X += d with d from GMRES on
// M⁻¹A·d = M⁻¹r. Returns the Arnoldi steps taken (at most `budget`);
// *hopeless is set (and X left alone) when, at any step from kGmProbe on, the
// residual's average reduction per step so far would need more than `budget`
// steps to reach kGmTol.
static int gmres_sweep(Ctx &c, bool spd, char uplo, long long n, long long nrhs, MixedWork &w, GmWork &gw,
                       double *X, long long ldx, int budget, bool *hopeless) {
    *hopeless = false;
    const dim3 g2(blocks(n), (unsigned)nrhs);
    const double *cs = spd ? w.s1 : w.s2;
    const long long blk = n * nrhs;
    // V_0 = M⁻¹r / ||M⁻¹r||
    correction(c, spd, uplo, n, nrhs, w);
    hipLaunchKernelGGL(scale_rows_k, g2, dim3(256), 0, c.stream, n, nrhs, cs, (const double *)w.D, n, gw.V, n);
    hipLaunchKernelGGL(gm_norm_scale_k, dim3((unsigned)nrhs), dim3(256), 0, c.stream, n, gw.V, gw.hv, (long long)kGmH);
    hipLaunchKernelGGL(gm_init_k, dim3(1), dim3(256), 0, c.stream, nrhs, gw);
    RL_CHECK(hipGetLastError());
    int steps = 0;
    for (int j = 0; j < kGmMax && steps < budget; ++j) {
        double *Vj = gw.V + (long long)j * blk, *Vn = gw.V + (long long)(j + 1) * blk;
        matvec(c, n, nrhs, w, Vj, n, w.R);
        correction(c, spd, uplo, n, nrhs, w);
        hipLaunchKernelGGL(scale_rows_k, g2, dim3(256), 0, c.stream, n, nrhs, cs, (const double *)w.D, n, Vn, n);
        // classical Gram-Schmidt, twice
        double *Hj = gw.H + (long long)j * kGmH;   // column j of column 0's matrix; stride kGmH·kGmMax per column
        hipLaunchKernelGGL(gm_dot_k, dim3((unsigned)(j + 1), (unsigned)nrhs), dim3(256), 0, c.stream, n, nrhs,
                           (const double *)gw.V, (const double *)Vn, Hj, (long long)kGmH * kGmMax);
        hipLaunchKernelGGL(gm_orth_k, g2, dim3(256), 0, c.stream, n, nrhs, (const double *)gw.V, j + 1,
                           (const double *)Hj, (long long)kGmH * kGmMax, Vn);
        hipLaunchKernelGGL(gm_dot_k, dim3((unsigned)(j + 1), (unsigned)nrhs), dim3(256), 0, c.stream, n, nrhs,
                           (const double *)gw.V, (const double *)Vn, gw.hv, (long long)kGmH);
        hipLaunchKernelGGL(gm_orth_k, g2, dim3(256), 0, c.stream, n, nrhs, (const double *)gw.V, j + 1,
                           (const double *)gw.hv, (long long)kGmH, Vn);
        hipLaunchKernelGGL(gm_norm_scale_k, dim3((unsigned)nrhs), dim3(256), 0, c.stream, n, Vn, gw.hv + (j + 1),
                           (long long)kGmH);
        hipLaunchKernelGGL(gm_givens_k, dim3(1), dim3(256), 0, c.stream, nrhs, j, gw);
        RL_CHECK(hipGetLastError());
        ++steps;
        const double ratio = fetch_scalar(c, gw.flag);
        if (ratio == 0.0) break;   // every column has finished
        if (steps >= kGmProbe) {
            // steps needed at the rate so far: log(kGmTol) / (log(ratio) / steps); checked
            // again after every later step, since a GMRES residual that slows down after a
            // fast start would otherwise spend the whole budget before failing
            const bool slow = !(ratio < 1.0) || std::log(kGmTol) * steps / std::log(ratio) > (double)budget;
            if (slow) { *hopeless = true; return steps; }
        }
    }
    hipLaunchKernelGGL(gm_backsolve_k, dim3(1), dim3(256), 0, c.stream, nrhs, gw);
    hipLaunchKernelGGL(gm_update_k, g2, dim3(256), 0, c.stream, n, nrhs, gw, X, ldx);
    RL_CHECK(hipGetLastError());
    return steps;
}

thread_local MixedStats t_mixed_stats;
MixedStats mixed_last_stats() { return t_mixed_stats; }

// Returns info; *iter and *berr as documented in relapack.h.
int mixed_solve(Ctx &c, bool spd, char uplo, long long n, long long nrhs, const double *A, long long lda,
                int *ipiv_out, const double *B, long long ldb, double *X, long long ldx, int prec, int *iter,
                double *berr) {
    const double tol = 1e-14;
    const int max_sweeps = 30;
    MixedStats &st = t_mixed_stats;
    st = MixedStats();
    MixedWork w;
    w.S = (float *)workspace(c, SL_LP, (size_t)n * n * sizeof(float));
    w.ldaf = spd ? n : lda;
    if (spd) w.Af = (double *)workspace(c, SL_FULL, (size_t)n * n * sizeof(double));
    else w.Af = const_cast<double *>(A);
    const long long nchunk = (n + 255) / 256;
    const size_t vec = (size_t)(2 * n + 2 * n * nrhs + nrhs + 2 + nchunk * n + blocks(n));
    double *v = (double *)workspace(c, SL_VEC, vec * sizeof(double));
    w.ipiv = spd ? nullptr : (ipiv_out ? ipiv_out : (int *)workspace(c, SL_PIV, (size_t)n * sizeof(int)));
    if (!w.S || !w.Af || !v) return -1000 - (int)hipErrorOutOfMemory;
    w.s1 = v; w.s2 = v + n; w.R = v + 2 * n; w.D = w.R + n * nrhs; w.eta = w.D + n * nrhs;
    w.scal = w.eta + nrhs; w.part = w.scal + 2;

    // scaling + conversion, FP64 copy for the residual, ||A||inf
    if (spd) {
        scale_spd_f32(c, uplo, n, A, lda, w.s1, w.S, n);
        const unsigned nt = (unsigned)((n + 63) / 64);
        hipLaunchKernelGGL(symmetrize_k, dim3(nt, nt), dim3(256), 0, c.stream, n, A, lda, w.Af, (int)(uplo == 'L'));
    } else {
        scale_ge_f32(c, n, A, lda, w.s1, w.s2, w.S, n);
    }
    inf_norm(c, n, w.Af, w.ldaf, w);

    // low-precision factorization (status reset: its info is its own)
    const Mfma mode = prec_mode(prec);
    c.abort_on_info = spd;
    if (spd) potrf_rec<float>(c, mode, uplo, n, w.S, n, 0);
    else getrf_top<float>(c, mode, n, n, w.S, n, w.ipiv);
    c.abort_on_info = false;
    if (!spd && c.lu_tracked) {
        // the factorization's row tracker is the gather map itself
        w.perm = c.pv + (size_t)c.pcur * c.pv_m;
    } else if (!spd) {
        w.perm = (int *)workspace(c, SL_PERM, (size_t)n * sizeof(int));
        if (!w.perm) return -1000 - (int)hipErrorOutOfMemory;
        const size_t shm = n <= 16384 ? (size_t)2 * n * sizeof(int) : 0;
        static size_t attr = 0;
        if (shm > attr) {
            RL_CHECK(hipFuncSetAttribute((const void *)ipiv_to_perm_k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)shm));
            attr = shm;
        }
        hipLaunchKernelGGL(ipiv_to_perm_k, dim3(1), dim3(256), (unsigned)shm, c.stream, n, (const int *)w.ipiv,
                           w.perm);
        RL_CHECK(hipGetLastError());
    }
    const int lp_info = fetch_info(c);
    const bool overflow = c.hstat->ovf != 0;   // set by the conversion or a half-precision operand
    int status = 0;  // 0 running, 1 converged, -2 overflow, -3 lp failed, -31 stalled
    double eta = INFINITY;
    int sweeps = 0;
    if (overflow) status = -2;
    else if (lp_info != 0) status = -3;

    if (status == 0) {
        prepare_correction(c, spd, uplo, n, nrhs, w);
        // x0 = A_lp⁻¹·b (as a correction of x = 0, residual r = b)
        hipLaunchKernelGGL(copy_cols_k, dim3(blocks(n), (unsigned)nrhs), dim3(256), 0, c.stream, n, nrhs, B, ldb,
                           w.R, n);
        correction(c, spd, uplo, n, nrhs, w);
        const double *cs = spd ? w.s1 : w.s2;
        hipLaunchKernelGGL(scale_rows_k, dim3(blocks(n), (unsigned)nrhs), dim3(256), 0, c.stream, n, nrhs, cs,
                           w.D, n, X, ldx);
        // plain refinement while each sweep at least halves eta; then GMRES-IR,
        // until eta stops halving (twice) or the Arnoldi budget is spent (at
        // n = 16384 with FP16 factors of a general system, plain sweeps that
        // cut eta about 2.5-fold reach 1e-14 sooner than GMRES-IR does)
        double prev = INFINITY;
        bool use_gmres = false;
        int gm_left = kGmTotal, slow = 0;
        GmWork gw;
        for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
            eta = residual_eta(c, n, nrhs, w, B, ldb, X, ldx);
            if (eta <= tol) { status = 1; break; }
            if (!(eta == eta)) { status = -31; break; }
            if (!use_gmres && sweeps >= 2 && eta > 0.5 * prev) {
                gw = gmres_work(c, n, nrhs);
                if (!gw.V) return -1000 - (int)hipErrorOutOfMemory;
                use_gmres = true;
                st.switched_at = sweeps;
            } else if (use_gmres && eta > 0.5 * prev) {
                if (++slow >= 2) { status = -31; break; }
            }
            if (use_gmres && gm_left <= 0) { status = -31; break; }
            prev = eta;
            if (use_gmres) {
                bool hopeless = false;
                const int k = gmres_sweep(c, spd, uplo, n, nrhs, w, gw, X, ldx, gm_left, &hopeless);
                gm_left -= k;
                st.gmres_steps += k;
                st.gmres_sweeps++;
                if (hopeless) { status = -31; break; }
            } else {
                correction(c, spd, uplo, n, nrhs, w);
                hipLaunchKernelGGL(axpy_rows_k, dim3(blocks(n), (unsigned)nrhs), dim3(256), 0, c.stream, n, nrhs, cs,
                                   w.D, n, X, ldx);
            }
        }
        if (status == 0) status = -31;
    }

    st.sweeps = sweeps;
    st.status = status;
    if (status == 1) {
        *iter = sweeps;
        *berr = eta;
        return 0;
    }
    // FP64 fallback on a copy of A (A itself is never modified)
    double *F = (double *)workspace(c, SL_FB, (size_t)n * n * sizeof(double));
    if (!F) return -1000 - (int)hipErrorOutOfMemory;
    hipLaunchKernelGGL(copy_cols_k, dim3(blocks(n), (unsigned)n), dim3(256), 0, c.stream, n, n, A, lda, F, n);
    hipLaunchKernelGGL(copy_cols_k, dim3(blocks(n), (unsigned)nrhs), dim3(256), 0, c.stream, n, nrhs, B, ldb, X,
                       ldx);
    hipLaunchKernelGGL(reset_info_k, dim3(1), dim3(64), 0, c.stream, c.dstat);
    int info = 0;
    if (spd) {
        c.abort_on_info = true;
        potrf_rec<double>(c, Mfma::F64, uplo, n, F, n, 0);
        c.abort_on_info = false;
        info = fetch_info(c);
        if (info == 0) {
            if (uplo == 'L') {
                trsm<double, double>(c, Mfma::F64, 'L', 'L', 'N', 'N', n, nrhs, F, n, X, ldx);
                trsm<double, double>(c, Mfma::F64, 'L', 'L', 'T', 'N', n, nrhs, F, n, X, ldx);
            } else {
                trsm<double, double>(c, Mfma::F64, 'L', 'U', 'T', 'N', n, nrhs, F, n, X, ldx);
                trsm<double, double>(c, Mfma::F64, 'L', 'U', 'N', 'N', n, nrhs, F, n, X, ldx);
            }
        }
    } else {
        getrf_top<double>(c, Mfma::F64, n, n, F, n, w.ipiv);
        info = fetch_info(c);
        laswp_rows<double>(c, nrhs, X, ldx, w.ipiv, 0, n, false);
        trsm<double, double>(c, Mfma::F64, 'L', 'L', 'N', 'U', n, nrhs, F, n, X, ldx);
        trsm<double, double>(c, Mfma::F64, 'L', 'U', 'N', 'N', n, nrhs, F, n, X, ldx);
    }
    *iter = status;
    *berr = (spd && info != 0) ? INFINITY : residual_eta(c, n, nrhs, w, B, ldb, X, ldx);
    return info;
}

}  // namespace rl
