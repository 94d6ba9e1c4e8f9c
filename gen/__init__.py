"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only *constructs* matrices and right-hand sides. It holds none of
the factorization arithmetic: no Cholesky, no elimination, no triangular
solve. Both the CPU oracle (``oracle/``) and the HIP path
(``paper_1602_06763_amd``) are fed from here, and neither imports the other.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` in a fixed,
documented order and returns column-major (Fortran-order) float64 arrays, the
LAPACK storage that the library's C ABI expects.

Workload recipes (the paper measures on unspecified random square matrices;
these stand in for them):

* ``spd_bbt``       A = B·Bᵀ + n·I, B i.i.d. uniform[-1, 1]   (Cholesky workload)
* ``general_uniform`` A i.i.d. uniform[-1, 1], any m×n           (LU workload)
* ``exact_chol``    A = L·Lᵀ with a small-integer L whose diagonal is a power of
                    two: every Cholesky step is exact in binary64, so L must come
                    back bit-for-bit under any summation order.
* ``exact_lu``      A = Pᵀ·L·U with dyadic |l_ij| ≤ 1/2 and a power-of-two
                    diagonal in U: partial pivoting must pick exactly P and
                    reproduce L and U bit-for-bit.
* ``wilkinson``     the growth matrix (every pivot an exact tie).
* ``diag_dominant`` column diagonally dominant (no row interchange at all).
* ``conditioned``   A = Q·diag(σ)·Qᵀ (SPD) or U·diag(σ)·Vᵀ (general) with a
                    prescribed 2-norm condition number κ, and b = A·x₀.
* ``triangular``    a row-diagonally-dominant triangle (triangular inverse and
                    product inputs); ``unit_bidiagonal`` a triangle with a
                    closed-form inverse.
* ``batch_sizes`` / ``batch_seeds``  the uneven batched workload: sizes
                    uniform in [lo, hi] and one seed per matrix, both from one
                    master seed; matrix i is then ``spd_bbt(n_i, seed_i)`` or
                    ``general_uniform(n_i, n_i, seed_i)``.
"""
from __future__ import annotations

import numpy as np

GEN_VERSION = 1


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _fortran(a: np.ndarray) -> np.ndarray:
    return np.asfortranarray(a, dtype=np.float64)


def spd_bbt(n: int, seed: int = 0) -> np.ndarray:
    """A = B·Bᵀ + n·I with B (n×n) i.i.d. uniform[-1, 1].

    Draw order: one ``uniform(-1, 1, size=(n, n))`` call, read as B in C order.
    The product is mirrored from its lower triangle so that A is exactly
    symmetric. κ₂(A) ≈ 7/3 for large n (Marchenko–Pastur edge 4n/3 over n).
    """
    b = spd_bbt_draws(n, seed)
    a = b @ b.T
    a = np.tril(a) + np.tril(a, -1).T
    a[np.diag_indices(n)] += float(n)
    return _fortran(a)


def spd_bbt_draws(n: int, seed: int = 0) -> np.ndarray:
    """The B of ``spd_bbt(n, seed)``: one ``uniform(-1, 1, size=(n, n))`` call."""
    return rng(seed).uniform(-1.0, 1.0, size=(n, n))


def general_uniform(m: int, n: int | None = None, seed: int = 0) -> np.ndarray:
    """A (m×n) i.i.d. uniform[-1, 1]; one ``uniform`` call of shape (n, m), transposed,
    so that the draws fill A column by column."""
    if n is None:
        n = m
    g = rng(seed)
    return _fortran(g.uniform(-1.0, 1.0, size=(n, m)).T)


def exact_chol_factor(n: int, seed: int = 0) -> np.ndarray:
    """Lower-triangular L: diagonal in {1, 2, 4, 8}, strict lower part integers in [-3, 3].

    Draw order: diagonal exponents (n ints in [0, 3]), then an (n, n) block of
    ints in [-3, 3] of which the strict lower triangle is kept.
    """
    g = rng(seed)
    diag = 2.0 ** g.integers(0, 4, size=n)
    off = g.integers(-3, 4, size=(n, n)).astype(np.float64)
    lo = np.tril(off, -1)
    lo[np.diag_indices(n)] = diag
    return _fortran(lo)


def exact_chol(n: int, seed: int = 0):
    """(A, L) with A = L·Lᵀ formed exactly in binary64.

    Every entry of A and every partial sum of L·Lᵀ is an integer of magnitude
    below 9n + 64, far below 2^53, so the product is exact whatever the
    summation order and A is exactly symmetric.
    """
    lo = exact_chol_factor(n, seed)
    a = lo @ lo.T
    a = np.tril(a) + np.tril(a, -1).T
    return _fortran(a), lo


def exact_lu(m: int, n: int | None = None, seed: int = 0):
    """(A, perm, L, U) with A = Pᵀ·L·U formed exactly in binary64.

    * L (m×k, k = min(m, n)) unit lower trapezoidal, strictly-lower entries drawn
      from {0, ±1/2, ±1/4};
    * U (k×n) upper trapezoidal, entries integers in [-4, 4], diagonal ±{1,2,4,8};
    * ``perm`` is a random permutation of range(m): row i of A is row perm[i] of L·U.

    All values are dyadic with denominator ≤ 4 and magnitude ≤ 8·k + 8, so the
    product and every Schur complement of it are exact in binary64.

    Draw order: perm, then L's (m, k) block, then U's (k, n) block, then U's
    diagonal exponents, then its diagonal signs.
    """
    if n is None:
        n = m
    k = min(m, n)
    g = rng(seed)
    perm = g.permutation(m)
    choices = np.array([0.0, 0.5, -0.5, 0.25, -0.25])
    lo = choices[g.integers(0, len(choices), size=(m, k))]
    lo = np.tril(lo, -1)
    lo[np.arange(k), np.arange(k)] = 1.0
    up = g.integers(-4, 5, size=(k, n)).astype(np.float64)
    up = np.triu(up)
    dexp = g.integers(0, 4, size=k)
    dsgn = np.where(g.integers(0, 2, size=k) == 0, 1.0, -1.0)
    up[np.arange(k), np.arange(k)] = dsgn * 2.0 ** dexp
    lu = lo @ up
    a = np.empty_like(lu)
    a[:, :] = lu[perm, :]
    return _fortran(a), perm, _fortran(lo), _fortran(up)


def exact_lu_pivots(perm: np.ndarray, k: int):
    """(ipiv, rows) that partial pivoting produces on ``exact_lu``'s A.

    At step j the pivot is the current position of the row that holds row j of
    L·U (its multiplier is 1, every other one is ≤ 1/2). ``ipiv`` is the
    1-based LAPACK interchange sequence; ``rows[pos]`` is the row of L·U that
    ends at position pos, so the factor partial pivoting returns is
    ``L[rows]`` (equal to L itself when A is square).

    This replays row interchanges only; it performs no arithmetic on A.
    """
    m = len(perm)
    content = np.array(perm, dtype=np.int64)  # content[pos] = row of L·U at pos
    where = np.empty(m, dtype=np.int64)
    where[content] = np.arange(m)
    ipiv = np.empty(k, dtype=np.int32)
    for j in range(k):
        p = int(where[j])
        ipiv[j] = p + 1
        cj, cp = content[j], content[p]
        content[j], content[p] = cp, cj
        where[cp], where[cj] = j, p
    return ipiv, content


def exact_lu_ipiv(perm: np.ndarray, k: int) -> np.ndarray:
    return exact_lu_pivots(perm, k)[0]


def wilkinson(n: int) -> np.ndarray:
    """1 on the diagonal, -1 strictly below it, 1 in the last column."""
    a = -np.tril(np.ones((n, n)), -1) + np.eye(n)
    a[:, n - 1] = 1.0
    return _fortran(a)


def diag_dominant(n: int, seed: int = 0) -> np.ndarray:
    """Uniform[-1, 1] off the diagonal; a_jj = ±(Σ_i≠j |a_ij| + n), a wide margin of
    column diagonal dominance, under which partial pivoting never swaps."""
    a = general_uniform(n, n, seed).copy(order="F")
    np.fill_diagonal(a, 0.0)
    colsum = np.abs(a).sum(axis=0)
    sgn = np.where(rng(seed + 1).integers(0, 2, size=n) == 0, 1.0, -1.0)
    a[np.diag_indices(n)] = sgn * (colsum + n)
    return _fortran(a)


def triangular(n: int, uplo: str = "L", diag: str = "N", seed: int = 0) -> np.ndarray:
    """A well-conditioned triangle (the input of the triangular inverse and
    product). Strict ``uplo`` part uniform[-1, 1]; diag = 'N': diagonal
    n·(1 + uniform[0, 1]), so every row is diagonally dominant with a margin;
    diag = 'U': the strict part is divided by n and the diagonal is 1. The
    strict other triangle is 0.

    Draw order: an (n, n) block of uniform[-1, 1], then n uniform[0, 1].
    """
    g = rng(seed)
    off = g.uniform(-1.0, 1.0, size=(n, n))
    d = g.uniform(0.0, 1.0, size=n)
    t = np.tril(off, -1) if uplo in ("L", "l") else np.triu(off, 1)
    if diag in ("U", "u"):
        t = t / max(n, 1)
        t[np.diag_indices(n)] = 1.0
    else:
        t[np.diag_indices(n)] = n * (1.0 + d)
    return _fortran(t)


def unit_bidiagonal(n: int, s: float = 1.0) -> np.ndarray:
    """L = I + s·(ones on the first subdiagonal): inv(L)_ij = (-s)^(i-j) for
    i >= j, and A = L·Lᵀ is the tridiagonal matrix with diagonal (1, 1+s², …)
    and off-diagonal s, whose Cholesky factor is L itself."""
    lo = np.eye(n) + s * np.eye(n, k=-1)
    return _fortran(lo)


def tridiag_121(n: int) -> np.ndarray:
    """T = tridiag(-1, 2, -1)."""
    a = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return _fortran(a)


def _haar_orthogonal(g: np.random.Generator, n: int) -> np.ndarray:
    z = g.standard_normal(size=(n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))


def conditioned(n: int, kappa: float, kind: str = "spd", nrhs: int = 1, seed: int = 0):
    """(A, b, x0) with κ₂(A) = kappa and b = A·x0, built on the host.

    σ_i = kappa^(-(i-1)/(n-1)); SPD: A = Q·diag(σ)·Qᵀ (mirrored to exact
    symmetry); general: A = U·diag(σ)·Vᵀ with U and V from two Gaussians drawn in
    that order. Q/U/V are Haar orthogonal (QR of a Gaussian, columns signed by
    diag(R)). Then x0 ~ N(0, 1)^(n×nrhs) and b = A·x0.

    Host QR costs O(n³); the benchmark builds its n = 16384 instances with
    ``conditioned_torch`` instead (same recipe, computed on the device).
    """
    g = rng(seed)
    sig = kappa ** (-np.arange(n) / max(n - 1, 1))
    if kind == "spd":
        q = _haar_orthogonal(g, n)
        a = (q * sig) @ q.T
        a = np.tril(a) + np.tril(a, -1).T
    elif kind == "general":
        u = _haar_orthogonal(g, n)
        v = _haar_orthogonal(g, n)
        a = (u * sig) @ v.T
    else:
        raise ValueError(kind)
    x0 = g.standard_normal(size=(n, nrhs))
    b = a @ x0
    return _fortran(a), _fortran(b), _fortran(x0)


# ---------------------------------------------------------------------------
# Device-side builders for the large benchmark sizes. They use torch only as a
# dense-algebra calculator for *constructing* inputs (B·Bᵀ, QR); the library
# under test is never called here.
# ---------------------------------------------------------------------------

def spd_bbt_torch(n: int, seed: int = 0, device: str = "cuda"):
    """Same recipe as ``spd_bbt`` (B drawn on the host with PCG64, so the draws
    are identical), product formed on the device. Returns a column-major
    (n×n) float64 tensor, i.e. a tensor whose ``.T`` is contiguous."""
    import torch

    g = rng(seed)
    b = torch.from_numpy(g.uniform(-1.0, 1.0, size=(n, n))).to(device)
    a = b @ b.T
    a = torch.tril(a) + torch.tril(a, -1).T
    a.diagonal().add_(float(n))
    del b
    return a.T.contiguous().T  # symmetric, so this is the same matrix stored column-major


def general_uniform_torch(m: int, n: int | None = None, seed: int = 0, device: str = "cuda"):
    """Same draws as ``general_uniform``, placed on the device column-major."""
    import torch

    a = general_uniform(m, n, seed)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device).T


def conditioned_torch(n: int, kappa: float, kind: str = "spd", nrhs: int = 1, seed: int = 0,
                      device: str = "cuda"):
    """``conditioned``'s recipe with the Gaussians drawn on the host (PCG64) and the
    QR and products done on the device in float64. Returns column-major tensors
    (A, b, x0)."""
    import torch

    g = rng(seed)

    def haar():
        z = torch.from_numpy(g.standard_normal(size=(n, n))).to(device)
        q, r = torch.linalg.qr(z)
        return q * torch.sign(torch.diagonal(r))

    sig = torch.from_numpy(kappa ** (-np.arange(n) / max(n - 1, 1))).to(device)
    if kind == "spd":
        q = haar()
        a = (q * sig) @ q.T.contiguous()
        a = torch.tril(a) + torch.tril(a, -1).T
    elif kind == "general":
        u = haar()
        v = haar()
        a = (u * sig) @ v.T.contiguous()
    else:
        raise ValueError(kind)
    x0 = torch.from_numpy(g.standard_normal(size=(n, nrhs))).to(device)
    b = a @ x0
    colmajor = lambda t: t.T.contiguous().T
    return colmajor(a), colmajor(b), colmajor(x0)


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Sizes of a batch: ``count`` integers uniform in [lo, hi] (one
    ``integers`` call of the master generator)."""
    return rng(seed).integers(lo, hi + 1, size=count).astype(np.int64)


def batch_seeds(count: int, seed: int) -> np.ndarray:
    """Per-matrix seeds of a batch: ``count`` 62-bit integers from the
    generator of ``seed + 1`` (the sizes use ``seed`` itself)."""
    return rng(seed + 1).integers(0, 2**62, size=count, dtype=np.int64)


# -- complex inputs (the c/z instances) ------------------------------------------

def hpd_bbh(n: int, seed: int = 0) -> np.ndarray:
    """Hermitian positive definite A = B·Bᴴ + n·I, B with real and imaginary
    parts i.i.d. uniform[-1, 1] (one ``uniform`` call of shape (2, n, n): real
    parts, then imaginary parts). Lower triangle mirrored (conjugated) so that
    A is exactly Hermitian with a real diagonal."""
    g = rng(seed)
    d = g.uniform(-1.0, 1.0, size=(2, n, n))
    b = d[0] + 1j * d[1]
    a = b @ b.conj().T
    a = np.tril(a) + np.tril(a, -1).conj().T
    a[np.diag_indices(n)] = a[np.diag_indices(n)].real + float(n)
    return np.asfortranarray(a, dtype=np.complex128)


def general_complex(m: int, n: int | None = None, seed: int = 0) -> np.ndarray:
    """A (m×n) with real and imaginary parts i.i.d. uniform[-1, 1] (one
    ``uniform`` call of shape (2, n, m), transposed)."""
    if n is None:
        n = m
    d = rng(seed).uniform(-1.0, 1.0, size=(2, n, m))
    return np.asfortranarray((d[0] + 1j * d[1]).T, dtype=np.complex128)


def exact_zchol(n: int, seed: int = 0):
    """A = L·Lᴴ with L lower triangular, a real diagonal in {1, 2, 4, 8} and
    Gaussian integers with parts in [-3, 3] below it: every step of the
    Cholesky is exact in binary64, so L comes back bit for bit. Returns (A, L)."""
    g = rng(seed)
    lo = np.tril(g.integers(-3, 4, size=(n, n)) + 1j * g.integers(-3, 4, size=(n, n)), -1)
    lo[np.diag_indices(n)] = 2.0 ** g.integers(0, 4, size=n)
    a = lo @ lo.conj().T
    return np.asfortranarray(a, dtype=np.complex128), np.asfortranarray(lo, dtype=np.complex128)


_ZL_VALUES = np.array([0, 0.5, -0.5, 0.25, -0.25, 0.5j, -0.5j, 0.25j, -0.25j,
                       0.25 + 0.25j, 0.25 - 0.25j, -0.25 + 0.25j, -0.25 - 0.25j])


def exact_zlu(n: int, seed: int = 0):
    """A = Pᵀ·L·U with a random permutation P, L unit lower with dyadic
    Gaussian entries (|re| + |im| <= 1/2) and U upper with Gaussian integers
    in [-4, 4] and a real diagonal in ±{1, 2, 4, 8}: partial pivoting by
    |re| + |im| picks exactly P and every step is exact. Returns
    (A, perm, L, U) with row i of A = row perm[i] of L·U, as ``exact_lu``, so
    ``exact_lu_pivots`` gives the expected ipiv and row order. Draw order:
    perm, L's entries, U's upper entries (real, then imaginary parts), U's
    diagonal signs, then its exponents."""
    g = rng(seed)
    perm = g.permutation(n)
    lo = np.tril(_ZL_VALUES[g.integers(0, len(_ZL_VALUES), size=(n, n))], -1) + np.eye(n)
    up = np.triu(g.integers(-4, 5, size=(n, n)) + 1j * g.integers(-4, 5, size=(n, n)), 1)
    up = up + np.diag(g.choice([-1, 1], size=n) * 2.0 ** g.integers(0, 4, size=n))
    lu = lo @ up
    a = lu[perm, :]
    return (np.asfortranarray(a, dtype=np.complex128), perm, np.asfortranarray(lo, dtype=np.complex128),
            np.asfortranarray(up, dtype=np.complex128))


def hpd_bbh_torch(n: int, seed: int = 0, device: str = "cuda"):
    """The draws of ``hpd_bbh`` with A = B·Bᴴ + n·I formed on the device (the
    product rounds differently from numpy's), lower triangle mirrored,
    diagonal real; column-major complex128."""
    import torch

    d = rng(seed).uniform(-1.0, 1.0, size=(2, n, n))
    b = torch.complex(torch.from_numpy(d[0]), torch.from_numpy(d[1])).to(device)
    a = b @ b.conj().T.contiguous()
    a = torch.tril(a) + torch.tril(a, -1).conj().T
    a.diagonal().copy_(a.diagonal().real + float(n))
    return a.T.contiguous().T


def general_complex_torch(m: int, n: int | None = None, seed: int = 0, device: str = "cuda"):
    """Same draws as ``general_complex``, placed on the device column-major."""
    import torch

    a = general_complex(m, n, seed)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device).T
