"""Exact-rational brute force for tiny matrices, used to pin the CPU oracle.

Nothing here eliminates: every quantity is a ratio of minors (determinants by
cofactor expansion), the closed forms of the Cholesky and LU factors in terms
of leading minors. Binary64 inputs convert to ``Fraction`` exactly; square
roots are taken in 60-digit decimal arithmetic and rounded once to binary64.
"""
from __future__ import annotations

import decimal
from fractions import Fraction
from functools import lru_cache

import numpy as np

_CTX = decimal.Context(prec=60)


def to_fractions(a) -> list[list[Fraction]]:
    a = np.asarray(a, dtype=np.float64)
    return [[Fraction(float(v)) for v in row] for row in a]


def det(F, rows, cols) -> Fraction:
    """det F[rows, cols] by cofactor (Laplace) expansion along the rows in order."""
    rows = tuple(rows)
    cols = tuple(cols)
    k = len(rows)
    assert k == len(cols)

    @lru_cache(maxsize=None)
    def f(r, mask):
        if r == k:
            return Fraction(1)
        total = Fraction(0)
        pos = 0
        for ci in range(k):
            if mask >> ci & 1:
                continue
            v = F[rows[r]][cols[ci]]
            if v != 0:
                term = v * f(r + 1, mask | (1 << ci))
                total += term if pos % 2 == 0 else -term
            pos += 1
        return total

    return f(0, 0)


def _dec(fr: Fraction) -> decimal.Decimal:
    return _CTX.divide(decimal.Decimal(fr.numerator), decimal.Decimal(fr.denominator))


def cholesky_lower(a) -> np.ndarray:
    """L of A = L·Lᵀ from leading minors D_j:
    l_jj = sqrt(D_j / D_{j-1}),  l_ij = det A[{0..j-1, i}, {0..j}] / sqrt(D_j·D_{j-1})."""
    F = to_fractions(a)
    n = len(F)
    D = [Fraction(1)] + [det(F, range(j), range(j)) for j in range(1, n + 1)]
    L = np.zeros((n, n))
    for j in range(n):
        dj, dj1 = D[j + 1], D[j]
        assert dj > 0, "not positive definite"
        root = _CTX.sqrt(_dec(dj * dj1))
        L[j, j] = float(_CTX.sqrt(_dec(dj / dj1)))
        for i in range(j + 1, n):
            num = det(F, list(range(j)) + [i], range(j + 1))
            L[i, j] = float(_CTX.divide(_dec(num), root))
    return L


def lu_partial_pivoting(a, min_gap: float = 1e-6):
    """(ipiv 1-based, L, U) of partial-pivoting LU from minors, or None when two
    pivot candidates are within a relative ``min_gap`` (a near-tie whose winner
    rounding may legitimately flip).

    With R the ordered pivot rows chosen so far, the Schur complement entry of
    row i in column k is det A[R+[i], 0..k] / det A[R, 0..k-1]; the pivot is its
    largest magnitude; u_kj = det A[R_k, {0..k-1, j}] / det A[R_{k-1}, 0..k-1].
    """
    F = to_fractions(a)
    m, n = len(F), len(F[0])
    kk = min(m, n)
    R: list[int] = []
    pos = list(range(m))  # pos[row] = current position of original row
    at = list(range(m))  # at[position] = original row there
    ipiv = np.zeros(kk, dtype=np.int32)
    U = np.zeros((kk, n))
    Lf: dict[tuple[int, int], Fraction] = {}
    prev = Fraction(1)
    for k in range(kk):
        cand = [i for i in range(m) if i not in R]
        s = {i: det(F, R + [i], range(k + 1)) / prev for i in cand}
        mags = sorted((abs(v) for v in s.values()), reverse=True)
        if len(mags) > 1 and mags[0] != 0 and (mags[0] - mags[1]) <= Fraction(min_gap) * mags[0]:
            return None
        best = max(abs(v) for v in s.values())
        if best == 0:
            return None  # singular leading block: not a brute-force case
        p = min((i for i in cand if abs(s[i]) == best), key=lambda i: pos[i])
        ipiv[k] = pos[p] + 1
        # the row interchange of step k, tracked on positions only
        rk, pk = at[k], p
        at[k], at[pos[p]] = p, rk
        pos[rk], pos[pk] = pos[pk], k
        for i in cand:
            if i != p:
                Lf[(i, k)] = s[i] / s[p]
        R.append(p)
        cur = det(F, R, range(k + 1))
        for j in range(k, n):
            U[k, j] = float(det(F, R, list(range(k)) + [j]) / prev)
        prev = cur
    L = np.zeros((m, kk))
    for k in range(kk):
        L[k, k] = 1.0
    for (i, k), v in Lf.items():
        L[pos[i], k] = float(v)
    return ipiv, L, U


def inverse(a) -> list[list[Fraction]]:
    """A⁻¹ by the adjugate: (A⁻¹)_ij = (-1)^(i+j)·det(A without row j and
    column i) / det(A), every determinant by cofactor expansion."""
    F = to_fractions(a)
    n = len(F)
    full = tuple(range(n))
    d = det(F, full, full)
    out = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            rows = tuple(r for r in full if r != j)
            cols = tuple(c for c in full if c != i)
            minor = det(F, rows, cols) if n > 1 else Fraction(1)
            out[i][j] = (-1) ** (i + j) * minor / d
    return out
