"""CPU oracle for the recursive factorizations -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``oracle.c`` (plain unblocked
FP64 Cholesky and partial-pivoting LU, their solves, the mixed-precision
scaling and the FP64 backward error) through ctypes and shares no code with
the HIP library.

Parity status of each function (what pins it is in ``tests/test_oracle_pins.py``):

* ``potrf``            pinned: exact integer factors, brute-force rationals
                       (n <= 7), tridiag(-1, 2, -1) closed form, special cases,
                       residual bound, upper/lower transposition.
* ``getrf``            pinned: exact dyadic P·L·U, brute-force rationals
                       (n <= 6), Wilkinson ties, diagonal dominance,
                       permutation matrices, residual bound, zero pivots.
* ``getrf_margin``     pinned: the same factorization as ``getrf`` bit for bit,
                       Wilkinson ties (lead 0), the exact dyadic construction
                       (lead >= 1/2), a hand-checked 3×3 column.
* ``potrs``/``getrs``  pinned: exact solutions on the exact constructions,
                       residual bound on random inputs.
* ``scale_spd_f32``/``scale_ge_f32`` pinned: powers of two, scaled ranges,
                       exactness of the binary64 scaling, RNE rounding.
* ``backward_error``   pinned: exact solutions give 0, hand-checked 2×2 case,
                       scaling invariance.
* ``trtri``            pinned: closed-form inverse of integer bidiagonal
                       triangles (exact), exact rational inverses by brute
                       force (n <= 6), reciprocals of a diagonal, unit
                       diagonal never read, zero pivot reported before any
                       write, residual bound, upper/lower transposition.
* ``lauum``            pinned: exact integer products against integer matrix
                       multiplication, identity, strict other triangle untouched.
* ``potri``            pinned: exact integer inverse of A = L·Lᵀ with unit
                       bidiagonal L, residual bound ‖A·X − I‖.
* ``zpotrf``           pinned: exact Gaussian-integer factors with a
                       power-of-two diagonal, a hand-checked 2×2 closed form,
                       real symmetric inputs (equal to ``potrf`` bit for bit),
                       upper = conjugate transpose of lower, failure index,
                       residual bound.
* ``zgetrf``           pinned: exact dyadic Gaussian P·L·U, a hand-checked
                       column where |re| + |im| and |z| pick different rows,
                       real inputs (same pivots as ``getrf``), zero pivots,
                       residual bound and every multiplier's modulus <= √2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
             "-std=c11", "-Wall"]


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int)
        c_int, c_char, c_double = ctypes.c_int, ctypes.c_char, ctypes.c_double
        L.oracle_dpotrf.argtypes = [c_char, c_int, dp, c_int]
        L.oracle_dpotrf.restype = c_int
        L.oracle_dgetrf.argtypes = [c_int, c_int, dp, c_int, ip]
        L.oracle_dgetrf.restype = c_int
        L.oracle_dgetrf_margin.argtypes = [c_int, c_int, dp, c_int, ip, dp]
        L.oracle_dgetrf_margin.restype = c_int
        L.oracle_dpotrs.argtypes = [c_char, c_int, c_int, dp, c_int, dp, c_int]
        L.oracle_dpotrs.restype = None
        L.oracle_dgetrs.argtypes = [c_char, c_int, c_int, dp, c_int, ip, dp, c_int]
        L.oracle_dgetrs.restype = None
        L.oracle_scale_spd_f32.argtypes = [c_char, c_int, dp, c_int, dp, fp, c_int]
        L.oracle_scale_spd_f32.restype = None
        L.oracle_scale_ge_f32.argtypes = [c_int, dp, c_int, dp, dp, fp, c_int]
        L.oracle_scale_ge_f32.restype = None
        L.oracle_backward_error.argtypes = [c_char, c_int, c_int, dp, c_int, dp, c_int, dp, c_int, dp]
        L.oracle_backward_error.restype = c_double
        L.oracle_dtrtri.argtypes = [c_char, c_char, c_int, dp, c_int]
        L.oracle_dtrtri.restype = c_int
        L.oracle_dlauum.argtypes = [c_char, c_int, dp, c_int]
        L.oracle_dlauum.restype = None
        L.oracle_set_threads.argtypes = [c_int]
        L.oracle_set_threads.restype = None
        L.oracle_zpotrf.argtypes = [c_char, c_int, dp, c_int]
        L.oracle_zpotrf.restype = c_int
        L.oracle_zgetrf.argtypes = [c_int, c_int, dp, c_int, ip]
        L.oracle_zgetrf.restype = c_int
        L.oracle_get_threads.argtypes = []
        L.oracle_get_threads.restype = c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    a = np.array(a, dtype=np.float64, order="F", copy=True)
    return a


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def potrf(a, uplo: str = "L"):
    """Cholesky of a copy of ``a``; returns (factored array, info)."""
    a = _f64(a)
    n = a.shape[0]
    info = lib().oracle_dpotrf(uplo.encode(), n, _dp(a), max(n, 1))
    return a, int(info)


def getrf(a):
    """Partial-pivoting LU of a copy of ``a`` (m×n); returns (LU array, ipiv (1-based), info)."""
    a = _f64(a)
    m, n = a.shape
    ipiv = np.zeros(max(min(m, n), 1), dtype=np.int32)
    info = lib().oracle_dgetrf(m, n, _dp(a), max(m, 1), _ip(ipiv))
    return a, ipiv[: min(m, n)], int(info)


def _c128(a):
    return np.array(a, dtype=np.complex128, order="F", copy=True)


def zpotrf(a, uplo: str = "L"):
    """Cholesky of a copy of the Hermitian ``a`` (complex, A = L·Lᴴ or Uᴴ·U);
    returns (factored array, info)."""
    a = _c128(a)
    n = a.shape[0]
    info = lib().oracle_zpotrf(uplo.encode(), n, _dp(a), max(n, 1))
    return a, int(info)


def zgetrf(a):
    """Partial-pivoting LU of a copy of the complex ``a`` (m×n), pivots by
    |re| + |im|; returns (LU array, ipiv (1-based), info)."""
    a = _c128(a)
    m, n = a.shape
    ipiv = np.zeros(max(min(m, n), 1), dtype=np.int32)
    info = lib().oracle_zgetrf(m, n, _dp(a), max(m, 1), _ip(ipiv))
    return a, ipiv[: min(m, n)], int(info)


def getrf_margin(a):
    """As ``getrf``, also returning each step's pivot lead over the runner-up,
    (|a_pk| - max_{i != p} |a_ik|) / |a_pk|: (LU, ipiv, info, margin)."""
    a = _f64(a)
    m, n = a.shape
    k = max(min(m, n), 1)
    ipiv = np.zeros(k, dtype=np.int32)
    margin = np.zeros(k)
    info = lib().oracle_dgetrf_margin(m, n, _dp(a), max(m, 1), _ip(ipiv), _dp(margin))
    return a, ipiv[: min(m, n)], int(info), margin[: min(m, n)]


def potrs(fac, b, uplo: str = "L"):
    fac = _f64(fac)
    b = _f64(b)
    if b.ndim == 1:
        b = b.reshape(-1, 1, order="F")
    n, nrhs = b.shape
    lib().oracle_dpotrs(uplo.encode(), n, nrhs, _dp(fac), max(n, 1), _dp(b), max(n, 1))
    return b


def getrs(lu, ipiv, b, trans: str = "N"):
    lu = _f64(lu)
    b = _f64(b)
    if b.ndim == 1:
        b = b.reshape(-1, 1, order="F")
    n, nrhs = b.shape
    ip = np.ascontiguousarray(ipiv, dtype=np.int32)
    lib().oracle_dgetrs(trans.encode(), n, nrhs, _dp(lu), max(n, 1), _ip(ip), _dp(b), max(n, 1))
    return b


def trtri(a, uplo: str = "L", diag: str = "N"):
    """Inverse of the ``uplo`` triangle of a copy of ``a`` in place; returns (array, info)."""
    a = _f64(a)
    n = a.shape[0]
    info = lib().oracle_dtrtri(uplo.encode(), diag.encode(), n, _dp(a), max(n, 1))
    return a, int(info)


def lauum(a, uplo: str = "L"):
    """Lᵀ·L (uplo 'L') or U·Uᵀ (uplo 'U') of the triangle of a copy of ``a``, in that triangle."""
    a = _f64(a)
    n = a.shape[0]
    lib().oracle_dlauum(uplo.encode(), n, _dp(a), max(n, 1))
    return a


def potri(a, uplo: str = "L"):
    """Inverse of an SPD matrix through its Cholesky factor: potrf, then trtri
    of the factor, then lauum (the LAPACK composition xpotri, which the paper
    names as the user of xtrtri and xlauum in Sec. 5). Returns (array, info);
    only the ``uplo`` triangle of the result is meaningful."""
    f, info = potrf(a, uplo)
    if info:
        return f, info
    f, info = trtri(f, uplo, "N")
    if info:
        return f, info
    return lauum(f, uplo), 0


def scale_spd_f32(a, uplo: str = "L"):
    """(d, S32): S = D·A·D rounded to float32 in the ``uplo`` triangle (other triangle 0)."""
    a = _f64(a)
    n = a.shape[0]
    d = np.zeros(n)
    s = np.zeros((n, n), dtype=np.float32, order="F")
    lib().oracle_scale_spd_f32(uplo.encode(), n, _dp(a), max(n, 1), _dp(d), _fp(s), max(n, 1))
    return d, s


def scale_ge_f32(a):
    """(r, c, S32): S = R·A·C rounded to float32."""
    a = _f64(a)
    n = a.shape[0]
    r = np.zeros(n)
    c = np.zeros(n)
    s = np.zeros((n, n), dtype=np.float32, order="F")
    lib().oracle_scale_ge_f32(n, _dp(a), max(n, 1), _dp(r), _dp(c), _fp(s), max(n, 1))
    return r, c, s


def backward_error(a, x, b, sym: str = "N"):
    """(max_j eta_j, eta per column), eta_j = ||b_j - A x_j||_inf / (||A||_inf ||x_j||_inf + ||b_j||_inf)."""
    a = _f64(a)
    x = _f64(x)
    b = _f64(b)
    if x.ndim == 1:
        x = x.reshape(-1, 1, order="F")
    if b.ndim == 1:
        b = b.reshape(-1, 1, order="F")
    n, nrhs = x.shape
    eta = np.zeros(nrhs)
    worst = lib().oracle_backward_error(sym.encode(), n, nrhs, _dp(a), max(n, 1), _dp(x), max(n, 1),
                                        _dp(b), max(n, 1), _dp(eta))
    return float(worst), eta


# -- helpers that unpack LAPACK-format results (no arithmetic of the method) --

def unpack_lu(lu, k=None):
    """(L, U) from a packed m×n LU array: L unit lower m×k, U upper k×n, k = min(m, n)."""
    m, n = lu.shape
    k = min(m, n) if k is None else k
    lo = np.tril(lu[:, :k], -1)
    lo[np.arange(k), np.arange(k)] = 1.0
    up = np.triu(lu[:k, :])
    return lo, up


def apply_ipiv(a, ipiv):
    """P·A: the rows of ``a`` after the interchanges ipiv (1-based) in order."""
    a = np.array(a, copy=True)
    for k, p in enumerate(np.asarray(ipiv) - 1):
        if p != k:
            a[[k, p], :] = a[[p, k], :]
    return a
