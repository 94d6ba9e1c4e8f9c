"""Python binding of librelapack_mi355x.so (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/relapack.h``
with the same name minus the ``relapack_`` prefix. Matrices are passed as
device pointers: either raw integers or torch CUDA tensors (their
``data_ptr()``), column-major, i.e. a tensor ``t`` whose ``t.T`` is
contiguous (``t.stride() == (1, ld)``). Nothing here computes: there is no
CPU fallback, and loading fails loudly if the library has not been built.

Tensor arguments are checked before anything reaches the library: each must
be a CUDA tensor of the routine's dtype (float64 for the ``d`` routines,
float32 for the ``s`` ones, int32 pivots and per-matrix sizes, int64 arrays
of addresses) whose storage covers the column-major extent the call will
touch, ``ld·(cols − 1) + rows`` elements from its start; a ValueError is
raised otherwise. Raw integer addresses are passed through unchecked.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librelapack_mi355x.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "relapack.h")

_lib = None

_c_int, _c_char, _c_double, _c_ll = ctypes.c_int, ctypes.c_char, ctypes.c_double, ctypes.c_longlong
_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)
_llp = ctypes.POINTER(ctypes.c_longlong)

_SIGS = {
    "relapack_version": ([], _c_int),
    "relapack_set_stream": ([_vp], _c_int),
    "relapack_get_stream": ([], _vp),
    "relapack_finalize": ([], None),
    "relapack_dpotrf": ([_c_char, _c_int, _vp, _c_int, _ip], None),
    "relapack_dgetrf": ([_c_int, _c_int, _vp, _c_int, _vp, _ip], None),
    "relapack_dgetrf_noalloc": ([_c_int, _c_int, _vp, _c_int, _vp, _ip], None),
    "relapack_zpotrf": ([_c_char, _c_int, _vp, _c_int, _ip], None),
    "relapack_cpotrf": ([_c_char, _c_int, _vp, _c_int, _ip], None),
    "relapack_zgetrf": ([_c_int, _c_int, _vp, _c_int, _vp, _ip], None),
    "relapack_cgetrf": ([_c_int, _c_int, _vp, _c_int, _vp, _ip], None),
    "relapack_zgemm": ([_c_char, _c_char, _c_int, _c_int, _c_int, _c_double, _vp, _c_int, _vp, _c_int,
                        _c_double, _vp, _c_int, _ip], None),
    "relapack_dpotrs": ([_c_char, _c_int, _c_int, _vp, _c_int, _vp, _c_int, _ip], None),
    "relapack_dgetrs": ([_c_char, _c_int, _c_int, _vp, _c_int, _vp, _vp, _c_int, _ip], None),
    "relapack_dposv_mixed": ([_c_char, _c_int, _c_int, _vp, _c_int, _vp, _c_int, _vp, _c_int, _c_int,
                              _ip, _dp, _ip], None),
    "relapack_dgesv_mixed": ([_c_int, _c_int, _vp, _c_int, _vp, _vp, _c_int, _vp, _c_int, _c_int, _ip,
                              _dp, _ip], None),
    "relapack_mixed_last": ([_ip, _ip, _ip, _ip], None),
    "relapack_dgemm": ([_c_char, _c_char, _c_int, _c_int, _c_int, _c_double, _vp, _c_int, _vp, _c_int,
                        _c_double, _vp, _c_int, _ip], None),
    "relapack_dsyrk": ([_c_char, _c_char, _c_int, _c_int, _c_double, _vp, _c_int, _c_double, _vp, _c_int,
                        _ip], None),
    "relapack_dtrsm": ([_c_char, _c_char, _c_char, _c_char, _c_int, _c_int, _vp, _c_int, _vp, _c_int, _ip],
                       None),
    "relapack_dtrmm": ([_c_char, _c_char, _c_char, _c_char, _c_int, _c_int, _c_double, _vp, _c_int, _vp,
                        _c_int, _ip], None),
    "relapack_dtrtri": ([_c_char, _c_char, _c_int, _vp, _c_int, _ip], None),
    "relapack_dlauum": ([_c_char, _c_int, _vp, _c_int, _ip], None),
    "relapack_dpotri": ([_c_char, _c_int, _vp, _c_int, _ip], None),
    "relapack_scale_spd_f32": ([_c_char, _c_int, _vp, _c_int, _vp, _vp, _c_int, _ip], None),
    "relapack_scale_ge_f32": ([_c_int, _vp, _c_int, _vp, _vp, _vp, _c_int, _ip], None),
    "relapack_spotrf_lp": ([_c_char, _c_int, _vp, _c_int, _c_int, _ip], None),
    "relapack_spotrf": ([_c_char, _c_int, _vp, _c_int, _ip], None),
    "relapack_sgetrf": ([_c_int, _c_int, _vp, _c_int, _vp, _ip], None),
    "relapack_sgetrf_lp": ([_c_int, _c_int, _vp, _c_int, _vp, _c_int, _ip], None),
    "relapack_dpotrf_batched": ([_c_char, _c_int, _vp, _vp, _vp, _vp], _c_int),
    "relapack_spotrf_batched": ([_c_char, _c_int, _vp, _vp, _vp, _vp], _c_int),
    "relapack_dgetrf_batched": ([_c_int, _vp, _vp, _vp, _vp, _vp], _c_int),
    "relapack_sgetrf_batched": ([_c_int, _vp, _vp, _vp, _vp, _vp], _c_int),
    "relapack_batched_tune": ([_c_int, _c_int, _c_int, _c_int], _c_int),
    "relapack_batched_tune_get": ([_c_int, _c_int, _ip, _ip], _c_int),
    "relapack_batched_graphs": ([_c_int], None),
    "relapack_lookahead": ([_c_int], None),
    "relapack_trace_enable": ([_c_int], None),
    "relapack_trace_collect": ([_dp, _c_int], _c_int),
    "relapack_plan": ([ctypes.c_char_p, _c_ll, _c_ll, _c_int, _llp, _c_ll], _c_ll),
    "relapack_split": ([_c_ll], _c_ll),
}

TRACE_FAMILIES = {1: "potf2", 2: "trsm_leaf", 3: "gemm", 4: "syrk", 5: "getf2_panel", 6: "laswp",
                  7: "convert", 8: "residual", 10: "gemm_lowprec", 11: "syrk_lowprec", 12: "gemm128",
                  13: "trti2", 14: "trmm_leaf", 15: "lauu2", 16: "zgemm", 17: "complex_leaf", 18: "trmm"}

PREC = {"fp32": 32, "32": 32, 32: 32, "fp16": 16, "16": 16, 16: 16, "bf16": ord("b"), "b": ord("b")}


class LibraryNotBuilt(RuntimeError):
    pass


def lib() -> ctypes.CDLL:
    """Load the built library (never builds, never falls back)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryNotBuilt(
                f"{LIB_PATH} is missing: run `python -c 'import __graft_entry__ as g; g.build()'` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


_F64, _F32, _I32, _I64 = "float64", "float32", "int32", "int64"
_C128, _C64 = "complex128", "complex64"


def _check(t, dtype: str, rows: int, cols: int, ld: int | None = None, what: str = "matrix") -> None:
    """Refuse a tensor the kernels would read or write out of bounds: it must
    be a CUDA tensor of ``dtype`` whose storage holds a column-major rows×cols
    array with leading dimension ``ld`` starting at its data pointer. Raw
    integer addresses and illegal sizes (which the library itself rejects
    through info) pass unchecked."""
    if t is None or isinstance(t, int):
        return
    if rows <= 0 or cols <= 0:
        return
    ld = rows if ld is None else ld
    if ld < rows:
        return   # the library reports the illegal leading dimension
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a CUDA tensor, got one on {t.device}")
    if str(t.dtype).replace("torch.", "") != dtype:
        raise ValueError(f"{what}: expected dtype {dtype}, got {t.dtype}")
    item = t.element_size()
    start = t.storage_offset()
    need = start + (cols - 1) * ld + rows
    have = t.untyped_storage().nbytes() // item
    if need > have:
        raise ValueError(f"{what}: a {rows}x{cols} array with leading dimension {ld} needs {need} "
                         f"elements of storage from the tensor's start, it has {have}")


def _check_vec(t, dtype: str, count: int, what: str) -> None:
    """A CUDA vector of ``dtype`` with at least ``count`` elements of storage."""
    _check(t, dtype, count, 1, count, what)


def _ld(t, rows):
    """Leading dimension of a column-major tensor (stride(0) == 1)."""
    if isinstance(t, int):
        return rows
    if t.dim() == 1:
        return max(rows, 1)
    if t.stride(0) != 1 and t.shape[0] > 1:
        raise ValueError("matrix must be column-major: use t.T.contiguous().T")
    return max(int(t.stride(1)), 1) if t.shape[1] > 1 else max(rows, 1)


def _b(ch: str) -> bytes:
    return ch.encode() if isinstance(ch, str) else bytes([ch])


def _cur_stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def set_stream(stream=None) -> int:
    """Set the library stream; default: torch's current stream."""
    if stream is None:
        s = _cur_stream()
    elif isinstance(stream, int):
        s = ctypes.c_void_p(stream)
    else:
        s = ctypes.c_void_p(stream.cuda_stream)
    return lib().relapack_set_stream(s)


def version() -> int:
    return lib().relapack_version()


def finalize() -> None:
    lib().relapack_finalize()


def potrf(A, uplo: str = "L", n: int | None = None, lda: int | None = None) -> int:
    n = A.shape[0] if n is None else n
    lda = _ld(A, n) if lda is None else lda
    _check(A, _F64, n, n, lda, "A")
    info = ctypes.c_int(0)
    lib().relapack_dpotrf(_b(uplo), n, _ptr(A), lda, ctypes.byref(info))
    return info.value


def getrf(A, ipiv, m: int | None = None, n: int | None = None, lda: int | None = None) -> int:
    m = A.shape[0] if m is None else m
    n = A.shape[1] if n is None else n
    lda = _ld(A, m) if lda is None else lda
    _check(A, _F64, m, n, lda, "A")
    _check_vec(ipiv, _I32, min(m, n), "ipiv")
    info = ctypes.c_int(0)
    lib().relapack_dgetrf(m, n, _ptr(A), lda, _ptr(ipiv), ctypes.byref(info))
    return info.value


def getrf_noalloc(A, ipiv, m: int | None = None, n: int | None = None, lda: int | None = None) -> int:
    """relapack_dgetrf_noalloc: the LU on the library's fixed workspace (m <= 32768)."""
    m = A.shape[0] if m is None else m
    n = A.shape[1] if n is None else n
    lda = _ld(A, m) if lda is None else lda
    _check(A, _F64, m, n, lda, "A")
    _check_vec(ipiv, _I32, min(m, n), "ipiv")
    info = ctypes.c_int(0)
    lib().relapack_dgetrf_noalloc(m, n, _ptr(A), lda, _ptr(ipiv), ctypes.byref(info))
    return info.value


def zpotrf(A, uplo: str = "L", n: int | None = None, lda: int | None = None) -> int:
    """relapack_zpotrf (complex128 tensor) or relapack_cpotrf (complex64)."""
    n = A.shape[0] if n is None else n
    lda = _ld(A, n) if lda is None else lda
    single = not isinstance(A, int) and str(A.dtype) == "torch.complex64"
    _check(A, _C64 if single else _C128, n, n, lda, "A")
    info = ctypes.c_int(0)
    f = lib().relapack_cpotrf if single else lib().relapack_zpotrf
    f(_b(uplo), n, _ptr(A), lda, ctypes.byref(info))
    return info.value


def zgetrf(A, ipiv, m: int | None = None, n: int | None = None, lda: int | None = None) -> int:
    """relapack_zgetrf (complex128 tensor) or relapack_cgetrf (complex64)."""
    m = A.shape[0] if m is None else m
    n = A.shape[1] if n is None else n
    lda = _ld(A, m) if lda is None else lda
    single = not isinstance(A, int) and str(A.dtype) == "torch.complex64"
    _check(A, _C64 if single else _C128, m, n, lda, "A")
    _check_vec(ipiv, _I32, min(m, n), "ipiv")
    info = ctypes.c_int(0)
    f = lib().relapack_cgetrf if single else lib().relapack_zgetrf
    f(m, n, _ptr(A), lda, _ptr(ipiv), ctypes.byref(info))
    return info.value


def zgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc) -> int:
    """relapack_zgemm on complex128 tensors (or raw addresses)."""
    ta, tb = str(transa).upper(), str(transb).upper()
    if k > 0:
        _check(A, _C128, k if ta != "N" else m, m if ta != "N" else k, lda, "A")
        _check(B, _C128, n if tb != "N" else k, k if tb != "N" else n, ldb, "B")
    _check(C, _C128, m, n, ldc, "C")
    info = ctypes.c_int(0)
    lib().relapack_zgemm(_b(ta), _b(tb), m, n, k, float(alpha), _ptr(A), lda, _ptr(B), ldb, float(beta), _ptr(C),
                         ldc, ctypes.byref(info))
    return info.value


def potrs(A, B, uplo: str = "L") -> int:
    n, nrhs = B.shape[0], (B.shape[1] if B.dim() > 1 else 1)
    _check(A, _F64, n, n, _ld(A, n), "A")
    _check(B, _F64, n, nrhs, _ld(B, n), "B")
    info = ctypes.c_int(0)
    lib().relapack_dpotrs(_b(uplo), n, nrhs, _ptr(A), _ld(A, n), _ptr(B), _ld(B, n), ctypes.byref(info))
    return info.value


def getrs(A, ipiv, B, trans: str = "N") -> int:
    n, nrhs = B.shape[0], (B.shape[1] if B.dim() > 1 else 1)
    _check(A, _F64, n, n, _ld(A, n), "A")
    _check_vec(ipiv, _I32, n, "ipiv")
    _check(B, _F64, n, nrhs, _ld(B, n), "B")
    info = ctypes.c_int(0)
    lib().relapack_dgetrs(_b(trans), n, nrhs, _ptr(A), _ld(A, n), _ptr(ipiv), _ptr(B), _ld(B, n),
                          ctypes.byref(info))
    return info.value


def posv_mixed(A, B, X, uplo: str = "L", prec=16):
    n, nrhs = B.shape[0], (B.shape[1] if B.dim() > 1 else 1)
    _check(A, _F64, n, n, _ld(A, n), "A")
    _check(B, _F64, n, nrhs, _ld(B, n), "B")
    _check(X, _F64, n, nrhs, _ld(X, n), "X")
    it, berr, info = ctypes.c_int(0), ctypes.c_double(0.0), ctypes.c_int(0)
    lib().relapack_dposv_mixed(_b(uplo), n, nrhs, _ptr(A), _ld(A, n), _ptr(B), _ld(B, n), _ptr(X),
                               _ld(X, n), PREC.get(prec, prec), ctypes.byref(it), ctypes.byref(berr),
                               ctypes.byref(info))
    return info.value, it.value, berr.value


def gesv_mixed(A, ipiv, B, X, prec=16):
    n, nrhs = B.shape[0], (B.shape[1] if B.dim() > 1 else 1)
    _check(A, _F64, n, n, _ld(A, n), "A")
    _check_vec(ipiv, _I32, n, "ipiv")
    _check(B, _F64, n, nrhs, _ld(B, n), "B")
    _check(X, _F64, n, nrhs, _ld(X, n), "X")
    it, berr, info = ctypes.c_int(0), ctypes.c_double(0.0), ctypes.c_int(0)
    lib().relapack_dgesv_mixed(n, nrhs, _ptr(A), _ld(A, n), _ptr(ipiv), _ptr(B), _ld(B, n), _ptr(X),
                               _ld(X, n), PREC.get(prec, prec), ctypes.byref(it), ctypes.byref(berr),
                               ctypes.byref(info))
    return info.value, it.value, berr.value


def mixed_last() -> dict:
    """relapack_mixed_last: what the calling thread's last mixed solve did."""
    v = [ctypes.c_int(0) for _ in range(4)]
    lib().relapack_mixed_last(*[ctypes.byref(x) for x in v])
    return {"sweeps": v[0].value, "gmres_from": v[1].value, "gmres_sweeps": v[2].value,
            "gmres_steps": v[3].value}


def gemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc) -> int:
    ta, tb = str(transa).upper() == "T", str(transb).upper() == "T"
    if k > 0:
        _check(A, _F64, k if ta else m, m if ta else k, lda, "A")
        _check(B, _F64, n if tb else k, k if tb else n, ldb, "B")
    _check(C, _F64, m, n, ldc, "C")
    info = ctypes.c_int(0)
    lib().relapack_dgemm(_b(transa), _b(transb), m, n, k, alpha, _ptr(A), lda, _ptr(B), ldb, beta,
                         _ptr(C), ldc, ctypes.byref(info))
    return info.value


def syrk(uplo, trans, n, k, alpha, A, lda, beta, C, ldc) -> int:
    tr = str(trans).upper() == "T"
    if k > 0:
        _check(A, _F64, k if tr else n, n if tr else k, lda, "A")
    _check(C, _F64, n, n, ldc, "C")
    info = ctypes.c_int(0)
    lib().relapack_dsyrk(_b(uplo), _b(trans), n, k, alpha, _ptr(A), lda, beta, _ptr(C), ldc,
                         ctypes.byref(info))
    return info.value


def trsm(side, uplo, transa, diag, m, n, A, lda, B, ldb) -> int:
    t = m if str(side).upper() == "L" else n
    if m > 0 and n > 0:
        _check(A, _F64, t, t, lda, "A")
    _check(B, _F64, m, n, ldb, "B")
    info = ctypes.c_int(0)
    lib().relapack_dtrsm(_b(side), _b(uplo), _b(transa), _b(diag), m, n, _ptr(A), lda, _ptr(B), ldb,
                         ctypes.byref(info))
    return info.value


def trmm(side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb) -> int:
    t = m if str(side).upper() == "L" else n
    if m > 0 and n > 0:
        _check(A, _F64, t, t, lda, "A")
    _check(B, _F64, m, n, ldb, "B")
    info = ctypes.c_int(0)
    lib().relapack_dtrmm(_b(side), _b(uplo), _b(transa), _b(diag), m, n, alpha, _ptr(A), lda, _ptr(B), ldb,
                         ctypes.byref(info))
    return info.value


def trtri(A, uplo: str = "L", diag: str = "N", n: int | None = None, lda: int | None = None) -> int:
    n = A.shape[0] if n is None else n
    lda = _ld(A, n) if lda is None else lda
    _check(A, _F64, n, n, lda, "A")
    info = ctypes.c_int(0)
    lib().relapack_dtrtri(_b(uplo), _b(diag), n, _ptr(A), lda, ctypes.byref(info))
    return info.value


def lauum(A, uplo: str = "L", n: int | None = None, lda: int | None = None) -> int:
    n = A.shape[0] if n is None else n
    lda = _ld(A, n) if lda is None else lda
    _check(A, _F64, n, n, lda, "A")
    info = ctypes.c_int(0)
    lib().relapack_dlauum(_b(uplo), n, _ptr(A), lda, ctypes.byref(info))
    return info.value


def potri(A, uplo: str = "L", n: int | None = None, lda: int | None = None) -> int:
    n = A.shape[0] if n is None else n
    lda = _ld(A, n) if lda is None else lda
    _check(A, _F64, n, n, lda, "A")
    info = ctypes.c_int(0)
    lib().relapack_dpotri(_b(uplo), n, _ptr(A), lda, ctypes.byref(info))
    return info.value


def scale_spd_f32(A, d, S, uplo: str = "L") -> int:
    n = A.shape[0]
    _check(A, _F64, n, n, _ld(A, n), "A")
    _check_vec(d, _F64, n, "d")
    _check(S, _F32, n, n, _ld(S, n), "S")
    info = ctypes.c_int(0)
    lib().relapack_scale_spd_f32(_b(uplo), n, _ptr(A), _ld(A, n), _ptr(d), _ptr(S), _ld(S, n),
                                 ctypes.byref(info))
    return info.value


def scale_ge_f32(A, r, c, S) -> int:
    n = A.shape[0]
    _check(A, _F64, n, n, _ld(A, n), "A")
    _check_vec(r, _F64, n, "r")
    _check_vec(c, _F64, n, "c")
    _check(S, _F32, n, n, _ld(S, n), "S")
    info = ctypes.c_int(0)
    lib().relapack_scale_ge_f32(n, _ptr(A), _ld(A, n), _ptr(r), _ptr(c), _ptr(S), _ld(S, n),
                                ctypes.byref(info))
    return info.value


def spotrf_lp(A, uplo: str = "L", prec=32) -> int:
    n = A.shape[0]
    _check(A, _F32, n, n, _ld(A, n), "A")
    info = ctypes.c_int(0)
    lib().relapack_spotrf_lp(_b(uplo), n, _ptr(A), _ld(A, n), PREC.get(prec, prec), ctypes.byref(info))
    return info.value


def sgetrf_lp(A, ipiv, prec=32) -> int:
    m, n = A.shape
    _check(A, _F32, m, n, _ld(A, m), "A")
    _check_vec(ipiv, _I32, min(m, n), "ipiv")
    info = ctypes.c_int(0)
    lib().relapack_sgetrf_lp(m, n, _ptr(A), _ld(A, m), _ptr(ipiv), PREC.get(prec, prec),
                             ctypes.byref(info))
    return info.value


def spotrf(A, uplo: str = "L", n: int | None = None, lda: int | None = None) -> int:
    n = A.shape[0] if n is None else n
    lda = _ld(A, n) if lda is None else lda
    _check(A, _F32, n, n, lda, "A")
    info = ctypes.c_int(0)
    lib().relapack_spotrf(_b(uplo), n, _ptr(A), lda, ctypes.byref(info))
    return info.value


def potrf_batched(uplo: str, count: int, n, A_ptrs, lda, info, single: bool = False) -> int:
    """Batched Cholesky: n, lda, info are device int32 arrays, A_ptrs a device int64 array of matrix
    addresses (count entries each). Returns the call status; per-matrix info lands in `info`."""
    for t, dt, what in ((n, _I32, "n"), (A_ptrs, _I64, "A_ptrs"), (lda, _I32, "lda"), (info, _I32, "info")):
        _check_vec(t, dt, count, what)
    f = lib().relapack_spotrf_batched if single else lib().relapack_dpotrf_batched
    return f(_b(uplo), count, _ptr(n), _ptr(A_ptrs), _ptr(lda), _ptr(info))


BATCH_ROUTINES = {"dpotrf": 0, "spotrf": 1, "dgetrf": 2, "sgetrf": 3}


def batched_tune(routine, bucket: int, leaf: int, tile: int) -> int:
    """relapack_batched_tune: set one size bucket's leaf size and tile edge."""
    return lib().relapack_batched_tune(BATCH_ROUTINES.get(routine, routine), bucket, leaf, tile)


def batched_tune_get(routine, bucket: int):
    """(leaf, tile) of one size bucket."""
    leaf, tile = ctypes.c_int(0), ctypes.c_int(0)
    r = lib().relapack_batched_tune_get(BATCH_ROUTINES.get(routine, routine), bucket, ctypes.byref(leaf),
                                        ctypes.byref(tile))
    if r != 0:
        raise ValueError(f"routine {routine!r} / bucket {bucket}: {r}")
    return leaf.value, tile.value


def lookahead(on: bool) -> None:
    """relapack_lookahead: the LU recursion's look-ahead on or off."""
    lib().relapack_lookahead(1 if on else 0)


def batched_graphs(on: bool) -> None:
    lib().relapack_batched_graphs(1 if on else 0)


def getrf_batched(count: int, n, A_ptrs, lda, ipiv_ptrs, info, single: bool = False) -> int:
    """Batched LU: as potrf_batched, with ipiv_ptrs a device int64 array of int32 pivot-array addresses."""
    for t, dt, what in ((n, _I32, "n"), (A_ptrs, _I64, "A_ptrs"), (lda, _I32, "lda"),
                        (ipiv_ptrs, _I64, "ipiv_ptrs"), (info, _I32, "info")):
        _check_vec(t, dt, count, what)
    f = lib().relapack_sgetrf_batched if single else lib().relapack_dgetrf_batched
    return f(count, _ptr(n), _ptr(A_ptrs), _ptr(lda), _ptr(ipiv_ptrs), _ptr(info))


def sgetrf(A, ipiv, m: int | None = None, n: int | None = None, lda: int | None = None) -> int:
    m = A.shape[0] if m is None else m
    n = A.shape[1] if n is None else n
    lda = _ld(A, m) if lda is None else lda
    _check(A, _F32, m, n, lda, "A")
    _check_vec(ipiv, _I32, min(m, n), "ipiv")
    info = ctypes.c_int(0)
    lib().relapack_sgetrf(m, n, _ptr(A), lda, _ptr(ipiv), ctypes.byref(info))
    return info.value


def trace_enable(on: bool = True) -> None:
    lib().relapack_trace_enable(1 if on else 0)


def trace_collect() -> dict:
    cap = 19
    out = (ctypes.c_double * (4 * cap))()
    if lib().relapack_trace_collect(out, cap) < 0:
        raise RuntimeError("relapack_trace_collect failed")
    res = {}
    for k, name in TRACE_FAMILIES.items():
        cnt, ms, fl, by = out[4 * k: 4 * k + 4]
        if cnt:
            res[name] = {"launches": int(cnt), "ms": ms, "flops": fl, "bytes": by}
    return res


def plan(routine: str, m: int, n: int, leaf: int = 0):
    """Kernel-call sequence of one factorization as a list of (kind, depth, m, n, k)."""
    cnt = lib().relapack_plan(routine.encode(), m, n, leaf, None, 0)
    if cnt < 0:
        raise ValueError(routine)
    buf = (ctypes.c_longlong * (5 * max(cnt, 1)))()
    lib().relapack_plan(routine.encode(), m, n, leaf, buf, cnt)
    return [tuple(buf[5 * i: 5 * i + 5]) for i in range(cnt)]


def split(n: int) -> int:
    return int(lib().relapack_split(n))
