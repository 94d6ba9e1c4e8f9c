"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/relapack.h declares, rejects bad arguments with LAPACK's
info = -k before launching anything, and its recursion plan (recorded without
launching) has the structure the paper describes."""
import ctypes
import re

import numpy as np
import pytest

import paper_1602_06763_amd as rl


def _declared():
    text = open(rl.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(relapack_\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = rl.lib()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert rl.version() == 1


def _info(fn, *args):
    info = ctypes.c_int(12345)
    fn(*args, ctypes.byref(info))
    return info.value


def test_argument_checks_without_gpu():
    L = rl.lib()
    assert _info(L.relapack_dpotrf, b"X", 4, 0, 4) == -1
    assert _info(L.relapack_dpotrf, b"L", -1, 0, 4) == -2
    assert _info(L.relapack_dpotrf, b"L", 8, 0, 7) == -4
    assert _info(L.relapack_dpotrf, b"U", 0, 0, 1) == 0  # quick return
    assert _info(L.relapack_dgetrf, -1, 4, 0, 4, 0) == -1
    assert _info(L.relapack_dgetrf, 4, -1, 0, 4, 0) == -2
    assert _info(L.relapack_dgetrf, 9, 4, 0, 8, 0) == -4
    assert _info(L.relapack_dgetrf, 0, 5, 0, 1, 0) == 0
    # complex instances
    assert _info(L.relapack_zpotrf, b"X", 4, 0, 4) == -1
    assert _info(L.relapack_cpotrf, b"L", -3, 0, 4) == -2
    assert _info(L.relapack_zpotrf, b"U", 8, 0, 7) == -4
    assert _info(L.relapack_zgetrf, -1, 4, 0, 4, 0) == -1
    assert _info(L.relapack_cgetrf, 4, -1, 0, 4, 0) == -2
    assert _info(L.relapack_zgetrf, 9, 4, 0, 8, 0) == -4
    assert _info(L.relapack_zgemm, b"N", b"Q", 2, 2, 2, 1.0, 0, 2, 0, 2, 0.0, 0, 2) == -2
    assert _info(L.relapack_zgemm, b"C", b"N", 3, 2, 4, 1.0, 0, 3, 0, 4, 0.0, 0, 3) == -8
    # batched tuning table: only the offered leaf sizes and tile edges, read back as set
    assert L.relapack_batched_tune(0, 0, 16, 64) == -3
    assert L.relapack_batched_tune(2, 0, 64, 64) == -3
    assert L.relapack_batched_tune(0, 0, 64, 48) == -3
    assert L.relapack_batched_tune(0, 4, 64, 64) == -2
    assert L.relapack_batched_tune(5, 0, 64, 64) == -1
    lf, tl = ctypes.c_int(0), ctypes.c_int(0)
    assert L.relapack_batched_tune_get(2, 1, ctypes.byref(lf), ctypes.byref(tl)) == 0
    assert (lf.value, tl.value) in {(16, 32), (16, 64), (32, 32), (32, 64)}
    # the allocation-free LU: same checks, and m above its fixed workspace (32768 rows) is refused
    assert _info(L.relapack_dgetrf_noalloc, -1, 4, 0, 4, 0) == -1
    assert _info(L.relapack_dgetrf_noalloc, 32769, 4, 0, 32769, 0) == -1
    assert _info(L.relapack_dgetrf_noalloc, 4, -1, 0, 4, 0) == -2
    assert _info(L.relapack_dgetrf_noalloc, 9, 4, 0, 8, 0) == -4
    assert _info(L.relapack_dgetrf_noalloc, 0, 5, 0, 1, 0) == 0
    assert _info(L.relapack_dpotrs, b"Q", 4, 1, 0, 4, 0, 4) == -1
    assert _info(L.relapack_dpotrs, b"L", 4, -2, 0, 4, 0, 4) == -3
    assert _info(L.relapack_dpotrs, b"L", 4, 1, 0, 4, 0, 3) == -7
    assert _info(L.relapack_dgetrs, b"Z", 4, 1, 0, 4, 0, 0, 4) == -1
    assert _info(L.relapack_dgetrs, b"N", 4, 1, 0, 3, 0, 0, 4) == -5
    assert _info(L.relapack_dgetrs, b"N", 4, 1, 0, 4, 0, 0, 2) == -8
    assert _info(L.relapack_dgemm, b"N", b"X", 2, 2, 2, 1.0, 0, 2, 0, 2, 0.0, 0, 2) == -2
    assert _info(L.relapack_dgemm, b"T", b"N", 3, 2, 4, 1.0, 0, 3, 0, 4, 0.0, 0, 3) == -8
    assert _info(L.relapack_dsyrk, b"L", b"N", 5, 2, 1.0, 0, 4, 0.0, 0, 5) == -7
    assert _info(L.relapack_dtrsm, b"L", b"L", b"N", b"Q", 2, 2, 0, 2, 0, 2) == -4
    it, be = ctypes.c_int(0), ctypes.c_double(0)
    info = ctypes.c_int(0)
    L.relapack_dposv_mixed(b"L", 4, 1, 0, 4, 0, 4, 0, 4, 8, ctypes.byref(it), ctypes.byref(be), ctypes.byref(info))
    assert info.value == -10
    L.relapack_dgesv_mixed(4, 1, 0, 4, 0, 0, 4, 0, 3, 16, ctypes.byref(it), ctypes.byref(be), ctypes.byref(info))
    assert info.value == -9
    assert _info(L.relapack_spotrf_lp, b"L", 4, 0, 4, 7) == -5
    assert _info(L.relapack_sgetrf_lp, 4, 4, 0, 4, 0, 64) == -6


@pytest.mark.parametrize("n", [1, 2, 63, 64, 100, 127, 128, 129, 130, 200, 1000, 4096, 16385, 32768])
def test_split_rule(n):
    n1 = rl.split(n)
    n2 = n - n1
    assert 0 < n1 < n or n == 1
    if n >= 128:
        assert n1 % 64 == 0 and n2 >= 64 and abs(n1 - n / 2) <= 32
    else:
        assert n1 == n // 2


def _flops(kind, m, n, k):
    if kind == 3:   # gemm
        return 2.0 * m * n * k
    if kind == 4:   # syrk (leading order)
        return 1.0 * m * m * k
    if kind == 2:   # trsm leaf: t×t triangle, n vectors
        return 1.0 * m * m * n
    if kind == 1:   # potf2
        return m ** 3 / 3.0
    if kind == 5:   # getf2 panel (m rows, w cols)
        return m * n * n - n ** 3 / 3.0
    return 0.0


def test_potrf_plan_flop_shares_follow_the_papers_series():
    """Top-level TRSM + SYRK hold 3/4 of n^3/3 and level l holds 3/4^l: the
    series of the paper's flop-share analysis (Sec. 3), here for Cholesky."""
    n = 4096
    plan = rl.plan("potrf_L", n, n, 64)
    total = sum(_flops(k, m, nn, kk) for k, _, m, nn, kk in plan)
    assert total == pytest.approx(n ** 3 / 3.0, rel=1e-12)
    # the top-level SYRK, and the top-level TRSM with everything inside it
    top = [r for r in plan if r[1] == 0 and r[0] == 4]
    assert top == [(4, 0, 2048, 2048, 2048)]
    # level-l BLAS-3 work (syrk at depth l-1 plus its trsm subtree)
    shares = _level_shares(plan, n)
    for lvl, share in enumerate(shares[:5], start=1):
        assert share == pytest.approx(3.0 / 4 ** lvl, rel=1e-12)


def _level_shares(plan, n):
    """Group flops by the Cholesky level that issued them: walk the plan, where a
    potf2 or the syrk of depth d closes the current trsm subtree."""
    # in potrf the trsm (and its recursion) of depth d is followed by the syrk of depth d
    per = {}
    pending = 0.0
    for kind, depth, m, nn, kk in plan:
        f = _flops(kind, m, nn, kk)
        if kind in (2, 3):
            pending += f
        elif kind == 4:
            per[depth] = per.get(depth, 0.0) + pending + f
            pending = 0.0
    total = n ** 3 / 3.0
    return [per.get(d, 0.0) / total for d in sorted(per)]


def test_crossover_does_not_change_the_big_calls():
    """Changing c leaves the large BLAS calls untouched; only the shapes are
    determined by n (Sec. 3, analysis of the effect of c)."""
    n = 4096
    big = lambda p: [r for r in p if r[0] in (3, 4) and min(r[2], r[3]) >= 512]
    p32, p64, p128 = (rl.plan("potrf_L", n, n, c) for c in (32, 64, 128))
    assert big(p32) == big(p64) == big(p128)
    assert len(p32) > len(p64) > len(p128)


def test_getrf_plan_structure():
    n = 4096
    plan = rl.plan("getrf", n, n, 32)
    total = sum(_flops(k, m, nn, kk) for k, _, m, nn, kk in plan)
    assert total == pytest.approx(2.0 * n ** 3 / 3.0, rel=2e-3)
    top = [r for r in plan if r[1] == 0]
    # the top level: one unit-lower trsm subtree and one gemm of (n/2)^3
    assert (3, 0, 2048, 2048, 2048) in top
    panels = [r for r in plan if r[0] == 5]
    assert len(panels) == n // 32 and all(r[3] == 32 for r in panels)
    assert [r[2] for r in panels] == [n - 32 * i for i in range(n // 32)]
    # every interchange reaches every column outside its own panel exactly
    # once: leaf records (2w, columns, w), batch records (rows, columns, pivots)
    swaps = [r for r in plan if r[0] == 6]
    assert sum(r[4] * r[3] for r in swaps) == sum(r[3] * (n - r[3]) for r in panels)
    # wide nodes batch their pivots: one batch per half per node wider than 512
    batches = [r for r in swaps if r[4] > 32]
    assert len(batches) == 2 * (1 + 2 + 4)          # nodes of width 4096, 2048, 1024
    assert max(r[3] for r in swaps if r[4] == 32) <= 512 - 32


@pytest.mark.parametrize("m,n", [(4096, 4096), (300, 5000), (5000, 300), (2000, 3000), (3000, 2000),
                                 (65536, 4096), (1000, 1000), (513, 513)])
def test_getrf_plan_interchanges_reach_every_column_once(m, n):
    plan = rl.plan("getrf", m, n, 0)
    panels = [r for r in plan if r[0] == 5]
    swaps = [r for r in plan if r[0] == 6]
    assert sum(r[4] * r[3] for r in swaps) == sum(r[3] * (n - r[3]) for r in panels)
    if m > 32768:
        assert all(r[4] <= 32 for r in swaps)      # no batches: a column's rows exceed the batch kernel

def test_getrf_plan_rectangular():
    plan = rl.plan("getrf", 5000, 300, 32)
    panels = [r for r in plan if r[0] == 5]
    assert sum(r[3] for r in panels) == 300
    wide = rl.plan("getrf", 300, 5000, 32)
    assert sum(r[3] for r in wide if r[0] == 5) == 300
    # the columns beyond the square part get one unit-lower solve with L11
    assert any(r[0] == 2 for r in wide[-5:]) or any(r[0] == 3 for r in wide[-5:])


class _FakeStorage:
    def __init__(self, nbytes):
        self._n = nbytes

    def nbytes(self):
        return self._n


class _FakeCudaTensor:
    """Just the attributes the binding's argument check reads (no GPU needed)."""

    def __init__(self, dtype, elems, offset=0, item=8):
        self.is_cuda = True
        self.dtype = dtype
        self.device = "cuda:0"
        self._elems, self._off, self._item = elems, offset, item

    def element_size(self):
        return self._item

    def storage_offset(self):
        return self._off

    def untyped_storage(self):
        return _FakeStorage(self._elems * self._item)


def test_binding_refuses_bad_tensors():
    import torch

    import paper_1602_06763_amd as rl

    # a CPU tensor never reaches the library
    with pytest.raises(ValueError, match="CUDA"):
        rl._check(torch.zeros(4, 4, dtype=torch.float64), "float64", 4, 4, 4, "A")
    # wrong dtype
    with pytest.raises(ValueError, match="dtype"):
        rl._check(_FakeCudaTensor("torch.float32", 16, item=4), "float64", 4, 4, 4, "A")
    # storage too small for ld·(cols−1) + rows from the view's start
    rl._check(_FakeCudaTensor("torch.float64", 6 * 7 + 5), "float64", 5, 8, 6, "A")
    with pytest.raises(ValueError, match="storage"):
        rl._check(_FakeCudaTensor("torch.float64", 6 * 7 + 4), "float64", 5, 8, 6, "A")
    with pytest.raises(ValueError, match="storage"):
        rl._check(_FakeCudaTensor("torch.float64", 6 * 7 + 5, offset=1), "float64", 5, 8, 6, "A")
    # an int64 pivot vector is refused, int32 of the right length accepted
    with pytest.raises(ValueError, match="dtype"):
        rl._check_vec(_FakeCudaTensor("torch.int64", 10), "int32", 10, "ipiv")
    rl._check_vec(_FakeCudaTensor("torch.int32", 10, item=4), "int32", 10, "ipiv")
    with pytest.raises(ValueError, match="storage"):
        rl._check_vec(_FakeCudaTensor("torch.int32", 9, item=4), "int32", 10, "ipiv")
    # illegal sizes are left to the library's own info codes
    rl._check(_FakeCudaTensor("torch.float32", 1, item=4), "float64", 5, 5, 3, "A")
    rl._check(_FakeCudaTensor("torch.float32", 1, item=4), "float64", -1, 5, 3, "A")
    # through a wrapper: a CPU tensor raises before any library call
    with pytest.raises(ValueError):
        rl.potrf(torch.zeros(4, 4, dtype=torch.float64).T, "L")
