"""The matrix-core building blocks on the recursion's path (GEMM, triangular
update, triangular solve) through the C ABI against plain FP64 products and
solves, at ragged sizes spanning several tiles."""
import numpy as np
import pytest
import scipy.linalg as sl

import gen
import paper_1602_06763_amd as rl
from gpu_util import U64, rel_fro, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ta", ["N", "T"])
@pytest.mark.parametrize("tb", ["N", "T"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (65, 33, 17), (130, 257, 300), (1000, 600, 129), (1000, 600, 208),
                                   (64, 64, 0)])
def test_gemm(ta, tb, m, n, k):
    a = gen.general_uniform(m if ta == "N" else k, k if ta == "N" else m, seed=1)
    b = gen.general_uniform(k if tb == "N" else n, n if tb == "N" else k, seed=2)
    c = gen.general_uniform(m, n, seed=3)
    A, B, C = to_dev(a), to_dev(b), to_dev(c, ld=m + 5)
    info = rl.gemm(ta, tb, m, n, k, -1.0, A, max(a.shape[0], 1), B, max(b.shape[0], 1), 0.5, C, m + 5)
    assert info == 0
    opa = a if ta == "N" else a.T
    opb = b if tb == "N" else b.T
    ref = 0.5 * c - opa @ opb
    assert np.abs(to_host(C) - ref).max() <= 4 * (k + 2) * U64 * max(1.0, np.abs(ref).max())


def _dev_layout(a, layout):
    """Device copy of a for the large-tile tests: 'pairs' gives an even leading
    dimension and an aligned base (2-wide loads), 'odd_ld' an odd leading
    dimension, 'odd_base' a base one element past an aligned address."""
    rows = a.shape[0]
    if layout == "pairs":
        return to_dev(a, ld=rows + rows % 2), rows + rows % 2
    if layout == "odd_ld":
        return to_dev(a, ld=rows + 1 - rows % 2), rows + 1 - rows % 2
    padded = np.vstack([np.zeros((1, a.shape[1])), a])
    ld = rows + 2 - rows % 2
    return to_dev(padded, ld=ld)[1:, :], ld


@pytest.mark.parametrize("ta", ["N", "T"])
@pytest.mark.parametrize("tb", ["N", "T"])
@pytest.mark.parametrize("layout", ["pairs", "odd_ld", "odd_base"])
@pytest.mark.parametrize("k", [37, 160])
def test_gemm_large_tiles(ta, tb, layout, k):
    """Sizes that take the 128x128 tiles (at least two per CU), ragged in M and
    N, with operands whose adjacent elements pair up and with operands that
    force element-wise loads; K = 160 (a multiple of the K step) sends the
    interior tiles down the unguarded path and the edge tiles down the
    guarded one."""
    m, n = 2900, 2836
    a = gen.general_uniform(m if ta == "N" else k, k if ta == "N" else m, seed=11)
    b = gen.general_uniform(k if tb == "N" else n, n if tb == "N" else k, seed=12)
    c = gen.general_uniform(m, n, seed=13)
    (A, lda), (B, ldb) = _dev_layout(a, layout), _dev_layout(b, layout)
    C = to_dev(c, ld=m + 3)
    assert rl.gemm(ta, tb, m, n, k, -1.0, A, lda, B, ldb, 0.5, C, m + 3) == 0
    ref = 0.5 * c - (a if ta == "N" else a.T) @ (b if tb == "N" else b.T)
    assert np.abs(to_host(C) - ref).max() <= 4 * (k + 2) * U64 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("layout", ["pairs", "odd_ld"])
@pytest.mark.parametrize("k", [20, 48])
def test_syrk_large_tiles(uplo, trans, layout, k):
    """A triangular update on 128x128 tiles whose last, partly filled round runs
    as 64x64 quarters (n = 4100: 561 tiles for 512 slots); K = 48 takes the
    unguarded path on the interior tiles."""
    n = 4100
    a = gen.general_uniform(n if trans == "N" else k, k if trans == "N" else n, seed=14)
    c = gen.general_uniform(n, n, seed=15)
    A, lda = _dev_layout(a, layout)
    C = to_dev(c)
    assert rl.syrk(uplo, trans, n, k, -1.0, A, lda, 1.0, C, n) == 0
    op = a if trans == "N" else a.T
    ref = c - op @ op.T
    got = to_host(C)
    tri = np.tril_indices(n) if uplo == "L" else np.triu_indices(n)
    other = np.triu_indices(n, 1) if uplo == "L" else np.tril_indices(n, -1)
    assert np.abs(got[tri] - ref[tri]).max() <= 4 * (k + 2) * U64 * np.abs(ref).max()
    assert np.array_equal(got[other], c[other])


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", ["N", "T"])
def test_syrk_touches_one_triangle(uplo, trans):
    n, k = 300, 130
    a = gen.general_uniform(n if trans == "N" else k, k if trans == "N" else n, seed=4)
    c = gen.general_uniform(n, n, seed=5)
    C = to_dev(c)
    assert rl.syrk(uplo, trans, n, k, -1.0, to_dev(a), a.shape[0], 1.0, C, n) == 0
    op = a if trans == "N" else a.T
    ref = c - op @ op.T
    got = to_host(C)
    tri = np.tril_indices(n) if uplo == "L" else np.triu_indices(n)
    other = np.triu_indices(n, 1) if uplo == "L" else np.tril_indices(n, -1)
    assert np.abs(got[tri] - ref[tri]).max() <= 4 * k * U64 * np.abs(ref).max()
    assert np.array_equal(got[other], c[other])


@pytest.mark.parametrize("side", ["L", "R"])
@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("diag", ["N", "U"])
def test_trsm(side, uplo, trans, diag):
    m, n = 333, 150
    t = m if side == "L" else n
    tri = np.tril(gen.general_uniform(t, t, seed=6)) if uplo == "L" else np.triu(gen.general_uniform(t, t, seed=6))
    tri[np.diag_indices(t)] = 2.0 + np.abs(tri[np.diag_indices(t)])
    b = gen.general_uniform(m, n, seed=7)
    B = to_dev(b)
    assert rl.trsm(side, uplo, trans, diag, m, n, to_dev(tri), t, B, m) == 0
    op = tri if trans == "N" else tri.T
    if diag == "U":
        op = op.copy()
        op[np.diag_indices(t)] = 1.0
    x = to_host(B)
    resid = (op @ x - b) if side == "L" else (x @ op - b)
    assert np.abs(resid).max() <= 64 * t * U64 * max(1.0, np.abs(b).max()) * np.abs(op).max() * np.abs(x).max()
    ref = sl.solve_triangular(op, b, lower=(uplo == "L") == (trans == "N")) if side == "L" else \
        sl.solve_triangular(op.T, b.T, lower=(uplo == "L") != (trans == "N")).T
    assert rel_fro(x, ref) <= 1e-10


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("diag", ["N", "U"])
@pytest.mark.parametrize("m,nrhs", [(1000, 1), (333, 3), (64, 8), (65, 9), (700, 20), (129, 33), (515, 47), (1000, 64)])
def test_trsm_few_rhs(uplo, trans, diag, m, nrhs):
    """Left-side solves with few right-hand sides (the single-launch blocked solve)."""
    tri = np.tril(gen.general_uniform(m, m, seed=16)) if uplo == "L" else np.triu(gen.general_uniform(m, m, seed=16))
    tri[np.diag_indices(m)] = 2.0 + np.abs(tri[np.diag_indices(m)])
    b = gen.general_uniform(m, nrhs, seed=17)
    B = to_dev(b, ld=m + 3)
    assert rl.trsm("L", uplo, trans, diag, m, nrhs, to_dev(tri), m, B, m + 3) == 0
    op = tri if trans == "N" else tri.T
    if diag == "U":
        op = op.copy()
        op[np.diag_indices(m)] = 1.0
    ref = sl.solve_triangular(op, b, lower=(uplo == "L") == (trans == "N"))
    assert rel_fro(to_host(B), ref) <= 1e-12


def test_trsm_few_rhs_exact():
    """Integer triangle with power-of-two diagonal: substitution is exact."""
    n = 2000
    lo = gen.exact_chol_factor(n, seed=3)
    x = gen.rng(3).integers(-3, 4, size=(n, 2)).astype(np.float64)
    b = lo @ x
    B = to_dev(b)
    assert rl.trsm("L", "L", "N", "N", n, 2, to_dev(lo), n, B, n) == 0
    assert np.array_equal(to_host(B), x)
    b2 = lo.T @ x
    B = to_dev(b2)
    assert rl.trsm("L", "L", "T", "N", n, 2, to_dev(lo), n, B, n) == 0
    assert np.array_equal(to_host(B), x)
