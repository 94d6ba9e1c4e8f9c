"""Triangular product, triangular inverse, Lᵀ·L and the SPD inverse through the
C ABI: against the oracle (trtri, lauum, potri) and plain FP64 products
(trmm), at ragged sizes around the 64 leaf and across several recursion
levels, on exact integer inputs (bit-exact), on a zero pivot, and at the
n = 8192 size of the SPD-inverse follow-on through A·A⁻¹ = I."""
import numpy as np
import pytest

import gen
import oracle
import paper_1602_06763_amd as rl
from gpu_util import U64, to_dev, to_host

pytestmark = pytest.mark.gpu


def _other(n, uplo):
    return np.triu_indices(n, 1) if uplo == "L" else np.tril_indices(n, -1)


def _tri(uplo):
    return np.tril if uplo == "L" else np.triu


@pytest.mark.parametrize("side", ["L", "R"])
@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("diag", ["N", "U"])
@pytest.mark.parametrize("m,n", [(1, 1), (64, 64), (65, 33), (200, 130), (300, 257), (1030, 90), (1000, 2100)])
def test_trmm(side, uplo, trans, diag, m, n):
    """Up to 64 rows the leaf; above, one launch per triangle of up to 1024
    rows (ragged tiles at 200, 257, 300) under the recursion's splits
    (1030, 2100), on 32×32 output tiles or, with enough of them (1000 rows
    by 2100 vectors), 64×64 ones."""
    t = m if side == "L" else n
    tri = gen.triangular(t, uplo, "N", seed=t)
    stored = tri.copy(order="F")
    stored[_other(t, uplo)] = np.nan            # never read
    if diag == "U":
        stored[np.diag_indices(t)] = np.nan     # never read either
    b = gen.general_uniform(m, n, seed=m + n)
    B = to_dev(b, ld=m + 3)
    assert rl.trmm(side, uplo, trans, diag, m, n, -1.5, to_dev(stored), t, B, m + 3) == 0
    op = tri.copy()
    if diag == "U":
        op[np.diag_indices(t)] = 1.0
    op = op if trans == "N" else op.T
    ref = -1.5 * (op @ b if side == "L" else b @ op)
    scale = 1.5 * (np.abs(op) @ np.abs(b) if side == "L" else np.abs(b) @ np.abs(op))
    err = np.abs(to_host(B) - ref)
    assert (err <= 4 * (t + 2) * U64 * scale + 1e-300).all()


@pytest.mark.parametrize("n", [1, 17, 64, 65, 200, 517, 1500, 2300])
@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("diag", ["N", "U"])
def test_trtri_vs_oracle(n, uplo, diag):
    t = gen.triangular(n, uplo, diag, seed=n + 1)
    t[_other(n, uplo)] = np.nan
    ref, info = oracle.trtri(t, uplo, diag)
    assert info == 0
    A = to_dev(t, ld=n + 1)
    assert rl.trtri(A, uplo, diag, n=n, lda=n + 1) == 0
    got = to_host(A)
    tri = _tri(uplo)
    k = 0 if diag == "N" else (-1 if uplo == "L" else 1)
    g, r = tri(np.nan_to_num(got, nan=0.0), k), tri(np.nan_to_num(ref, nan=0.0), k)
    assert np.abs(g - r).max() <= 16 * n * U64 * max(np.abs(r).max(), 1.0)
    # the strict other triangle (and a unit diagonal) is neither read nor written
    assert np.isnan(got[_other(n, uplo)]).all()
    if diag == "U":
        assert np.array_equal(np.diag(got), np.diag(t))


@pytest.mark.parametrize("n,s", [(40, 2.0), (300, 1.0), (130, -1.0)])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_trtri_exact(n, s, uplo):
    lo = gen.unit_bidiagonal(n, s)
    t = lo if uplo == "L" else lo.T.copy(order="F")
    A = to_dev(t)
    assert rl.trtri(A, uplo, "N") == 0
    ref, info = oracle.trtri(t, uplo, "N")
    assert info == 0
    assert np.array_equal(_tri(uplo)(to_host(A)), _tri(uplo)(ref))


@pytest.mark.parametrize("uplo", ["L", "U"])
def test_trtri_zero_pivot(uplo):
    n = 300
    t = gen.triangular(n, uplo, "N", seed=3)
    t[100, 100] = 0.0
    t[250, 250] = 0.0
    A = to_dev(t)
    assert rl.trtri(A, uplo, "N") == 101
    got = to_host(A)
    assert np.array_equal(got, t)        # nothing was written
    assert rl.trtri(A, uplo, "U") == 0   # a unit diagonal is not inspected


@pytest.mark.parametrize("n", [1, 33, 64, 65, 300, 517, 1500, 2300])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_lauum_vs_oracle(n, uplo):
    t = gen.triangular(n, uplo, "N", seed=n + 2) / n
    t[_other(n, uplo)] = np.nan
    ref = oracle.lauum(t, uplo)
    A = to_dev(t, ld=n + 2)
    assert rl.lauum(A, uplo, n=n, lda=n + 2) == 0
    got = to_host(A)
    tri = _tri(uplo)
    g, r = tri(np.nan_to_num(got, nan=0.0)), tri(np.nan_to_num(ref, nan=0.0))
    assert np.abs(g - r).max() <= 8 * n * U64 * max(np.abs(r).max(), 1.0)
    assert np.isnan(got[_other(n, uplo)]).all()


@pytest.mark.parametrize("uplo", ["L", "U"])
def test_lauum_exact_integers(uplo):
    n = 257
    g = np.random.default_rng(11)
    t = g.integers(-3, 4, size=(n, n))
    t = np.tril(t) if uplo == "L" else np.triu(t)
    ref = t.T @ t if uplo == "L" else t @ t.T
    A = to_dev(t.astype(np.float64, order="F"))
    assert rl.lauum(A, uplo) == 0
    assert np.array_equal(_tri(uplo)(to_host(A)), _tri(uplo)(ref).astype(np.float64))


@pytest.mark.parametrize("n", [512, 1000])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_potri_vs_oracle(n, uplo):
    a = gen.spd_bbt(n, seed=0)
    ref, info = oracle.potri(a, uplo)
    assert info == 0
    A = to_dev(a)
    assert rl.potrf(A, uplo) == 0
    assert rl.potri(A, uplo) == 0
    tri = _tri(uplo)
    got = tri(to_host(A))
    r = tri(ref)
    assert np.abs(got - r).max() <= 32 * n * U64 * np.abs(r).max()


def test_potri_exact_bidiagonal():
    n = 700
    lo = gen.unit_bidiagonal(n, 1.0)
    a = lo @ lo.T
    A = to_dev(a)
    assert rl.potrf(A, "L") == 0
    assert rl.potri(A, "L") == 0
    ref, info = oracle.potri(a, "L")
    assert info == 0
    assert np.array_equal(np.tril(to_host(A)), np.tril(ref))


def test_potri_zero_factor_diagonal():
    a = np.tril(gen.triangular(200, "L", "N", seed=4))
    a[57, 57] = 0.0
    A = to_dev(a)
    assert rl.potri(A, "L") == 58
    assert np.array_equal(to_host(A), a)


def test_potri_n8192_identity_residual():
    import torch

    torch.cuda.set_device(0)
    rl.set_stream(torch.cuda.current_stream())
    n = 8192
    A0 = gen.spd_bbt_torch(n, seed=0, device="cuda")
    A = A0.clone()
    assert rl.potrf(A, "L") == 0
    assert rl.potri(A, "L") == 0
    torch.cuda.synchronize()
    X = torch.tril(A) + torch.tril(A, -1).T
    R = A0 @ X
    R.diagonal().sub_(1.0)
    bound = 10 * n * U64 * float(A0.abs().sum(1).max()) * float(X.abs().sum(1).max())
    assert float(R.abs().max()) <= bound
    # the strict upper triangle keeps A's values
    iu = torch.triu_indices(n, n, 1, device="cuda")
    assert torch.equal(A[iu[0], iu[1]], A0[iu[0], iu[1]])
