"""GPU parity of the recursive Cholesky (relapack_dpotrf / dpotrs) against the
CPU oracle, through the C ABI. Bars: exact constructions bit-exact; L within
1e-12 normwise of the oracle on the well-conditioned A = B·Bᵀ + n·I inputs;
||A - L·Lᵀ||_F <= 10·n·u·||A||_F; the other triangle untouched."""
import numpy as np
import pytest

import gen
import paper_1602_06763_amd as rl
from gpu_util import U64, ipiv_dev, rel_fro, to_dev, to_host

pytestmark = pytest.mark.gpu


def _run(a, uplo="L", ld=None):
    t = to_dev(a, ld)
    info = rl.potrf(t, uplo)
    return to_host(t), info


def test_config0_n512(orc):
    """n = 512, lda = 512, A = B·Bᵀ + 512·I from seed 0: the small parity case."""
    a = gen.spd_bbt(512, seed=0)
    f, info = _run(a)
    ref, rinfo = orc.potrf(a)
    assert info == rinfo == 0
    L = np.tril(f)
    assert rel_fro(L, np.tril(ref)) <= 1e-12
    assert np.linalg.norm(a - L @ L.T) <= 10 * 512 * U64 * np.linalg.norm(a)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 63, 64, 65, 100, 127, 128, 129, 191, 300, 777, 1031, 2100])
def test_lower_ragged_sizes(orc, n):
    a = gen.spd_bbt(n, seed=n)
    s = a.copy(order="F")
    s[np.triu_indices(n, 1)] = np.nan  # strict upper: must be neither read nor written
    f, info = _run(s, "L", ld=n + (7 if n % 2 else 0))
    ref, _ = orc.potrf(a)
    assert info == 0
    assert rel_fro(np.tril(f), np.tril(ref)) <= 1e-12
    assert np.isnan(f[np.triu_indices(n, 1)]).all()


@pytest.mark.parametrize("n", [5, 64, 65, 300, 1000])
def test_upper(orc, n):
    a = gen.spd_bbt(n, seed=100 + n)
    s = a.copy(order="F")
    s[np.tril_indices(n, -1)] = np.nan
    f, info = _run(s, "U")
    ref, _ = orc.potrf(a, "U")
    assert info == 0
    assert rel_fro(np.triu(f), np.triu(ref)) <= 1e-12
    assert np.isnan(f[np.tril_indices(n, -1)]).all()


@pytest.mark.parametrize("n", [1, 64, 200, 1000, 2500])
def test_exact_integer_factor(n):
    a, lo = gen.exact_chol(n, seed=7 * n)
    f, info = _run(a)
    assert info == 0
    assert np.array_equal(np.tril(f), lo)


@pytest.mark.parametrize("n,k", [(40, 1), (200, 70), (300, 300), (1000, 513)])
def test_not_positive_definite(orc, n, k):
    a = gen.spd_bbt(n, seed=3)
    a[k - 1, k - 1] = -1.0
    f, info = _run(a)
    ref, rinfo = orc.potrf(a)
    assert info == rinfo == k
    # the leading (k-1)×(k-1) block is the factor's
    if k > 1:
        assert rel_fro(np.tril(f[: k - 1, : k - 1]), np.tril(ref[: k - 1, : k - 1])) <= 1e-12
    nanm = gen.spd_bbt(n, seed=3)
    nanm[k - 1, k - 1] = np.nan
    assert _run(nanm)[1] == k


@pytest.mark.parametrize("n,k", [(200, 30), (200, 70), (130, 100)])
def test_not_positive_definite_upper(orc, n, k):
    """'U' failures inside the one-launch bottom node: in its first block
    (200, 30), its second (200, 70), and a 66-row node split 33 + 33
    (130, 100)."""
    a = gen.spd_bbt(n, seed=5)
    a[k - 1, k - 1] = -1.0
    f, info = _run(a, "U")
    ref, rinfo = orc.potrf(a, "U")
    assert info == rinfo == k
    if k > 1:
        assert rel_fro(np.triu(f[: k - 1, : k - 1]), np.triu(ref[: k - 1, : k - 1])) <= 1e-12


def test_zero_and_one():
    import torch

    t = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    assert rl.potrf(t, "L", n=0, lda=1) == 0
    t.fill_(16.0)
    assert rl.potrf(t) == 0 and float(t[0, 0]) == 4.0


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("nrhs", [1, 3, 64])
def test_potrs_exact_and_random(orc, uplo, nrhs):
    n = 700
    a, lo = gen.exact_chol(n, seed=5)
    x = gen.rng(5).integers(-5, 6, size=(n, nrhs)).astype(np.float64)
    b = a @ x
    t = to_dev(a)
    assert rl.potrf(t, uplo) == 0
    bt = to_dev(b)
    assert rl.potrs(t, bt, uplo) == 0
    assert np.array_equal(to_host(bt), x)
    s = gen.spd_bbt(n, seed=6)
    b2 = gen.general_uniform(n, nrhs, seed=8)
    t = to_dev(s)
    rl.potrf(t, uplo)
    bt = to_dev(b2)
    rl.potrs(t, bt, uplo)
    fac, _ = orc.potrf(s, uplo)
    xr = orc.potrs(fac, b2, uplo)
    assert rel_fro(to_host(bt), xr) <= 1e-12
    assert orc.backward_error(s, to_host(bt), b2)[0] <= 10 * n * U64
