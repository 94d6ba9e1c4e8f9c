"""The complex instances (relapack_zpotrf / cpotrf, relapack_zgetrf / cgetrf,
relapack_zgemm) through the C ABI against the complex oracle: ragged sizes
around the 64-wide leaves and 16-column panels, exact Gaussian-integer and
dyadic constructions bit for bit, the pivot rule |re| + |im|, failure and
zero-pivot info, the other triangle never written, single precision within
its own tolerance."""
import numpy as np
import pytest

import gen
import paper_1602_06763_amd as rl
from gpu_util import U32, U64, rel_fro

pytestmark = pytest.mark.gpu


def _dev(a, ld=None, single=False):
    import torch

    m, n = a.shape
    ld = m if ld is None else ld
    dt = torch.complex64 if single else torch.complex128
    buf = torch.full((max(n, 1), max(ld, 1)), complex(float("nan"), float("nan")), dtype=dt)
    buf[:n, :m] = torch.from_numpy(np.ascontiguousarray(a.T)).to(dt)
    return buf.cuda().T[:m, :n]


def _host(t):
    return np.asfortranarray(t.T.contiguous().cpu().numpy().T).astype(np.complex128)


def _setup():
    import torch

    torch.cuda.set_device(0)
    rl.set_stream(torch.cuda.current_stream())


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("N", "C"), ("C", "N"), ("T", "N"), ("N", "T"), ("C", "C")])
def test_zgemm_against_numpy(ta, tb):
    _setup()
    m, n, k = 150, 97, 83
    g = np.random.default_rng(3)
    op = lambda x, t: x if t == "N" else (x.T if t == "T" else x.conj().T)
    A = gen.general_complex(*((m, k) if ta == "N" else (k, m)), seed=1)
    B = gen.general_complex(*((k, n) if tb == "N" else (n, k)), seed=2)
    C = gen.general_complex(m, n, seed=3)
    dA, dB, dC = _dev(A), _dev(B), _dev(C)
    assert rl.zgemm(ta, tb, m, n, k, -1.0, dA, A.shape[0], dB, B.shape[0], 0.5, dC, m) == 0
    ref = 0.5 * C - op(A, ta) @ op(B, tb)
    assert rel_fro(_host(dC), ref) <= 1e-14


@pytest.mark.parametrize("n", [1, 7, 64, 65, 130, 257, 600])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_zpotrf_vs_oracle(orc, n, uplo):
    _setup()
    a = gen.hpd_bbh(n, seed=n)
    s = a.copy(order="F")
    other = np.triu_indices(n, 1) if uplo == "L" else np.tril_indices(n, -1)
    s[other] = complex(np.nan, np.nan)
    d = _dev(s, ld=n + 3)
    assert rl.zpotrf(d, uplo) == 0
    got = _host(d)
    ref, info = orc.zpotrf(a, uplo)
    assert info == 0
    tri = np.tril if uplo == "L" else np.triu
    assert rel_fro(tri(got), tri(ref)) <= 1e-12, n
    assert np.isnan(got[other]).all()


@pytest.mark.parametrize("n", [5, 64, 200])
def test_zpotrf_exact_and_failure(orc, n):
    _setup()
    a, lo = gen.exact_zchol(n, seed=n)
    d = _dev(a)
    assert rl.zpotrf(d, "L") == 0
    assert np.array_equal(np.tril(_host(d)), lo)
    bad = gen.hpd_bbh(n, seed=1)
    k = n // 2
    bad[k, k] = -1e6
    d = _dev(bad)
    _, rinfo = orc.zpotrf(bad, "L")
    assert rl.zpotrf(d, "L") == rinfo == k + 1


@pytest.mark.parametrize("m,n", [(1, 1), (16, 16), (17, 17), (100, 100), (300, 300), (500, 320), (250, 400),
                                 (1100, 1100)])
def test_zgetrf_vs_oracle(orc, m, n):
    _setup()
    import torch

    a = gen.general_complex(m, n, seed=m * 7 + n)
    d = _dev(a, ld=m + 2)
    piv = torch.zeros(max(min(m, n), 1), dtype=torch.int32, device="cuda")
    assert rl.zgetrf(d, piv) == 0
    ref, rpiv, info = orc.zgetrf(a)
    assert info == 0
    assert np.array_equal(piv.cpu().numpy()[: min(m, n)], rpiv)
    assert rel_fro(_host(d), ref) <= 1e-10


@pytest.mark.parametrize("n", [6, 40, 130])
def test_zgetrf_exact_and_pivot_rule(orc, n):
    _setup()
    import torch

    a, perm, lo, up = gen.exact_zlu(n, seed=n)
    d = _dev(a)
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert rl.zgetrf(d, piv) == 0
    ipiv_ref, rows = gen.exact_lu_pivots(perm, n)
    f = _host(d)
    assert np.array_equal(piv.cpu().numpy(), ipiv_ref)
    assert np.array_equal(np.tril(f, -1) + np.eye(n), lo[rows]) and np.array_equal(np.triu(f), up)
    # |re| + |im| decides, not |z|
    a = np.array([[3.0, 1.0], [2 + 2j, 1.0]], dtype=np.complex128, order="F")
    d = _dev(a)
    piv = torch.zeros(2, dtype=torch.int32, device="cuda")
    assert rl.zgetrf(d, piv) == 0 and piv.cpu().numpy()[0] == 2


@pytest.mark.parametrize("m,n", [(1600, 40), (5500, 16), (7000, 24), (13000, 33)])
def test_zgetrf_tall_panels(orc, m, n):
    """Tall panels spread their rows over several cooperating workgroups of
    512 rows (4, 11, 14 and 26 of them: records read whole up to 12, headers
    then the winner's row above), with a ragged last workgroup."""
    _setup()
    import torch

    a = gen.general_complex(m, n, seed=m + n)
    d = _dev(a, ld=m + 3)
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert rl.zgetrf(d, piv) == 0
    ref, rpiv, info = orc.zgetrf(a)
    assert info == 0
    assert np.array_equal(piv.cpu().numpy(), rpiv)
    assert rel_fro(_host(d), ref) <= 1e-10


def test_zgetrf_panel_beyond_the_grid(orc):
    """A panel of more rows than the chip's CUs can hold as 512-row workgroups
    (140000 rows: 274 of them) is factored by the one-workgroup panel
    instead, with its interchanges applied one by one."""
    _setup()
    import torch

    m, n = 140000, 20
    a = gen.general_complex(m, n, seed=17)
    d = _dev(a)
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert rl.zgetrf(d, piv) == 0
    ref, rpiv, info = orc.zgetrf(a)
    assert info == 0
    assert np.array_equal(piv.cpu().numpy(), rpiv)
    assert rel_fro(_host(d), ref) <= 1e-10


def test_zgetrf_tall_zero_pivot(orc):
    _setup()
    import torch

    a = gen.general_complex(3000, 48, seed=11)
    a[:, 20] = 0.0
    d = _dev(a)
    piv = torch.zeros(48, dtype=torch.int32, device="cuda")
    info = rl.zgetrf(d, piv)
    ref, rpiv, rinfo = orc.zgetrf(a)
    assert info == rinfo == 21
    assert np.array_equal(piv.cpu().numpy(), rpiv)
    assert rel_fro(_host(d), ref) <= 1e-10


def test_zgetrf_zero_pivot_completes(orc):
    _setup()
    import torch

    a = gen.general_complex(90, 90, seed=4)
    a[:, 33] = 0.0
    d = _dev(a)
    piv = torch.zeros(90, dtype=torch.int32, device="cuda")
    info = rl.zgetrf(d, piv)
    ref, rpiv, rinfo = orc.zgetrf(a)
    assert info == rinfo == 34
    assert np.array_equal(piv.cpu().numpy(), rpiv)
    assert rel_fro(_host(d), ref) <= 1e-10


def test_single_precision_complex(orc):
    _setup()
    import torch

    n = 300
    a = gen.hpd_bbh(n, seed=2).astype(np.complex64).astype(np.complex128)
    d = _dev(a, single=True)
    assert rl.zpotrf(d, "L") == 0
    lo = np.tril(_host(d))
    assert np.linalg.norm(a - lo @ lo.conj().T) / np.linalg.norm(a) <= 20 * n * U32
    g = gen.general_complex(n, n, seed=5).astype(np.complex64).astype(np.complex128)
    d = _dev(g, single=True)
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert rl.zgetrf(d, piv) == 0
    f = _host(d)
    lo = np.tril(f, -1) + np.eye(n)
    up = np.triu(f)
    import oracle

    pa = oracle.apply_ipiv(g, piv.cpu().numpy())
    assert np.linalg.norm(pa - lo @ up) / np.linalg.norm(g) <= 20 * n * U32
    # a tall single-precision panel over 12 cooperating workgroups
    m, n = 6000, 20
    g = gen.general_complex(m, n, seed=6).astype(np.complex64).astype(np.complex128)
    d = _dev(g, single=True)
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert rl.zgetrf(d, piv) == 0
    f = _host(d)
    lo = np.tril(f, -1)[:, :n] + np.eye(m, n)
    up = np.triu(f[:n])
    pa = oracle.apply_ipiv(g, piv.cpu().numpy())
    assert np.linalg.norm(pa - lo @ up) / np.linalg.norm(g) <= 20 * n * U32
