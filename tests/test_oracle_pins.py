"""Pins for the CPU oracle, none of which re-derives it from itself.

Each test fixes the oracle's output by something the mathematics or the
construction of the input decides: exact factors (binary64-exact integer and
dyadic constructions), ratios of minors in exact rational arithmetic, closed
forms, special cases, invariants (residual bounds, |l_ij| <= 1, untouched
triangles), and the failure semantics LAPACK defines. A dropped term, a wrong
sign or index, a transposed operand or a wrong tie-break fails at least one.
"""
import numpy as np
import pytest

import gen
import exact

U64 = 2.0 ** -53


# --------------------------------------------------------------------- Cholesky

@pytest.mark.parametrize("n", [1, 2, 7, 64, 257])
def test_chol_exact_integer_factor(orc, n):
    a, lo = gen.exact_chol(n, seed=n)
    sentinel = a.copy(order="F")
    sentinel[np.triu_indices(n, 1)] = np.nan  # strict upper must be neither read nor written
    f, info = orc.potrf(sentinel, "L")
    assert info == 0
    assert np.array_equal(np.tril(f), lo)
    assert np.isnan(f[np.triu_indices(n, 1)]).all()


def test_chol_upper_is_transpose(orc):
    a = gen.spd_bbt(90, seed=3)
    fl, il = orc.potrf(a, "L")
    s = a.copy(order="F")
    s[np.tril_indices(90, -1)] = np.nan
    fu, iu = orc.potrf(s, "U")
    assert il == iu == 0
    assert np.array_equal(np.triu(fu), np.tril(fl).T)
    assert np.isnan(fu[np.tril_indices(90, -1)]).all()


@pytest.mark.parametrize("n", [1, 2, 50, 500])
def test_chol_tridiag_closed_form(orc, n):
    f, info = orc.potrf(gen.tridiag_121(n))
    assert info == 0
    k = np.arange(1, n + 1, dtype=np.float64)
    diag = np.sqrt((k + 1) / k)
    sub = -np.sqrt(k[:-1] / (k[:-1] + 1))
    np.testing.assert_allclose(np.diag(f), diag, rtol=32 * U64, atol=0)
    np.testing.assert_allclose(np.diag(f, -1), sub, rtol=32 * U64, atol=0)
    assert np.all(np.tril(f, -2) == 0)


def test_chol_special_cases(orc):
    f, info = orc.potrf(np.array([[9.0]]))
    assert info == 0 and f[0, 0] == 3.0
    d = np.diag([4.0, 2.0, 0.25, 1e6])
    f, info = orc.potrf(d)
    assert info == 0 and np.array_equal(np.tril(f), np.diag(np.sqrt([4.0, 2.0, 0.25, 1e6])))
    f, info = orc.potrf(np.eye(17))
    assert info == 0 and np.array_equal(np.tril(f), np.eye(17))
    f, info = orc.potrf(np.zeros((0, 0)))
    assert info == 0


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (4, 3), (5, 4), (6, 5), (6, 6)])
def test_chol_bruteforce_minors(orc, n, seed):
    a = gen.spd_bbt(n, seed=seed)
    ref = exact.cholesky_lower(a)
    f, info = orc.potrf(a)
    assert info == 0
    np.testing.assert_allclose(np.tril(f), ref, rtol=0, atol=16 * n * U64 * np.abs(ref).max())


@pytest.mark.parametrize("n", [300])
def test_chol_residual_bound(orc, n):
    a = gen.spd_bbt(n, seed=11)
    f, info = orc.potrf(a)
    lo = np.tril(f)
    assert info == 0
    res = np.linalg.norm(a - lo @ lo.T) / np.linalg.norm(a)
    assert res <= 10 * n * U64


@pytest.mark.parametrize("k", [1, 5, 40])
def test_chol_not_positive_definite(orc, k):
    n = 40
    a = gen.spd_bbt(n, seed=2)
    good, _ = orc.potrf(a)
    bad = a.copy(order="F")
    bad[k - 1, k - 1] = -1.0
    f, info = orc.potrf(bad)
    assert info == k
    # the failing pivot keeps its updated (Schur complement) value, which is not > 0
    assert f[k - 1, k - 1] <= -1.0 and (k > 1 or f[0, 0] == -1.0)
    # columns before k are the true factor's leading columns
    np.testing.assert_array_equal(np.tril(f[: k - 1, : k - 1]), np.tril(good[: k - 1, : k - 1]))
    nanm = a.copy(order="F")
    nanm[k - 1, k - 1] = np.nan
    assert orc.potrf(nanm)[1] == k
    zero = a.copy(order="F")
    zero[k - 1, k - 1] = 0.0
    zero[k - 1, : k - 1] = 0.0
    zero[:, k - 1] = 0.0
    assert orc.potrf(zero)[1] == k


# --------------------------------------------------------------------- LU

@pytest.mark.parametrize("m,n", [(1, 1), (7, 7), (64, 64), (200, 200), (300, 120), (120, 300), (1, 5), (5, 1)])
def test_lu_exact_dyadic(orc, m, n):
    a, perm, lo, up = gen.exact_lu(m, n, seed=m * 1000 + n)
    lu, ipiv, info = orc.getrf(a)
    k = min(m, n)
    assert info == 0
    ipiv_ref, rows = gen.exact_lu_pivots(perm, k)
    assert np.array_equal(ipiv, ipiv_ref)
    L, U = orc.unpack_lu(lu)
    assert np.array_equal(L, lo[rows])
    assert np.array_equal(U, up)


@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (2, 2, 1), (3, 3, 2), (4, 4, 3), (5, 5, 4), (5, 3, 5), (3, 5, 6), (6, 6, 7)])
def test_lu_bruteforce_minors(orc, m, n, seed):
    s = seed
    while True:
        a = gen.general_uniform(m, n, seed=s)
        ref = exact.lu_partial_pivoting(a)
        if ref is not None:
            break
        s += 100
    ipiv_ref, L_ref, U_ref = ref
    lu, ipiv, info = orc.getrf(a)
    L, U = orc.unpack_lu(lu)
    assert info == 0
    assert np.array_equal(ipiv, ipiv_ref)
    tol = 64 * max(m, n) * U64
    np.testing.assert_allclose(L, L_ref, rtol=0, atol=tol)
    np.testing.assert_allclose(U, U_ref, rtol=0, atol=tol * max(1.0, np.abs(U_ref).max()))


@pytest.mark.parametrize("n", [2, 10, 53])
def test_lu_wilkinson_ties(orc, n):
    lu, ipiv, info = orc.getrf(gen.wilkinson(n))
    assert info == 0
    assert np.array_equal(ipiv, np.arange(1, n + 1))  # every pivot is an exact tie: lowest index wins
    L, U = orc.unpack_lu(lu)
    assert np.array_equal(U[:, n - 1], 2.0 ** np.arange(n))
    assert np.array_equal(np.tril(L, -1), -np.tril(np.ones((n, n)), -1))
    assert np.array_equal(np.diag(U)[:-1], np.ones(n - 1))


def test_lu_margin_pins(orc):
    """The pivot lead reported for the near-tie triage: every Wilkinson pivot is
    an exact tie (lead 0, the last step has no rival: lead 1); on the exact
    dyadic construction the pivot's multiplier is 1 and every other one at most
    1/2 (lead >= 1/2); a hand-checked 3x3 first column (3, -2, 1) gives 1/3;
    and the factorization itself is the plain oracle's, bit for bit."""
    n = 40
    lu, ipiv, info, margin = orc.getrf_margin(gen.wilkinson(n))
    assert info == 0 and np.array_equal(ipiv, np.arange(1, n + 1))
    assert np.array_equal(margin, np.r_[np.zeros(n - 1), 1.0])
    a, perm, _, _ = gen.exact_lu(60, 60, seed=3)
    lu, ipiv, info, margin = orc.getrf_margin(a)
    assert (margin >= 0.5).all()
    ref, rpiv, rinfo = orc.getrf(a)
    assert np.array_equal(lu, ref) and np.array_equal(ipiv, rpiv) and info == rinfo
    h = np.asfortranarray([[3.0, 1.0, 0.0], [-2.0, 4.0, 1.0], [1.0, 0.0, 5.0]])
    _, ipiv, _, margin = orc.getrf_margin(h)
    assert ipiv[0] == 1 and margin[0] == (3.0 - 2.0) / 3.0
    g = gen.general_uniform(257, 190, seed=9)
    lu, ipiv, info, margin = orc.getrf_margin(g)
    ref, rpiv, rinfo = orc.getrf(g)
    assert np.array_equal(lu, ref) and np.array_equal(ipiv, rpiv)
    assert ((margin > 0) & (margin <= 1)).all()


def test_lu_diag_dominant_no_interchange(orc):
    n = 300
    lu, ipiv, info = orc.getrf(gen.diag_dominant(n, seed=5))
    assert info == 0 and np.array_equal(ipiv, np.arange(1, n + 1))


def _swap_sequence_of_permutation(pm):
    """ipiv that partial pivoting takes on the permutation matrix pm: at step k the
    single nonzero of column k sits at the current position of that row."""
    n = pm.shape[0]
    rows = pm.copy()
    ipiv = []
    for k in range(n):
        p = int(np.flatnonzero(rows[:, k])[0])
        ipiv.append(p + 1)
        rows[[k, p]] = rows[[p, k]]
    return np.array(ipiv)


@pytest.mark.parametrize("n", [1, 6, 33])
def test_lu_permutation_matrices(orc, n):
    pm = np.eye(n)[gen.rng(n).permutation(n)]
    for a in (pm, np.eye(n)[::-1]):
        lu, ipiv, info = orc.getrf(a)
        L, U = orc.unpack_lu(lu)
        assert info == 0
        assert np.array_equal(L, np.eye(n)) and np.array_equal(U, np.eye(n))
        assert np.array_equal(ipiv, _swap_sequence_of_permutation(a))


@pytest.mark.parametrize("m,n", [(300, 300), (400, 250), (250, 400)])
def test_lu_residual_and_multipliers(orc, m, n):
    a = gen.general_uniform(m, n, seed=m + n)
    lu, ipiv, info = orc.getrf(a)
    L, U = orc.unpack_lu(lu)
    assert info == 0
    assert np.abs(L).max() <= 1.0
    assert np.all(ipiv >= np.arange(1, min(m, n) + 1)) and np.all(ipiv <= m)
    res = np.linalg.norm(orc.apply_ipiv(a, ipiv) - L @ U) / np.linalg.norm(a)
    assert res <= 10 * max(m, n) * U64


def test_lu_zero_pivot_completes(orc):
    n = 30
    a = gen.general_uniform(n, n, seed=9)
    a[:, 4] = 0.0      # column 5 (1-based) is zero: U(5,5) = 0 exactly
    a[:, 17] = a[:, 3]  # column 18 duplicates column 4: another exact zero pivot, later
    lu, ipiv, info = orc.getrf(a)
    assert info == 5
    L, U = orc.unpack_lu(lu)
    assert U[4, 4] == 0.0
    res = np.linalg.norm(orc.apply_ipiv(a, ipiv) - L @ U) / np.linalg.norm(a)
    assert res <= 10 * n * U64


def test_lu_lapack_context(orc):
    """Context, not the pin: LAPACK's dgetrf (SciPy) follows the same definition."""
    from scipy.linalg import lapack

    a = gen.general_uniform(150, 150, seed=21)
    lu, ipiv, _ = orc.getrf(a)
    lu2, piv2, info2 = lapack.dgetrf(a)
    assert info2 == 0 and np.array_equal(ipiv, piv2 + 1)
    np.testing.assert_allclose(lu, lu2, atol=1e-12)
    s = gen.spd_bbt(150, seed=21)
    f, _ = orc.potrf(s)
    f2, info3 = lapack.dpotrf(s, lower=1)
    assert info3 == 0
    np.testing.assert_allclose(np.tril(f), np.tril(f2), atol=1e-12)


def test_bitwise_independent_of_threads(orc):
    a = gen.general_uniform(257, 257, seed=1)
    s = gen.spd_bbt(257, seed=1)
    prev = orc.get_threads()
    try:
        orc.set_threads(1)
        r1 = orc.getrf(a), orc.potrf(s)
        orc.set_threads(4)
        r4 = orc.getrf(a), orc.potrf(s)
    finally:
        orc.set_threads(prev)
    assert np.array_equal(r1[0][0], r4[0][0]) and np.array_equal(r1[0][1], r4[0][1])
    assert np.array_equal(r1[1][0], r4[1][0])


# --------------------------------------------------------------------- solves

@pytest.mark.parametrize("uplo", ["L", "U"])
def test_potrs_exact(orc, uplo):
    n = 120
    a, lo = gen.exact_chol(n, seed=4)
    x = gen.rng(4).integers(-5, 6, size=(n, 3)).astype(np.float64)
    b = a @ x  # exact: small integers
    f, info = orc.potrf(a, uplo)
    assert info == 0
    assert np.array_equal(orc.potrs(f, b, uplo), x)


@pytest.mark.parametrize("trans", ["N", "T"])
def test_getrs_exact(orc, trans):
    n = 150
    a, perm, lo, up = gen.exact_lu(n, n, seed=8)
    x = gen.rng(8).integers(-5, 6, size=(n, 2)).astype(np.float64)
    b = (a if trans == "N" else a.T) @ x
    lu, ipiv, info = orc.getrf(a)
    assert np.array_equal(orc.getrs(lu, ipiv, b, trans), x)


def test_solves_residual(orc):
    n = 200
    a = gen.general_uniform(n, n, seed=2)
    b = gen.general_uniform(n, 4, seed=3)
    lu, ipiv, _ = orc.getrf(a)
    for trans, op in (("N", a), ("T", a.T)):
        x = orc.getrs(lu, ipiv, b, trans)
        eta, _ = orc.backward_error(op, x, b)
        assert eta <= 10 * n * U64
    s = gen.spd_bbt(n, seed=2)
    f, _ = orc.potrf(s)
    x = orc.potrs(f, b)
    assert orc.backward_error(s, x, b)[0] <= 10 * n * U64


# --------------------------------------------------------------------- mixed precision pre/post

def test_scale_spd_properties(orc):
    n = 64
    a, _, _ = gen.conditioned(n, 1e6, "spd", seed=1)
    a = a * np.exp(gen.rng(2).uniform(-20, 20, size=n))[:, None]
    a = a * np.exp(gen.rng(2).uniform(-20, 20, size=n))[None, :] * 0 + a  # keep symmetric input
    a = (a + a.T) / 2
    a[np.diag_indices(n)] = np.abs(a[np.diag_indices(n)]) + 1e-3
    d, s = orc.scale_spd_f32(a, "L")
    e = np.log2(d)
    assert np.array_equal(e, np.round(e))  # powers of two
    sd = np.diag(s).astype(np.float64)
    assert np.all(sd >= 1.0) and np.all(sd < 4.0)
    s64 = (d[:, None] * a) * d[None, :]
    lo = np.tril_indices(n)
    # the binary64 scaling is exact: dividing back recovers A bit for bit
    assert np.array_equal((s64 / d[:, None] / d[None, :])[lo], a[lo])
    # float32 is the round-to-nearest of the exact scaled value
    err = np.abs(s[lo].astype(np.float64) - s64[lo])
    assert np.all(err <= np.spacing(np.abs(s[lo])).astype(np.float64) / 2 * (1 + 1e-12))
    assert np.all(s[np.triu_indices(n, 1)] == 0)


def test_scale_ge_properties(orc):
    n = 50
    a = gen.general_uniform(n, n, seed=3) * np.exp(gen.rng(7).uniform(-30, 30, size=n))[:, None]
    a[:, 7] = 0.0
    r, c, s = orc.scale_ge_f32(a)
    for v in (r, c):
        e = np.log2(v)
        assert np.array_equal(e, np.round(e))
    ra = r[:, None] * a
    rowmax = np.abs(ra).max(axis=1)
    assert np.all((rowmax >= 1) & (rowmax < 2))
    colmax = np.abs(ra * c[None, :]).max(axis=0)
    nz = colmax > 0
    assert np.all((colmax[nz] >= 1) & (colmax[nz] < 2)) and c[7] == 1.0
    s64 = ra * c[None, :]
    assert np.array_equal(s.astype(np.float64), s64.astype(np.float32).astype(np.float64))


def test_backward_error_definition(orc):
    a = np.array([[2.0, 1.0], [0.0, 4.0]])
    x = np.array([1.0, 1.0])
    b = np.array([3.0, 4.0])
    assert orc.backward_error(a, x, b)[0] == 0.0
    b2 = np.array([3.5, 4.0])  # r = (0.5, 0); ||A||inf = 4, ||x|| = 1, ||b|| = 4
    assert orc.backward_error(a, x, b2)[0] == 0.5 / (4.0 + 4.0)
    s = gen.spd_bbt(20, seed=1)
    y = gen.general_uniform(20, 2, seed=4)
    bb = s @ y + 1e-9
    e1 = orc.backward_error(s, y, bb, "L")[0]
    e2 = orc.backward_error(4.0 * s, y, 4.0 * bb, "N")[0]
    assert e1 == pytest.approx(e2, rel=1e-12)


# ------------------------------------------------ triangular inverse / product

@pytest.mark.parametrize("n,s", [(1, 2.0), (9, 2.0), (40, 2.0), (300, 1.0), (120, -1.0)])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_trtri_bidiagonal_closed_form(orc, n, s, uplo):
    lo = gen.unit_bidiagonal(n, s)
    t = lo if uplo == "L" else lo.T.copy(order="F")
    x, info = orc.trtri(t, uplo, "N")
    assert info == 0
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    closed = np.where(i >= j, (-s) ** np.maximum(i - j, 0), 0.0)
    if uplo == "U":
        closed = closed.T
    tri = np.tril if uplo == "L" else np.triu
    assert np.array_equal(tri(x), closed)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (4, 2), (6, 3)])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_trtri_bruteforce_adjugate(orc, n, seed, uplo):
    g = np.random.default_rng(seed)
    t = g.integers(-5, 6, size=(n, n)).astype(np.float64)
    t = np.tril(t) if uplo == "L" else np.triu(t)
    t[np.diag_indices(n)] = g.choice([-3.0, -2.0, 1.0, 3.0, 5.0, 7.0], size=n)
    x, info = orc.trtri(t, uplo, "N")
    assert info == 0
    inv = exact.inverse(t)
    ref = np.array([[float(v) for v in row] for row in inv])
    tri = np.tril if uplo == "L" else np.triu
    # each entry is within a few rounding errors of the exact rational value
    scale = np.abs(ref).max()
    assert np.abs(tri(x) - ref).max() <= 64 * n * U64 * scale
    # the other triangle of the exact inverse is zero
    assert np.all(ref[np.triu_indices(n, 1) if uplo == "L" else np.tril_indices(n, -1)] == 0)


def test_trtri_diagonal_and_unit(orc):
    d = np.array([4.0, -2.0, 3.0, 0.1, 7.0])
    x, info = orc.trtri(np.diag(d), "L", "N")
    assert info == 0 and np.array_equal(np.diag(x), 1.0 / d)
    # unit diagonal: the stored diagonal is never read and never written
    t = gen.triangular(30, "L", "U", seed=4)
    t[np.diag_indices(30)] = np.nan
    x, info = orc.trtri(t, "L", "U")
    assert info == 0 and np.isnan(np.diag(x)).all()
    ref = t.copy()
    ref[np.diag_indices(30)] = 1.0
    xx = np.tril(x, -1) + np.eye(30)
    assert np.abs(ref @ xx - np.eye(30)).max() <= 30 * 30 * U64


@pytest.mark.parametrize("uplo", ["L", "U"])
def test_trtri_zero_pivot_reported_before_writing(orc, uplo):
    t = gen.triangular(12, uplo, "N", seed=5)
    t[7, 7] = 0.0
    t[9, 9] = 0.0
    x, info = orc.trtri(t, uplo, "N")
    assert info == 8
    assert np.array_equal(x, t)
    # the same matrix with diag = 'U' has nothing to report
    _, info = orc.trtri(t, uplo, "U")
    assert info == 0


@pytest.mark.parametrize("n", [50, 333])
def test_trtri_residual_and_transpose(orc, n):
    t = gen.triangular(n, "L", "N", seed=n)
    x, info = orc.trtri(t, "L", "N")
    assert info == 0
    xl = np.tril(x)
    res = np.abs(t @ xl - np.eye(n)).max()
    assert res <= 4 * n * U64 * np.abs(t).max() * np.abs(xl).max() * n
    # T upper = Lᵀ: its inverse is the transpose (up to summation order)
    xu, info = orc.trtri(t.T.copy(order="F"), "U", "N")
    assert info == 0
    assert np.abs(np.triu(xu) - xl.T).max() <= 8 * n * U64 * np.abs(xl).max()
    # strict other triangle untouched
    assert np.all(np.triu(x, 1) == 0)


@pytest.mark.parametrize("n", [1, 5, 64, 129])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_lauum_exact_integers(orc, n, uplo):
    g = np.random.default_rng(n)
    t = g.integers(-3, 4, size=(n, n))
    t = np.tril(t) if uplo == "L" else np.triu(t)
    ref = t.T @ t if uplo == "L" else t @ t.T          # integer matrix product, exact
    s = t.astype(np.float64, order="F")
    other = np.triu_indices(n, 1) if uplo == "L" else np.tril_indices(n, -1)
    s[other] = np.nan
    out = orc.lauum(s, uplo)
    tri = np.tril if uplo == "L" else np.triu
    assert np.array_equal(tri(np.nan_to_num(out, nan=0.0)), tri(ref).astype(np.float64))
    assert np.isnan(out[other]).all()


def test_lauum_identity_and_diagonal(orc):
    assert np.array_equal(orc.lauum(np.eye(7), "L"), np.eye(7))
    d = np.diag([3.0, -2.0, 0.5])
    assert np.array_equal(orc.lauum(d, "U"), d * d)


@pytest.mark.parametrize("n", [1, 7, 200])
@pytest.mark.parametrize("uplo", ["L", "U"])
def test_potri_exact_bidiagonal(orc, n, uplo):
    lo = gen.unit_bidiagonal(n, 1.0)
    a = lo @ lo.T                        # tridiagonal, integers
    x, info = orc.potri(a, uplo)
    assert info == 0
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    closed = ((-1.0) ** (i + j)) * (n - np.maximum(i, j))   # inv(L)ᵀ·inv(L)
    tri = np.tril if uplo == "L" else np.triu
    assert np.array_equal(tri(x), tri(closed))
    assert np.abs(a @ closed - np.eye(n)).max() == 0


def test_potri_residual(orc):
    n = 160
    a = gen.spd_bbt(n, seed=9)
    x, info = orc.potri(a, "L")
    assert info == 0
    full = np.tril(x) + np.tril(x, -1).T
    assert np.abs(a @ full - np.eye(n)).max() <= 10 * n * U64 * np.abs(a).sum(1).max() * np.abs(full).sum(1).max()
    _, info = orc.potri(-a, "L")
    assert info == 1


# ---- complex instances (c/z types) --------------------------------------------------

U64C = 2.0 ** -53


@pytest.mark.parametrize("n", [1, 5, 33, 120])
def test_zpotrf_exact_gaussian_integer_factor(orc, n):
    a, lo = gen.exact_zchol(n, seed=n)
    f, info = orc.zpotrf(a, "L")
    assert info == 0
    assert np.array_equal(np.tril(f), lo)
    # upper: A = Uᴴ·U with U = Lᴴ, the strict lower triangle never touched
    s = a.copy(order="F")
    s[np.tril_indices(n, -1)] = np.nan
    f, info = orc.zpotrf(s, "U")
    assert info == 0 and np.array_equal(np.triu(f), lo.conj().T)
    assert np.isnan(f[np.tril_indices(n, -1)]).all()


def test_zpotrf_2x2_closed_form(orc):
    # A = [[4, conj(b)], [b, 6]], b = 2+2i: l11 = 2, l21 = b/2 = 1+i, l22 = sqrt(6 - |b|²/4) = 2
    a = np.array([[4.0, 2 - 2j], [2 + 2j, 6.0]], dtype=np.complex128, order="F")
    f, info = orc.zpotrf(a, "L")
    assert info == 0
    assert np.array_equal(np.tril(f), np.array([[2, 0], [1 + 1j, 2]], dtype=np.complex128))


def test_zpotrf_real_input_is_the_real_cholesky(orc):
    a = gen.spd_bbt(70, seed=3)
    f, info = orc.zpotrf(a.astype(np.complex128), "L")
    fr, rinfo = orc.potrf(a, "L")
    assert info == rinfo == 0
    assert np.array_equal(np.tril(f).real, np.tril(fr)) and not np.tril(f).imag.any()


def test_zpotrf_residual_and_failure(orc):
    n = 150
    a = gen.hpd_bbh(n, seed=1)
    f, info = orc.zpotrf(a, "L")
    lo = np.tril(f)
    assert info == 0
    assert np.linalg.norm(a - lo @ lo.conj().T) <= 10 * n * U64C * np.linalg.norm(a)
    assert not np.diag(lo).imag.any() and (np.diag(lo).real > 0).all()
    bad = a.copy(order="F")
    bad[40, 40] = -1.0e4
    _, info = orc.zpotrf(bad, "L")
    assert info == 41


@pytest.mark.parametrize("n", [1, 6, 40, 100])
def test_zgetrf_exact_dyadic(orc, n):
    a, perm, lo, up = gen.exact_zlu(n, seed=n)
    f, ipiv, info = orc.zgetrf(a)
    assert info == 0
    ipiv_ref, rows = gen.exact_lu_pivots(perm, n)
    assert np.array_equal(ipiv, ipiv_ref)
    assert np.array_equal(np.tril(f, -1) + np.eye(n), lo[rows]) and np.array_equal(np.triu(f), up)


def test_zgetrf_pivot_rule_is_re_plus_im(orc):
    # |3| = 3 > |2+2i| = 2.83, but |re| + |im| picks 2+2i (LAPACK's izamax)
    a = np.array([[3.0, 1.0], [2 + 2j, 1.0]], dtype=np.complex128, order="F")
    _, ipiv, _ = orc.zgetrf(a)
    assert ipiv[0] == 2
    # a tie in |re| + |im| (3 against 1.5+1.5i) keeps the first row
    a = np.array([[3.0, 1.0], [1.5 + 1.5j, 1.0]], dtype=np.complex128, order="F")
    _, ipiv, _ = orc.zgetrf(a)
    assert ipiv[0] == 1


def test_zgetrf_real_input_and_zero_pivot(orc):
    a = gen.general_uniform(90, 90, seed=4)
    f, ipiv, info = orc.zgetrf(a.astype(np.complex128))
    fr, ipr, infor = orc.getrf(a)
    assert info == infor == 0 and np.array_equal(ipiv, ipr)
    assert np.abs(f.imag).max() == 0.0
    assert np.linalg.norm(f.real - fr) <= 1e-13 * np.linalg.norm(fr)
    z = gen.general_complex(30, 30, seed=5)
    z[:, 7] = 0.0
    _, _, info = orc.zgetrf(z)
    assert info == 8


def test_zgetrf_residual(orc):
    m, n = 160, 120
    a = gen.general_complex(m, n, seed=6)
    f, ipiv, info = orc.zgetrf(a)
    assert info == 0
    k = min(m, n)
    lo = np.tril(f[:, :k], -1) + np.eye(m, k)
    up = np.triu(f[:k, :])
    # |re| + |im| of every candidate is at most the pivot's, so
    # |l| <= (|re| + |im| of a) / |p| <= √2 (the modulus bound of izamax pivoting)
    assert np.abs(lo).max() <= np.sqrt(2.0) * (1 + 1e-15)
    pa = orc.apply_ipiv(a, ipiv)
    assert np.linalg.norm(pa - lo @ up) <= 10 * n * U64C * np.linalg.norm(a)
