"""The seeded input generators: determinism, layout and the properties each
recipe promises (they feed both the oracle and the HIP path)."""
import numpy as np

import gen


def test_deterministic_and_column_major():
    a1, a2 = gen.spd_bbt(64, seed=5), gen.spd_bbt(64, seed=5)
    assert np.array_equal(a1, a2) and a1.flags.f_contiguous
    assert not np.array_equal(a1, gen.spd_bbt(64, seed=6))
    g = gen.general_uniform(33, 17, seed=2)
    assert g.shape == (33, 17) and g.flags.f_contiguous
    assert np.abs(g).max() <= 1.0


def test_spd_bbt_is_symmetric_and_well_conditioned():
    a = gen.spd_bbt(256, seed=1)
    assert np.array_equal(a, a.T)
    w = np.linalg.eigvalsh(a)
    assert w.min() > 0 and w.max() / w.min() < 4.0


def test_exact_constructions_are_exact():
    a, lo = gen.exact_chol(300, seed=3)
    assert np.array_equal(a, a.T)
    assert np.array_equal(np.round(a), a)
    a2, perm, L, U = gen.exact_lu(100, 100, seed=2)
    assert np.array_equal(a2 * 4, np.round(a2 * 4))  # dyadic, denominator <= 4
    assert np.abs(np.tril(L, -1)).max() <= 0.5
    assert np.array_equal(np.sort(perm), np.arange(100))


def test_conditioned_has_requested_kappa():
    for kind in ("spd", "general"):
        a, b, x0 = gen.conditioned(80, 1e6, kind, nrhs=2, seed=1)
        s = np.linalg.svd(a, compute_uv=False)
        assert abs(np.log10(s[0] / s[-1]) - 6.0) < 1e-6
        np.testing.assert_allclose(a @ x0, b, rtol=1e-12, atol=1e-12)
