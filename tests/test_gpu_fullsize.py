"""Full-size checks: dpotrf / dgetrf on the benchmark's matrices (n = 16384, the
launch configuration bench.py times), the n = 32768 target size and the tall
65536 × 4096 LU, through the C ABI.

The oracle cannot factor these sizes in test time, so the checks are the
properties that hold at any size, on sampled entries computed one by one in
FP64 from the returned factors:

* Cholesky: (L·Lᵀ)_ij = a_ij within 10·n·u·(|L|·|Lᵀ|)_ij, a positive diagonal,
  and the strict upper triangle untouched.
* LU: (L·U)_ij = (P·A)_ij within 10·n·u·(|L|·|U|)_ij with P replayed from ipiv,
  |l_ij| <= 1, and k+1 <= ipiv[k] <= m.
"""
import numpy as np
import pytest

import gen
import paper_1602_06763_amd as rl
from gpu_util import U64

pytestmark = pytest.mark.gpu

SAMPLES = 512


def _samples(n, m=None, seed=7, lower=False):
    g = np.random.default_rng(seed)
    m = n if m is None else m
    i = g.integers(0, m, size=SAMPLES)
    j = g.integers(0, n, size=SAMPLES)
    # always include the corners and the last row/column
    i[:4] = [0, m - 1, m - 1, min(m, n) - 1]
    j[:4] = [0, 0, n - 1, min(m, n) - 1]
    if lower:
        i, j = np.maximum(i, j), np.minimum(i, j)
    return i, j


def _replay(ipiv, m):
    perm = np.arange(m)
    for k, p in enumerate(ipiv):
        p -= 1
        if p != k:
            perm[k], perm[p] = perm[p], perm[k]
    return perm


def _check_potrf(n, seed):
    import torch

    torch.cuda.set_device(0)
    rl.set_stream(torch.cuda.current_stream())
    A0 = gen.spd_bbt_torch(n, seed=seed, device="cuda")
    A = A0.clone()
    assert A.stride() == (1, n)
    assert rl.potrf(A, "L") == 0
    torch.cuda.synchronize()
    i, j = _samples(n, lower=True)
    ii = torch.from_numpy(i).cuda()
    jj = torch.from_numpy(j).cuda()
    Li = A[ii, :]
    Lj = A[jj, :]
    k = torch.arange(n, device="cuda")
    mask = (k[None, :] <= jj[:, None]).to(torch.float64)
    s = (Li * Lj * mask).sum(1)
    bound = 10 * n * U64 * (Li.abs() * Lj.abs() * mask).sum(1)
    err = (s - A0[ii, jj]).abs()
    assert bool((err <= bound).all()), float((err / bound).max())
    assert bool((torch.diagonal(A) > 0).all())
    # the strict upper triangle is neither read nor written
    iu, ju = _samples(n, seed=11)
    up = torch.from_numpy(np.minimum(iu, ju)).cuda(), torch.from_numpy(np.maximum(iu, ju)).cuda()
    sel = up[0] < up[1]
    assert torch.equal(A[up[0][sel], up[1][sel]], A0[up[0][sel], up[1][sel]])


def _check_getrf(m, n, seed):
    import torch

    torch.cuda.set_device(0)
    rl.set_stream(torch.cuda.current_stream())
    A0 = gen.general_uniform_torch(m, n, seed=seed, device="cuda")
    A = A0.clone()
    assert A.stride() == (1, m)
    mn = min(m, n)
    piv = torch.zeros(mn, dtype=torch.int32, device="cuda")
    assert rl.getrf(A, piv) == 0
    torch.cuda.synchronize()
    ipiv = piv.cpu().numpy()
    ks = np.arange(mn)
    assert (ipiv >= ks + 1).all() and (ipiv <= m).all()
    perm = _replay(ipiv, m)
    i, j = _samples(n, m)
    ii = torch.from_numpy(i).cuda()
    jj = torch.from_numpy(j).cuda()
    k = torch.arange(mn, device="cuda")
    Fi = A[ii, :mn]                     # row i: L(i, k) for k < i, U(i, k) for k >= i
    Fj = A[:mn, jj].T                   # column j: U(k, j) for k <= j, L(k, j) for k > j
    Lik = torch.where(k[None, :] < ii[:, None], Fi, (k[None, :] == ii[:, None]).to(torch.float64))
    Ukj = torch.where(k[None, :] <= jj[:, None], Fj, torch.zeros_like(Fj))
    s = (Lik * Ukj).sum(1)
    bound = 10 * max(m, n) * U64 * (Lik.abs() * Ukj.abs()).sum(1)
    pa = A0[torch.from_numpy(perm[i]).cuda(), jj]
    err = (s - pa).abs()
    assert bool((err <= bound).all()), float((err / bound).max())
    # multipliers of partial pivoting are bounded by one
    below = ii > jj
    assert bool((A[ii[below], jj[below]].abs() <= 1.0).all())


def test_potrf_n16384_bench_matrix():
    _check_potrf(16384, seed=0)


def test_getrf_n16384_bench_matrix():
    _check_getrf(16384, 16384, seed=1)


def test_getrf_tall_65536x4096():
    _check_getrf(65536, 4096, seed=5)


def test_potrf_n32768():
    _check_potrf(32768, seed=0)


def test_getrf_n32768():
    _check_getrf(32768, 32768, seed=1)
