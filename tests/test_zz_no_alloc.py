"""The allocation-free LU (relapack_dgetrf_noalloc) against relapack_dgetrf.

Both run the same kernels in the same order on the same input, one on the
library's grow-only workspace and one on its fixed device array, so ipiv and
the factors must agree bit for bit. Two calls in a row, the second on a
smaller matrix, check that the fixed array's leftover contents (the previous
call's row bookkeeping and exchange records) do not leak into the next call.
The sizes take the batched-interchange path (more than 512 columns) with
several panel workgroups, a ragged tail, and m > n / m < n shapes.
"""
import numpy as np
import pytest

import gen
import paper_1602_06763_amd as rl
from gpu_util import ipiv_dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def _both(a):
    import torch

    m, n = a.shape
    A1, A2 = to_dev(a), to_dev(a)
    p1, p2 = ipiv_dev(min(m, n)), ipiv_dev(min(m, n))
    i1 = rl.getrf(A1, p1)
    i2 = rl.getrf_noalloc(A2, p2)
    torch.cuda.synchronize()
    return (i1, p1.cpu().numpy(), to_host(A1)), (i2, p2.cpu().numpy(), to_host(A2))


def test_noalloc_matches_getrf_twice_shrinking():
    import torch

    torch.cuda.set_device(0)
    rl.set_stream(torch.cuda.current_stream())
    for (m, n, seed) in [(3000, 2100, 11), (1100, 700, 12), (600, 900, 13)]:
        print(f"getrf_noalloc {m}x{n} seed {seed}", flush=True)
        a = gen.general_uniform(m, n, seed)
        (i1, p1, f1), (i2, p2, f2) = _both(a)
        assert i1 == i2 == 0, (i1, i2)
        k = min(m, n)
        assert np.array_equal(p1[:k], p2[:k])
        assert np.array_equal(f1, f2)


def test_noalloc_zero_pivot():
    import torch

    torch.cuda.set_device(0)
    rl.set_stream(torch.cuda.current_stream())
    a = gen.general_uniform(300, 300, 21)
    a[:, 37] = 0.0   # column 38 has no nonzero pivot candidate
    (i1, p1, f1), (i2, p2, f2) = _both(a)
    assert i1 == i2 == 38
    assert np.array_equal(p1, p2) and np.array_equal(f1, f2)
