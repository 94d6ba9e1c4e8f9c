"""Calls from several host threads on one device: each thread has its own
stream and its own matrices; the library runs the calls one at a time per
device (they share the device's status block, exchange records and
workspace), so every thread's results equal the ones of a lone call."""
import threading

import numpy as np
import pytest

import gen
import paper_1602_06763_amd as rl
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def test_concurrent_threads_match_serial():
    import torch

    torch.cuda.set_device(0)
    n = 700
    spd = [gen.spd_bbt(n, seed=s) for s in range(4)]
    ge = [gen.general_uniform(n, n, seed=10 + s) for s in range(4)]

    def run(i, out):
        torch.cuda.set_device(0)
        s = torch.cuda.Stream()
        rl.set_stream(s)
        with torch.cuda.stream(s):
            A = to_dev(spd[i])
            G = to_dev(ge[i])
            piv = torch.zeros(n, dtype=torch.int32, device="cuda")
            s.synchronize()
            ok = []
            for _ in range(3):
                A2 = A.clone()
                G2 = G.clone()
                s.synchronize()
                ok.append((rl.potrf(A2, "L"), rl.getrf(G2, piv)))
            out[i] = (to_host(A2), to_host(G2), piv.cpu().numpy(), ok)

    serial = {}
    for i in range(4):
        run(i, serial)
    par = {}
    th = [threading.Thread(target=run, args=(i, par)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(4):
        assert all(r == (0, 0) for r in par[i][3])
        assert np.array_equal(np.tril(par[i][0]), np.tril(serial[i][0]))
        assert np.array_equal(par[i][1], serial[i][1])
        assert np.array_equal(par[i][2], serial[i][2])
    rl.set_stream(torch.cuda.current_stream())
