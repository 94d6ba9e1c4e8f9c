"""Autotuner of the batched factorizations: per routine and size bucket, the
leaf size (Cholesky: potf2 crossover 32 or 64; LU: panel width 16 or 32) and
the edge of the workgroup's matrix-core product tiles (32 or 64).

For every routine (dpotrf, spotrf, dgetrf, sgetrf) and bucket (n <= 64,
<= 128, <= 256, <= 512; LU stops at 256) it builds a batch of matrices with
sizes uniform over the bucket (the seeded recipes of the benchmark), times one
batched call per candidate (median of a few after an untimed one, inputs
restored before each), and keeps the fastest. The table is written as the
C++ header the library compiles its defaults from
(``csrc/batched_tune.hpp``, or the path given), with the measured times as
comments. Each matrix's recursion stays free of tuning: these two sizes are
all that is chosen, per bucket.

Usage (on the GPU): python -m paper_1602_06763_amd.autotune [--out PATH] [--count N]
"""
from __future__ import annotations

import argparse
import datetime
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BUCKETS = [(8, 64), (65, 128), (129, 256), (257, 512)]
ROUTINES = ["dpotrf", "spotrf", "dgetrf", "sgetrf"]
LEAVES = {"dpotrf": (32, 64), "spotrf": (32, 64), "dgetrf": (16, 32), "sgetrf": (16, 32)}
TILES = (32, 64)
DEFAULT_LEAF = {"dpotrf": 64, "spotrf": 64, "dgetrf": 32, "sgetrf": 32}


def batch_buffer(ns, seeds, spd, dtype):
    """The batch in one device buffer, matrix i column-major at offset
    sum_{k<i} n_k^2: SPD A = B·Bᵀ + n·I with B the PCG64 draws of gen.spd_bbt
    (the product formed on the device, lower triangle mirrored), general A
    from gen.general_uniform."""
    import numpy as np
    import torch

    import gen

    ns = np.asarray(ns, dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(ns ** 2)])
    buf = torch.empty(int(offs[-1]), dtype=torch.float64, device="cuda")
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(16) as ex:
        for n in np.unique(ns):
            idx = np.nonzero(ns == n)[0]
            n = int(n)
            if spd:
                draws = list(ex.map(lambda i: gen.spd_bbt_draws(n, int(seeds[i])), idx))
                B = torch.from_numpy(np.stack(draws)).cuda()
                A = torch.bmm(B, B.transpose(1, 2).contiguous())
                A = torch.tril(A) + torch.tril(A, -1).transpose(1, 2)
                A.diagonal(dim1=1, dim2=2).add_(float(n))
                for q, i in enumerate(idx):
                    # symmetric: the row-major rows are the columns
                    buf[int(offs[i]):int(offs[i + 1])].copy_(A[q].reshape(-1))
                del B, A
            else:
                mats = list(ex.map(lambda i: gen.general_uniform(n, n, int(seeds[i])), idx))
                for q, i in enumerate(idx):
                    buf[int(offs[i]):int(offs[i + 1])].copy_(torch.from_numpy(mats[q].ravel(order="F")))
    if dtype != torch.float64:
        buf = buf.to(dtype)
    return buf, offs


def time_call(call, buf, src, stream, reps):
    import numpy as np
    import torch

    ts = []
    for r in range(reps + 1):
        buf.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st = call()
        e1.record(stream)
        torch.cuda.synchronize()
        assert st == 0
        if r:
            ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(count: int, reps: int, seed: int = 11):
    import numpy as np
    import torch

    import gen
    import paper_1602_06763_amd as rl

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rl.set_stream(stream)
    table, notes = {}, []
    for routine in ROUTINES:
        lu = routine.endswith("getrf")
        single = routine.startswith("s")
        dtype = torch.float32 if single else torch.float64
        rows = []
        for b, (lo, hi) in enumerate(BUCKETS):
            if lu and lo > 256:
                rows.append((DEFAULT_LEAF[routine], 64, None))
                continue
            ns = gen.batch_sizes(count, lo, hi, seed + 10 * b)
            seeds = gen.batch_seeds(count, seed + 10 * b)
            buf, offs = batch_buffer(ns, seeds, not lu, dtype)
            src = buf.clone()
            esz = buf.element_size()
            ptrs = torch.tensor(buf.data_ptr() + esz * offs[:-1], dtype=torch.int64, device="cuda")
            nv = torch.tensor(ns, dtype=torch.int32, device="cuda")
            info = torch.zeros(count, dtype=torch.int32, device="cuda")
            if lu:
                piv = torch.zeros(int(ns.sum()), dtype=torch.int32, device="cuda")
                pp = torch.tensor(piv.data_ptr() + 4 * np.concatenate([[0], np.cumsum(ns)[:-1]]),
                                  dtype=torch.int64, device="cuda")
                call = lambda: rl.getrf_batched(count, nv, ptrs, nv, pp, info, single=single)
            else:
                call = lambda: rl.potrf_batched("L", count, nv, ptrs, nv, info, single=single)
            best = None
            for leaf in LEAVES[routine]:
                for tile in TILES:
                    assert rl.batched_tune(routine, b, leaf, tile) == 0
                    ms = time_call(call, buf, src, stream, reps)
                    assert int(info.abs().max()) == 0
                    notes.append(f"{routine} n in [{lo}, {hi}] leaf {leaf} tile {tile}: {ms:.3f} ms")
                    print(notes[-1], flush=True)
                    if best is None or ms < best[2]:
                        best = (leaf, tile, ms)
            assert rl.batched_tune(routine, b, best[0], best[1]) == 0
            rows.append(best)
            del buf, src
            torch.cuda.empty_cache()
        table[routine] = rows
    return table, notes


def header(table, notes, count):
    import torch

    dev = torch.cuda.get_device_name(0)
    date = datetime.date.today().isoformat()
    lines = [
        "// Per-size-bucket choices of the batched factorizations: the crossover of",
        "// each matrix's recursion (Cholesky: potf2 leaf 32 or 64; LU: panel width 16",
        "// or 32) and the edge of the workgroup's matrix-core product tiles (32 or 64),",
        "// for the buckets n <= 64, <= 128, <= 256 and above. Each matrix's recursion",
        "// itself stays free of tuning (splits at n/2, rounded to 64); only these two",
        "// sizes are chosen per bucket.",
        "//",
        f"// Written by paper_1602_06763_amd/autotune.py on {dev}, {date}: one batched call",
        f"// of {count} matrices per bucket (sizes uniform over the bucket), median time per",
        "// candidate; the fastest is kept.",
    ]
    lines += [f"//   {t}" for t in notes]
    lines += [
        "#pragma once",
        "",
        "namespace rl {",
        "",
        "constexpr int kBatchBuckets = 4;",
        "__host__ __device__ constexpr int batch_bucket(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3; }",
        "",
        "struct BatchTune {",
        "    unsigned char leaf[kBatchBuckets];",
        "    unsigned char tile[kBatchBuckets];",
        "};",
        "",
        "// routines: dpotrf, spotrf, dgetrf, sgetrf",
        "constexpr BatchTune kTuneDefault[4] = {",
    ]
    for r in ROUTINES:
        rows = table[r]
        leaf = ", ".join(str(x[0]) for x in rows)
        tile = ", ".join(str(x[1]) for x in rows)
        lines.append(f"    {{{{{leaf}}}, {{{tile}}}}},   // {r}")
    lines += ["};", "", "}  // namespace rl", ""]
    return "\n".join(lines)


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--out", default=os.path.join(HERE, "csrc", "batched_tune.hpp"))
    p.add_argument("--count", type=int, default=3000)
    p.add_argument("--reps", type=int, default=3)
    a = p.parse_args(argv)
    table, notes = tune(a.count, a.reps)
    text = header(table, notes, a.count)
    with open(a.out, "w") as f:
        f.write(text)
    print(f"wrote {a.out}")


if __name__ == "__main__":
    main()
