"""Write the stored oracle results that the full-size GPU parity tests compare
against. Calls only ``gen`` (seeded inputs) and ``oracle`` (the CPU
reference); nothing here touches the HIP library.

Files (gzip-compressed JSON text, one per case):

* ``getrf_m{m}_n{n}_seed{s}.json.gz``: the partial-pivoting LU (Sec. 5,
  xgetrf, with partial row pivoting and the lowest-index tie-break) of
  ``gen.general_uniform(m, n, seed)``: the full ipiv, info, every step whose
  pivot leads the runner-up by a relative margin below 1e-9 (the only steps
  where a differently rounded elimination may legitimately pick another row),
  the smallest margin, ||LU||_F and sampled entries of the packed factors.
* ``potrf_n{n}_seed{s}.json.gz``: the Cholesky factor (Sec. 5, xpotrf, lower)
  of ``gen.spd_bbt(n, seed)``: sampled entries of L (hex floats, exact),
  ||L||_F and info.

Usage: python tests/golden/make_golden.py [case ...]   (default: every case)
The largest case (n = 32768 LU) runs for about an hour on 8 cores.
"""
from __future__ import annotations

import gzip
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

NEAR_TIE = 1e-9
SAMPLE_SEED = 7

GETRF_CASES = {
    "getrf_4096": (4096, 4096, 1),
    "getrf_65536x4096": (65536, 4096, 5),
    "getrf_16384": (16384, 16384, 1),
    "getrf_32768": (32768, 32768, 1),
}
POTRF_CASES = {
    "potrf_4096": (4096, 0),
    "potrf_8192": (8192, 0),
    "potrf_16384": (16384, 0),
}


def path_getrf(m, n, seed):
    return os.path.join(HERE, f"getrf_m{m}_n{n}_seed{seed}.json.gz")


def path_potrf(n, seed):
    return os.path.join(HERE, f"potrf_n{n}_seed{seed}.json.gz")


def sample_positions(m, n, count, lower):
    """Seeded positions (rows i, columns j), the four corners first."""
    g = np.random.default_rng(SAMPLE_SEED)
    i = g.integers(0, m, size=count)
    j = g.integers(0, n, size=count)
    k = min(m, n)
    i[:4] = [0, m - 1, m - 1, k - 1]
    j[:4] = [0, 0, n - 1, k - 1]
    if lower:
        i, j = np.maximum(i, j), np.minimum(i, j)
    return i.astype(np.int64), j.astype(np.int64)


def _write(path, obj):
    tmp = path + ".tmp"
    with gzip.open(tmp, "wt", encoding="ascii") as f:
        json.dump(obj, f, separators=(",", ":"))
    os.replace(tmp, path)


def make_getrf(m, n, seed):
    a = gen.general_uniform(m, n, seed)
    t0 = time.time()
    lu, ipiv, info, margin = oracle.getrf_margin(a)
    dt = time.time() - t0
    del a
    ties = np.nonzero(margin < NEAR_TIE)[0]
    i, j = sample_positions(m, n, 1024, lower=False)
    obj = {
        "what": "partial-pivoting LU (xgetrf, Sec. 5) of gen.general_uniform(m, n, seed) by the CPU oracle",
        "m": m, "n": n, "seed": seed, "gen_version": gen.GEN_VERSION, "info": info,
        "ipiv": [int(v) for v in ipiv],
        "near_tie_threshold": NEAR_TIE,
        "near_ties": {str(int(k)): float(margin[k]) for k in ties},
        "min_margin": float(margin.min()) if margin.size else 1.0,
        "fro": float(np.linalg.norm(lu)).hex(),
        "samples": {"i": i.tolist(), "j": j.tolist(), "v": [float(v).hex() for v in lu[i, j]]},
        "oracle_seconds": round(dt, 1), "oracle_threads": oracle.get_threads(),
    }
    _write(path_getrf(m, n, seed), obj)
    return dt


def make_potrf(n, seed):
    a = gen.spd_bbt(n, seed)
    t0 = time.time()
    f, info = oracle.potrf(a, "L")
    dt = time.time() - t0
    del a
    i, j = sample_positions(n, n, 2048, lower=True)
    obj = {
        "what": "Cholesky factor L (xpotrf, Sec. 5, lower) of gen.spd_bbt(n, seed) by the CPU oracle",
        "n": n, "seed": seed, "gen_version": gen.GEN_VERSION, "info": info,
        "fro": float(np.linalg.norm(np.tril(f))).hex(),
        "samples": {"i": i.tolist(), "j": j.tolist(), "v": [float(v).hex() for v in f[i, j]]},
        "oracle_seconds": round(dt, 1), "oracle_threads": oracle.get_threads(),
    }
    _write(path_potrf(n, seed), obj)
    return dt


def main(argv):
    names = argv or list(POTRF_CASES) + list(GETRF_CASES)
    for name in names:
        if name in POTRF_CASES:
            dt = make_potrf(*POTRF_CASES[name])
        elif name in GETRF_CASES:
            dt = make_getrf(*GETRF_CASES[name])
        else:
            raise SystemExit(f"unknown case {name}")
        print(f"{name}: oracle {dt:.1f} s on {oracle.get_threads()} threads", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
