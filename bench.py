#!/usr/bin/env python3
"""Benchmark: recursive FP64 dpotrf / dgetrf at n = 16384 on one MI355X, plus
the mixed-precision + FP64-refinement solves against the FP64 solves.

One step = the whole hot path over one synthetic input set:
  1. dpotrf (lower) of A = B·Bᵀ + n·I, then dpotrs with nrhs right-hand sides
  2. dgetrf of A ~ uniform[-1, 1], then dgetrs
  3. dposv_mixed and dgesv_mixed (low-precision matrix-core updates, FP64
     refinement to eta <= 1e-14) on kappa-conditioned test matrices, same n
Every matrix is restored from a pristine device copy before it is factored
(untimed). ``value`` is the FP64 factorization throughput
(n³/3 + 2n³/3) / (t_potrf + t_getrf) in TFLOP/s, from HIP events around each
library call on the library stream; inputs are resident in HBM before timing
starts. The timed steps run without per-kernel instrumentation; one more
dpotrf + dgetrf pass right after them records HIP events around every kernel
launch (library tracing) for the kernel-family breakdown and the roofline of
the dominant kernel, the FP64 matrix-core GEMM on 128×128 tiles.

``target_size`` additionally times one dpotrf and one dgetrf at n = 32768
(``--target-n``), the size at which the FP64 matrix-core fraction is targeted;
``spd_inverse`` times dpotri (dtrtri + dlauum of the Cholesky factor) at
n = 8192 (``--inv-n``); ``variants`` times dpotrf with uplo = 'U' and the
single-precision spotrf / sgetrf at the benchmark size (``--no-variants``
skips them); ``batched`` times one call of each batched routine over 20000
matrices of uneven sizes (``--batch-count``; SPD n in [8, 512], general n in
[8, 256]) in FP64 and FP32; ``--mixed-sweep`` adds the mixed solves over
kappa in {1e2, 1e6, 1e10} x nrhs in {1, 16, 64} x {fp32, fp16, bf16}.

Prints ONE JSON line. ``--gpus N`` with N > 1 exits: the library runs on one GPU.
``--copy-calib MB`` only runs a plain device copy of that size 20 times (the
reference point for the HBM byte counters) and prints nothing else.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6   # TFLOP/s, MI355X FP64 matrix (published, dense)
PEAK_FP32 = 157.3  # TFLOP/s, MI355X FP32 matrix (published, dense)
PEAK_HBM = 8000.0  # GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_k1_fp64_traffic_potrf_getrf_n16384.md")
GEMM_SOURCES = [os.path.join(ROOT, "paper_1602_06763_amd", "csrc", "gemm.hip")]   # the GEMM kernel's source


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--nrhs", type=int, default=1)
    p.add_argument("--kappa", type=float, default=1e2)
    p.add_argument("--prec", default="fp16")
    p.add_argument("--no-mixed", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-n", type=int, default=8192)
    p.add_argument("--cpu-n1", type=int, default=2048, help="size of the one-thread oracle sample (0 skips it)")
    p.add_argument("--copy-calib", type=float, default=0.0, help="MB; run only a plain device copy")
    p.add_argument("--target-n", type=int, default=32768,
                   help="also time one dpotrf + dgetrf at this size (0: skip)")
    p.add_argument("--no-variants", action="store_true", help="skip the uplo = 'U' and FP32 timings")
    p.add_argument("--mixed-sweep", action="store_true",
                   help="also time the mixed solves over kappa x nrhs x precision (about a minute)")
    p.add_argument("--batch-count", type=int, default=20000,
                   help="matrices per batched routine (SPD n in [8, 512], general n in [8, 256]); 0 skips")
    p.add_argument("--inv-n", type=int, default=8192,
                   help="also time the SPD inverse (dtrtri + dlauum of a dpotrf factor) at this size (0: skip)")
    return p.parse_args()


def gemm_source_hash() -> str:
    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the FP64 GEMM family from the FETCH_SIZE /
    WRITE_SIZE counter runs, if they were taken on the current GEMM source."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    kv = dict(re.findall(r"^\s*([a-z_0-9]+):\s*(\S+)\s*$", text, flags=re.M))
    if kv.get("gemm_source_sha256") != gemm_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_pass(n: int):
    import gen
    import oracle

    a = gen.spd_bbt(n, seed=0)
    g = gen.general_uniform(n, n, seed=0)
    t0 = time.perf_counter()
    _, i1 = oracle.potrf(a)
    t1 = time.perf_counter()
    _, _, i2 = oracle.getrf(g)
    t2 = time.perf_counter()
    assert i1 == 0 and i2 == 0
    flops = n ** 3 / 3.0 + 2.0 * n ** 3 / 3.0
    return flops / (t2 - t0) / 1e12, t1 - t0, t2 - t1


def cpu_baseline(n: int, n1: int):
    """The oracle (unblocked FP64 Cholesky + partial-pivoting LU) on one n×n
    instance of each workload on all of this host's cores, and on one n1×n1
    instance of each with one thread."""
    import oracle

    oracle.build(force=False)
    threads = oracle.get_threads()
    v, tp, tg = _oracle_pass(n)
    out = {"value": v, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"oracle dpotrf + dgetrf, one n={n} instance each (same generators), "
                     f"{tp:.1f} s + {tg:.1f} s"}
    if n1 > 0:
        oracle.set_threads(1)
        try:
            v1, tp1, tg1 = _oracle_pass(n1)
        finally:
            oracle.set_threads(threads)
        out["single_core"] = {"value": v1, "unit": "TFLOP/s", "cores": 1,
                              "sample": f"one n={n1} instance each, {tp1:.1f} s + {tg1:.1f} s"}
    return out


def target_size(n: int, stream):
    """One dpotrf and one dgetrf at the target size (same generators), each
    after an untimed warm-up call on the same input."""
    import torch

    import gen
    import paper_1602_06763_amd as rl

    res = {"n": n}
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for name, make, flops in (("potrf", lambda: gen.spd_bbt_torch(n, seed=0, device="cuda"), n ** 3 / 3.0),
                              ("getrf", lambda: gen.general_uniform_torch(n, n, seed=1, device="cuda"),
                               2.0 * n ** 3 / 3.0)):
        A0 = make()
        A = A0.clone()
        piv = torch.zeros(n, dtype=torch.int32, device="cuda")
        call = (lambda: rl.potrf(A, "L")) if name == "potrf" else (lambda: rl.getrf(A, piv))
        assert call() == 0
        A.copy_(A0)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        info = call()
        e1.record(stream)
        torch.cuda.synchronize()
        assert info == 0
        ms = e0.elapsed_time(e1)
        res[name + "_ms"] = round(ms, 3)
        res[name + "_tflops"] = round(flops / (ms * 1e-3) / 1e12, 3)
        res[name + "_frac_of_fp64_peak"] = round(flops / (ms * 1e-3) / 1e12 / PEAK_FP64, 4)
        del A0, A
        torch.cuda.empty_cache()
    return res


def spd_inverse(n: int, stream, reps: int = 3):
    """dpotri = dtrtri + dlauum on the Cholesky factor of the n×n SPD input
    (same generator as dpotrf), the factor restored from a pristine copy before
    each untimed-then-timed call; median of ``reps`` timed calls, each with
    the normwise residual ‖A·X − I‖_max of the last one."""
    import numpy as np
    import torch

    import gen
    import paper_1602_06763_amd as rl

    A0 = gen.spd_bbt_torch(n, seed=0, device="cuda")
    F0 = A0.clone()
    assert rl.potrf(F0, "L") == 0
    A = F0.clone()
    ts, tt, tl = [], [], []
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for r in range(reps + 1):
        A.copy_(F0)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        info = rl.potri(A, "L")
        e1.record(stream)
        torch.cuda.synchronize()
        assert info == 0
        if r > 0:
            ts.append(e0.elapsed_time(e1))
    # the two halves separately, for the breakdown
    for r in range(reps):
        A.copy_(F0)
        torch.cuda.synchronize()
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        assert rl.trtri(A, "L", "N") == 0
        e1.record(stream)
        assert rl.lauum(A, "L") == 0
        e2.record(stream)
        torch.cuda.synchronize()
        tt.append(e0.elapsed_time(e1))
        tl.append(e1.elapsed_time(e2))
    X = torch.tril(A) + torch.tril(A, -1).T
    R = A0 @ X
    R.diagonal().sub_(1.0)
    resid = float(R.abs().max()) / (float(A0.abs().sum(1).max()) * float(X.abs().sum(1).max()))
    ms, mt, ml = float(np.median(ts)), float(np.median(tt)), float(np.median(tl))
    fl = 2.0 * n ** 3 / 3.0
    del A0, F0, A, X, R
    torch.cuda.empty_cache()
    return {"n": n, "potri_ms": round(ms, 3), "potri_tflops": round(fl / (ms * 1e-3) / 1e12, 3),
            "potri_frac_of_fp64_peak": round(fl / (ms * 1e-3) / 1e12 / PEAK_FP64, 4),
            "trtri_ms": round(mt, 3), "lauum_ms": round(ml, 3),
            "residual_AX_minus_I_rel": resid,
            "flops": "n^3/3 (dtrtri) + n^3/3 (dlauum)"}


def variants(n: int, stream, reps: int = 3):
    """The other instances at the benchmark size: dpotrf with uplo = 'U' on the
    same SPD input, the single-precision spotrf / sgetrf (FP32 storage and
    FP32 matrix cores) on the FP32-rounded inputs, and the complex zpotrf /
    zgetrf at n = 8192 (the Hermitian and general recipes of ``gen``);
    medians of ``reps`` calls after an untimed one, the input restored before
    each."""
    import numpy as np
    import torch

    import gen
    import paper_1602_06763_amd as rl

    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(call, src, dst):
        ts = []
        for r in range(reps + 1):
            dst.copy_(src)
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record(stream)
            info = call()
            e1.record(stream)
            torch.cuda.synchronize()
            assert info == 0
            if r:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    out = {"n": n}
    A0 = gen.spd_bbt_torch(n, seed=0, device="cuda")
    A = A0.clone()
    ms = timed(lambda: rl.potrf(A, "U"), A0, A)
    out["dpotrf_upper_ms"] = round(ms, 3)
    out["dpotrf_upper_tflops"] = round(n ** 3 / 3.0 / (ms * 1e-3) / 1e12, 3)
    S0 = A0.float().T.contiguous().T
    del A0, A
    S = S0.clone()
    ms = timed(lambda: rl.spotrf(S, "L"), S0, S)
    out["spotrf_ms"] = round(ms, 3)
    out["spotrf_tflops"] = round(n ** 3 / 3.0 / (ms * 1e-3) / 1e12, 3)
    del S0, S
    G0 = gen.general_uniform_torch(n, n, seed=1, device="cuda").float().T.contiguous().T
    G = G0.clone()
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    ms = timed(lambda: rl.sgetrf(G, piv), G0, G)
    out["sgetrf_ms"] = round(ms, 3)
    out["sgetrf_tflops"] = round(2.0 * n ** 3 / 3.0 / (ms * 1e-3) / 1e12, 3)
    out["fp32_matrix_peak_tflops"] = PEAK_FP32
    del G0, G
    torch.cuda.empty_cache()
    # complex instances at n = 8192 (complex flops counted in real operations:
    # 4n³/3 for the Cholesky, 8n³/3 for the LU), against the FP64 matrix peak
    nz = min(n, 8192)
    Z0 = gen.hpd_bbh_torch(nz, seed=0, device="cuda")
    Z = Z0.clone()
    ms = timed(lambda: rl.zpotrf(Z, "L"), Z0, Z)
    out["complex_n"] = nz
    out["zpotrf_ms"] = round(ms, 3)
    out["zpotrf_tflops"] = round(4.0 * nz ** 3 / 3.0 / (ms * 1e-3) / 1e12, 3)
    del Z0, Z
    Z0 = gen.general_complex_torch(nz, nz, seed=1, device="cuda")
    Z = Z0.clone()
    piv = torch.zeros(nz, dtype=torch.int32, device="cuda")
    ms = timed(lambda: rl.zgetrf(Z, piv), Z0, Z)
    out["zgetrf_ms"] = round(ms, 3)
    out["zgetrf_tflops"] = round(8.0 * nz ** 3 / 3.0 / (ms * 1e-3) / 1e12, 3)
    del Z0, Z
    torch.cuda.empty_cache()
    return out


def batched(count: int, stream, reps: int = 3, seed: int = 4):
    """The batched workload of uneven sizes: ``count`` SPD matrices with n
    uniform in [8, 512] and ``count`` general matrices with n uniform in
    [8, 256], sizes and per-matrix seeds from one master seed
    (``gen.batch_sizes`` / ``gen.batch_seeds``), each matrix from the PCG64
    recipes (SPD: the draws of ``gen.spd_bbt``, B·Bᵀ + n·I formed on the
    device; general: ``gen.general_uniform``); each routine one call over its
    whole batch, in FP64 and FP32 (the FP64 inputs rounded). Median of
    ``reps`` calls after an untimed one (the first call captures the launch
    graph), the inputs restored before each. The bound is the per-matrix
    roofline summed over the batch: max(flops / matrix peak, bytes / HBM
    bandwidth) with n³/3 flops and 8n² B (Cholesky), 2n³/3 flops and 16n² B
    (LU), halved bytes in FP32."""
    import numpy as np
    import torch

    import gen
    import paper_1602_06763_amd as rl
    from paper_1602_06763_amd.autotune import batch_buffer

    ev = lambda: torch.cuda.Event(enable_timing=True)
    out = {"count_spd": count, "count_general": count, "n_spd": "U{8..512}", "n_general": "U{8..256}",
           "inputs": "PCG64 per matrix (gen.batch_sizes / batch_seeds, master seeds %d and %d)" % (seed, seed + 2)}

    def build(ns, spd):
        seeds = gen.batch_seeds(len(ns), seed if spd else seed + 2)
        return batch_buffer(ns, seeds, spd, torch.float64)

    def run(name, ns, buf, offs, call, flops, nbytes, peak, ipiv=None):
        esz = buf.element_size()
        ptrs = torch.tensor(buf.data_ptr() + esz * offs[:-1], dtype=torch.int64, device="cuda")
        nv = torch.tensor(ns, dtype=torch.int32, device="cuda")
        info = torch.zeros(len(ns), dtype=torch.int32, device="cuda")
        src = buf.clone()
        ts = []
        for r in range(reps + 1):
            buf.copy_(src)
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record(stream)
            st = call(nv, ptrs, info)
            e1.record(stream)
            torch.cuda.synchronize()
            assert st == 0 and int(info.abs().max()) == 0
            if r:
                ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        n = ns.astype(np.float64)
        fl = float(np.sum(flops(n)))
        bound_s = float(np.sum(np.maximum(flops(n) / (peak * 1e12), nbytes(n) / (PEAK_HBM * 1e9))))
        out[name] = {"ms": round(ms, 3), "matrices_per_s": round(len(ns) / (ms * 1e-3), 1),
                     "tflops": round(fl / (ms * 1e-3) / 1e12, 3), "roofline_bound_ms": round(bound_s * 1e3, 3),
                     "frac_of_bound": round(bound_s * 1e3 / ms, 4)}
        del src
        return ms

    ns_spd = gen.batch_sizes(count, 8, 512, seed)
    ns_ge = gen.batch_sizes(count, 8, 256, seed + 2)
    chol_f, lu_f = (lambda n: n ** 3 / 3.0), (lambda n: 2.0 * n ** 3 / 3.0)
    buf, offs = build(ns_spd, True)
    run("dpotrf", ns_spd, buf, offs, lambda nv, p, info: rl.potrf_batched("L", count, nv, p, nv, info),
        chol_f, lambda n: 8.0 * n * n, PEAK_FP64)
    sb = buf.float()
    del buf
    torch.cuda.empty_cache()
    run("spotrf", ns_spd, sb, offs, lambda nv, p, info: rl.potrf_batched("L", count, nv, p, nv, info, single=True),
        chol_f, lambda n: 4.0 * n * n, PEAK_FP32)
    del sb
    torch.cuda.empty_cache()
    poffs = np.concatenate([[0], np.cumsum(ns_ge.astype(np.int64))])
    piv = torch.zeros(int(poffs[-1]), dtype=torch.int32, device="cuda")
    pp = torch.tensor(piv.data_ptr() + 4 * poffs[:-1], dtype=torch.int64, device="cuda")
    buf, offs = build(ns_ge, False)
    run("dgetrf", ns_ge, buf, offs, lambda nv, p, info: rl.getrf_batched(count, nv, p, nv, pp, info),
        lu_f, lambda n: 16.0 * n * n, PEAK_FP64)
    sb = buf.float()
    del buf
    torch.cuda.empty_cache()
    run("sgetrf", ns_ge, sb, offs, lambda nv, p, info: rl.getrf_batched(count, nv, p, nv, pp, info, single=True),
        lu_f, lambda n: 8.0 * n * n, PEAK_FP32)
    del sb, piv
    torch.cuda.empty_cache()
    return out


def mixed_sweep(n: int, stream, reps: int = 2):
    """The mixed-precision solves over the grid of condition numbers (1e2, 1e6,
    1e10), right-hand-side counts (1, 16, 64) and factorization precisions
    (fp32, fp16, bf16), SPD and general, against the FP64 solve of the same
    system (potrf + potrs, getrf + getrs); each time the median of ``reps``
    calls after an untimed one. One conditioned matrix per kind and condition
    number; smaller right-hand-side counts take the leading columns of b."""
    import numpy as np
    import torch

    import gen
    import paper_1602_06763_amd as rl

    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(call):
        ts, r = [], None
        for i in range(reps + 1):
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record(stream)
            r = call()
            e1.record(stream)
            torch.cuda.synchronize()
            if i:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), r

    rows = []
    for kind in ("spd", "general"):
        fp64 = {}
        for kappa in (1e2, 1e6, 1e10):
            M, b, _ = gen.conditioned_torch(n, kappa, kind, nrhs=64, seed=5, device="cuda")
            for nrhs in (1, 16, 64):
                bb = b[:, :nrhs]
                if nrhs not in fp64:
                    W = torch.empty_like(M.T).T
                    Bw = torch.empty_like(bb.T).T
                    piv = torch.zeros(n, dtype=torch.int32, device="cuda")

                    def solve64():
                        W.copy_(M)
                        Bw.copy_(bb)
                        if kind == "spd":
                            return rl.potrf(W, "L") or rl.potrs(W, Bw, "L")
                        return rl.getrf(W, piv) or rl.getrs(W, piv, Bw, "N")

                    fp64[nrhs], info = timed(solve64)
                    assert info == 0
                    del W, Bw
                X = torch.zeros_like(bb.T).T
                pv = torch.zeros(n, dtype=torch.int32, device="cuda")
                for prec in ("fp32", "fp16", "bf16"):
                    if kind == "spd":
                        ms, r = timed(lambda: rl.posv_mixed(M, bb, X, "L", prec))
                    else:
                        ms, r = timed(lambda: rl.gesv_mixed(M, pv, bb, X, prec))
                    st = rl.mixed_last()
                    rows.append({"kind": kind, "kappa": kappa, "nrhs": nrhs, "prec": prec, "ms": round(ms, 3),
                                 "fp64_solve_ms": round(fp64[nrhs], 3), "speedup": round(fp64[nrhs] / ms, 3),
                                 "info": r[0], "iter": r[1], "berr": r[2], "gmres_from": st["gmres_from"],
                                 "gmres_steps": st["gmres_steps"]})
                del X
            del M, b
            torch.cuda.empty_cache()
    return {"n": n, "cases": rows}


def copy_calibration(mb: float):
    import torch

    n = int(mb * 1e6 / 8)
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(20):
        dst.copy_(src)
    torch.cuda.synchronize()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calib > 0:
        copy_calibration(args.copy_calib)
        return
    import numpy as np
    import torch

    import gen
    import paper_1602_06763_amd as rl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    rl.set_stream(stream)
    n, nrhs = args.n, args.nrhs

    # ---- inputs, resident in HBM before timing ----
    t_gen = time.perf_counter()
    A_spd0 = gen.spd_bbt_torch(n, seed=0, device="cuda")
    A_ge0 = gen.general_uniform_torch(n, n, seed=1, device="cuda")
    colmaj = lambda t: t.T.contiguous().T
    B0 = colmaj(torch.from_numpy(gen.general_uniform(n, nrhs, seed=2)).cuda())
    A_spd = torch.empty_like(A_spd0.T).T
    A_ge = torch.empty_like(A_ge0.T).T
    Bw = torch.empty_like(B0.T).T
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    mixed = not args.no_mixed
    if mixed:
        Ms, bs, _ = gen.conditioned_torch(n, args.kappa, "spd", nrhs=nrhs, seed=3, device="cuda")
        Mg, bg, _ = gen.conditioned_torch(n, args.kappa, "general", nrhs=nrhs, seed=4, device="cuda")
        Xs = torch.zeros_like(bs.T).T
        Xg = torch.zeros_like(bg.T).T
        pivm = torch.zeros(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step():
        out = {}
        A_spd.copy_(A_spd0)
        Bw.copy_(B0)
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        info = rl.potrf(A_spd, "L")
        e1.record(stream)
        info2 = rl.potrs(A_spd, Bw, "L")
        e2.record(stream)
        assert info == 0 and info2 == 0, (info, info2)
        A_ge.copy_(A_ge0)
        Bw.copy_(B0)
        e3, e4, e5 = ev(), ev(), ev()
        e3.record(stream)
        info = rl.getrf(A_ge, piv)
        e4.record(stream)
        info2 = rl.getrs(A_ge, piv, Bw, "N")
        e5.record(stream)
        assert info == 0 and info2 == 0, (info, info2)
        torch.cuda.synchronize()
        out["potrf"] = e0.elapsed_time(e1)
        out["potrs"] = e1.elapsed_time(e2)
        out["getrf"] = e3.elapsed_time(e4)
        out["getrs"] = e4.elapsed_time(e5)
        if mixed:
            f0, f1, f2 = ev(), ev(), ev()
            f0.record(stream)
            r1 = rl.posv_mixed(Ms, bs, Xs, "L", args.prec)
            f1.record(stream)
            r2 = rl.gesv_mixed(Mg, pivm, bg, Xg, args.prec)
            f2.record(stream)
            torch.cuda.synchronize()
            out["posv_mixed"] = f0.elapsed_time(f1)
            out["gesv_mixed"] = f1.elapsed_time(f2)
            out["mixed_spd"] = r1
            out["mixed_ge"] = r2
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res.append(step())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # ---- one traced factorization pass: per-kernel HIP events on the library stream ----
    A_spd.copy_(A_spd0)
    A_ge.copy_(A_ge0)
    torch.cuda.synchronize()
    rl.trace_enable(True)
    assert rl.potrf(A_spd, "L") == 0
    assert rl.getrf(A_ge, piv) == 0
    fam = rl.trace_collect()
    rl.trace_enable(False)

    med = lambda key: float(np.median([r[key] for r in res]))
    t_potrf, t_getrf = med("potrf"), med("getrf")
    fl_potrf, fl_getrf = n ** 3 / 3.0, 2.0 * n ** 3 / 3.0
    value = (fl_potrf + fl_getrf) / ((t_potrf + t_getrf) * 1e-3) / 1e12

    # dominant kernel: the FP64 matrix-core GEMM on 128×128 tiles (the
    # recursion's large Schur-complement updates; the smaller-tile launches
    # are the "gemm" family)
    d = fam.get("gemm128", {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
    launches = max(d["launches"], 1)
    avg_s = d["ms"] * 1e-3 / launches
    achieved = (d["flops"] / launches) / avg_s / 1e12 if d["ms"] > 0 else 0.0
    traffic = measured_traffic()
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64, 4),
                "traffic": round(traffic, 1) if traffic is not None else None,
                "kernel": "gemm_k1<double,...,TRI=0,128,128,*> (FP64 GEMM, 128x128 tiles)",
                "launches": d["launches"], "avg_launch_us": round(avg_s * 1e6, 3),
                "flops_per_launch": round(d["flops"] / launches, 1),
                "algorithmic_bytes_per_launch": round(d["bytes"] / launches, 1)}
    families = {k: {"launches": v["launches"],
                    "ms": round(v["ms"], 3),
                    "avg_us": round(v["ms"] * 1e3 / max(v["launches"], 1), 2),
                    "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) if v["ms"] > 0 and v["flops"] > 0 else None,
                    "gbps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 and v["bytes"] > 0 else None}
                for k, v in fam.items()}
    # the leaves' pivot chains are latency-bound: time per factored column
    # (every column of the matrix passes through exactly one potf2 and one LU panel)
    for k in ("potf2", "getf2_panel"):
        if k in families:
            families[k]["us_per_column"] = round(fam[k]["ms"] * 1e3 / n, 3)

    out = {
        "metric": "dpotrf/dgetrf TFLOP/s at n=16384; mixed+IR vs FP64 solve speedup at 1e-14",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded PCG64 inputs built on the device; no dataset)",
        "config": {"workload": f"recursive dpotrf (lower) + dgetrf, FP64, n={n}, lda=n; "
                               f"A_spd = B·Bᵀ + n·I, A_ge ~ U[-1,1]; solves with nrhs={nrhs}",
                   "n": n, "nrhs": nrhs},
        "potrf_ms": round(t_potrf, 3),
        "potrf_tflops": round(fl_potrf / (t_potrf * 1e-3) / 1e12, 3),
        "getrf_ms": round(t_getrf, 3),
        "getrf_tflops": round(fl_getrf / (t_getrf * 1e-3) / 1e12, 3),
        "potrs_ms": round(med("potrs"), 3),
        "getrs_ms": round(med("getrs"), 3),
        "frac_of_fp64_peak": round(value / PEAK_FP64, 4),
        "roofline": roofline,
        "kernel_families_one_pass": families,
        "input_build_s": round(t_gen, 1),
    }
    if mixed:
        ms, mg = med("posv_mixed"), med("gesv_mixed")
        fs = med("potrf") + med("potrs")
        fg = med("getrf") + med("getrs")
        last = res[-1]
        out["mixed"] = {
            "prec": args.prec, "kappa": args.kappa, "nrhs": nrhs,
            "spd": {"ms": round(ms, 3), "fp64_solve_ms": round(fs, 3), "speedup": round(fs / ms, 3),
                    "info": last["mixed_spd"][0], "iter": last["mixed_spd"][1], "berr": last["mixed_spd"][2]},
            "general": {"ms": round(mg, 3), "fp64_solve_ms": round(fg, 3), "speedup": round(fg / mg, 3),
                        "info": last["mixed_ge"][0], "iter": last["mixed_ge"][1], "berr": last["mixed_ge"][2]},
        }
    if args.target_n > 0:
        out["target_size"] = target_size(args.target_n, stream)
    if args.inv_n > 0:
        out["spd_inverse"] = spd_inverse(args.inv_n, stream)
    if not args.no_variants:
        out["variants"] = variants(n, stream)
    if args.batch_count > 0:
        out["batched"] = batched(args.batch_count, stream)
    if args.mixed_sweep:
        out["mixed_sweep"] = mixed_sweep(n, stream)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.cpu_n1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
