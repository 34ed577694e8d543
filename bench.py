#!/usr/bin/env python3
"""Benchmark of the block recursive inverse on one MI355X.

One step = one ``invert_block`` call on the n = 4096, k = 4 workload
(b = 1024, Q Lam Q^T with Lam log-uniform in [1, 100], Haar Q, seed 2),
FP64, target block (0, 0), inputs resident in HBM.  The throughput is the
algorithmic flop count of one block,
    F = T(k) (14/3) b^3 + 2 b^3 (+ 2 b^3 for an off-diagonal block),
    T(k) = (4^(k-1) - 1) / 3 Schur operations (Theorem "C_BRI"),
divided by the measured time.  The line also carries variants (the
off-diagonal target, FP32, the n = 256, k = 2 latency case), the roofline of
the dominant kernel (HIP events around every plan step, summed per kernel
role) and the FP64 CPU oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "block-inverse TFLOP/s + % MFMA peak, mixed vs FP64 at stated rel. error"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "f16": 2500.0, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0
KIND_NAMES = {1: "load", 2: "getrf", 3: "trtri", 4: "trmm_lower", 5: "trmm_upper", 6: "gemm_schur",
              7: "gemm_acc", 8: "gemm_neg"}


class ProfEntry(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double)]


def profile_read(lib):
    arr = (ProfEntry * 9)()
    lib.bri_profile_read.restype = ctypes.c_int
    lib.bri_profile_read.argtypes = [ctypes.POINTER(ProfEntry), ctypes.c_int]
    n = lib.bri_profile_read(arr, 9)
    return {t: (arr[t].steps, arr[t].launches, arr[t].ms, arr[t].flops) for t in range(1, n)}


def rel_err(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def time_calls(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return ev0.elapsed_time(ev1) / steps, wall


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the block recursive inverse runs on a single MI355X "
              "(see the sharding notes in DESIGN.md); use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1612_00001_amd as bri
    import workloads

    dev = torch.device("cuda:0")
    lib = bri.lib()
    wl = workloads.WORKLOADS["spd_n4096_k4"]
    n, k = wl.n, wl.k
    m_host = workloads.workload_matrix(wl.name)
    M64 = torch.from_numpy(m_host).to(dev)
    M32 = M64.float()

    def setup(M, i, j, precision):
        need = bri.workspace_size(n, k, i, j, precision)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        b = bri.block_size(n, k)
        out = torch.empty(b, b, dtype=M.dtype, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)

        def call():
            bri.invert_block(M, k, i, j, precision=precision, out=out, info=info, workspace=ws)
        return call, out, info

    # ---- headline: FP64, block (0, 0) ------------------------------------
    i, j = wl.targets[0]
    stats = bri.plan_describe(n, k, i, j, "f64")
    flops = stats["algorithmic_flops"]
    call, out, info = setup(M64, i, j, "f64")
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    lib.bri_profile_enable(1)
    profile_read(lib)  # clear
    ms, wall_ms = time_calls(call, args.steps, 0, torch)
    prof = profile_read(lib)
    lib.bri_profile_enable(0)
    assert int(info.item()) == 0, "device status"
    got = out.cpu().numpy()

    value = flops / (ms * 1e-3) / 1e12
    breakdown = {}
    for t, (st, la, pms, pfl) in prof.items():
        if st:
            breakdown[KIND_NAMES[t]] = {"ms_per_step": pms / args.steps, "launches_per_step": la / args.steps,
                                        "tflops": (pfl / (pms * 1e-3) / 1e12) if pms > 0 else None}
    # Dominant kernel: the MFMA product kernel in its explicit-item instance
    # (triangular products and Schur updates, one launch per plan step).
    prod_kinds = (4, 5, 6, 7, 8)
    p_ms = sum(prof[t][2] for t in prod_kinds if t in prof)
    p_fl = sum(prof[t][3] for t in prod_kinds if t in prof)
    p_la = sum(prof[t][1] for t in prod_kinds if t in prof)
    achieved = p_fl / (p_ms * 1e-3) / 1e12 if p_ms > 0 else 0.0
    roofline = {
        "kernel": "k_gemm<double, GEMM_EXPLICIT, 128x128> (Schur and triangular products)",
        "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
        "frac": achieved / PEAK_TFLOPS["f64"], "traffic": None,
        "launches_per_step": p_la / args.steps, "avg_launch_ms": (p_ms / p_la) if p_la else None,
        "flops_per_launch": (p_fl / p_la) if p_la else None,
    }

    line = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "spd_n4096_k4: n=4096 k=4 b=1024, block (0,0), Q Lam Q^T, Lam in [1,100]",
                   "n": n, "k": k, "b": stats["block"], "block": [i, j], "precision": "f64",
                   "concurrency": stats["batch_width"]},
        "pct_fp64_mfma_peak": 100.0 * value / PEAK_TFLOPS["f64"],
        "wall_ms_per_step": wall_ms,
        "schur_ops": stats["schur_ops"], "algorithmic_flops": flops, "executed_flops": stats["executed_flops"],
        "workspace_bytes": stats["workspace_bytes"], "workspace_blocks": stats["slots"],
        "kernel_launches_per_step": stats["kernel_launches"],
        "roofline": roofline, "breakdown": breakdown,
    }

    # ---- CPU baseline (the FP64 oracle) -------------------------------------
    ref = None
    if not args.no_cpu_baseline:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = sum(x.get("num_threads", 0) for x in threadpool_info() if x.get("user_api") == "blas")
        except Exception:  # threadpoolctl missing: report the process's CPU count
            cores = os.cpu_count()
        t0 = time.perf_counter()
        ref = oracle.invert_block(m_host, k, i, j)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
                                "sample": f"the whole step: oracle recursion for block ({i},{j}) of the "
                                          f"n={n}, k={k} workload ({stats['schur_ops']} Schur operations), "
                                          f"{dt:.2f} s"}
        line["rel_error"] = rel_err(got, ref)

    # ---- variants -------------------------------------------------------------
    if not args.no_variants:
        variants = []
        import oracle
        refs = {(i, j): ref}
        for (vi, vj, prec) in [(1, 2, "f64"), (0, 0, "f32"), (1, 2, "f32")]:
            M = M64 if prec == "f64" else M32
            st = bri.plan_describe(n, k, vi, vj, prec)
            c2, o2, inf2 = setup(M, vi, vj, prec)
            vms, _ = time_calls(c2, args.steps, args.warmup, torch)
            entry = {"block": [vi, vj], "precision": prec, "ms_per_step": vms,
                     "tflops": st["algorithmic_flops"] / (vms * 1e-3) / 1e12,
                     "pct_mfma_peak": 100.0 * st["algorithmic_flops"] / (vms * 1e-3) / 1e12 / PEAK_TFLOPS[prec]}
            if not args.no_cpu_baseline:
                if refs.get((vi, vj)) is None:
                    refs[(vi, vj)] = oracle.invert_block(m_host, k, vi, vj)
                entry["rel_error"] = rel_err(o2.double().cpu().numpy(), refs[(vi, vj)])
            variants.append(entry)
        # latency case n = 256, k = 2 (FP64)
        m1 = workloads.workload_matrix("dd_n256_k2")
        M1 = torch.from_numpy(m1).to(dev)
        st1 = bri.plan_describe(256, 2, 0, 0, "f64")
        o1 = torch.empty(128, 128, dtype=torch.float64, device=dev)
        w1 = torch.empty(bri.workspace_size(256, 2, 0, 0), dtype=torch.uint8, device=dev)
        c1 = lambda: bri.invert_block(M1, 2, 0, 0, out=o1, workspace=w1)  # noqa: E731
        ms1, _ = time_calls(c1, 50, 5, torch)
        e1 = {"workload": "dd_n256_k2: n=256 k=2 b=128 block (0,0), Gaussian + nI", "precision": "f64",
              "us_per_call": ms1 * 1e3, "tflops": st1["algorithmic_flops"] / (ms1 * 1e-3) / 1e12}
        if not args.no_cpu_baseline:
            e1["rel_error"] = rel_err(o1.cpu().numpy(), oracle.invert_block(m1, 2, 0, 0))
        variants.append(e1)
        line["variants"] = variants

    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
