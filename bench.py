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


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_gemm_explicit_hbm_traffic_spd_n4096_k4_f64.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1612_00001_amd", "csrc", "bri_kernels.hip")


def gemm_source_digest():
    """sha256 over the source of the product kernel: its operand loaders and
    kernel bodies, register-staged and direct-to-LDS (from the "Operand
    tiles." section to the low-precision kernel) and its tile-shape selection
    (launch_gemm_mode, launch_gemm)."""
    import hashlib
    text = open(KERNEL_SOURCE).read()
    a = text.index("// Operand tiles.")
    e = text.index("// Low-precision products")
    c = text.index("hipError_t launch_gemm_mode(")
    d = text.index("\n}\n", c)
    f = text.index("hipError_t launch_gemm(const GemmLaunch& L")
    g = text.index("\n}\n", f)
    return hashlib.sha256((text[a:e] + text[c:d] + text[f:g]).encode()).hexdigest()


def counted_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size),
    or None when the summary is missing or the kernel source has changed
    since the counters were taken."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
        digest = gemm_source_digest()
    except (OSError, ValueError):
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith(("traffic_bytes", "source_sha256")))
    if fields.get("source_sha256", "").strip() != digest:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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


def precision_workload(bri, workloads, torch, np) -> int:
    """n = 16384, k = 8 (b = 2048), Q Lam Q^T with cond 1e4 (generated on the
    device, same recipe as the host generator), block (0,0): the plain FP64
    path and the mixed paths, each timed once, against a dense FP64 solve of
    M X = E_0 on the device (torch.linalg.solve, not this library)."""
    wl = workloads.WORKLOADS["spd_n16384_k8"]
    n, k = wl.n, wl.k
    i, j = wl.targets[0]
    b = bri.block_size(n, k)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    M = workloads.haar_spd_device(n, wl.seed, 0.0, 4.0, pin_endpoints=True, device=dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    e = torch.zeros(n, b, dtype=torch.float64, device=dev)
    e[j * b:(j + 1) * b] = torch.eye(b, dtype=torch.float64, device=dev)
    ref = torch.linalg.solve(M, e)[i * b:(i + 1) * b].contiguous()
    del e
    torch.cuda.synchronize()
    flops = bri.plan_describe(n, k, i, j, "f64")["algorithmic_flops"]
    runs = []
    for prec, reuse in (("f64", False), ("mixed_f16", False), ("mixed_bf16", False), ("mixed_f32", False),
                        ("f64", True), ("mixed_f16", True), ("mixed_bf16", True)):
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        ws = torch.empty(bri.workspace_size(n, k, i, j, prec, reuse=reuse), dtype=torch.uint8, device=dev)
        print(f"precision workload: {prec} reuse={reuse}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = bri.invert_block(M, k, i, j, precision=prec, info=info, workspace=ws, reuse=reuse)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
        sweeps = bri.refine_last()[0] if prec.startswith("mixed") else 0
        runs.append({"precision": prec, "reuse_pivots": reuse, "s": dt, "paper_equivalent_tflops": flops / dt / 1e12,
                     "rel_error_vs_dense_solve": err,
                     "refine_sweeps": sweeps, "info": int(info.item()), "workspace_bytes": ws.numel()})
        print(json.dumps(runs[-1]), file=sys.stderr, flush=True)
        del ws, out
    print(json.dumps({"workload": "spd_n16384_k8: n=16384 k=8 b=2048, Q Lam Q^T, cond 1e4 (Lam pinned at 1 and 1e4), "
                                  "block (0,0), matrix generated on the device",
                      "algorithmic_flops": flops, "generation_s": gen_s, "runs": runs}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--precision-workload", action="store_true",
                    help="run only the n=16384, k=8 (cond 1e4) precision workload once per precision and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the block recursive inverse runs on a single MI355X "
              "(its independent subtrees could be spread over GPUs, but no multi-GPU path is built); "
              "use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.calibrate_copy:
        # A plain copy of known size: the HBM counters of its kernel give the
        # scale between counted and actual bytes.
        src = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 8, "launches": 5}), flush=True)
        return 0

    import paper_1612_00001_amd as bri
    import workloads

    if args.precision_workload:
        return precision_workload(bri, workloads, torch, np)

    dev = torch.device("cuda:0")
    lib = bri.lib()
    wl = workloads.WORKLOADS["spd_n4096_k4"]
    n, k = wl.n, wl.k
    m_host = workloads.workload_matrix(wl.name)
    M64 = torch.from_numpy(m_host).to(dev)
    M32 = M64.float()

    def setup(M, i, j, precision, reuse=False):
        need = bri.workspace_size(n, k, i, j, precision, reuse=reuse)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        b = bri.block_size(n, k)
        out = torch.empty(b, b, dtype=M.dtype, device=dev)
        info = torch.zeros(1, dtype=torch.int32, device=dev)

        def call():
            bri.invert_block(M, k, i, j, precision=precision, out=out, info=info, workspace=ws, reuse=reuse)
        return call, out, info

    # ---- headline: FP64, block (0, 0) ------------------------------------
    i, j = wl.targets[0]
    stats = bri.plan_describe(n, k, i, j, "f64")
    flops = stats["algorithmic_flops"]
    call, out, info = setup(M64, i, j, "f64")
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    # Timed steps without instrumentation, then the same steps again with HIP
    # events around every plan step for the per-kernel breakdown.
    ms, wall_ms = time_calls(call, args.steps, 0, torch)
    lib.bri_profile_enable(1)
    profile_read(lib)  # clear
    prof_ms, _ = time_calls(call, args.steps, 0, torch)
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
        "kernel": "explicit-item FP64 products (Schur and triangular): k_gemm_dl (direct-to-LDS loads, 128x128 tiles) "
                  "where every item of a step has stored, aligned operands, else k_gemm<double, GEMM_EXPLICIT> "
                  "(128x256, 128x128 or 64x64 tiles)",
        "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
        "frac": achieved / PEAK_TFLOPS["f64"], "traffic": counted_traffic(),
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
        "wall_ms_per_step": wall_ms, "profiled_ms_per_step": prof_ms,
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
        # mixed precision on the same workload: float recursion (FP32, split
        # FP16 or split BF16 MFMA products) with FP64 refinement of the block
        # column; value = F / time including refinement (extra work not credited)
        f64_ms = ms
        for prec in ("mixed_f32", "mixed_f16", "mixed_bf16"):
            c2, o2, inf2 = setup(M64, i, j, prec)
            vms, _ = time_calls(c2, max(1, args.steps // 3), 1, torch)
            sweeps, last = bri.refine_last()
            entry = {"block": [i, j], "precision": prec, "ms_per_step": vms,
                     "tflops": flops / (vms * 1e-3) / 1e12, "speed_vs_f64": f64_ms / vms,
                     "refine_sweeps": sweeps, "last_rel_correction": last, "info": int(inf2.item())}
            if not args.no_cpu_baseline:
                entry["rel_error"] = rel_err(o2.cpu().numpy(), refs[(i, j)])
            variants.append(entry)
        # the paper's suggested reuse across branches (elimination pivots kept
        # and factored once); value still counts the paper's operations F
        for prec in ("f64", "mixed_f16"):
            c2, o2, inf2 = setup(M64, i, j, prec, reuse=True)
            vms, _ = time_calls(c2, max(1, args.steps // 3), 1, torch)
            entry = {"block": [i, j], "precision": prec, "reuse_pivots": True, "ms_per_step": vms,
                     "paper_equivalent_tflops": flops / (vms * 1e-3) / 1e12, "speed_vs_f64": f64_ms / vms,
                     "executed_flops": bri.plan_describe(n, k, i, j, prec, reuse=True)["executed_flops"],
                     "info": int(inf2.item())}
            if prec.startswith("mixed"):
                entry["refine_sweeps"] = bri.refine_last()[0]
            if not args.no_cpu_baseline:
                entry["rel_error"] = rel_err(o2.cpu().numpy(), refs[(i, j)])
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

    # ---- batched workload: 512 problems, n in [64, 1024], k in {2,3,4} ---------
    if not args.no_batched:
        probs = workloads.batch_problems()
        mats = [workloads.batch_matrix(p) for p in probs]
        bflops = sum(bri.plan_describe(p.n, p.k, p.i, p.j, "f64")["algorithmic_flops"] for p in probs)
        ks, ii, jj = [p.k for p in probs], [p.i for p in probs], [p.j for p in probs]
        sample = list(range(0, len(probs), 32))
        dense = {}
        for t in sample:
            p = probs[t]
            b = bri.block_size(p.n, p.k)
            g = np.eye(p.k * b)
            g[:p.n, :p.n] = mats[t]
            dense[t] = np.linalg.inv(g)[p.i * b:(p.i + 1) * b, p.j * b:(p.j + 1) * b]
        batched = []
        for prec in ("mixed_f32", "f64", "f32"):
            dt = torch.float32 if prec == "f32" else torch.float64
            Ms = [torch.from_numpy(m).to(dev, dt) for m in mats]
            binfo = torch.zeros(len(probs), dtype=torch.int32, device=dev)
            outs = bri.invert_block_batched(Ms, ks, ii, jj, precision=prec, info=binfo)
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                outs = bri.invert_block_batched(Ms, ks, ii, jj, precision=prec, info=binfo)
            torch.cuda.synchronize()
            bms = (time.perf_counter() - t0) * 1e3 / reps
            err = max(rel_err(outs[t].double().cpu().numpy(), dense[t]) for t in sample)
            batched.append({"precision": prec, "ms_per_batch": bms, "tflops": bflops / (bms * 1e-3) / 1e12,
                            "problems_per_s": len(probs) / (bms * 1e-3), "max_rel_error_sampled": err,
                            "info_nonzero": int((binfo != 0).sum().item()),
                            "refine_sweeps": bri.refine_last()[0] if prec.startswith("mixed") else 0})
            del Ms, outs
        line["batched"] = {"workload": "512 problems, n ~ U[64,1024], k ~ U{2,3,4}, random block, Gaussian + n I, "
                                       "seeds SeedSequence(5).spawn(512); error vs dense inverse on every 32nd problem",
                           "algorithmic_flops": bflops, "runs": batched}

    # ---- adjoint: n = 8192, k = 4, FP32, dL/dM for L = sum(W * N_00) --------
    if not args.no_backward:
        wlg = workloads.WORKLOADS["dd_n8192_k4_grad"]
        mg = torch.from_numpy(workloads.workload_matrix(wlg.name)).to(dev, torch.float32)
        bg = bri.block_size(wlg.n, wlg.k)
        W = torch.from_numpy(workloads.cotangent(bg, seed=4)).to(dev, torch.float32)
        gi, gj = wlg.targets[0]
        grad = bri.invert_block_backward(mg, wlg.k, gi, gj, W, precision="f32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grad = bri.invert_block_backward(mg, wlg.k, gi, gj, W, precision="f32")
        torch.cuda.synchronize()
        gms = (time.perf_counter() - t0) * 1e3
        line["backward"] = {"workload": "dd_n8192_k4_grad: n=8192 k=4 b=2048, Gaussian + n I, block (0,0), FP32",
                            "ms": gms, "finite": bool(torch.isfinite(grad).all().item())}
        del grad, mg

    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
