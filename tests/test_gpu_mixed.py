"""GPU parity of the mixed-precision paths against the FP64 CPU oracle.

Mixed paths: M and the result in FP64, the recursion in float storage with
its products on FP32 MFMA (mixed_f32) or on split FP16 / BF16 MFMA with FP32
accumulation (mixed_f16 / mixed_bf16), and FP64 iterative refinement of the
block column.  After refinement the target block must match the oracle to
1e-10 (relative Frobenius error); the refinement stops when the correction is
below 1e-12 of the iterate.

Split products: x = hi + lo 2^-11 (FP16, three products) or hi + mid + lo
(BF16, six products).  Their rounding error is bounded by a few units of
2^-22 (FP16 split, the dropped lo*lo term and the hi/lo rounding) or 2^-24
(BF16 split) relative to sum |a||b|, plus FP32 accumulation; the bound used
below, 2^-20 * sqrt(K) relative to ||A|| ||B||, holds with a wide margin.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import paper_1612_00001_amd as bri
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu(m, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(m)).to(DEV, dtype)


@pytest.mark.parametrize("products", ["f16", "bf16", None])
@pytest.mark.parametrize("m,n,kk", [(64, 64, 32), (200, 130, 77), (512, 256, 1024)])
def test_split_product_gemm(products, m, n, kk):
    rng = np.random.default_rng(m + n + kk)
    a = rng.standard_normal((m, kk))
    b = rng.standard_normal((kk, n))
    c0 = rng.standard_normal((m, n))
    A, B = gpu(a, torch.float32), gpu(b, torch.float32)
    C = gpu(c0, torch.float32)
    bri.gemm([A], [B], [C], alpha=-1.0, beta=1.0, products=products)
    torch.cuda.synchronize()
    a32 = a.astype(np.float32).astype(np.float64)
    b32 = b.astype(np.float32).astype(np.float64)
    want = c0.astype(np.float32).astype(np.float64) - a32 @ b32
    err = np.abs(C.double().cpu().numpy() - want).max()
    scale = np.abs(a32).max() * np.abs(b32).max() * kk
    print(f"products={products} {m}x{n}x{kk}: max err {err:.2e} (scale {scale:.1e})", flush=True)
    assert err <= 2.0 ** -20 * scale / np.sqrt(kk) * 8


@pytest.mark.parametrize("products", ["f16", "bf16"])
@pytest.mark.parametrize("count,m,n,kk,chunk", [(64, 1024, 1024, 1024, 20), (80, 1000, 776, 1000, 23),
                                                 (1100, 64, 136, 200, 300)])
def test_split_once_products(products, count, m, n, kk, chunk):
    # Split products of launches with at least 2048 output tiles of 256 x 128:
    # operands split once into scratch (chunk items at a time; 2 FP16 or 3
    # BF16 planes), then the products of the split planes; against the FP64
    # product of the float operands, and against the same launch without
    # scratch (operands split inside the product kernel).
    rng = np.random.default_rng(7 * count + m + n + kk)
    a = [rng.standard_normal((m, kk)).astype(np.float32) for _ in range(count)]
    b = [rng.standard_normal((kk, n)).astype(np.float32) for _ in range(count)]
    c0 = [rng.standard_normal((m, n)).astype(np.float32) for _ in range(count)]
    kp = (kk + 63) // 64 * 64
    per = 2 * (2 if products == "f16" else 3) * (m + n) * kp
    A = [gpu(x, torch.float32) for x in a]
    B = [gpu(x, torch.float32) for x in b]
    C1 = [gpu(x, torch.float32) for x in c0]
    C2 = [gpu(x, torch.float32) for x in c0]
    print(f"split once ({products}): {count} x {m}x{n}x{kk}, {chunk} items per part", flush=True)
    bri.gemm(A, B, C1, alpha=-1.0, beta=1.0, products=products, split_bytes=chunk * per)
    bri.gemm(A, B, C2, alpha=-1.0, beta=1.0, products=products)
    torch.cuda.synchronize()
    worst = 0.0
    for t in range(count):
        want = c0[t].astype(np.float64) - a[t].astype(np.float64) @ b[t].astype(np.float64)
        got = C1[t].double().cpu().numpy()
        scale = np.abs(a[t]).max() * np.abs(b[t]).max() * kk
        err = np.abs(got - want).max()
        worst = max(worst, err / scale)
        assert err <= 2.0 ** -20 * scale / np.sqrt(kk) * 8
        assert np.abs(got - C2[t].double().cpu().numpy()).max() <= 2.0 ** -20 * scale / np.sqrt(kk)
    print(f"  worst err / (max|a| max|b| kk) = {worst:.2e}", flush=True)


def run_mixed(m, k, i, j, precision, iters=10, tol=1e-12):
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    out = bri.invert_block(gpu(m), k, i, j, precision=precision, info=info, refine_max_iters=iters,
                           refine_tol=tol)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(info.item())


@pytest.mark.parametrize("precision", ["mixed_f32", "mixed_f16", "mixed_bf16"])
@pytest.mark.parametrize("n,k", [(384, 4), (130, 4), (257, 2), (300, 5)])
def test_mixed_refined_matches_oracle(precision, n, k):
    m = workloads.haar_spd(n, 40 + n, 0.0, 2.0).m
    for (i, j) in [(0, 0), (k - 1, 1)]:
        print(f"case {precision} n={n} k={k} ({i},{j})", flush=True)
        got, info = run_mixed(m, k, i, j, precision)
        assert info == 0
        err = rel(got, oracle.invert_block(m, k, i, j))
        print(f"  rel err {err:.2e}", flush=True)
        assert err < 1e-10


@pytest.mark.parametrize("precision", ["mixed_f16", "mixed_bf16"])
def test_mixed_cond_1e4(precision):
    # Q Lam Q^T with Lam log-uniform in [1, 1e4] (condition number 1e4).
    n, k = 512, 4
    m = workloads.haar_spd(n, 91, 0.0, 4.0, pin_endpoints=True).m
    for (i, j) in [(1, 1), (2, 0)]:
        got, info = run_mixed(m, k, i, j, precision)
        assert info == 0
        err = rel(got, oracle.invert_block(m, k, i, j))
        print(f"{precision} cond 1e4 ({i},{j}): rel err {err:.2e}", flush=True)
        assert err < 1e-10


def test_mixed_without_refinement_is_float_accurate():
    n, k = 256, 4
    m = workloads.gaussian_dd(n, 17)
    want = oracle.invert_block(m, k, 1, 2)
    got, info = run_mixed(m, k, 1, 2, "mixed_f32", iters=0)
    assert info == 0
    err = rel(got, want)
    assert 1e-12 < err < 1e-4  # float-level only: no FP64 refinement ran
    got2, _ = run_mixed(m, k, 1, 2, "mixed_f32", iters=3)
    assert rel(got2, want) < 1e-12


def test_mixed_unreachable_tolerance_reports_minus_one():
    n, k = 128, 2
    m = workloads.gaussian_dd(n, 18)
    got, info = run_mixed(m, k, 0, 1, "mixed_bf16", iters=1, tol=0.0)
    assert info == -1
    assert rel(got, oracle.invert_block(m, k, 0, 1)) < 1e-6  # one sweep still improved it


def test_mixed_batched_problems():
    probs = workloads.batch_problems(count=6, seed=5, n_lo=64, n_hi=200)
    Ms = [gpu(workloads.batch_matrix(p)) for p in probs]
    info = torch.zeros(len(probs), dtype=torch.int32, device=DEV)
    outs = bri.invert_block_batched(Ms, [p.k for p in probs], [p.i for p in probs], [p.j for p in probs],
                                    precision="mixed_f32", info=info)
    torch.cuda.synchronize()
    assert int(info.abs().sum().item()) == 0
    for p, o in zip(probs, outs):
        want = oracle.invert_block(workloads.batch_matrix(p), p.k, p.i, p.j)
        assert rel(o.cpu().numpy(), want) < 1e-10, (p.n, p.k, p.i, p.j)


def test_mixed_f32_batched_512_problems_merged():
    # The batched workload in its stated precision (FP32 recursion with FP64
    # refinement): every block against the dense inverse of its matrix.
    probs = workloads.batch_problems()
    mats = [workloads.batch_matrix(p) for p in probs]
    Ms = [gpu(m) for m in mats]
    info = torch.zeros(len(probs), dtype=torch.int32, device=DEV)
    print("mixed_f32 batched 512 problems", flush=True)
    outs = bri.invert_block_batched(Ms, [p.k for p in probs], [p.i for p in probs], [p.j for p in probs],
                                    precision="mixed_f32", info=info)
    torch.cuda.synchronize()
    assert int(info.abs().sum().item()) == 0
    worst = 0.0
    for p, m, o in zip(probs, mats, outs):
        b = -(-p.n // p.k)
        g = np.eye(p.k * b)
        g[:p.n, :p.n] = m
        want = np.linalg.inv(g)[p.i * b:(p.i + 1) * b, p.j * b:(p.j + 1) * b]
        worst = max(worst, rel(o.cpu().numpy(), want))
    print(f"  worst rel err {worst:.2e}, sweeps {bri.refine_last()[0]}", flush=True)
    assert worst < 1e-10


@pytest.mark.parametrize("precision", ["mixed_f32", "mixed_f16"])
def test_mixed_with_reused_pivots(precision):
    n, k = 300, 5
    m = workloads.haar_spd(n, 12, 0.0, 2.0).m
    for (i, j) in [(0, 0), (3, 2)]:
        info = torch.zeros(1, dtype=torch.int32, device=DEV)
        got = bri.invert_block(gpu(m), k, i, j, precision=precision, info=info, reuse=True)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert rel(got.cpu().numpy(), oracle.invert_block(m, k, i, j)) < 1e-10


def test_mixed_f16_cond_1e6_stays_in_range():
    # cond 1e6: after the power-of-two scaling of M (largest entry in
    # [0.5, 1)) the largest magnitude the products meet is about 1e4, inside
    # the FP16 range: FP16 split products and refinement reach the target.
    # The corrections stop shrinking near cond(M) u64 ~ 1e-10 (the FP64
    # residual's own rounding), so the stopping tolerance is the accuracy
    # target itself rather than the default 1e-12.
    n, k = 512, 4
    m = workloads.haar_spd(n, 61, 0.0, 6.0, pin_endpoints=True).m
    got, info = run_mixed(m, k, 0, 0, "mixed_f16", iters=30, tol=1e-10)
    err = rel(got, oracle.invert_block(m, k, 0, 0))
    print(f"mixed_f16 cond 1e6: rel err {err:.2e}, info {info}", flush=True)
    assert info == 0 and not bri.refine_last_bf16_fallback()
    assert err < 1e-10


def test_mixed_f16_out_of_range_falls_back_to_bf16():
    # A badly scaled matrix D A D (A diagonally dominant, the last 64 rows and
    # columns scaled by 1e-4): its inverse D^-1 A^-1 D^-1 has entries around
    # 1e8 times the scaled matrix's, far outside the FP16 range (65504).  The
    # split FP16 products flag it and the call is computed again with BF16
    # split products (FP32's exponent range), which reach the target.
    n, k = 512, 4
    d = np.ones(n)
    d[-64:] = 1e-4
    m = d[:, None] * workloads.gaussian_dd(n, 63) * d[None, :]
    for (i, j) in [(3, 3), (0, 3)]:
        got, info = run_mixed(m, k, i, j, "mixed_f16", iters=30)
        err = rel(got, oracle.invert_block(m, k, i, j))
        fell_back = bri.refine_last_bf16_fallback()
        print(f"mixed_f16 scaled ({i},{j}): rel err {err:.2e}, info {info}, bf16 fallback {fell_back}", flush=True)
        assert fell_back
        assert info == 0
        assert err < 1e-10


def test_mixed_f16_range_fallback_on_split_once_products():
    # The same fallback where the explicit products run on operands split
    # once (n = 4096, k = 8: launches of 256 items of order 512): the FP16
    # split pass flags the range, the BF16 pass reuses the split scratch with
    # three planes.  D A D with A = Q Lam Q^T (cond 1e2) and the last 64 rows
    # and columns scaled by 1e-4; reference D^-1 (Q Lam^-1 Q^T) D^-1.
    n, k = 4096, 8
    b = n // k
    w = workloads.haar_spd(n, 71, 0.0, 2.0)
    d = np.ones(n)
    d[-64:] = 1e-4
    m = d[:, None] * w.m * d[None, :]
    for (i, j) in [(7, 7), (0, 7)]:
        qi, qj = w.q[i * b:(i + 1) * b], w.q[j * b:(j + 1) * b]
        want = ((qi / w.lam[None, :]) @ qj.T) / d[i * b:(i + 1) * b, None] / d[None, j * b:(j + 1) * b]
        got, info = run_mixed(m, k, i, j, "mixed_f16", iters=30)
        err = rel(got, want)
        fell_back = bri.refine_last_bf16_fallback()
        print(f"mixed_f16 n=4096 k=8 scaled ({i},{j}): rel err {err:.2e}, info {info}, bf16 fallback {fell_back}",
              flush=True)
        assert fell_back
        assert info == 0
        assert err < 1e-10


@pytest.mark.parametrize("precision", ["mixed_f16", "mixed_bf16"])
def test_mixed_recursive_lu_with_split_products(precision):
    # The recursive LU of the float recursion forced on b = 512 pivot blocks:
    # its products of order 256 and 128 run as split FP16 / BF16 products
    # (row-permuted and triangular operands), the smaller ones in FP32.  Tile
    # pivoting, so the element-growth check must stay quiet.
    n, k = 2048, 4
    m = workloads.haar_spd(n, 77, 0.0, 2.0).m
    for (i, j) in [(0, 0), (2, 1)]:
        info = torch.zeros(1, dtype=torch.int32, device=DEV)
        print(f"recursive LU {precision} ({i},{j})", flush=True)
        got = bri.invert_block(gpu(m), k, i, j, precision=precision, info=info, pivoting="tile",
                               factorization="recursive")
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        err = rel(got.cpu().numpy(), oracle.invert_block(m, k, i, j))
        print(f"  rel err {err:.2e}", flush=True)
        assert err < 1e-10
