"""GPU parity of the two factorisation variants of the pivot blocks.

The tile-step LU (one launch per 32-column diagonal tile, then a triangular
inversion) and the recursive LU with inverted factors (halving down to
32 x 32 tiles; every other step an MFMA product, the inverses of the
triangular factors formed on the way) must give the same blocks of M^{-1}
as the FP64 oracle.  Block orders b = 32 * 2^m take the recursive variant
when forced; other orders fall back to tile steps.
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
EPS32 = 2.0 ** -24


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu(m, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(m)).to(DEV, dtype)


def run(m, k, i, j, precision="f64", factorization="recursive", concurrency=0):
    dtype = torch.float64 if precision == "f64" else torch.float32
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    out = bri.invert_block(gpu(m, dtype), k, i, j, precision=precision, info=info,
                           factorization=factorization, concurrency=concurrency)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), int(info.item())


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("b", [64, 128, 256, 512, 1024])
def test_recursive_lu_block_orders(b, precision):
    # k = 2: the root pivot and the final inversion are both factored by the
    # variant under test; all four blocks.
    n = 2 * b
    m = workloads.gaussian_dd(n, 40 + b)
    tol = 1e-12 if precision == "f64" else 64 * EPS32 * 2
    print(f"recursive LU b={b} {precision}", flush=True)
    for i in range(2):
        for j in range(2):
            got, info = run(m, 2, i, j, precision)
            assert info == 0
            assert rel(got, oracle.invert_block(m, 2, i, j)) < tol, (b, i, j)


def test_recursive_lu_spd_pivot_blocks_k4():
    # Q Lam Q^T (cond 1e2) with b = 256: pivot blocks of every depth.
    n, k = 1024, 4
    m = workloads.haar_spd(n, 12, 0.0, 2.0).m
    for (i, j) in [(0, 0), (1, 2), (3, 3)]:
        for fac in ("recursive", "tile"):
            got, info = run(m, k, i, j, factorization=fac)
            assert info == 0
            assert rel(got, oracle.invert_block(m, k, i, j)) < 1e-12, (i, j, fac)


@pytest.mark.parametrize("i,j", [(0, 0), (1, 2)])
def test_recursive_lu_config_n4096_k4_fp64(i, j):
    m = workloads.workload_matrix("spd_n4096_k4")
    got, info = run(m, 4, i, j)
    assert info == 0
    err = rel(got, oracle.invert_block(m, 4, i, j))
    print(f"n=4096 k=4 ({i},{j}) recursive LU: rel err {err:.2e}", flush=True)
    assert err < 1e-12


def test_recursive_lu_ragged_order_falls_back():
    # b = 100 is not 32 * 2^m: the recursive choice takes tile steps.
    n, k = 300, 3
    m = workloads.gaussian_dd(n, 303)
    got, info = run(m, k, 2, 0)
    assert info == 0
    assert rel(got, oracle.invert_block(m, k, 2, 0)) < 1e-12


def test_recursive_lu_singular_pivot_reports_info():
    # The first pivot (block (1,1)) is exactly zero: the first 32 x 32 tile
    # of the recursion reports it.
    b = 64
    rng = np.random.default_rng(3)
    a = rng.standard_normal((b, b)) + 8 * np.eye(b)
    m = np.block([[a, np.eye(b)], [np.eye(b), np.zeros((b, b))]])
    _, info = run(m, 2, 0, 0)
    assert info == 1


def test_recursive_lu_merged_batch_uniform_and_mixed_orders():
    # Sixteen problems of one order (their factorisations take the
    # recursive variant) and a group of mixed orders (tile steps).
    mats, ks, iis, jjs = [], [], [], []
    for t in range(16):
        mats.append(workloads.gaussian_dd(512, 900 + t))
        ks.append(2)
        iis.append(t % 2)
        jjs.append((t // 2) % 2)
    for t, n in enumerate((200, 260, 333)):
        mats.append(workloads.gaussian_dd(n, 950 + t))
        ks.append(3)
        iis.append(t)
        jjs.append((t + 1) % 3)
    info = torch.zeros(len(mats), dtype=torch.int32, device=DEV)
    outs = bri.invert_block_batched([gpu(m) for m in mats], ks, iis, jjs, info=info, factorization="recursive")
    torch.cuda.synchronize()
    assert int(info.abs().sum().item()) == 0
    for m, k, i, j, o in zip(mats, ks, iis, jjs, outs):
        assert rel(o.cpu().numpy(), oracle.invert_block(m, k, i, j)) < 1e-12, (m.shape[0], k, i, j)


def test_recursive_lu_block_column():
    n, k = 512, 4
    m = workloads.gaussian_dd(n, 77)
    x = bri.block_column(gpu(m), k, 1, factorization="recursive").cpu().numpy()
    assert rel(x, oracle.block_column(m, k, 1)) < 1e-12


def test_recursive_lu_large_halves_merged():
    # Eight problems of order 4096, k = 2 (b = 2048), merged: the recursive
    # LU's top-level products (halves of 1024, 8 x 2 items) take the
    # 256 x 128 tile shape.  Three of the blocks against the oracle.
    mats = [workloads.gaussian_dd(4096, 900 + t) for t in range(8)]
    ks, iis, jjs = [2] * 8, [t % 2 for t in range(8)], [(t // 2) % 2 for t in range(8)]
    info = torch.zeros(8, dtype=torch.int32, device=DEV)
    print("recursive LU, 8 x b=2048 merged", flush=True)
    outs = bri.invert_block_batched([gpu(m) for m in mats], ks, iis, jjs, info=info, factorization="recursive",
                                    pivoting="tile")
    torch.cuda.synchronize()
    assert int(info.abs().sum().item()) == 0
    for t in (0, 3, 6):
        err = rel(outs[t].cpu().numpy(), oracle.invert_block(mats[t], 2, iis[t], jjs[t]))
        print(f"  problem {t}: rel err {err:.2e}", flush=True)
        assert err < 1e-12
