"""GPU parity at the precision workload's full size and at k = 8.

* n = 16384, k = 8 (b = 2048), M = Q Lam Q^T with cond(M) = 1e4 exactly
  (eigenvalues log-uniform, endpoints pinned at 1 and 1e4), target block
  (0, 0).  The oracle would need about half an hour here, so the reference
  is the closed form of this matrix's inverse, Q Lam^{-1} Q^T, restricted to
  the block: N_00 = Q[0:b] Lam^{-1} Q[0:b]^T, formed by torch in FP64 from
  the generator's own factors (not by this library).  M itself is
  0.5 (Q Lam Q^T + (Q Lam Q^T)^T) in FP64, so its exact inverse differs from
  the closed form by about cond(M) * 1e-16 = 1e-12, below the 1e-10 bar.
  The plain FP64 path and the mixed paths with split FP16 / BF16 products and
  FP64 refinement must all reach 1e-10 (relative Frobenius error, and every
  element within 1e-10 of the block's largest magnitude).
* n = 2048, k = 8 (b = 256), same family: checked against the FP64 oracle.
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


@pytest.fixture(scope="module")
def spd_n16384_k8():
    wl = workloads.WORKLOADS["spd_n16384_k8"]
    b = bri.block_size(wl.n, wl.k)
    print("generating spd_n16384_k8 on the device", flush=True)
    m, q, lam = workloads.haar_spd_device(wl.n, wl.seed, 0.0, 4.0, pin_endpoints=True, device=DEV,
                                          return_factors=True)
    qb = q[0:b].contiguous()
    del q
    inv_lam = torch.from_numpy(1.0 / lam).to(DEV)
    ref = (qb * inv_lam[None, :]) @ qb.T.contiguous()
    del qb
    torch.cuda.synchronize()
    return m, ref.cpu().numpy(), wl


@pytest.mark.parametrize("precision", ["f64", "mixed_f16", "mixed_bf16"])
def test_precision_workload_n16384_k8(spd_n16384_k8, precision):
    m, ref, wl = spd_n16384_k8
    print(f"n=16384 k=8 block (0,0) {precision}", flush=True)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    out = bri.invert_block(m, wl.k, 0, 0, precision=precision, info=info)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    err = rel(got, ref)
    emax = float(np.abs(got - ref).max() / np.abs(ref).max())
    sweeps = bri.refine_last()[0] if precision.startswith("mixed") else 0
    print(f"  rel err {err:.2e}, max elementwise {emax:.2e}, sweeps {sweeps}, info {int(info.item())}", flush=True)
    assert int(info.item()) == 0
    assert err < 1e-10
    assert emax < 1e-10


@pytest.fixture(scope="module")
def spd_n2048_k8():
    m = workloads.haar_spd(2048, 31, 0.0, 4.0, pin_endpoints=True).m
    targets = [(0, 0), (3, 5)]
    print("oracle n=2048 k=8", flush=True)
    return m, {t: oracle.invert_block(m, 8, *t) for t in targets}


@pytest.mark.parametrize("precision", ["f64", "mixed_f16", "mixed_bf16", "mixed_f32"])
def test_k8_n2048_against_oracle(spd_n2048_k8, precision):
    m, refs = spd_n2048_k8
    g = torch.from_numpy(m).to(DEV)
    for (i, j), want in refs.items():
        info = torch.zeros(1, dtype=torch.int32, device=DEV)
        out = bri.invert_block(g, 8, i, j, precision=precision, info=info)
        torch.cuda.synchronize()
        err = rel(out.cpu().numpy(), want)
        print(f"n=2048 k=8 ({i},{j}) {precision}: rel err {err:.2e}", flush=True)
        assert int(info.item()) == 0
        assert err < 1e-10


@pytest.fixture(scope="module")
def spd_n4096_k8():
    w = workloads.haar_spd(4096, 37, 0.0, 4.0, pin_endpoints=True)
    b = 512
    qb = w.q[:b]
    # closed form of block (0, 0) of M^{-1} = Q Lam^{-1} Q^T
    return w.m, (qb / w.lam[None, :]) @ qb.T


@pytest.mark.parametrize("precision", ["mixed_f16", "mixed_bf16", "mixed_f32"])
def test_k8_n4096_unrefined_float_recursion(spd_n4096_k8, precision):
    # The float recursion alone (no FP64 sweep) at n = 4096, k = 8: its
    # explicit product launches (256 items of order 512, 2048 tiles of
    # 256 x 128) run on operands split once for FP16 and BF16, triangular
    # multiplies included.  Its error is the float recursion's, about
    # cond(M) = 1e4 times the unit roundoff of the products (2^-22 for the
    # split FP16 products, 2^-24 for split BF16 and FP32).
    m, want = spd_n4096_k8
    g = torch.from_numpy(m).to(DEV)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    out = bri.invert_block(g, 8, 0, 0, precision=precision, info=info, refine_max_iters=0)
    torch.cuda.synchronize()
    err = rel(out.cpu().numpy(), want)
    print(f"n=4096 k=8 (0,0) {precision} without refinement: rel err {err:.2e}", flush=True)
    assert int(info.item()) == 0
    assert err < 1e4 * 2.0 ** -22 * 16
    # and with the FP64 sweeps
    out = bri.invert_block(g, 8, 0, 0, precision=precision, info=info)
    torch.cuda.synchronize()
    err = rel(out.cpu().numpy(), want)
    print(f"  refined: rel err {err:.2e}", flush=True)
    assert int(info.item()) == 0
    assert err < 1e-10
