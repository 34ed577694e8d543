"""GPU parity of several blocks of one matrix (invert_blocks): all k^2 blocks
or a band of them, computed as one merged batch over the same M, against the
FP64 oracle and, at n = 4096, against the matrix's known inverse."""
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


@pytest.mark.parametrize("n,k,family", [(1024, 4, "spd"), (1000, 4, "dd"), (300, 3, "dd")])
def test_all_blocks_against_oracle(n, k, family):
    m = workloads.haar_spd(n, 5 + n, 0.0, 2.0).m if family == "spd" else workloads.gaussian_dd(n, 7 + n)
    info = torch.zeros(k * k, dtype=torch.int32, device=DEV)
    print(f"all blocks n={n} k={k} {family}", flush=True)
    outs = bri.invert_blocks(gpu(m), k, info=info)
    torch.cuda.synchronize()
    assert int(info.abs().sum().item()) == 0
    t = 0
    for i in range(k):
        for j in range(k):
            assert rel(outs[t].cpu().numpy(), oracle.invert_block(m, k, i, j)) < 1e-12, (i, j)
            t += 1


def test_band_selection_against_oracle():
    n, k = 600, 6
    m = workloads.gaussian_dd(n, 606)
    band = bri.band_blocks(k, 1)
    assert len(band) == k + 2 * (k - 1)
    outs = bri.invert_blocks(gpu(m), k, band)
    torch.cuda.synchronize()
    for (i, j), o in zip(band, outs):
        assert rel(o.cpu().numpy(), oracle.invert_block(m, k, i, j)) < 1e-12, (i, j)


def test_all_blocks_n4096_k4_known_inverse():
    # The n = 4096, k = 4 workload: every block against Q[rows] Lam^{-1} Q[cols]^T.
    wl = workloads.WORKLOADS["spd_n4096_k4"]
    spd = workloads.haar_spd(wl.n, wl.seed, 0.0, 2.0)
    b = wl.n // wl.k
    outs = bri.invert_blocks(gpu(spd.m), wl.k)
    torch.cuda.synchronize()
    t = 0
    worst = 0.0
    for i in range(wl.k):
        for j in range(wl.k):
            want = (spd.q[i * b:(i + 1) * b] / spd.lam[None, :]) @ spd.q[j * b:(j + 1) * b].T
            worst = max(worst, rel(outs[t].cpu().numpy(), want))
            t += 1
    print(f"all 16 blocks n=4096 k=4: worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-12


def test_all_blocks_mixed_precision():
    n, k = 384, 3
    m = workloads.haar_spd(n, 38, 0.0, 2.0).m
    outs = bri.invert_blocks(gpu(m), k, precision="mixed_f16")
    torch.cuda.synchronize()
    t = 0
    for i in range(k):
        for j in range(k):
            assert rel(outs[t].cpu().numpy(), oracle.invert_block(m, k, i, j)) < 1e-10, (i, j)
            t += 1
