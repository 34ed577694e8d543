"""GPU parity of the paper's literal frame order (BRI_ORDER_PAPER) against
the oracle's literal procedure, and its behaviour where it pivots on
non-principal blocks (Sections "Forward recursive procedure" and "Backward
recursive procedure"; the reformulation with respect to (M/A) that the
Conclusion proposes is the principal order, the default)."""
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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(m, k, i, j, precision="f64", order="paper", concurrency=0, pivoting="auto"):
    # Automatic pivoting: the literal order's non-principal pivots are
    # plain Gaussian blocks here, on which tile pivoting reports its element
    # growth and the call falls back to panel pivoting.
    dtype = torch.float64 if precision == "f64" else torch.float32
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    M = torch.from_numpy(np.ascontiguousarray(m)).to(DEV, dtype)
    out = bri.invert_block(M, k, i, j, precision=precision, concurrency=concurrency, info=info,
                           pivoting=pivoting, order=order)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), int(info.item())


@pytest.mark.parametrize("n,k,targets", [(192, 3, [(0, 0), (2, 1), (1, 2)]), (256, 4, [(0, 0), (1, 2), (3, 3)]),
                                         (320, 5, [(0, 0), (4, 1), (2, 2)]), (384, 6, [(0, 0), (5, 2)]),
                                         (1024, 4, [(0, 0), (2, 3)])])
@pytest.mark.parametrize("W", [1, 0])
def test_literal_order_matches_the_literal_oracle(n, k, targets, W):
    m = workloads.gaussian_dd(n, 70 * n + k)
    for (i, j) in targets:
        print(f"literal n={n} k={k} ({i},{j}) W={W}", flush=True)
        got, info = run(m, k, i, j, concurrency=W)
        assert info == 0
        want = oracle.literal_invert_block(m, k, i, j)
        # Off-diagonal targets: the literal order pivots on Gaussian
        # off-diagonal blocks (no diagonal shift; condition numbers in the
        # hundreds at these orders) and finally inverts N_ij^{-1}, so the two
        # rounding orders differ by more than for the principal pivots.
        assert rel(got, want) < (1e-12 if i == j else 1e-10), (i, j)


def test_literal_order_fp32():
    # Diagonal target (1, 1), k = 4: the literal order exchanges block row
    # and column 0 with 1 alike, so its pivots are principal Schur
    # complements of the permuted matrix and the FP32 bound of the principal
    # path applies (c eps32 cond(M), c = 64).
    m = workloads.gaussian_dd(256, 91)
    got, info = run(m, 4, 1, 1, precision="f32")
    assert info == 0
    assert rel(got, oracle.literal_invert_block(m, 4, 1, 1)) < 64 * 2.0 ** -24 * np.linalg.cond(m)


def test_literal_order_reports_its_singular_pivot():
    # Tridiagonal M: a non-principal pivot of the literal order at k = 5 is
    # exactly singular (the oracle fails there too); the device status
    # reports it, under tile and under panel pivoting, and the principal
    # order gets the block.
    n, k = 320, 5
    m = workloads.tridiag_toeplitz(n)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.literal_invert_block(workloads.tridiag_toeplitz(20), k, 0, 0)
    for piv in ("tile", "panel"):
        _, info = run(m, k, 0, 0, pivoting=piv)
        print(f"tridiagonal literal {piv}: info {info}", flush=True)
        assert info > 0
    got, info = run(m, k, 0, 0, order="principal")
    assert info == 0
    assert rel(got, np.linalg.inv(m)[:64, :64]) < 1e-12
