"""GPU parity of the matrix-free path (invert_block_rbf): blocks of the
inverse of the LS-SVM cross-validation matrix A_gamma (Section "Experimental
results", eq. A), whose elements the block loads evaluate from the data
points, against the FP64 oracle on the same matrix built densely here from
the equation.  The paper does not give its sigma, gamma or input sizes, so
the values below are choices; what is checked is that the matrix-free
evaluation and the recursion give the blocks of the dense A_gamma's inverse."""
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


@pytest.mark.parametrize("npts,d,k,sigma,gamma", [(255, 4, 4, 1.0, 10.0), (299, 7, 3, 2.0, 100.0),
                                                  (1023, 16, 4, 3.0, 1.0)])
def test_rbf_blocks_against_oracle(npts, d, k, sigma, gamma):
    x = workloads.lssvm_points(npts, d, npts + d)
    a = workloads.lssvm_matrix(x, sigma, gamma)
    X = torch.from_numpy(x).to(DEV)
    print(f"A_gamma npts={npts} d={d} k={k}", flush=True)
    for (i, j) in [(0, 0), (k - 1, k - 1), (1, 0), (k - 1, 1)]:
        info = torch.zeros(1, dtype=torch.int32, device=DEV)
        got = bri.invert_block_rbf(X, k, i, j, sigma, gamma, info=info).cpu().numpy()
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        err = rel(got, oracle.invert_block(a, k, i, j))
        print(f"  ({i},{j}) rel err {err:.2e}", flush=True)
        assert err < 1e-10


def test_rbf_diagonal_band_for_cross_validation():
    # The cross-validation only needs the diagonal blocks (Section
    # "Introduction"): every diagonal block, the matrix never stored.
    npts, d, k = 511, 8, 4
    x = workloads.lssvm_points(npts, d, 5)
    a = workloads.lssvm_matrix(x, 1.5, 20.0)
    X = torch.from_numpy(x).to(DEV)
    for i in range(k):
        got = bri.invert_block_rbf(X, k, i, i, 1.5, 20.0).cpu().numpy()
        assert rel(got, oracle.invert_block(a, k, i, i)) < 1e-10


def test_rbf_workspace_holds_no_copy_of_the_matrix():
    # At width 1 the workspace is a few b x b blocks, far below m^2 doubles.
    npts, d, k = 8191, 16, 8
    m = npts + 1
    need = bri.rbf_workspace_size(npts, d, k, 0, 0, concurrency=1)
    assert 0 < need < 8 * m * m // 4
