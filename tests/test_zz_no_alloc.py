"""The entry point that allocates nothing (invert_block_noalloc), through the
C ABI: its blocks against invert_block's on the same inputs, on two calls in
a row (the second smaller), and its size limit."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import paper_1612_00001_amd as bri
import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def noalloc_call(M, k, i, j, out, info):
    o = bri.make_opts("f64")
    o.d_info = info.data_ptr()
    o.stream = torch.cuda.current_stream().cuda_stream
    return bri.lib().invert_block_noalloc(M.data_ptr(), M.shape[0], M.stride(0), k, i, j, out.data_ptr(),
                                          out.stride(0), ctypes.byref(o))


@pytest.mark.parametrize("pivoting_case", ["spd_then_dd"])
def test_noalloc_matches_invert_block_two_calls(pivoting_case):
    cases = [(workloads.haar_spd(1024, 91, 0.0, 2.0).m, 4, 1, 2),   # b = 256
             (workloads.gaussian_dd(256, 92), 2, 0, 0)]              # smaller: b = 128
    for m, k, i, j in cases:
        M = torch.from_numpy(m).to(DEV)
        b = bri.block_size(m.shape[0], k)
        out = torch.full((b, b), float("nan"), dtype=torch.float64, device=DEV)
        info = torch.full((1,), 7, dtype=torch.int32, device=DEV)
        print(f"noalloc n={m.shape[0]} k={k} ({i},{j})", flush=True)
        rc = noalloc_call(M, k, i, j, out, info)
        assert rc == 0, bri.status_string(rc)
        want = bri.invert_block(M, k, i, j)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        err = rel(out.cpu().numpy(), want.cpu().numpy())
        print(f"  rel diff vs invert_block {err:.2e}", flush=True)
        assert err < 1e-12


def test_noalloc_rejects_sizes_beyond_the_scratch():
    # n = 16384, k = 8 needs far more than the static array even at width 1:
    # a clear error, nothing enqueued.
    assert bri.lib().bri_noalloc_scratch_bytes() == 64 << 20
    M = torch.empty(16384, 16384, dtype=torch.float64, device=DEV)
    out = torch.empty(2048, 2048, dtype=torch.float64, device=DEV)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert noalloc_call(M, 8, 0, 0, out, info) == bri.BRI_ERR_WORKSPACE
