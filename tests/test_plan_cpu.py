"""Host-side checks of libbri.so that need no GPU.

* every function declared in include/bri.h is exported by the library;
* invalid arguments are rejected synchronously with LAPACK-style codes;
* the planner's step list, executed step by step by a small NumPy
  interpreter written here (test-only; it is neither the oracle nor the
  product), reproduces blocks of inv(Gamma) -- this checks the scheduling,
  slot reuse and operand bookkeeping of the host planner on the CPU;
* the plan performs sum_{i=1}^{k-1} 4^{k-1-i} Schur operations (Theorem
  "C_BRI") and its live workspace stays within (k + 1) blocks per branch
  evaluated side by side.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg

import paper_1612_00001_amd as bri
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bri.h")

ST_LOAD, ST_GETRF, ST_TRTRI, ST_TRMM_L, ST_TRMM_U, ST_GEMM, ST_GEMM_ACC, ST_GEMM_NEG = range(1, 9)
O_NONE, O_SLOT, O_MBLK, O_IDENT, O_OUT, O_RHS = range(6)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(bri.LIB_PATH)
    names = declared_functions()
    assert "invert_block" in names and "invert_block_batched" in names and "invert_block_backward" in names
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    assert bri.version().startswith("bri-mi355x")
    assert "workspace" in bri.status_string(bri.BRI_ERR_WORKSPACE)
    assert "argument" in bri.status_string(-4)


def _call_invert(M_ptr, n, ldm, k, i, j, out_ptr, ldo, opts):
    return bri.lib().invert_block(M_ptr, n, ldm, k, i, j, out_ptr, ldo, opts)


def test_argument_validation_codes():
    o = bri.make_opts("f64")
    fake = 0x1000  # never dereferenced: validation happens before any work
    assert _call_invert(None, 8, 8, 2, 0, 0, fake, 4, ctypes.byref(o)) == -1
    assert _call_invert(fake, 0, 8, 2, 0, 0, fake, 4, ctypes.byref(o)) == -2
    assert _call_invert(fake, 8, 7, 2, 0, 0, fake, 4, ctypes.byref(o)) == -3
    assert _call_invert(fake, 8, 8, 1, 0, 0, fake, 4, ctypes.byref(o)) == -4
    assert _call_invert(fake, 8, 8, 9, 0, 0, fake, 4, ctypes.byref(o)) == -4
    assert _call_invert(fake, 8, 8, 2, 2, 0, fake, 4, ctypes.byref(o)) == -5
    assert _call_invert(fake, 8, 8, 2, 0, -1, fake, 4, ctypes.byref(o)) == -6
    assert _call_invert(fake, 8, 8, 2, 0, 0, None, 4, ctypes.byref(o)) == -7
    assert _call_invert(fake, 8, 8, 2, 0, 0, fake, 3, ctypes.byref(o)) == -8
    assert _call_invert(fake, 8, 8, 2, 0, 0, fake, 4, None) == -9
    # workspace missing / too small
    assert _call_invert(fake, 8, 8, 2, 0, 0, fake, 4, ctypes.byref(o)) == bri.BRI_ERR_WORKSPACE
    o.workspace = fake
    o.workspace_bytes = 16
    assert _call_invert(fake, 8, 8, 2, 0, 0, fake, 4, ctypes.byref(o)) == bri.BRI_ERR_WORKSPACE
    # block larger than the supported maximum
    assert bri.lib().bri_workspace_size(10000, 2, 0, 0, ctypes.byref(o)) == 0


def test_theorem_schur_counts_and_workspace_bound():
    for (n, k) in [(64, 2), (96, 3), (128, 4), (160, 5), (192, 6), (224, 7), (256, 8)]:
        T = sum(4 ** (k - 1 - i) for i in range(1, k))
        for (i, j) in [(0, 0), (k - 1, 0), (1, 1)]:
            for W in (1, 4, 16):
                d = bri.plan_describe(n, k, i, j, "f64", W)
                assert d["schur_ops"] == T
                assert d["final_inversions"] == 1
                w_eff = d["batch_width"]
                batch = 1
                while batch * 4 <= w_eff:
                    batch *= 4
                if W == 1:
                    # one pending block per recursion level + the leaf's
                    # working set: (k + 1) blocks, one more for i != j
                    assert d["slots"] <= k + 1 + (1 if i != j else 0)
                # breadth-first top (< 4/3 batch blocks per level above the
                # lock-step depth) plus (k + 1) per lock-step branch
                assert d["slots"] <= batch * (k + 1) + (4 * batch) // 3 * k + 2


def test_binding_lays_out_bri_opts_like_the_library():
    # The ctypes structure of the binding and the C struct agree in size (a
    # field missing on either side changes it).
    assert ctypes.sizeof(bri.BriOpts) == bri.lib().bri_opts_size()


def test_auto_width_is_a_power_of_four():
    d = bri.plan_describe(4096, 4, 0, 0, "f64", 0)
    assert d["batch_width"] == 16
    d = bri.plan_describe(16384, 8, 0, 0, "f64", 0)
    assert d["batch_width"] == 256
    # the estimated live workspace stays within 48 GiB
    assert d["workspace_bytes"] <= 48 * 2**30
    d = bri.plan_describe(32768, 8, 0, 0, "f64", 0)
    assert d["batch_width"] == 64
    assert d["workspace_bytes"] <= 48 * 2**30 + 2**28


def test_flop_accounting():
    b = 1024
    d = bri.plan_describe(4096, 4, 0, 0, "f64", 0)
    assert d["algorithmic_flops"] == pytest.approx(21 * 14 / 3 * b ** 3 + 2 * b ** 3)
    d2 = bri.plan_describe(4096, 4, 1, 2, "f64", 0)
    assert d2["algorithmic_flops"] == pytest.approx(21 * 14 / 3 * b ** 3 + 4 * b ** 3)
    assert d["executed_flops"] > d["algorithmic_flops"]


# ---------------------------------------------------------------------------
# Test-only interpreter of the step list
# ---------------------------------------------------------------------------

def run_plan(m: np.ndarray, k: int, steps, transpose=False, rhs=None, state=None):
    """Executes a step list; ``state`` (a dict) carries the slots and factors
    from one plan to the next (the refinement plans share kept pivots)."""
    n = m.shape[0]
    b = -(-n // k)
    g = np.eye(k * b)
    g[:n, :n] = m
    if transpose:
        g = g.T.copy()
    state = {} if state is None else state
    slots = state.setdefault("slots", {})
    factors = state.setdefault("factors", {})   # slot -> (perm, L, U) or ("inv", perm, Linv, Uinv)
    out = {}

    def blk(r, c):
        return g[r * b:(r + 1) * b, c * b:(c + 1) * b]

    def get(op):
        kind, a, bb = op
        if kind == O_SLOT:
            return slots[a]
        if kind == O_MBLK:
            return blk(a, bb)
        if kind == O_IDENT:
            return np.eye(b)
        if kind == O_OUT:
            return out[a]
        if kind == O_RHS:
            return rhs[a * b:(a + 1) * b]
        raise AssertionError(op)

    def put(op, val):
        kind, a, _ = op
        if kind == O_SLOT:
            slots[a] = val
            factors.pop(a, None)
        elif kind == O_OUT:
            out[a] = val
        else:
            raise AssertionError(op)

    for kind, items in steps:
        for dst, x, y, cin, sub, node in items:
            if kind == ST_LOAD:
                put(dst, get(x).copy())
            elif kind == ST_GETRF:
                p, l_, u = scipy.linalg.lu(slots[dst[1]])
                perm = np.argmax(p, axis=0)       # row r of P^T A is A[perm[r]]
                f = (perm, l_, u)
                slots[dst[1]] = np.full((b, b), np.nan)   # contents are now factors
                factors[dst[1]] = f
            elif kind == ST_TRTRI:
                perm, l_, u = factors[dst[1]]
                slots[x[1]] = np.full((b, b), np.nan)     # scratch
                factors.pop(x[1], None)
                factors[dst[1]] = ("inv", perm, np.linalg.inv(l_), np.linalg.inv(u))
            elif kind == ST_TRMM_L:
                _, perm, linv, _ = factors[x[1]]
                put(dst, linv @ get(y)[perm])
            elif kind == ST_TRMM_U:
                _, _, _, uinv = factors[x[1]]
                put(dst, uinv @ get(y))
            elif kind == ST_GEMM:
                v = -(get(x) @ get(y))
                if cin[0] != O_NONE:
                    v = get(cin) + v
                if sub[0] != O_NONE:
                    v = v - get(sub)
                put(dst, v)
            elif kind == ST_GEMM_ACC:
                v = get(x) @ get(y)
                if cin[0] != O_NONE:
                    v = get(cin) + v
                put(dst, v)
            elif kind == ST_GEMM_NEG:
                put(dst, -(get(x) @ get(y)))
            else:
                raise AssertionError(kind)
            for v in slots.values():
                pass
    return out


PLAN_CASES = [
    (16, 2, 0, 0, 1), (16, 2, 1, 0, 1), (16, 2, 0, 1, 1), (16, 2, 1, 1, 1),
    (18, 3, 0, 0, 1), (18, 3, 2, 1, 1), (18, 3, 1, 2, 4), (17, 3, 0, 2, 4),
    (24, 4, 0, 0, 1), (24, 4, 1, 2, 1), (24, 4, 3, 0, 4), (24, 4, 2, 2, 16), (23, 4, 3, 3, 16),
    (25, 5, 0, 0, 1), (25, 5, 4, 1, 4), (26, 5, 2, 3, 16), (25, 5, 1, 1, 64),
    (18, 6, 0, 0, 1), (18, 6, 5, 2, 16), (14, 7, 3, 3, 4),
]


@pytest.mark.parametrize("n,k,i,j,W", PLAN_CASES)
def test_plan_interpreter_reproduces_inverse_blocks(n, k, i, j, W):
    m = workloads.gaussian_dd(n, 1000 + 7 * n + k)
    steps = bri.plan_dump(n, k, i, j, "f64", W)
    out = run_plan(m, k, steps)
    b = -(-n // k)
    full = np.eye(k * b)
    full[:n, :n] = np.linalg.inv(m)
    want = full[i * b:(i + 1) * b, j * b:(j + 1) * b]
    assert np.abs(out[0] - want).max() < 1e-12


# ---------------------------------------------------------------------------
# Mixed-precision refinement plans (block column that keeps its pivots, then
# the correction solve with a general right-hand side)
# ---------------------------------------------------------------------------
REFINE_CASES = [(16, 2, 0, 1), (16, 2, 1, 4), (18, 3, 1, 1), (17, 3, 2, 4), (24, 4, 0, 1), (24, 4, 2, 16),
                (23, 4, 3, 4), (25, 5, 1, 1), (26, 5, 4, 64), (18, 6, 2, 16), (14, 7, 6, 4)]


@pytest.mark.parametrize("n,k,j,W", REFINE_CASES)
def test_refine_plans_column_then_general_solve(n, k, j, W):
    m = workloads.gaussian_dd(n, 2000 + 5 * n + k)
    b = -(-n // k)
    full = np.eye(k * b)
    full[:n, :n] = m
    inv = np.linalg.inv(full)
    state = {}
    col = run_plan(m, k, bri.refine_plan_dump(n, k, j, "column", W), state=state)
    x = np.vstack([col[t] for t in range(k)])
    assert np.abs(x - inv[:, j * b:(j + 1) * b]).max() < 1e-12
    kept = bri.refine_plan_dump(n, k, j, "kept", W)
    assert len(set(kept)) == k and all(s in state["factors"] for s in kept)
    rng = np.random.default_rng(n + k + j)
    for _ in range(2):  # the solve plan runs once per refinement sweep
        r = rng.standard_normal((k * b, b))
        sol = run_plan(m, k, bri.refine_plan_dump(n, k, j, "solve", W), rhs=r, state=state)
        y = np.vstack([sol[t] for t in range(k)])
        assert np.abs(y - np.linalg.solve(full, r)).max() < 1e-10
    # The correction solve never refactors: no getrf / trtri steps.
    kinds = {kind for kind, _ in bri.refine_plan_dump(n, k, j, "solve", W)}
    assert ST_GETRF not in kinds and ST_TRTRI not in kinds


def test_refine_solve_uses_three_way_recursion():
    # With the pivots kept, a depth-d value costs (3^d - 1) / 2 Schur steps
    # instead of (4^d - 1) / 3: count the triangular-solve pairs of the plan.
    for k in (3, 4, 5, 6):
        steps = bri.refine_plan_dump(32 * k, k, 0, "solve", 1)
        trmm_l = sum(len(items) for kind, items in steps if kind == ST_TRMM_L)
        c3 = [(3 ** d - 1) // 2 for d in range(k)]
        # x_last: value of depth k-1 (+1 solve); x_q at position p: (k - p) values of depth p (+1 solve)
        want = c3[k - 1] + 1 + sum((k - p) * c3[p] + 1 for p in range(k - 1))
        assert trmm_l == want, (k, trmm_l, want)


def test_no_kernel_spills_to_scratch():
    # The build records every kernel's register and scratch use (hipcc
    # resource remarks); a spill to scratch memory turns register traffic
    # into memory traffic in the hot loops.
    build_dir = os.path.join(ROOT, "paper_1612_00001_amd", "_build")
    reports = [os.path.join(build_dir, f) for f in ("bri_kernels.resources.txt", "bri_refine.resources.txt")]
    if not all(os.path.exists(r) for r in reports):
        pytest.skip("kernel resource report not built (run __graft_entry__.build())")
    spills = []
    for r in reports:
        for line in open(r):
            name, *fields = line.split()
            kv = dict(f.split("=") for f in fields)
            if int(kv["scratch"]) > 0:
                spills.append(name)
    assert not spills, spills


# ---------------------------------------------------------------------------
# Reuse of the elimination pivots (kept, factored once)
# ---------------------------------------------------------------------------
REUSE_CASES = [(16, 2, 0, 0, 1), (18, 3, 0, 0, 1), (18, 3, 2, 1, 4), (24, 4, 0, 0, 1), (24, 4, 1, 2, 4),
               (23, 4, 3, 3, 16), (25, 5, 0, 0, 4), (26, 5, 4, 1, 16), (18, 6, 5, 2, 64), (14, 7, 3, 3, 16)]


@pytest.mark.parametrize("n,k,i,j,W", REUSE_CASES)
def test_reuse_plan_interpreter_reproduces_inverse_blocks(n, k, i, j, W):
    m = workloads.gaussian_dd(n, 3000 + 7 * n + k)
    steps = bri.plan_dump(n, k, i, j, "f64", W, reuse=True)
    out = run_plan(m, k, steps)
    b = -(-n // k)
    full = np.eye(k * b)
    full[:n, :n] = m
    want = np.linalg.inv(full)[i * b:(i + 1) * b, j * b:(j + 1) * b]
    assert np.abs(out[0] - want).max() < 1e-12


def test_reuse_factorises_only_the_elimination_pivots():
    for k in (3, 4, 5, 6, 8):
        n = 16 * k
        d = bri.plan_describe(n, k, 0, 0, "f64", 1, reuse=True)
        steps = bri.plan_dump(n, k, 0, 0, "f64", 1, reuse=True)
        getrf = sum(len(items) for kind, items in steps if kind == ST_GETRF)
        # k - 2 kept pivots, the root pivot and the final inverse
        assert getrf == k, (k, getrf)
        assert d["final_inversions"] == k - 1
        # three children per node: the four root values of depth k - 2, the
        # kept pivots of depths 0 .. k - 3, and the root pivot's solve
        c3 = [(3 ** t - 1) // 2 for t in range(k)]
        assert d["schur_ops"] == 4 * c3[k - 2] + sum(c3[:k - 2]) + 1, (k, d["schur_ops"])
        assert d["schur_ops"] <= (4 ** (k - 1) - 1) // 3


@pytest.mark.parametrize("n,k,j,W", [(16, 2, 1, 1), (18, 3, 1, 4), (24, 4, 0, 1), (25, 5, 4, 16), (18, 6, 2, 16)])
def test_reuse_refine_plans(n, k, j, W):
    m = workloads.gaussian_dd(n, 4000 + 5 * n + k)
    b = -(-n // k)
    full = np.eye(k * b)
    full[:n, :n] = m
    inv = np.linalg.inv(full)
    state = {}
    run_plan(m, k, bri.refine_plan_dump(n, k, j, "column", W, reuse=True), state=state)
    kept = bri.refine_plan_dump(n, k, j, "kept", W, reuse=True)
    assert len(set(kept)) == k and all(s in state["factors"] for s in kept)
    ej = np.zeros((k * b, b))
    ej[j * b:(j + 1) * b] = np.eye(b)
    solve = bri.refine_plan_dump(n, k, j, "solve", W, reuse=True)
    x = run_plan(m, k, solve, rhs=ej, state=state)
    assert np.abs(np.vstack([x[t] for t in range(k)]) - inv[:, j * b:(j + 1) * b]).max() < 1e-12
    r = np.random.default_rng(n).standard_normal((k * b, b))
    y = run_plan(m, k, solve, rhs=r, state=state)
    assert np.abs(np.vstack([y[t] for t in range(k)]) - inv @ r).max() < 1e-10


@pytest.mark.parametrize("precision", ["f64", "mixed_f16"])
def test_workspace_budget_narrows_the_width(precision):
    # The memory / time trade-off of Theorem "MC_BRI": with a budget the
    # automatic width shrinks (by factors of 4) until the workspace fits;
    # below the width-1 workspace nothing fits.
    n, k = 16384, 8
    m_bytes = 8 * n * n
    free = bri.workspace_size(n, k, 0, 0, precision)
    w_free = bri.plan_describe(n, k, 0, 0, precision)["batch_width"]
    last_w = w_free
    for frac in (2.0, 1.0, 0.5, 0.25):
        budget = int(frac * m_bytes)
        need = bri.workspace_size(n, k, 0, 0, precision, workspace_budget=budget)
        if need == 0:
            continue
        assert need <= budget
        w = bri.plan_describe(n, k, 0, 0, precision, workspace_budget=budget)["batch_width"]
        assert w <= last_w
        last_w = w
        if free <= budget:
            assert need == free
    w1 = bri.workspace_size(n, k, 0, 0, precision, concurrency=1)
    assert bri.workspace_size(n, k, 0, 0, precision, workspace_budget=w1) == w1
    assert bri.workspace_size(n, k, 0, 0, precision, workspace_budget=w1 - 1) == 0
    # the FP64 path fits a quarter of M at width 1
    if precision == "f64":
        assert w1 <= m_bytes // 4


def test_mixed_workspace_below_the_matrix_at_width_one():
    # The mixed paths read M in place (block loads convert and scale it), so
    # at the precision workload's shape (k = 8) their workspace at width 1
    # stays below the size of M itself (about 0.67 of it: the FP64 block
    # column and residual of the refinement, 2 k b^2 doubles = 2 / k of M,
    # their float images, and the float slots with the k kept pivots).  At
    # k = 4 the column buffers alone are half of M's size.
    n, k = 16384, 8
    need = bri.workspace_size(n, k, 0, 0, "mixed_f16", concurrency=1)
    assert 0 < need < 0.75 * 8 * n * n


def test_tuning_cache_drives_the_lu_choice(tmp_path):
    # Tuning cache entries for factorisation launches of up to 256 matrices of
    # order 2048 override the built-in rule (which takes the recursive LU
    # there): the plan's launch count changes accordingly; an empty cache
    # restores it.
    n, k = 16384, 8
    auto = bri.plan_describe(n, k, 0, 0, "f64")["kernel_launches"]
    cache = tmp_path / "tune.txt"
    lines = [f"lu {c} 2048 0" for c in (1, 2, 4, 8, 16, 32, 64, 128, 256)] + ["product 8 0 256 2048 2048 3"]
    cache.write_text("# test\n" + "\n".join(lines) + "\n")
    try:
        assert bri.tune_load(str(cache)) == 10
        tiled = bri.plan_describe(n, k, 0, 0, "f64")["kernel_launches"]
        forced = bri.plan_describe(n, k, 0, 0, "f64", factorization="tile")["kernel_launches"]
        assert tiled == forced and tiled != auto
    finally:
        empty = tmp_path / "empty.txt"
        empty.write_text("")
        assert bri.tune_load(str(empty)) == 0
    assert bri.plan_describe(n, k, 0, 0, "f64")["kernel_launches"] == auto
    with pytest.raises(bri.BriError):
        bri.tune_load(str(tmp_path / "missing.txt"))


# ---------------------------------------------------------------------------
# The paper's literal frame order (typed frames, non-principal pivots)
# ---------------------------------------------------------------------------
LITERAL_CASES = [(16, 2, 0, 0, 1), (16, 2, 1, 0, 1), (18, 3, 0, 0, 1), (18, 3, 2, 1, 4), (24, 4, 0, 0, 1),
                 (24, 4, 1, 2, 4), (23, 4, 3, 3, 16), (25, 5, 0, 0, 1), (25, 5, 4, 1, 16), (25, 5, 2, 2, 64),
                 (18, 6, 5, 2, 64), (14, 7, 3, 3, 16)]


@pytest.mark.parametrize("n,k,i,j,W", LITERAL_CASES)
def test_literal_plan_follows_the_literal_oracle(n, k, i, j, W):
    import oracle
    m = workloads.gaussian_dd(n, 4000 + 7 * n + k)
    steps = bri.plan_dump(n, k, i, j, "f64", W, order="paper")
    out = run_plan(m, k, steps)
    want = oracle.literal_invert_block(m, k, i, j)
    assert np.abs(out[0] - want).max() < 1e-12
    d = bri.plan_describe(n, k, i, j, "f64", W, order="paper")
    assert d["schur_ops"] == (4 ** (k - 1) - 1) // 3 and d["final_inversions"] == 1


def test_literal_plan_pivots_on_non_principal_blocks():
    # Tridiagonal M (4 on the diagonal, -1 beside it), n = 20, k = 5: every
    # off-diagonal block has rank <= 1 and every principal Schur complement
    # is SPD.  The literal order's typed frames (M/C) and (M/B) pivot on
    # non-principal Schur complements, and for k = 5 one of them is exactly
    # singular here (as in the oracle); the principal order is not affected.
    import oracle
    m = workloads.tridiag_toeplitz(20)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.literal_invert_block(m, 5, 0, 0)
    with pytest.raises(np.linalg.LinAlgError):
        run_plan(m, 5, bri.plan_dump(20, 5, 0, 0, "f64", 4, order="paper"))
    out = run_plan(m, 5, bri.plan_dump(20, 5, 0, 0, "f64", 4))
    assert np.abs(out[0] - np.linalg.inv(m)[:4, :4]).max() < 1e-12


def test_literal_order_meets_a_singular_padded_pivot():
    # n = 26, k = 5 (b = 6): the last block row and column carry four rows of
    # Gamma's identity padding, so a non-principal pivot block taken from
    # them has zero rows.  The literal order meets such a pivot for block
    # (4, 1) (the oracle's dense solves fail there too); the principal order
    # pivots on principal blocks only and is unaffected.
    import oracle
    m = workloads.gaussian_dd(26, 4000 + 7 * 26 + 5)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.literal_invert_block(m, 5, 4, 1)
    with pytest.raises(np.linalg.LinAlgError):
        run_plan(m, 5, bri.plan_dump(26, 5, 4, 1, "f64", 16, order="paper"))
    out = run_plan(m, 5, bri.plan_dump(26, 5, 4, 1, "f64", 16))
    full = np.eye(30)
    full[:26, :26] = m
    assert np.abs(out[0] - np.linalg.inv(full)[24:30, 6:12]).max() < 1e-12


def test_literal_order_is_rejected_where_it_does_not_apply():
    assert bri.workspace_size(64, 4, 0, 0, "mixed_f16", order="paper") == 0
    assert bri.workspace_size(64, 4, 0, 0, "f64", reuse=True, order="paper") == 0
    assert bri.workspace_size(64, 4, 0, 0, "f64", order="paper") > 0
    with pytest.raises(ValueError):
        bri.make_opts("f64", order="literal")
