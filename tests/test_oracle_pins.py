"""Pins of the FP64 oracle against results fixed by the paper and by mathematics.

None of these checks goes back through the oracle's own arithmetic: the
expected values come from exact rational Gauss-Jordan elimination, closed-form
inverses (orthogonal diagonalisation, Usmani's tridiagonal formula), the
worked 4 x 4 example printed in the paper, dense LAPACK solves of the whole
matrix, and invariants (operation counts, Gamma X = E_j, finite
differences).  The last group plants plausible mistakes in the oracle and
checks that the pins catch each of them.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import bri_oracle as ob
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Independent references
# ---------------------------------------------------------------------------

def gauss_jordan_exact(a_int):
    """Exact inverse of an integer matrix by Gauss-Jordan with partial pivoting (Fractions)."""
    n = len(a_int)
    a = [[Fraction(int(a_int[r][c])) for c in range(n)] + [Fraction(int(r == c)) for c in range(n)]
         for r in range(n)]
    for col in range(n):
        piv = max(range(col, n), key=lambda r: abs(a[r][col]))
        if a[piv][col] == 0:
            raise ZeroDivisionError("singular")
        a[col], a[piv] = a[piv], a[col]
        inv = 1 / a[col][col]
        a[col] = [x * inv for x in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [x - f * y for x, y in zip(a[r], a[col])]
    return [[a[r][n + c] for c in range(n)] for r in range(n)]


def gamma_block(inv_exact, n, k, i, j):
    """Block (i, j) of Gamma^{-1} = diag(M^{-1}, I) (eq. inverse_M_augmented) as floats."""
    b = -(-n // k)
    out = np.zeros((b, b))
    for r in range(b):
        for c in range(b):
            gr, gc = i * b + r, j * b + c
            if gr < n and gc < n:
                out[r, c] = float(inv_exact[gr][gc])
            elif gr == gc:
                out[r, c] = 1.0
    return out


def int_matrix(n, seed, shift):
    r = np.random.default_rng(seed)
    a = r.integers(-5, 6, size=(n, n))
    a[np.diag_indices(n)] += shift
    return a


def usmani_inverse(diag, sup, sub):
    """Inverse of a tridiagonal matrix by Usmani's theta/phi recurrences (1-based formulas)."""
    n = len(diag)
    theta = [1.0, diag[0]]
    for i in range(2, n + 1):
        theta.append(diag[i - 1] * theta[i - 1] - sup[i - 2] * sub[i - 2] * theta[i - 2])
    phi = [0.0] * (n + 2)
    phi[n + 1] = 1.0
    phi[n] = diag[n - 1]
    for i in range(n - 1, 0, -1):
        phi[i] = diag[i - 1] * phi[i + 1] - sup[i - 1] * sub[i - 1] * phi[i + 2]
    t = np.zeros((n, n))
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if i < j:
                prod = np.prod([sup[q - 1] for q in range(i, j)])
                t[i - 1, j - 1] = (-1) ** (i + j) * prod * theta[i - 1] * phi[j + 1] / theta[n]
            elif i == j:
                t[i - 1, j - 1] = theta[i - 1] * phi[i + 1] / theta[n]
            else:
                prod = np.prod([sub[q - 1] for q in range(j, i)])
                t[i - 1, j - 1] = (-1) ** (i + j) * prod * theta[j - 1] * phi[i + 1] / theta[n]
    return t


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ---------------------------------------------------------------------------
# Whole result: brute force
# ---------------------------------------------------------------------------

CASES_EXACT = [(8, 2), (9, 3), (8, 4), (10, 3), (10, 4), (7, 4), (10, 5), (6, 6)]


@pytest.mark.parametrize("n,k", CASES_EXACT)
@pytest.mark.parametrize("order", ["principal", "paper"])
def test_every_block_matches_exact_gauss_jordan(n, k, order):
    if order == "paper" and k > 4:
        # For k >= 5 the literal frames invert non-principal blocks, which
        # small-integer matrices make exactly singular; the literal order is
        # checked on Gaussian matrices for k = 5, 6 below.
        pytest.skip("literal order inverts non-principal blocks for k >= 5")
    a = int_matrix(n, seed=n * 31 + k, shift=3 * n)
    exact = gauss_jordan_exact(a.tolist())
    for i in range(k):
        for j in range(k):
            if order == "paper" and n % k and i != j:
                # The literal corner permutation inverts N_ij^{-1}, which is
                # singular when N_ij meets the identity padding of Gamma.
                continue
            got = oracle.invert_block(a.astype(np.float64), k, i, j, order=order)
            want = gamma_block(exact, n, k, i, j)
            assert np.allclose(got, want, rtol=1e-13, atol=1e-15), (i, j)


def test_general_gaussian_matches_exact_gauss_jordan():
    # Non-dominant integer matrix: pivots are general (non-symmetric, not dominant).
    a = int_matrix(8, seed=7, shift=0)
    exact = gauss_jordan_exact(a.tolist())
    for (i, j) in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        got = oracle.invert_block(a.astype(np.float64), 2, i, j)
        want = gamma_block(exact, 8, 2, i, j)
        assert rel(got, want) < 1e-11


# ---------------------------------------------------------------------------
# k = 2: the four blocks of eq. invSchur with explicit inverses
# ---------------------------------------------------------------------------

def test_two_by_two_closed_form():
    m = workloads.gaussian_dd(12, 11)
    a, bq, c, d = m[:6, :6], m[:6, 6:], m[6:, :6], m[6:, 6:]
    dinv = np.linalg.inv(d)
    e = np.linalg.inv(a - bq @ dinv @ c)
    f = -e @ bq @ dinv
    g = -dinv @ c @ e
    h = dinv + dinv @ c @ e @ bq @ dinv
    for (i, j), want in {(0, 0): e, (0, 1): f, (1, 0): g, (1, 1): h}.items():
        assert rel(oracle.invert_block(m, 2, i, j), want) < 1e-14


# ---------------------------------------------------------------------------
# Every internal node equals its closed-form generalised Schur complement
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_node_values_are_generalised_schur_complements(seed):
    k, b = 5, 3
    m = workloads.gaussian_dd(k * b, 100 + seed)
    rng = np.random.default_rng(seed)
    for _ in range(12):
        size = int(rng.integers(1, k - 1))
        elim = [int(t) for t in rng.permutation(k)[:size]]
        free = [t for t in range(k) if t not in elim]
        r, c = int(rng.choice(free)), int(rng.choice(free))
        idx = np.concatenate([np.arange(t * b, (t + 1) * b) for t in elim])
        rr = np.arange(r * b, (r + 1) * b)
        cc = np.arange(c * b, (c + 1) * b)
        want = m[np.ix_(rr, cc)] - m[np.ix_(rr, idx)] @ np.linalg.solve(m[np.ix_(idx, idx)],
                                                                       m[np.ix_(idx, cc)])
        got = oracle.principal_value(m, b, r, c, elim)
        assert rel(got, want) < 1e-13


# ---------------------------------------------------------------------------
# Orders and counts
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
def test_literal_order_equals_principal_order(k):
    m = workloads.gaussian_dd(2 * k, 200 + k)
    for (i, j) in {(0, 0), (k - 1, 0), (0, k - 1), (1, 1 % k)}:
        x = oracle.invert_block(m, k, i, j, order="principal")
        y = oracle.invert_block(m, k, i, j, order="paper")
        assert rel(x, y) < 1e-13


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("order", ["principal", "paper"])
def test_schur_operation_count_is_theorem_count(k, order):
    # Theorem C_BRI: sum_{i=1}^{k-1} 4^{k-1-i} Schur operations, one final inverse.
    expect = sum(4 ** (k - 1 - i) for i in range(1, k))
    assert oracle.schur_op_count(k) == expect
    m = workloads.gaussian_dd(k, 300 + k)
    for (i, j) in [(0, 0), (k - 1, 1)]:
        cnt = oracle.OpCounter()
        oracle.invert_block(m, k, i, j, order=order, counter=cnt)
        assert cnt.schur == expect
        assert cnt.inversions == 1


def test_paper_order_performs_the_papers_operations_for_k4():
    # For target (0,0) and k <= 4 the principal order eliminates M_22 first and
    # the last block last, exactly the operations of the worked example.
    assert oracle.elimination_plan(4, 0, 0) == (0, 3, [1, 2, 3])
    assert oracle.elimination_plan(3, 0, 0) == (0, 2, [1, 2])


# ---------------------------------------------------------------------------
# Gamma padding (eqs. M_augmented, inverse_M_augmented)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,k", [(10, 3), (11, 4), (5, 4), (13, 5)])
def test_gamma_padding_blocks(n, k):
    m = workloads.gaussian_dd(n, 400 + n)
    inv = np.linalg.inv(m)
    b = -(-n // k)
    full = np.eye(k * b)
    full[:n, :n] = inv
    for i in range(k):
        for j in range(k):
            got = oracle.invert_block(m, k, i, j)
            assert np.allclose(got, full[i * b:(i + 1) * b, j * b:(j + 1) * b], atol=1e-14)


# ---------------------------------------------------------------------------
# Known inverses
# ---------------------------------------------------------------------------

def test_orthogonal_diagonalisation_inverse():
    s = workloads.haar_spd(24, 5, 0.0, 2.0)
    inv = (s.q / s.lam[None, :]) @ s.q.T
    for k in (2, 3, 4):
        b = 24 // k
        for (i, j) in [(0, 0), (k - 1, k - 1), (0, k - 1), (k - 1, 1)]:
            got = oracle.invert_block(s.m, k, i, j)
            assert rel(got, inv[i * b:(i + 1) * b, j * b:(j + 1) * b]) < 1e-12


def test_tridiagonal_usmani_closed_form():
    n = 12
    t = workloads.tridiag_toeplitz(n, 4.0, -1.0)
    inv = usmani_inverse([4.0] * n, [-1.0] * (n - 1), [-1.0] * (n - 1))
    assert np.abs(inv @ t - np.eye(n)).max() < 1e-13   # the closed form itself
    for k in (2, 3, 4, 6):
        b = n // k
        for i in range(k):
            for j in range(k):
                got = oracle.invert_block(t, k, i, j)
                assert np.allclose(got, inv[i * b:(i + 1) * b, j * b:(j + 1) * b], atol=1e-14)


def test_literal_permutation_fails_where_principal_does_not():
    # Reading R2: the literal corner permutation inverts N_ij^{-1}; on a
    # tridiagonal matrix the off-diagonal blocks of the inverse have rank 1,
    # so that inversion is singular while the principal order is exact.
    t = workloads.tridiag_toeplitz(12, 4.0, -1.0)
    inv = np.linalg.inv(t)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.invert_block(t, 4, 1, 2, order="paper")
    assert np.allclose(oracle.invert_block(t, 4, 1, 2), inv[3:6, 6:9], atol=1e-15)


# ---------------------------------------------------------------------------
# Block column / row / solve and M X = E_j
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,k", [(12, 2), (12, 3), (12, 4), (11, 3), (15, 5)])
def test_block_column_satisfies_m_x_eq_ej(n, k):
    m = workloads.gaussian_dd(n, 500 + n + k)
    b = -(-n // k)
    g = np.eye(k * b)
    g[:n, :n] = m
    for j in range(k):
        x = oracle.block_column(m, k, j)
        ej = np.zeros((k * b, b))
        ej[j * b:(j + 1) * b] = np.eye(b)
        assert np.abs(g @ x - ej).max() < 1e-13
        for i in range(k):
            assert np.allclose(x[i * b:(i + 1) * b], oracle.invert_block(m, k, i, j), atol=1e-15)


def test_block_row_and_solve():
    m = workloads.gaussian_dd(12, 600)
    inv = np.linalg.inv(m)
    for k in (2, 3, 4):
        b = 12 // k
        for i in range(k):
            assert np.allclose(oracle.block_row(m, k, i), inv[i * b:(i + 1) * b], atol=1e-15)
        r = np.random.default_rng(k).standard_normal((12, 5))
        assert np.allclose(oracle.block_solve(m, k, r), np.linalg.solve(m, r), atol=1e-14)


def test_spine_cost_is_larger_than_one_block():
    # Recomputing the back-substitution nodes costs more than one block (k >= 3).
    m = workloads.gaussian_dd(12, 601)
    for k in (3, 4):
        cnt = oracle.OpCounter()
        oracle.block_column(m, k, 0, counter=cnt)
        assert cnt.schur > oracle.schur_op_count(k)


# ---------------------------------------------------------------------------
# Gradient: finite differences and the dense formula
# ---------------------------------------------------------------------------

def test_gradient_central_differences():
    n, k, i, j = 9, 3, 2, 1
    m = workloads.gaussian_dd(n, 700)
    w = workloads.cotangent(3, seed=701)
    grad = oracle.inverse_block_grad(m, k, i, j, w)
    h = 1e-6
    fd = np.zeros((n, n))
    for r in range(n):
        for c in range(n):
            mp = m.copy()
            mm = m.copy()
            mp[r, c] += h
            mm[r, c] -= h
            fp = np.sum(w * oracle.invert_block(mp, k, i, j))
            fm = np.sum(w * oracle.invert_block(mm, k, i, j))
            fd[r, c] = (fp - fm) / (2 * h)
    assert rel(grad, fd) < 1e-7


def test_gradient_dense_formula_with_padding():
    n, k, i, j = 10, 3, 0, 2
    m = workloads.gaussian_dd(n, 702)
    b = 4
    w = workloads.cotangent(b, seed=703)
    inv = np.linalg.inv(m)
    wbar = np.zeros((k * b, k * b))
    wbar[i * b:(i + 1) * b, j * b:(j + 1) * b] = w
    want = -inv.T @ wbar[:n, :n] @ inv.T
    assert rel(oracle.inverse_block_grad(m, k, i, j, w), want) < 1e-13


# ---------------------------------------------------------------------------
# The worked 4 x 4 example (Section "An example: inverse of 4 x 4 block matrices")
# ---------------------------------------------------------------------------

def _read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([p.strip() for p in line.split("|")])
    return rows


def test_frames_match_the_printed_example():
    frames = oracle.literal_frames(4)
    for path, rows, cols in _read_table("frames_4x4.txt"):
        r = [int(t) - 1 for t in rows.split()]
        c = [int(t) - 1 for t in cols.split()]
        assert frames[path] == (r, c), path


def test_exchange_rule_for_larger_k():
    # eq. F_k-1_ChangeM22: the first two columns of M>_B are (3, 2, 4, ...), the
    # first two rows of M>_C are (3, 2, 4, ...), both for M>_D.
    for k in (5, 6):
        f = oracle.literal_frames(k)
        assert f["B"] == (list(range(k - 1)), [2, 1] + list(range(3, k)))
        assert f["C"] == ([2, 1] + list(range(3, k)), list(range(k - 1)))
        assert f["D"] == ([2, 1] + list(range(3, k)), [2, 1] + list(range(3, k)))


def test_leaf_values_match_the_printed_formulas():
    b = 3
    m = workloads.gaussian_dd(4 * b, 800)

    def blk(pq):
        r, c = int(pq[0]) - 1, int(pq[1]) - 1
        return m[r * b:(r + 1) * b, c * b:(c + 1) * b]

    values = {}
    ob.literal_invert_block(m, 4, 0, 0, values=values)
    m22inv = np.linalg.inv(blk("22"))
    for path, pq, rs, tu in _read_table("leaf_formulas_4x4.txt"):
        want = blk(pq) - blk(rs) @ m22inv @ blk(tu)
        assert rel(values[path], want) < 1e-14, path
    for frame, p, q, r_, s in _read_table("level2_formulas_4x4.txt"):
        want = values[frame + p] - values[frame + q] @ np.linalg.inv(values[frame + r_]) @ values[frame + s]
        assert rel(values[frame], want) < 1e-13, frame
    # eq. blockmatrix4x4: N_11 = (<<A>> - <<B>> <<D>>^{-1} <<C>>)^{-1}
    n11 = np.linalg.inv(values["A"] - values["B"] @ np.linalg.inv(values["D"]) @ values["C"])
    assert rel(n11, np.linalg.inv(m)[:b, :b]) < 1e-13


# ---------------------------------------------------------------------------
# Planted mistakes: every one must be caught by a pin above
# ---------------------------------------------------------------------------

def _pins_hold():
    """A fast subset of the pins; False if any of them fails."""
    try:
        a = int_matrix(9, seed=9 * 31 + 3, shift=27)
        exact = gauss_jordan_exact(a.tolist())
        for (i, j) in [(0, 0), (1, 2), (2, 0), (2, 2)]:
            got = oracle.invert_block(a.astype(np.float64), 3, i, j)
            if not np.allclose(got, gamma_block(exact, 9, 3, i, j), rtol=1e-12, atol=1e-14):
                return False
        m = workloads.gaussian_dd(10, 401)
        full = np.eye(12)
        full[:10, :10] = np.linalg.inv(m)
        for (i, j) in [(2, 2), (2, 0)]:
            if not np.allclose(oracle.invert_block(m, 3, i, j), full[i * 4:(i + 1) * 4, j * 4:(j + 1) * 4],
                               atol=1e-13):
                return False
        x = oracle.block_column(m, 3, 1)
        if not np.allclose(x, full[:, 4:8], atol=1e-13):
            return False
        return True
    except (np.linalg.LinAlgError, ValueError, IndexError, KeyError):
        return False


def _mut_sign(g, b, r, c, elim, counter=None, _orig=ob.principal_value):
    if not elim:
        return _orig(g, b, r, c, elim, counter)
    p, rest = elim[-1], elim[:-1]
    return (_mut_sign(g, b, r, c, rest) + _mut_sign(g, b, r, p, rest)
            @ np.linalg.solve(_mut_sign(g, b, p, p, rest), _mut_sign(g, b, p, c, rest)))


def _mut_transpose(g, b, r, c, elim, counter=None, _orig=ob.principal_value):
    if not elim:
        return _orig(g, b, r, c, elim, counter)
    p, rest = elim[-1], elim[:-1]
    return (_mut_transpose(g, b, r, c, rest) - _mut_transpose(g, b, r, p, rest)
            @ np.linalg.solve(_mut_transpose(g, b, p, p, rest).T, _mut_transpose(g, b, p, c, rest)))


def _mut_index(g, b, r, c, elim, counter=None, _orig=ob.principal_value):
    if not elim:
        return _orig(g, b, r, c, elim, counter)
    p, rest = elim[-1], elim[:-1]
    return (_mut_index(g, b, r, c, rest) - _mut_index(g, b, r, p, rest)
            @ np.linalg.solve(_mut_index(g, b, p, p, rest), _mut_index(g, b, c, p, rest)))


def _mut_drop(g, b, r, c, elim, counter=None, _orig=ob.principal_value):
    return _orig(g, b, r, c, [], counter)


def _mut_plan(k, i, j, _orig=ob.elimination_plan):
    return _orig(k, j, i)


def _mut_augment(m, k, _orig=ob.augment):
    g = _orig(m, k)
    n = m.shape[0]
    for t in range(n, g.shape[0]):
        g[t, t] = 2.0
    return g


@pytest.mark.parametrize("name,attr,mutant", [
    ("sign", "principal_value", _mut_sign),
    ("transposed pivot", "principal_value", _mut_transpose),
    ("wrong index", "principal_value", _mut_index),
    ("dropped term", "principal_value", _mut_drop),
    ("swapped target", "elimination_plan", _mut_plan),
    ("padding", "augment", _mut_augment),
])
def test_planted_mistakes_are_caught(monkeypatch, name, attr, mutant):
    assert _pins_hold()
    monkeypatch.setattr(ob, attr, mutant)
    assert not _pins_hold(), name
