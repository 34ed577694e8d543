"""FP64 CPU oracle of the block recursive inverse (BRI).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the two meet only through the seeded inputs of ``workloads.py``.

Everything here is plain NumPy in float64.  ``np.linalg.solve`` / ``inv``
(LAPACK LU with partial pivoting, the same routine family the paper calls
through Armadillo ``inv()``, Section "Implementation") stand in for the b x b
"matrix inversion" step of every Schur complement.  There is no blocking,
fusion or reuse of sub-results: every node of the recursion is recomputed, as
the paper's branch-by-branch evaluation does (Section "Implementation";
Theorem "C_BRI" counts that recomputation).

Notation follows the paper (Section "Preliminaries"): M is m x m (here
``n x n``), partitioned into k x k square blocks of order b.  Block indices
are 0-based in this code; the paper's M_11 is block (0, 0) here.

Parity status of every public function is stated in its docstring; all of
them are pinned by ``tests/test_oracle_pins.py`` against brute-force inverses,
closed forms or invariants that do not go through this module.

Readings of the paper taken here (each is also listed in the design notes):

* (R1) elimination order.  The default "principal" order eliminates the
  blocks one at a time, always pivoting on a principal Schur complement
  v(p, p, I); for target (0, 0) and k <= 4 it performs exactly the paper's
  operations.  The frame bookkeeping of Section "Forward recursive procedure"
  is available as ``order="paper"`` (the literal frame splitting, swaps and
  typed Schur formulas) and must give the same block in exact arithmetic.
* (R2) arbitrary block (i, j).  The paper moves a block to the upper-left
  corner by a permutation (end of Section "Block Recursive Inversion
  algorithm").  Read literally for ``order="paper"``: swap block rows 0<->j
  and block columns 0<->i, then N_00 of the permuted matrix is N_ij.  The
  principal order instead finishes with the 2 x 2 inverse of eq. invSchur:
  with a = j and c = i (i != j), N_ij is the lower-left block
  G = -D^{-1} C (M/D)^{-1} of that equation.
* (R3) k does not divide n: the matrix is augmented with an identity block
  (eq. M_augmented) and the block of Gamma^{-1} is returned, b = ceil(n/k).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

__all__ = [
    "schur_op_count", "augment", "block_size", "principal_value", "elimination_plan",
    "invert_block", "literal_frames", "literal_invert_block", "block_column", "block_row",
    "block_solve", "inverse_block_grad", "OpCounter",
]


class OpCounter:
    """Counts executed Schur complement operations."""

    def __init__(self) -> None:
        self.schur = 0
        self.inversions = 0


def schur_op_count(k: int) -> int:
    """Schur operations BRI executes for one block: sum_{i=1}^{k-1} 4^{k-1-i}.

    Proof of Theorem "C_BRI" (Section "Complexity analysis"): step i of the
    backward procedure reduces 4^{k-1-i} 2 x 2 block matrices.
    """
    if k < 2:
        raise ValueError("k >= 2 required")
    return (4 ** (k - 1) - 1) // 3


def block_size(n: int, k: int) -> int:
    """b = ceil(n / k) (eq. M_augmented: the smallest l with (n + l)/k integral)."""
    return -(-n // k)


def augment(m: np.ndarray, k: int) -> np.ndarray:
    """Gamma = [[M, 0], [0^T, I_l]] of eq. M_augmented, l = k*b - n."""
    n = m.shape[0]
    b = block_size(n, k)
    size = k * b
    g = np.zeros((size, size), dtype=np.float64)
    g[:n, :n] = m
    for t in range(n, size):
        g[t, t] = 1.0
    return g


def _blk(g: np.ndarray, b: int, r: int, c: int) -> np.ndarray:
    return g[r * b:(r + 1) * b, c * b:(c + 1) * b]


# ---------------------------------------------------------------------------
# Principal elimination order
# ---------------------------------------------------------------------------

def principal_value(g: np.ndarray, b: int, r: int, c: int, elim: Sequence[int],
                    counter: OpCounter | None = None) -> np.ndarray:
    """v(r, c, I): block (r, c) left after eliminating the blocks in ``elim``.

    v(r, c, {}) = M_rc and, with p the last entry of I and I' the rest,
        v(r, c, I) = v(r, c, I') - v(r, p, I') v(p, p, I')^{-1} v(p, c, I'),
    i.e. the Schur complement (M/A) = D - C A^{-1} B of eq. SchurofA applied to
    the 2 x 2 block matrix [[v(p,p), v(p,c)], [v(r,p), v(r,c)]].  All four
    children are recomputed (no memoisation).
    """
    if len(elim) == 0:
        return _blk(g, b, r, c).copy()
    p = elim[-1]
    rest = elim[:-1]
    d = principal_value(g, b, r, c, rest, counter)
    cc = principal_value(g, b, r, p, rest, counter)
    a = principal_value(g, b, p, p, rest, counter)
    bb = principal_value(g, b, p, c, rest, counter)
    if counter is not None:
        counter.schur += 1
    return d - cc @ np.linalg.solve(a, bb)


def elimination_plan(k: int, i: int, j: int) -> Tuple[int, int, List[int]]:
    """(a, c, I): final 2 x 2 frame [[a, c], ...] and elimination sequence I.

    Target (i, i): a = i, c = the largest index != i, I = the other blocks in
    ascending order followed by c (the block eliminated last).
    Target (i, j), i != j: a = j, c = i, I = blocks other than i, j ascending,
    followed by i.  The last Schur step then pivots on v(c, c) and N_ij is the
    lower-left block of eq. invSchur (reading R2).
    """
    if not (0 <= i < k and 0 <= j < k):
        raise ValueError("block index out of range")
    if i == j:
        a = i
        c = max(t for t in range(k) if t != i)
    else:
        a, c = j, i
    rest = [t for t in range(k) if t not in (a, c)]
    return a, c, rest + [c]


def invert_block(m: np.ndarray, k: int, i: int, j: int, order: str = "principal",
                 counter: OpCounter | None = None) -> np.ndarray:
    """Block N_ij (b x b) of Gamma^{-1}, Gamma the augmented M (eq. M_augmented).

    ``order="principal"``: recursion of ``principal_value`` followed by the
    2 x 2 inverse of eq. invSchur:  Z = (M/D) of the final frame, N_aa = Z^{-1},
    and for i != j, N_ij = -v(c,c)^{-1} v(c,a) N_aa.
    ``order="paper"``: the literal frame procedure (``literal_invert_block``).

    Parity: pinned (brute-force Gauss-Jordan, closed forms, known inverses).
    """
    if order == "paper":
        return literal_invert_block(m, k, i, j, counter)
    if order != "principal":
        raise ValueError(order)
    if k < 2:
        raise ValueError("k >= 2 required")
    g = augment(np.asarray(m, dtype=np.float64), k)
    b = g.shape[0] // k
    a, c, elim = elimination_plan(k, i, j)
    rest = elim[:-1]
    s_aa = principal_value(g, b, a, a, rest, counter)
    s_ac = principal_value(g, b, a, c, rest, counter)
    s_cc = principal_value(g, b, c, c, rest, counter)
    s_ca = principal_value(g, b, c, a, rest, counter)
    x = np.linalg.solve(s_cc, s_ca)               # D^{-1} C
    if counter is not None:
        counter.schur += 1
    z = s_aa - s_ac @ x                           # (M/D), eq. SchurofD
    n_aa = np.linalg.inv(z)                       # E = (M/D)^{-1}, eq. invSchur
    if counter is not None:
        counter.inversions += 1
    if i == j:
        return n_aa
    return -x @ n_aa                              # G = -D^{-1} C (M/D)^{-1}


# ---------------------------------------------------------------------------
# Literal frame procedure (Sections "Forward/Backward recursive procedure")
# ---------------------------------------------------------------------------

def _exchange(rows: List[int], cols: List[int], ftype: str):
    """M_22 exchange of a frame with at least 3 blocks per side (Step 2).

    A frame of type B, C or D has its two leftmost block columns (B), its two
    uppermost block rows (C) or both (D) exchanged so that the original M_22
    returns to position (2, 2) (eq. F_k-1_ChangeM22).  The root frame and
    frames of type A are left as they are.
    """
    rows = list(rows)
    cols = list(cols)
    if len(rows) >= 3:
        if ftype in ("B", "D"):
            cols[0], cols[1] = cols[1], cols[0]
        if ftype in ("C", "D"):
            rows[0], rows[1] = rows[1], rows[0]
    return rows, cols


def _split(rows: List[int], cols: List[int]):
    """The four children of a frame (Step 1, eq. F_k-1).

    A drops the last block row and column, B the last row and first column,
    C the first row and last column, D the first row and first column.
    """
    return {
        "A": (rows[:-1], cols[:-1]),
        "B": (rows[:-1], cols[1:]),
        "C": (rows[1:], cols[:-1]),
        "D": (rows[1:], cols[1:]),
    }


def literal_frames(k: int) -> Dict[str, Tuple[List[int], List[int]]]:
    """Every frame of the forward procedure, keyed by its path ("", "B", "BA"...).

    Frames are returned *as they are split*, i.e. after the M_22 exchange of
    their own type when they have at least 3 blocks per side.  0-based
    block indices.  Pinned against the 4 x 4 worked example (Section "An
    example: inverse of 4 x 4 block matrices").
    """
    out: Dict[str, Tuple[List[int], List[int]]] = {}

    def visit(path, rows, cols, ftype):
        rows, cols = _exchange(rows, cols, ftype)
        out[path] = (rows, cols)
        if len(rows) >= 3:
            kids = _split(rows, cols)
            for t in "ABCD":
                visit(path + t, kids[t][0], kids[t][1], t)

    visit("", list(range(k)), list(range(k)), "R")
    return out


def _typed_schur(ftype: str, a, b_, c, d):
    """Schur complement of a typed 2 x 2 frame [[a, b], [c, d]].

    Types A, B, C, D use (M/D), (M/C), (M/B), (M/A) respectively
    (backward Step 1, eqs. SchurofD, SchurofC, SchurofB, SchurofA); the root
    frame uses (M/D) (backward Step k-1).
    """
    if ftype in ("A", "R"):
        return a - b_ @ np.linalg.solve(d, c)      # (M/D) = A - B D^{-1} C
    if ftype == "B":
        return b_ - a @ np.linalg.solve(c, d)      # (M/C) = B - A C^{-1} D
    if ftype == "C":
        return c - d @ np.linalg.solve(b_, a)      # (M/B) = C - D B^{-1} A
    if ftype == "D":
        return d - c @ np.linalg.solve(a, b_)      # (M/A) = D - C A^{-1} B
    raise ValueError(ftype)


def _literal_reduce(g, b, rows, cols, ftype, counter, values=None, path=""):
    if len(rows) == 2:
        a = _blk(g, b, rows[0], cols[0])
        b_ = _blk(g, b, rows[0], cols[1])
        c = _blk(g, b, rows[1], cols[0])
        d = _blk(g, b, rows[1], cols[1])
    else:
        rows, cols = _exchange(rows, cols, ftype)
        kids = _split(rows, cols)
        a = _literal_reduce(g, b, *kids["A"], "A", counter, values, path + "A")
        b_ = _literal_reduce(g, b, *kids["B"], "B", counter, values, path + "B")
        c = _literal_reduce(g, b, *kids["C"], "C", counter, values, path + "C")
        d = _literal_reduce(g, b, *kids["D"], "D", counter, values, path + "D")
    if counter is not None:
        counter.schur += 1
    s = _typed_schur(ftype, a, b_, c, d)
    if values is not None:
        values[path] = s
    return s


def literal_invert_block(m: np.ndarray, k: int, i: int, j: int,
                         counter: OpCounter | None = None,
                         values: Dict[str, np.ndarray] | None = None) -> np.ndarray:
    """N_ij by the paper's literal frame procedure (cross-check only).

    Block rows 0<->j and block columns 0<->i are exchanged (reading R2 of the
    permutation remark), the frames are split and reduced as in Sections
    "Forward/Backward recursive procedure", and N_00 of the permuted matrix is
    the inverse of the root's (M/D) (eq. blockmatrix_NxN).  ``values`` (if
    given) receives every reduced frame keyed by its path.

    Parity: pinned against brute force; it inverts non-principal blocks for
    k >= 5 and is singular on some matrices for which the principal order is
    not (see the tests).
    """
    if k < 2:
        raise ValueError("k >= 2 required")
    g = augment(np.asarray(m, dtype=np.float64), k)
    b = g.shape[0] // k
    rows = list(range(k))
    cols = list(range(k))
    rows[0], rows[j] = rows[j], rows[0]
    cols[0], cols[i] = cols[i], cols[0]
    z = _literal_reduce(g, b, rows, cols, "R", counter, values, "")
    if counter is not None:
        counter.inversions += 1
    return np.linalg.inv(z)


# ---------------------------------------------------------------------------
# Block column / block row / solve (back substitution with recomputed nodes)
# ---------------------------------------------------------------------------

def block_solve(m: np.ndarray, k: int, rhs: np.ndarray,
                counter: OpCounter | None = None) -> np.ndarray:
    """X = Gamma^{-1} R for an (k*b) x w right-hand side R, by block elimination.

    The blocks are eliminated in ascending order p = 0..k-1 on the bordered
    matrix [Gamma | R]; every Schur complement v(q, c, I) with c a block column
    of Gamma or the border column R is recomputed by the recursion of
    ``principal_value`` (the border column has leaves R_q).  Back substitution:
        x_q = v(q, q, I_q)^{-1} (v(q, R, I_q) - sum_{t after q} v(q, t, I_q) x_t),
    I_q the blocks before q.  ``rhs`` rows beyond n are the identity padding's
    rows and are returned unchanged (Gamma^{-1} = diag(M^{-1}, I)).

    Parity: pinned against ``np.linalg.solve`` on M.
    """
    g = augment(np.asarray(m, dtype=np.float64), k)
    b = g.shape[0] // k
    rhs = np.asarray(rhs, dtype=np.float64)
    if rhs.shape[0] != k * b:
        raise ValueError("rhs must have k*b rows")
    w = rhs.shape[1]

    def v(q, col, elim):
        # principal_value on the bordered matrix [Gamma | R]; the border is column k
        if col == k:
            if len(elim) == 0:
                return rhs[q * b:(q + 1) * b, :].copy()
            p = elim[-1]
            rest = elim[:-1]
            d = v(q, col, rest)
            cc = principal_value(g, b, q, p, rest, counter)
            a = principal_value(g, b, p, p, rest, counter)
            bb = v(p, col, rest)
            if counter is not None:
                counter.schur += 1
            return d - cc @ np.linalg.solve(a, bb)
        return principal_value(g, b, q, col, elim, counter)

    x: Dict[int, np.ndarray] = {}
    order = list(range(k))
    for pos in range(k - 1, -1, -1):
        q = order[pos]
        elim = order[:pos]
        acc = v(q, k, elim)
        for t in order[pos + 1:]:
            acc = acc - v(q, t, elim) @ x[t]
        x[q] = np.linalg.solve(v(q, q, elim), acc)
    return np.vstack([x[q] for q in range(k)])


def block_column(m: np.ndarray, k: int, j: int,
                 counter: OpCounter | None = None) -> np.ndarray:
    """Block column j of Gamma^{-1}: the (k*b) x b matrix X with Gamma X = E_j.

    "Spine" back substitution.  With P = (blocks != j, ascending) and
    I_q = the entries of P before q:
        x_j = v(j, j, P)^{-1},
        x_q = -v(q, q, I_q)^{-1} (v(q, j, I_q) x_j + sum_{t after q in P} v(q, t, I_q) x_t)
    for q = last of P down to the first; this is block elimination of
    Gamma X = E_j with j eliminated last, whose right-hand side stays zero in
    every block row other than j.  All v's are recomputed by the recursion.

    Parity: pinned (Gamma X = E_j, brute-force inverse).
    """
    g = augment(np.asarray(m, dtype=np.float64), k)
    b = g.shape[0] // k
    p_order = [t for t in range(k) if t != j]
    x: Dict[int, np.ndarray] = {}
    root = principal_value(g, b, j, j, p_order, counter)
    x[j] = np.linalg.inv(root)
    for pos in range(len(p_order) - 1, -1, -1):
        q = p_order[pos]
        elim = p_order[:pos]
        acc = principal_value(g, b, q, j, elim, counter) @ x[j]
        for t in p_order[pos + 1:]:
            acc = acc + principal_value(g, b, q, t, elim, counter) @ x[t]
        x[q] = -np.linalg.solve(principal_value(g, b, q, q, elim, counter), acc)
    return np.vstack([x[q] for q in range(k)])


def block_row(m: np.ndarray, k: int, i: int, counter: OpCounter | None = None) -> np.ndarray:
    """Block row i of Gamma^{-1} (b x (k*b)), the transposed block column of M^T."""
    return block_column(np.asarray(m).T, k, i, counter).T


def inverse_block_grad(m: np.ndarray, k: int, i: int, j: int, w: np.ndarray) -> np.ndarray:
    """dL/dM for L = sum(W * N_ij), N = M^{-1} (Gamma^{-1} when k does not divide n).

    dN = -N dM N gives dL/dM = -(N_{i,:})^T W (N_{:,j})^T, the n x n top-left
    part of -Gamma^{-T} Wbar Gamma^{-T} with W placed at block (i, j).  The
    block row and column are computed with ``block_row`` / ``block_column``.

    Parity: pinned (central finite differences, dense formula).
    """
    n = m.shape[0]
    u = block_row(m, k, i).T          # (k*b) x b
    v = block_column(m, k, j)         # (k*b) x b
    full = -(u @ np.asarray(w, dtype=np.float64)) @ v.T
    return full[:n, :n]
