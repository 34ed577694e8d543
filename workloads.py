"""Seeded synthetic inputs for the block recursive inverse.

This module only *constructs* input matrices; it contains none of the
inversion method's arithmetic.  It is the one module shared by the FP64 CPU
oracle (``oracle/``), the tests and ``bench.py``.

Matrix families (all dense, row-major, float64):

* ``gaussian_dd`` -- entries i.i.d. N(0, 1) with ``n`` added to the diagonal
  (diagonally dominant; the paper's own experiments draw N(0, 1) entries,
  Section "Experimental results").
* ``haar_spd`` -- ``Q diag(lam) Q^T`` with ``Q`` Haar-distributed orthogonal
  (QR of a Gaussian matrix with the sign of ``diag(R)`` folded into ``Q``,
  Mezzadri 2007) and ``lam`` log-uniform between two decades.
* ``gaussian`` -- plain N(0, 1) entries (the paper's ``randn`` matrices).
* ``tridiag_toeplitz`` -- constant tridiagonal matrix, used as a matrix with a
  closed-form inverse.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np


def rng_for(seed) -> np.random.Generator:
    """PCG64 generator for an integer seed or a ``SeedSequence``."""
    return np.random.default_rng(seed)


def gaussian(n: int, seed) -> np.ndarray:
    """n x n matrix with i.i.d. N(0, 1) entries."""
    return rng_for(seed).standard_normal((n, n))


def gaussian_dd(n: int, seed, shift: float | None = None) -> np.ndarray:
    """N(0, 1) entries with ``shift`` (default ``n``) added on the diagonal."""
    m = gaussian(n, seed)
    m[np.diag_indices(n)] += float(n if shift is None else shift)
    return m


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix (QR of a Gaussian, signs fixed)."""
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    q *= np.sign(np.diag(r))[None, :]
    return q


@dataclasses.dataclass
class SpdMatrix:
    m: np.ndarray      # Q diag(lam) Q^T
    q: np.ndarray      # the orthogonal factor
    lam: np.ndarray    # the eigenvalues


def haar_spd(n: int, seed, lo_exp: float = 0.0, hi_exp: float = 2.0,
             pin_endpoints: bool = False) -> SpdMatrix:
    """``Q diag(lam) Q^T`` with ``lam = 10**U(lo_exp, hi_exp)``.

    With ``pin_endpoints`` the smallest and largest eigenvalues are set to
    exactly ``10**lo_exp`` and ``10**hi_exp`` so that the 2-norm condition
    number is exactly ``10**(hi_exp - lo_exp)``.
    """
    rng = rng_for(seed)
    q = haar_orthogonal(n, rng)
    lam = 10.0 ** rng.uniform(lo_exp, hi_exp, size=n)
    if pin_endpoints and n >= 2:
        lam[0] = 10.0 ** lo_exp
        lam[-1] = 10.0 ** hi_exp
    m = (q * lam[None, :]) @ q.T
    m = 0.5 * (m + m.T)
    return SpdMatrix(m=m, q=q, lam=lam)


def haar_spd_device(n: int, seed, lo_exp: float = 0.0, hi_exp: float = 2.0, pin_endpoints: bool = False,
                    device="cuda:0", return_factors: bool = False):
    """The ``haar_spd`` recipe with the O(n^3) steps (QR, Q Lam Q^T) done by
    torch on ``device`` in float64, for sizes where the host would take
    minutes.  Same draws as ``haar_spd`` (the Gaussian and the eigenvalues
    come from the same seeded generator, in the same order); Q differs from
    the host one only by rounding (the QR is unique once the sign of
    diag(R) is fixed).  Returns a float64 device tensor, or with
    ``return_factors`` the tuple (M, Q, lam) with Q on the device and lam a
    host array."""
    import torch

    rng = rng_for(seed)
    z = torch.from_numpy(rng.standard_normal((n, n))).to(device)
    lam = 10.0 ** rng.uniform(lo_exp, hi_exp, size=n)
    if pin_endpoints and n >= 2:
        lam[0] = 10.0 ** lo_exp
        lam[-1] = 10.0 ** hi_exp
    q, r = torch.linalg.qr(z)
    del z
    q *= torch.sign(torch.diagonal(r))[None, :]
    del r
    m = (q * torch.from_numpy(lam).to(device)[None, :]) @ q.T.contiguous()
    m = 0.5 * (m + m.T)
    if return_factors:
        return m, q, lam
    del q
    return m


def lssvm_points(n: int, d: int, seed) -> np.ndarray:
    """n x d input points with i.i.d. N(0, 1) entries (the paper's LS-SVM
    experiment draws its inputs with randn)."""
    return rng_for(seed).standard_normal((n, d))


def lssvm_matrix(x: np.ndarray, sigma: float, gamma: float) -> np.ndarray:
    """The dense (n + 1) x (n + 1) LS-SVM cross-validation matrix
    A_gamma = [[0, 1^T], [1, K + I/gamma]], K_ij = exp(-|x_i - x_j|^2 / (2 sigma^2))
    of the points x (rows), for checking the matrix-free path."""
    n = x.shape[0]
    d2 = np.empty((n, n))
    for r0 in range(0, n, 256):  # squared distances from differences, by row chunks
        diff = x[r0:r0 + 256, None, :] - x[None, :, :]
        d2[r0:r0 + 256] = np.sum(diff * diff, axis=2)
    a = np.empty((n + 1, n + 1))
    a[0, 0] = 0.0
    a[0, 1:] = 1.0
    a[1:, 0] = 1.0
    a[1:, 1:] = np.exp(-d2 / (2.0 * sigma * sigma)) + np.eye(n) / gamma
    return a


def tridiag_toeplitz(n: int, diag: float = 4.0, off: float = -1.0) -> np.ndarray:
    """Constant tridiagonal matrix with ``diag`` on the diagonal and ``off`` beside it."""
    t = np.zeros((n, n))
    t[np.diag_indices(n)] = diag
    idx = np.arange(n - 1)
    t[idx, idx + 1] = off
    t[idx + 1, idx] = off
    return t


# ---------------------------------------------------------------------------
# Named workloads (sizes and recipes of the five measured configurations).
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    n: int
    k: int
    targets: List[Tuple[int, int]]   # 0-based block indices
    family: str
    seed: int
    precisions: List[str]


WORKLOADS = {
    # n=256, k=2, block (0,0), Gaussian + n I.
    "dd_n256_k2": Workload("dd_n256_k2", 256, 2, [(0, 0)], "gaussian_dd", 1, ["f64"]),
    # n=4096, k=4, blocks (0,0) and (1,2), Q Lam Q^T with Lam log-uniform in [1, 100].
    "spd_n4096_k4": Workload("spd_n4096_k4", 4096, 4, [(0, 0), (1, 2)], "haar_spd_1e2", 2,
                             ["f64", "f32"]),
    # n=16384, k=8, block (0,0), Q Lam Q^T with condition number exactly 1e4.
    "spd_n16384_k8": Workload("spd_n16384_k8", 16384, 8, [(0, 0)], "haar_spd_1e4", 3,
                              ["mixed_f16", "mixed_bf16"]),
    # n=8192, k=4, block (0,0), Gaussian + n I, FP32, gradient of sum(W * X00).
    "dd_n8192_k4_grad": Workload("dd_n8192_k4_grad", 8192, 4, [(0, 0)], "gaussian_dd", 4,
                                 ["f32"]),
}


def make_matrix(family: str, n: int, seed) -> np.ndarray:
    if family == "gaussian_dd":
        return gaussian_dd(n, seed)
    if family == "gaussian":
        return gaussian(n, seed)
    if family == "haar_spd_1e2":
        return haar_spd(n, seed, 0.0, 2.0).m
    if family == "haar_spd_1e4":
        return haar_spd(n, seed, 0.0, 4.0, pin_endpoints=True).m
    if family == "tridiag":
        return tridiag_toeplitz(n)
    raise ValueError(f"unknown matrix family {family!r}")


def workload_matrix(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    return make_matrix(w.family, w.n, w.seed)


def cotangent(b: int, seed: int = 44) -> np.ndarray:
    """W ~ N(0, 1), the b x b weight of the loss sum(W * X)."""
    return rng_for(seed).standard_normal((b, b))


@dataclasses.dataclass
class BatchProblem:
    n: int
    k: int
    i: int
    j: int
    matrix_seed: int


def batch_problems(count: int = 512, seed: int = 5, n_lo: int = 64, n_hi: int = 1024,
                   ks=(2, 3, 4)) -> List[BatchProblem]:
    """Problem list of the batched workload.

    Problem ``t`` draws its sizes (n uniform in [n_lo, n_hi], k uniform in
    ``ks``, target block uniform) and the seed of its matrix from the t-th
    child of ``SeedSequence(seed)``; its matrix is Gaussian + n I
    (``batch_matrix``).
    """
    out = []
    for child in np.random.SeedSequence(seed).spawn(count):
        r = np.random.default_rng(child)
        n = int(r.integers(n_lo, n_hi + 1))
        k = int(r.choice(np.asarray(ks)))
        i = int(r.integers(0, k))
        j = int(r.integers(0, k))
        out.append(BatchProblem(n, k, i, j, int(r.integers(0, 2**62))))
    return out


def batch_matrix(p: BatchProblem) -> np.ndarray:
    return gaussian_dd(p.n, p.matrix_seed)
