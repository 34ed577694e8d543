"""MI355X block recursive inverse (BRI): Python binding of ``libbri.so``.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libbri.so`` (see ``include/bri.h``).  PyTorch provides device
memory (tensors for inputs, outputs and the workspace) and the stream.  There
is no CPU fallback: the functions raise if the library is not built or the
tensors are not on a GPU.

Block indices are 0-based; the paper's N_11 is ``invert_block(M, k, 0, 0)``.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbri.so")

PRECISIONS = {"f64": 0, "f32": 1, "mixed_f32": 2, "mixed_f16": 3, "mixed_bf16": 4}
PIVOTING = {"tile": 0, "panel": 1, "auto": 2}
FACTORIZATIONS = {"auto": 0, "tile": 1, "recursive": 2}
ORDERS = {"principal": 0, "paper": 1}
_DTYPE_OF = {"f64": torch.float64, "f32": torch.float32, "mixed_f32": torch.float64,
             "mixed_f16": torch.float64, "mixed_bf16": torch.float64}

BRI_ERR_HIP = -1000
BRI_ERR_WORKSPACE = -1001
BRI_ERR_UNSUPPORTED = -1002


class BriOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("concurrency", ctypes.c_int),
        ("pivoting", ctypes.c_int),
        ("reuse", ctypes.c_int),
        ("refine_max_iters", ctypes.c_int),
        ("refine_tol", ctypes.c_double),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("d_info", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("factorization", ctypes.c_int),
        ("workspace_budget", ctypes.c_size_t),
        ("order", ctypes.c_int),
        ("d_stats", ctypes.c_void_p),
    ]


class BriPlanStats(ctypes.Structure):
    _fields_ = [
        ("schur_ops", ctypes.c_int64),
        ("final_inversions", ctypes.c_int64),
        ("slots", ctypes.c_int64),
        ("batch_width", ctypes.c_int64),
        ("steps", ctypes.c_int64),
        ("kernel_launches", ctypes.c_int64),
        ("block", ctypes.c_int64),
        ("algorithmic_flops", ctypes.c_double),
        ("executed_flops", ctypes.c_double),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class BriError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"BRI status {status}: {text}")
        self.status = status


_lib = None

# (name, restype, argtypes) of every exported entry point of include/bri.h.
_SIGNATURES = [
    ("bri_default_opts", None, [ctypes.POINTER(BriOpts)]),
    ("bri_workspace_size", ctypes.c_size_t,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BriOpts)]),
    ("invert_block", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(BriOpts)]),
    ("bri_block_column_workspace_size", ctypes.c_size_t,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BriOpts)]),
    ("bri_block_column", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(BriOpts)]),
    ("bri_batched_workspace_size", ctypes.c_size_t,
     [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(BriOpts)]),
    ("invert_block_batched", ctypes.c_int,
     [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
      ctypes.POINTER(BriOpts)]),
    ("bri_backward_workspace_size", ctypes.c_size_t,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BriOpts)]),
    ("invert_block_backward", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(BriOpts)]),
    ("bri_plan_describe", ctypes.c_int,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BriOpts),
      ctypes.POINTER(BriPlanStats)]),
    ("bri_plan_dump", ctypes.c_int64,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BriOpts),
      ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]),
    ("bri_refine_plan_dump", ctypes.c_int64,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BriOpts),
      ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]),
    ("bri_blocks_workspace_size", ctypes.c_size_t,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
      ctypes.POINTER(BriOpts)]),
    ("invert_blocks", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
      ctypes.POINTER(BriOpts)]),
    ("bri_rbf_workspace_size", ctypes.c_size_t,
     [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BriOpts)]),
    ("invert_block_rbf", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(BriOpts)]),
    ("bri_noalloc_scratch_bytes", ctypes.c_size_t, []),
    ("invert_block_noalloc", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
      ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(BriOpts)]),
    ("bri_gemm_workspace_size", ctypes.c_size_t, [ctypes.c_int]),
    ("bri_gemm", ctypes.c_int,
     [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
      ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64,
      ctypes.c_double, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int64, ctypes.POINTER(BriOpts)]),
    ("bri_profile_enable", ctypes.c_int, [ctypes.c_int]),
    ("bri_profile_read", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("bri_refine_last", ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int)]),
    ("bri_autotune", ctypes.c_int, [ctypes.POINTER(BriOpts), ctypes.c_char_p]),
    ("bri_tune_load", ctypes.c_int, [ctypes.c_char_p]),
    ("bri_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("bri_version", ctypes.c_char_p, []),
    ("bri_opts_size", ctypes.c_size_t, []),
]


def lib() -> ctypes.CDLL:
    """The loaded ``libbri.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status: int) -> str:
    return lib().bri_status_string(int(status)).decode()


def _check(status: int) -> None:
    if status != 0:
        raise BriError(status, status_string(status))


def make_opts(precision: str = "f64", concurrency: int = 0, refine_max_iters: int = 10,
              refine_tol: float = 1e-12, pivoting: str = "auto", reuse: bool = False,
              factorization: str = "auto", workspace_budget: int = 0, order: str = "principal") -> BriOpts:
    o = BriOpts()
    lib().bri_default_opts(ctypes.byref(o))
    if precision not in PRECISIONS:
        raise ValueError(f"unknown precision {precision!r}")
    if pivoting not in PIVOTING:
        raise ValueError(f"unknown pivoting {pivoting!r}")
    o.precision = PRECISIONS[precision]
    o.pivoting = PIVOTING[pivoting]
    o.concurrency = int(concurrency)
    o.reuse = int(bool(reuse))
    o.refine_max_iters = int(refine_max_iters)
    o.refine_tol = float(refine_tol)
    if factorization not in FACTORIZATIONS:
        raise ValueError(f"unknown factorization {factorization!r}")
    o.factorization = FACTORIZATIONS[factorization]
    o.workspace_budget = int(workspace_budget)
    if order not in ORDERS:
        raise ValueError(f"unknown order {order!r}")
    o.order = ORDERS[order]
    return o


def _require_gpu(t: torch.Tensor, name: str, dtype: torch.dtype) -> None:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (there is no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a row-major 2-D tensor with unit column stride")


def _stream_ptr(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def block_size(n: int, k: int) -> int:
    return -(-n // k)


def plan_describe(n: int, k: int, i: int, j: int, precision: str = "f64", concurrency: int = 0,
                  reuse: bool = False, factorization: str = "auto", workspace_budget: int = 0,
                  order: str = "principal") -> dict:
    """Host-only structure of the plan (no GPU needed)."""
    o = make_opts(precision, concurrency, reuse=reuse, factorization=factorization,
                  workspace_budget=workspace_budget, order=order)
    s = BriPlanStats()
    _check(lib().bri_plan_describe(n, k, i, j, ctypes.byref(o), ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in BriPlanStats._fields_}


def _decode_steps(words: List[int]) -> List[tuple]:
    steps, pos = [], 0
    while pos < len(words):
        kind, count = words[pos], words[pos + 1]
        pos += 2
        items = []
        for _ in range(count):
            w = words[pos:pos + 16]
            pos += 16
            items.append((tuple(w[0:3]), tuple(w[3:6]), tuple(w[6:9]), tuple(w[9:12]), tuple(w[12:15]), w[15]))
        steps.append((kind, items))
    return steps


def plan_dump(n: int, k: int, i: int, j: int, precision: str = "f64", concurrency: int = 0,
              reuse: bool = False, order: str = "principal") -> List[tuple]:
    """Host-only list of plan steps: [(kind, [items...])], item = (dst, x, y, cin, sub, node)."""
    o = make_opts(precision, concurrency, reuse=reuse, order=order)
    need = lib().bri_plan_dump(n, k, i, j, ctypes.byref(o), None, 0)
    if need < 0:
        raise BriError(int(need), status_string(int(need)))
    buf = (ctypes.c_int64 * need)()
    lib().bri_plan_dump(n, k, i, j, ctypes.byref(o), buf, need)
    return _decode_steps(list(buf))


def refine_plan_dump(n: int, k: int, j: int, which: str, concurrency: int = 0, reuse: bool = False):
    """Host-only plans of the mixed-precision refinement: which = "column"
    (float block column, keeps its pivots), "solve" (correction solve with the
    right-hand side as operand kind 5) or "kept" (pivot slot per position)."""
    w = {"column": 0, "solve": 1, "kept": 2}[which]
    o = make_opts("mixed_f32", concurrency, reuse=reuse)
    need = lib().bri_refine_plan_dump(n, k, j, w, ctypes.byref(o), None, 0)
    if need < 0:
        raise BriError(int(need), status_string(int(need)))
    buf = (ctypes.c_int64 * max(need, 1))()
    lib().bri_refine_plan_dump(n, k, j, w, ctypes.byref(o), buf, need)
    return list(buf)[:need] if which == "kept" else _decode_steps(list(buf)[:need])


def workspace_size(n: int, k: int, i: int, j: int, precision: str = "f64", concurrency: int = 0,
                   reuse: bool = False, workspace_budget: int = 0, order: str = "principal") -> int:
    o = make_opts(precision, concurrency, reuse=reuse, workspace_budget=workspace_budget, order=order)
    return int(lib().bri_workspace_size(n, k, i, j, ctypes.byref(o)))


def invert_block(M: torch.Tensor, k: int, i: int, j: int, precision: str = "f64", concurrency: int = 0,
                 out: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None,
                 workspace: Optional[torch.Tensor] = None, refine_max_iters: int = 10,
                 refine_tol: float = 1e-12, pivoting: str = "auto", reuse: bool = False,
                 factorization: str = "auto", workspace_budget: int = 0,
                 order: str = "principal", stats: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Block N_ij (b x b, b = ceil(n/k)) of M^{-1} (of Gamma^{-1} when k does not divide n).

    ``order="paper"`` runs the paper's literal frame procedure instead of the
    principal elimination order (f64 / f32, no reuse).

    ``info`` (optional int32 GPU tensor of one element) receives the device
    status of include/bri.h; it is not checked here (no synchronisation).

    ``stats`` (optional int64 GPU tensor of four elements) receives the
    device accounting of the executed work (bri_opts::d_stats in
    include/bri.h; ``stats_dict`` names its fields).
    """
    dtype = _DTYPE_OF[precision]
    _require_gpu(M, "M", dtype)
    n = M.shape[0]
    if M.shape[1] != n:
        raise ValueError("M must be square")
    b = block_size(n, k)
    o = make_opts(precision, concurrency, refine_max_iters, refine_tol, pivoting, reuse, factorization,
                  workspace_budget, order)
    need = lib().bri_workspace_size(n, k, i, j, ctypes.byref(o))
    if need == 0:
        # Invalid arguments: let the library name the offending one (it
        # validates before enqueuing anything).
        _check(lib().invert_block(M.data_ptr(), n, M.stride(0), k, i, j, M.data_ptr(), b, ctypes.byref(o))
               or BRI_ERR_UNSUPPORTED)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=M.device)
    if out is None:
        out = torch.empty(b, b, dtype=dtype, device=M.device)
    _require_gpu(out, "out", dtype)
    o.workspace = workspace.data_ptr()
    o.workspace_bytes = workspace.numel()
    o.d_info = info.data_ptr() if info is not None else None
    if stats is not None:
        if not isinstance(stats, torch.Tensor) or stats.device != M.device or stats.dtype != torch.int64 \
                or stats.numel() < 4 or not stats.is_contiguous():
            raise ValueError("stats must be a contiguous int64 tensor of at least 4 elements on M's device")
        o.d_stats = stats.data_ptr()
    o.stream = _stream_ptr(M.device)
    _check(lib().invert_block(M.data_ptr(), n, M.stride(0), k, i, j, out.data_ptr(), out.stride(0),
                              ctypes.byref(o)))
    return out


def stats_dict(stats: torch.Tensor) -> dict:
    """The device accounting words of ``invert_block(..., stats=...)`` by name
    (synchronises with the device to read them)."""
    v = [int(x) for x in stats[:4].cpu().tolist()]
    return {"factorizations": v[0], "schur_products": v[1], "other_products": v[2],
            "workspace_high_water": v[3]}


def rbf_workspace_size(npts: int, d: int, k: int, i: int, j: int, precision: str = "f64",
                       concurrency: int = 0, workspace_budget: int = 0) -> int:
    o = make_opts(precision, concurrency, workspace_budget=workspace_budget)
    return int(lib().bri_rbf_workspace_size(npts, d, k, i, j, ctypes.byref(o)))


def invert_block_rbf(X: torch.Tensor, k: int, i: int, j: int, sigma: float, gamma: float,
                     precision: str = "f64", info: Optional[torch.Tensor] = None, pivoting: str = "auto",
                     concurrency: int = 0, workspace_budget: int = 0) -> torch.Tensor:
    """Block (i, j) of A_gamma^{-1}, A_gamma the LS-SVM matrix of the points X
    (npts x d, rows), order npts + 1, evaluated element by element on the
    device (never stored)."""
    dtype = _DTYPE_OF[precision]
    _require_gpu(X, "X", dtype)
    npts, d = X.shape
    m = npts + 1
    b = block_size(m, k)
    o = make_opts(precision, concurrency, pivoting=pivoting, workspace_budget=workspace_budget)
    need = lib().bri_rbf_workspace_size(npts, d, k, i, j, ctypes.byref(o))
    out = torch.empty(b, b, dtype=dtype, device=X.device)
    if need == 0:
        _check(lib().invert_block_rbf(X.data_ptr(), npts, X.stride(0), d, sigma, gamma, k, i, j, out.data_ptr(),
                                      out.stride(0), ctypes.byref(o)) or BRI_ERR_UNSUPPORTED)
    ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = need
    o.d_info = info.data_ptr() if info is not None else None
    o.stream = _stream_ptr(X.device)
    _check(lib().invert_block_rbf(X.data_ptr(), npts, X.stride(0), d, sigma, gamma, k, i, j, out.data_ptr(),
                                  out.stride(0), ctypes.byref(o)))
    return out


def invert_block_noalloc(M: torch.Tensor, k: int, i: int, j: int, out: torch.Tensor,
                         precision: str = "f64", info: Optional[torch.Tensor] = None,
                         pivoting: str = "auto") -> torch.Tensor:
    """invert_block into a caller-provided ``out`` with the library's static
    device scratch as workspace: allocates no device memory."""
    dtype = _DTYPE_OF[precision]
    _require_gpu(M, "M", dtype)
    _require_gpu(out, "out", dtype)
    o = make_opts(precision, pivoting=pivoting)
    o.d_info = info.data_ptr() if info is not None else None
    o.stream = _stream_ptr(M.device)
    _check(lib().invert_block_noalloc(M.data_ptr(), M.shape[0], M.stride(0), k, i, j, out.data_ptr(),
                                      out.stride(0), ctypes.byref(o)))
    return out


def block_column(M: torch.Tensor, k: int, j: int, transpose: bool = False, precision: str = "f64",
                 concurrency: int = 0, factorization: str = "auto") -> torch.Tensor:
    """Block column j of Gamma^{-1} ((k*b) x b); with ``transpose`` the block
    column of (Gamma^T)^{-1}, i.e. the transposed block row j of Gamma^{-1}."""
    dtype = _DTYPE_OF[precision]
    _require_gpu(M, "M", dtype)
    n = M.shape[0]
    b = block_size(n, k)
    o = make_opts(precision, concurrency, factorization=factorization)
    need = lib().bri_block_column_workspace_size(n, k, j, ctypes.byref(o))
    if need == 0:
        raise BriError(BRI_ERR_UNSUPPORTED, "invalid arguments")
    ws = torch.empty(need, dtype=torch.uint8, device=M.device)
    X = torch.empty(k * b, b, dtype=dtype, device=M.device)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = need
    o.stream = _stream_ptr(M.device)
    _check(lib().bri_block_column(M.data_ptr(), n, M.stride(0), k, j, int(bool(transpose)), X.data_ptr(),
                                  X.stride(0), ctypes.byref(o)))
    return X


def invert_block_backward(M: torch.Tensor, k: int, i: int, j: int, G: torch.Tensor,
                          precision: str = "f64", concurrency: int = 0) -> torch.Tensor:
    """dL/dM for L = sum(G * N_ij): -(N_{i,:})^T G (N_{:,j})^T, recomputed through the recursion."""
    dtype = _DTYPE_OF[precision]
    _require_gpu(M, "M", dtype)
    G = G.contiguous()
    _require_gpu(G, "G", dtype)
    n = M.shape[0]
    o = make_opts(precision, concurrency)
    need = lib().bri_backward_workspace_size(n, k, i, j, ctypes.byref(o))
    if need == 0:
        raise BriError(BRI_ERR_UNSUPPORTED, "invalid arguments")
    ws = torch.empty(need, dtype=torch.uint8, device=M.device)
    grad = torch.empty(n, n, dtype=dtype, device=M.device)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = need
    o.stream = _stream_ptr(M.device)
    _check(lib().invert_block_backward(M.data_ptr(), n, M.stride(0), k, i, j, G.data_ptr(), G.stride(0),
                                       grad.data_ptr(), grad.stride(0), ctypes.byref(o)))
    return grad


def batched_workspace_size(ns: Sequence[int], ks: Sequence[int], iis: Sequence[int], jjs: Sequence[int],
                           precision: str = "f64", reuse: bool = False, pivoting: str = "auto") -> int:
    """Workspace bytes of invert_block_batched for these problems (0 when invalid)."""
    count = len(ns)
    o = make_opts(precision, 0, reuse=reuse, pivoting=pivoting)
    return int(lib().bri_batched_workspace_size(count, (ctypes.c_int64 * count)(*ns), (ctypes.c_int * count)(*ks),
                                                (ctypes.c_int * count)(*iis), (ctypes.c_int * count)(*jjs),
                                                ctypes.byref(o)))


def invert_block_batched(Ms: Sequence[torch.Tensor], ks: Sequence[int], iis: Sequence[int],
                         jjs: Sequence[int], precision: str = "f64", concurrency: int = 0,
                         info: Optional[torch.Tensor] = None, reuse: bool = False,
                         factorization: str = "auto", pivoting: str = "auto",
                         out: Optional[Sequence[torch.Tensor]] = None,
                         workspace: Optional[torch.Tensor] = None) -> List[torch.Tensor]:
    """One block per problem; all problems share one workspace and one call.
    ``out`` (one block per problem) and ``workspace`` may be passed in to be
    reused across calls."""
    count = len(Ms)
    dtype = _DTYPE_OF[precision]
    for t, m in enumerate(Ms):
        _require_gpu(m, f"Ms[{t}]", dtype)
    dev = Ms[0].device
    n = (ctypes.c_int64 * count)(*[m.shape[0] for m in Ms])
    ldm = (ctypes.c_int64 * count)(*[m.stride(0) for m in Ms])
    kk = (ctypes.c_int * count)(*ks)
    ii = (ctypes.c_int * count)(*iis)
    jj = (ctypes.c_int * count)(*jjs)
    if out is None:
        outs = [torch.empty(block_size(m.shape[0], k), block_size(m.shape[0], k), dtype=dtype, device=dev)
                for m, k in zip(Ms, ks)]
    else:
        outs = list(out)
        if len(outs) != count:
            raise ValueError("out must hold one block per problem")
        for t, (o_, m, k) in enumerate(zip(outs, Ms, ks)):
            _require_gpu(o_, f"out[{t}]", dtype)
            if o_.shape[0] < block_size(m.shape[0], k) or o_.shape[1] < block_size(m.shape[0], k):
                raise ValueError(f"out[{t}] is smaller than its block")
    ldo = (ctypes.c_int64 * count)(*[o_.stride(0) for o_ in outs])
    mp = (ctypes.c_void_p * count)(*[m.data_ptr() for m in Ms])
    op = (ctypes.c_void_p * count)(*[o_.data_ptr() for o_ in outs])
    o = make_opts(precision, concurrency, reuse=reuse, factorization=factorization, pivoting=pivoting)
    need = lib().bri_batched_workspace_size(count, n, kk, ii, jj, ctypes.byref(o))
    if need == 0 and count > 0:
        raise BriError(BRI_ERR_UNSUPPORTED, "invalid arguments")
    ws = workspace if workspace is not None and workspace.numel() >= need else \
        torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = need
    o.d_info = info.data_ptr() if info is not None else None
    o.stream = _stream_ptr(dev)
    _check(lib().invert_block_batched(count, mp, n, ldm, kk, ii, jj, op, ldo, ctypes.byref(o)))
    return outs


def band_blocks(k: int, width: int = 0) -> List[tuple]:
    """The blocks (i, j) with |i - j| <= width (width 0: the diagonal blocks)."""
    return [(i, j) for i in range(k) for j in range(k) if abs(i - j) <= width]


def invert_blocks(M: torch.Tensor, k: int, blocks: Optional[Sequence[tuple]] = None, precision: str = "f64",
                  info: Optional[torch.Tensor] = None, pivoting: str = "auto") -> List[torch.Tensor]:
    """Several blocks of M^{-1} (all k^2 when ``blocks`` is None), computed as
    one merged batch over the same M; returns them in the order of ``blocks``."""
    dtype = _DTYPE_OF[precision]
    _require_gpu(M, "M", dtype)
    n = M.shape[0]
    if M.shape[1] != n:
        raise ValueError("M must be square")
    if blocks is None:
        blocks = [(i, j) for i in range(k) for j in range(k)]
    count = len(blocks)
    b = block_size(n, k)
    ii = (ctypes.c_int * count)(*[int(x[0]) for x in blocks])
    jj = (ctypes.c_int * count)(*[int(x[1]) for x in blocks])
    outs = [torch.empty(b, b, dtype=dtype, device=M.device) for _ in range(count)]
    op = (ctypes.c_void_p * count)(*[o_.data_ptr() for o_ in outs])
    ldo = (ctypes.c_int64 * count)(*[o_.stride(0) for o_ in outs])
    o = make_opts(precision, pivoting=pivoting)
    need = lib().bri_blocks_workspace_size(n, k, count, ii, jj, ctypes.byref(o))
    if need == 0 and count > 0:
        _check(lib().invert_blocks(M.data_ptr(), n, M.stride(0), k, count, ii, jj, op, ldo, ctypes.byref(o))
               or BRI_ERR_UNSUPPORTED)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=M.device)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = need
    o.d_info = info.data_ptr() if info is not None else None
    o.stream = _stream_ptr(M.device)
    _check(lib().invert_blocks(M.data_ptr(), n, M.stride(0), k, count, ii, jj, op, ldo, ctypes.byref(o)))
    return outs


def gemm(A: Sequence[torch.Tensor], B: Sequence[torch.Tensor], C: Sequence[torch.Tensor],
         alpha: float = 1.0, beta: float = 0.0, workspace: Optional[torch.Tensor] = None,
         products: Optional[str] = None, split_bytes: int = 0) -> None:
    """C[t] = beta C[t] + alpha A[t] B[t] on the library's MFMA product kernel (in place on C).

    ``products`` (float operands only): None or "f32" for FP32 MFMA, "f16" or
    "bf16" for the split low-precision MFMA products of the mixed paths.
    ``split_bytes`` (FP16 products): scratch for operands split once before
    the products (see bri_gemm in include/bri.h), appended to the workspace."""
    count = len(A)
    if count == 0:
        return
    dtype = A[0].dtype
    prec = "f64" if dtype == torch.float64 else "f32"
    if products in ("f16", "bf16"):
        if dtype != torch.float32:
            raise TypeError("split low-precision products take float32 operands")
        prec = "mixed_" + products
    for t in range(count):
        for nm, x in (("A", A[t]), ("B", B[t]), ("C", C[t])):
            _require_gpu(x, f"{nm}[{t}]", dtype)
    m, kk = A[0].shape
    n = B[0].shape[1]
    o = make_opts(prec)
    need = lib().bri_gemm_workspace_size(count) + int(split_bytes)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=A[0].device)
    o.workspace = workspace.data_ptr()
    o.workspace_bytes = workspace.numel()
    o.stream = _stream_ptr(A[0].device)
    ap = (ctypes.c_void_p * count)(*[x.data_ptr() for x in A])
    bp = (ctypes.c_void_p * count)(*[x.data_ptr() for x in B])
    cp = (ctypes.c_void_p * count)(*[x.data_ptr() for x in C])
    _check(lib().bri_gemm(count, m, n, kk, alpha, ap, A[0].stride(0), bp, B[0].stride(0), beta, cp,
                          C[0].stride(0), ctypes.byref(o)))


class InvertBlock(torch.autograd.Function):
    """N_ij = block (i, j) of M^{-1} with a backward pass that recomputes the
    needed block row and column of M^{-1} instead of storing them."""

    @staticmethod
    def forward(ctx, M, k: int, i: int, j: int, precision: str = "f64"):
        ctx.k, ctx.i, ctx.j, ctx.precision = k, i, j, precision
        ctx.save_for_backward(M)
        return invert_block(M, k, i, j, precision=precision)

    @staticmethod
    def backward(ctx, grad_out):
        (M,) = ctx.saved_tensors
        g = invert_block_backward(M, ctx.k, ctx.i, ctx.j, grad_out, precision=ctx.precision)
        return g, None, None, None, None


class _ProfEntry(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double)]


def profile_read_clear() -> None:
    """Reads (and so clears) the step-timing record of bri_profile_*."""
    arr = (_ProfEntry * 9)()
    lib().bri_profile_read(ctypes.cast(arr, ctypes.c_void_p), 9)


def autotune(path: Optional[str] = None, workspace_bytes: int = 4 << 30, device: str = "cuda:0") -> int:
    """Measures the product tile shapes and LU variants on this GPU (see
    bri_autotune in include/bri.h), writes the tuning cache and loads it;
    returns the number of decisions."""
    ws = torch.empty(workspace_bytes, dtype=torch.uint8, device=device)
    o = make_opts("f64")
    o.workspace = ws.data_ptr()
    o.workspace_bytes = workspace_bytes
    o.stream = _stream_ptr(torch.device(device))
    rc = lib().bri_autotune(ctypes.byref(o), path.encode() if path else None)
    if rc < 0:
        raise BriError(rc, status_string(rc))
    return rc


def tune_load(path: Optional[str] = None) -> int:
    """(Re)loads a tuning cache; returns its number of decisions."""
    rc = lib().bri_tune_load(path.encode() if path else None)
    if rc < 0:
        raise BriError(rc, status_string(rc))
    return rc


def refine_last() -> tuple:
    """(sweeps, last relative correction) of this thread's last mixed-precision call."""
    s = ctypes.c_int(0)
    d = ctypes.c_double(0.0)
    lib().bri_refine_last(ctypes.byref(s), ctypes.byref(d), None)
    return s.value, d.value


def refine_last_bf16_fallback() -> bool:
    """Whether this thread's last mixed FP16 call met an operand outside the
    FP16 range and was computed again with BF16 split products."""
    f = ctypes.c_int(0)
    lib().bri_refine_last(None, None, ctypes.byref(f))
    return bool(f.value)


def version() -> str:
    return lib().bri_version().decode()
