"""Python binding of the C ABI in include/knn.h (ctypes; argument marshalling only).

Every step of the search runs in the HIP library ``libknn_mi355x.so``; torch is
used for device memory and the current stream.  The binding refuses to run when
the library is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknn_mi355x.so")

MIPS, L2, COSINE = 0, 1, 2
F32, BF16, FP8 = 0, 1, 2
METRICS = {"mips": MIPS, "l2": L2, "cosine": COSINE}
DTYPES = {"fp32": F32, "bf16": BF16, "fp8": FP8}
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of memory", 4: "HIP error"}

_lib = None


class KnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class KnnBatch(ctypes.Structure):
    _fields_ = [("Q", ctypes.c_void_p), ("M", ctypes.c_int64), ("db", ctypes.c_int32), ("K", ctypes.c_int32),
                ("out_val", ctypes.c_void_p), ("out_idx", ctypes.c_void_p)]


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_14286_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        SZ = ctypes.c_size_t
        sig = {
            "knn_bins_for_recall": (i64, [i32, f64, i64]),
            "knn_expected_recall_bound": (f64, [i32, i64]),
            "knn_bin_start": (i64, [i64, i64, i64]),
            "knn_status_string": (ctypes.c_char_p, [i32]),
            "knn_last_error": (ctypes.c_char_p, []),
            "knn_device_count": (i32, []),
            "knn_db_prepare_size": (SZ, [i64, i32, i32, i32]),
            "knn_db_prepare": (i32, [P, i32, i64, i32, i32, i32, P, SZ, P, ctypes.POINTER(P)]),
            "knn_db_destroy": (i32, [P]),
            "knn_db_export": (i32, [P, P, P, P, P]),
            "knn_search": (i32, [P, i64, P, i64, i32, i32, i64, i32, P, P, P]),
            "knn_db_search": (i32, [P, P, i32, i64, i32, i64, f64, i64, i32, P, P, P, P, P, SZ, P]),
            "knn_db_search_workspace_size": (i32, [P, i64, i32, i64, f64, i64, i32, i32, ctypes.POINTER(SZ)]),
            "knn_db_search_noalloc": (i32, [P, P, i32, i64, i32, i64, f64, i64, i32, P, P, P, P, P]),
            "knn_noalloc_scratch_bytes": (SZ, []),
            "knn_plan_create": (i32, [ctypes.POINTER(P), i32, ctypes.POINTER(KnnBatch), i32, i32, f64, i32,
                                      ctypes.c_char_p, ctypes.POINTER(P)]),
            "knn_plan_workspace_size": (i32, [P, ctypes.POINTER(SZ)]),
            "knn_plan_setup": (i32, [P, P, SZ, P]),
            "knn_search_batched": (i32, [P, P]),
            "knn_plan_info": (i32, [P, P, P, P]),
            "knn_plan_set_own_launches": (i32, [P, i64]),
            "knn_plan_destroy": (i32, [P]),
            "knn_backward": (i32, [P, P, P, P, i32, i64, i64, i32, i32, i32, P, P, P]),
            "knn_query_buffer_bytes": (SZ, [P, i64]),
            "knn_query_prepare": (i32, [P, P, i32, i64, P, SZ, P]),
            "knn_partial_reduce": (i32, [P, P, i64, i64, P, P, P]),
            "knn_resolve_rows": (i32, [P, P, i64, i64, P, i64, P]),
            "knn_approx_bins": (i64, [i64, i32, f64, i64]),
            "knn_approx_top_k": (i32, [P, i32, i64, i64, i64, i32, i32, f64, i64, i64, i32, i32, P, P, P, SZ, P]),
            "knn_approx_workspace_size": (i32, [i32, i64, i64, i64, i32, i32, f64, i64, i64, i32, i32,
                                                ctypes.POINTER(SZ)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise KnnError(status, lib().knn_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _metric(m):
    return METRICS[m] if isinstance(m, str) else int(m)


def _in_dtype(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"inputs must be float32 or bfloat16, got {t.dtype}")


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


# ------------------------------------------------------------------------------ helpers
def bins_for_recall(K: int, recall_target: float = 0.95, N: int = 1 << 62) -> int:
    return int(lib().knn_bins_for_recall(int(K), float(recall_target), int(N)))


def expected_recall_bound(K: int, L: int) -> float:
    return float(lib().knn_expected_recall_bound(int(K), int(L)))


def bin_start(b: int, N: int, L: int) -> int:
    return int(lib().knn_bin_start(int(b), int(N), int(L)))


def _device_buffer(nbytes: int, device) -> torch.Tensor:
    """Caller-owned device memory for the library (a torch allocation)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _same_device(*named):
    devs = {t.device for _, t in named if t is not None}
    if len(devs) > 1:
        raise ValueError("tensors on different devices: " + ", ".join(f"{n} on {t.device}" for n, t in named
                                                                       if t is not None))


# ------------------------------------------------------------------------------ search
def search(Q: torch.Tensor, X: torch.Tensor, k: int, L: int | None = None, metric="mips"):
    """The plain FP32 search (``knn_search``): returns (values, indices), each M x k."""
    if Q.dim() != 2 or X.dim() != 2 or Q.shape[1] != X.shape[1]:
        raise ValueError(f"Q (M x D) and X (N x D) must share the depth D: Q {tuple(Q.shape)}, X {tuple(X.shape)}")
    _same_device(("Q", Q), ("X", X))
    _dev(Q, "Q")
    _dev(X, "X")
    if Q.dtype != torch.float32 or X.dtype != torch.float32:
        raise TypeError("knn_search takes float32 inputs")
    M, D = Q.shape
    N = X.shape[0]
    ov = torch.empty((M, k), dtype=torch.float32, device=Q.device)
    oi = torch.empty((M, k), dtype=torch.int32, device=Q.device)
    _check(lib().knn_search(_ptr(Q), M, _ptr(X), N, D, int(k), int(L or 0), _metric(metric), _ptr(ov), _ptr(oi),
                            _stream()))
    return ov, oi


class Database:
    """A database prepared once (``knn_db_prepare``) into a device buffer this object owns
    (a torch allocation); keeps a reference to X, which the FP32 rerank reads."""

    def __init__(self, X: torch.Tensor, metric="mips", compute: str = "fp32"):
        if X.dim() != 2:
            raise ValueError("X must be N x D")
        _dev(X, "X")
        self.X = X
        self.metric = _metric(metric)
        self.compute = DTYPES[compute]
        self.N, self.D = X.shape
        nbytes = int(lib().knn_db_prepare_size(self.N, self.D, self.metric, self.compute))
        if nbytes == 0:
            _check(lib().knn_db_prepare(_ptr(X), _in_dtype(X), self.N, self.D, self.metric, self.compute, None, 0,
                                        _stream(), ctypes.byref(ctypes.c_void_p())))
        self.buf = _device_buffer(nbytes, X.device)
        h = ctypes.c_void_p()
        _check(lib().knn_db_prepare(_ptr(X), _in_dtype(X), self.N, self.D, self.metric, self.compute, _ptr(self.buf),
                                    nbytes, _stream(), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().knn_db_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self):
        """The prepared rows as the kernel sees them (host numpy): codes, exponents, half norms."""
        import numpy as np
        dt = {F32: np.float32, BF16: np.uint16, FP8: np.uint8}[self.compute]
        codes = np.empty((self.N, self.D), dt)
        e = np.empty(self.N, np.int32)
        hn = np.empty(self.N, np.float32)
        _check(lib().knn_db_export(self._h, codes.ctypes.data_as(ctypes.c_void_p),
                                   e.ctypes.data_as(ctypes.c_void_p), hn.ctypes.data_as(ctypes.c_void_p),
                                   _stream()))
        return codes, e, hn

    def workspace_size(self, M: int, k: int, L: int | None = None, rerank: int = 0, return_bins: bool = False,
                       recall_target: float = 0.95, input_size_override: int = -1) -> int:
        """``knn_db_search_workspace_size``: device bytes a search with these arguments needs."""
        n = ctypes.c_size_t()
        _check(lib().knn_db_search_workspace_size(self._h, int(M), int(k), int(L or 0), float(recall_target),
                                                  int(input_size_override), int(rerank), int(bool(return_bins)),
                                                  ctypes.byref(n)))
        return int(n.value)

    def bins(self, k: int, L: int | None = None, recall_target: float = 0.95, input_size_override: int = -1) -> int:
        """The bin count a search uses (L given, or derived as ``knn_db_search`` does)."""
        if L:
            return int(L)
        return approx_bins(self.N, k, recall_target, input_size_override)

    def search(self, Q: torch.Tensor, k: int, L: int | None = None, rerank: int = 0, return_bins: bool = False,
               out=None, recall_target: float = 0.95, input_size_override: int = -1, workspace=None):
        """``knn_db_search``: (values, indices[, bins_val, bins_idx]).  The workspace is a torch
        allocation unless ``workspace`` (a uint8 device tensor) is given."""
        if Q.dim() != 2 or Q.shape[1] != self.D:
            raise ValueError(f"Q must be M x {self.D} (got {tuple(Q.shape)})")
        _same_device(("Q", Q), ("X", self.X))
        _dev(Q, "Q")
        M = Q.shape[0]
        L = self.bins(k, L, recall_target, input_size_override)
        if out is None:
            ov = torch.empty((M, k), dtype=torch.float32, device=Q.device)
            oi = torch.empty((M, k), dtype=torch.int32, device=Q.device)
        else:
            ov, oi = out
        bv = bi = None
        if return_bins:
            bv = torch.empty((M, L), dtype=torch.float32, device=Q.device)
            bi = torch.empty((M, L), dtype=torch.int32, device=Q.device)
        if workspace is None:
            workspace = _device_buffer(self.workspace_size(M, k, L, rerank, return_bins), Q.device)
        _check(lib().knn_db_search(self._h, _ptr(Q), _in_dtype(Q), M, int(k), L, float(recall_target),
                                   int(input_size_override), int(rerank), _ptr(ov), _ptr(oi), _ptr(bv), _ptr(bi),
                                   _ptr(workspace), workspace.numel(), _stream()))
        return (ov, oi, bv, bi) if return_bins else (ov, oi)


    def prepare_queries(self, Q: torch.Tensor) -> torch.Tensor:
        """``knn_query_prepare``: a uint8 device buffer holding Q in the kernel's layout."""
        _dev(Q, "Q")
        M = Q.shape[0]
        nbytes = int(lib().knn_query_buffer_bytes(self._h, M))
        buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=Q.device)
        _check(lib().knn_query_prepare(self._h, _ptr(Q), _in_dtype(Q), M, _ptr(buf), nbytes, _stream()))
        return buf

    def partial_reduce(self, qbuf: torch.Tensor, M: int, L: int, out=None, resolve: bool = True):
        """``knn_partial_reduce`` (Algorithm 1 alone): bin winners (values, indices), M x L.
        With ``resolve`` the compact 4-row group entries are replaced by exact rows
        (``knn_resolve_rows``)."""
        if out is None:
            bv = torch.empty((M, L), dtype=torch.float32, device=qbuf.device)
            bi = torch.empty((M, L), dtype=torch.int32, device=qbuf.device)
        else:
            bv, bi = out
        _check(lib().knn_partial_reduce(self._h, _ptr(qbuf), int(M), int(L), _ptr(bv), _ptr(bi), _stream()))
        if resolve:
            _check(lib().knn_resolve_rows(self._h, _ptr(qbuf), int(M), int(L), _ptr(bi), int(L), _stream()))
        return bv, bi


class BatchedPlan:
    """``knn_plan_create`` / ``knn_plan_setup`` / ``knn_search_batched`` over several prepared
    databases; the plan's workspace is a torch allocation this object owns."""

    def __init__(self, dbs, batches, recall_target: float = 0.95, tune: bool = False, cache_path: str | None = None,
                 own_launch_min_items: int = 0):
        """batches: list of (Q tensor, db index, k).  Output tensors are allocated here and bound to the plan.
        own_launch_min_items > 0: ``knn_plan_set_own_launches`` (database groups with at least that many
        work items get a distance launch of their own; 0 keeps one persistent launch)."""
        self.dbs = list(dbs)
        self.outs = []
        arr = (KnnBatch * len(batches))()
        qdt = None
        self._keep = []
        for i, (Q, d, k) in enumerate(batches):
            if not 0 <= int(d) < len(self.dbs):
                raise ValueError(f"batch {i}: database index {d} out of range")
            if Q.dim() != 2 or Q.shape[1] != self.dbs[d].D:
                raise ValueError(f"batch {i}: Q must be M x {self.dbs[d].D} (got {tuple(Q.shape)})")
            _same_device(("Q", Q), ("X", self.dbs[d].X))
            _dev(Q, "Q")
            qdt = _in_dtype(Q) if qdt is None else qdt
            if _in_dtype(Q) != qdt:
                raise TypeError("all query batches must share a dtype")
            ov = torch.empty((Q.shape[0], k), dtype=torch.float32, device=Q.device)
            oi = torch.empty((Q.shape[0], k), dtype=torch.int32, device=Q.device)
            self.outs.append((ov, oi))
            self._keep.append(Q)
            arr[i] = KnnBatch(Q.data_ptr(), Q.shape[0], int(d), int(k), ov.data_ptr(), oi.data_ptr())
        hs = (ctypes.c_void_p * len(self.dbs))(*[d.handle.value for d in self.dbs])
        h = ctypes.c_void_p()
        _check(lib().knn_plan_create(hs, len(self.dbs), arr, len(batches), qdt, float(recall_target), int(tune),
                                     cache_path.encode() if cache_path else None, ctypes.byref(h)))
        self._h = h
        if own_launch_min_items:
            _check(lib().knn_plan_set_own_launches(self._h, int(own_launch_min_items)))
        n = ctypes.c_size_t()
        _check(lib().knn_plan_workspace_size(self._h, ctypes.byref(n)))
        self.workspace = _device_buffer(n.value, self.dbs[0].X.device)
        _check(lib().knn_plan_setup(self._h, _ptr(self.workspace), self.workspace.numel(), _stream()))

    def run(self):
        _check(lib().knn_search_batched(self._h, _stream()))
        return self.outs

    def info(self):
        import numpy as np
        n = len(self.dbs)
        L = np.zeros(n, np.int64)
        qb = np.zeros(n, np.int32)
        cr = np.zeros(n, np.int64)
        _check(lib().knn_plan_info(self._h, L.ctypes.data_as(ctypes.c_void_p), qb.ctypes.data_as(ctypes.c_void_p),
                                   cr.ctypes.data_as(ctypes.c_void_p)))
        return {"L": L.tolist(), "qblock": qb.tolist(), "chunk_rows": cr.tolist()}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().knn_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------ approx_max_k on scores
def approx_bins(n: int, k: int, recall_target: float = 0.95, reduction_input_size_override: int = -1) -> int:
    """``knn_approx_bins``: the bin count the op uses for a slice of n scores."""
    return int(lib().knn_approx_bins(int(n), int(k), float(recall_target), int(reduction_input_size_override)))


def approx_top_k(scores: torch.Tensor, k: int, reduction_dimension: int = -1, recall_target: float = 0.95,
                 reduction_input_size_override: int = -1, aggregate_to_topk: bool = True, minimize: bool = False,
                 L: int | None = None, out=None):
    """``knn_approx_top_k`` on a 2-D FP32 or BF16 device matrix whose rows may be strided
    (unit stride along the last dimension).  Returns (values FP32, indices int32) with the
    reduced dimension replaced by k (aggregate_to_topk) or by the bin count."""
    if not scores.is_cuda or scores.dim() != 2:
        raise ValueError("scores must be a 2-D device tensor")
    if scores.stride(1) != 1:
        raise ValueError("scores must have unit stride along its last dimension")
    rows, cols = scores.shape
    ld = max(int(scores.stride(0)), cols, 1)
    dim = 1 if reduction_dimension in (-1, 1) else int(reduction_dimension)
    n, B = (cols, rows) if dim == 1 else (rows, cols)
    if L is None:
        L = approx_bins(n, k, recall_target, reduction_input_size_override)
    R = int(k) if aggregate_to_topk else int(L)
    shape = (B, R) if dim == 1 else (R, B)
    if out is None:
        ov = torch.empty(shape, dtype=torch.float32, device=scores.device)
        oi = torch.empty(shape, dtype=torch.int32, device=scores.device)
    else:
        ov, oi = out
    args = (_in_dtype(scores), rows, cols, ld, dim, int(k), float(recall_target), int(reduction_input_size_override),
            int(L), int(bool(minimize)), int(bool(aggregate_to_topk)))
    n = ctypes.c_size_t()
    _check(lib().knn_approx_workspace_size(*args, ctypes.byref(n)))
    ws = _device_buffer(n.value, scores.device) if n.value else None
    _check(lib().knn_approx_top_k(_ptr(scores), *args[:11], _ptr(ov), _ptr(oi), _ptr(ws), n.value, _stream()))
    return ov, oi


def approx_max_k(scores, k, **kw):
    """The paper's approx_max_k on a score matrix (App. A.1 options as keywords)."""
    return approx_top_k(scores, k, minimize=False, **kw)


def approx_min_k(scores, k, **kw):
    """approx_min_k: the same reduction keeping the smallest scores."""
    return approx_top_k(scores, k, minimize=True, **kw)


# ------------------------------------------------------------------------------ backward
def backward(g: torch.Tensor, idx: torch.Tensor, Q: torch.Tensor, X: torch.Tensor, metric="mips",
             need_dX: bool = True, out=None):
    """``knn_backward``: (dQ, dX) FP32 for the retrieved-score gradient g (selection fixed).
    ``out=(dQ, dX)``: caller buffers; dQ is overwritten and dX accumulated into (as the C
    function does), so a fresh gradient needs a zeroed dX."""
    if g.dim() != 2 or idx.shape != g.shape:
        raise ValueError(f"g and idx must both be M x K (got {tuple(g.shape)} and {tuple(idx.shape)})")
    if Q.dim() != 2 or X.dim() != 2 or Q.shape[0] != g.shape[0] or Q.shape[1] != X.shape[1]:
        raise ValueError(f"need Q M x D and X N x D with M = {g.shape[0]} (got Q {tuple(Q.shape)}, "
                         f"X {tuple(X.shape)})")
    _same_device(("g", g), ("idx", idx), ("Q", Q), ("X", X))
    for t, n in ((g, "g"), (idx, "idx"), (Q, "Q"), (X, "X")):
        _dev(t, n)
    if g.dtype != torch.float32 or idx.dtype != torch.int32:
        raise TypeError("g must be float32 and idx int32")
    if Q.dtype != X.dtype:
        raise TypeError("Q and X must share a dtype")
    M, K = g.shape
    N, D = X.shape
    if out is not None:
        dQ, dX = out
    else:
        dQ = torch.empty((M, D), dtype=torch.float32, device=Q.device)
        dX = torch.zeros((N, D), dtype=torch.float32, device=Q.device) if need_dX else None
    _check(lib().knn_backward(_ptr(g), _ptr(idx), _ptr(Q), _ptr(X), _in_dtype(Q), M, N, D, K, _metric(metric),
                              _ptr(dQ), _ptr(dX), _stream()))
    return dQ, dX


class KNN(torch.autograd.Function):
    """Differentiable retrieval: forward runs the search, backward runs ``knn_backward``
    through the retrieved scores with the selected indices held fixed."""

    @staticmethod
    def forward(ctx, Q, X, k, L, metric, db):
        vals, idx = db.search(Q.detach(), k, L)
        ctx.save_for_backward(Q, X, idx)
        ctx.metric = metric
        ctx.mark_non_differentiable(idx)
        return vals, idx

    @staticmethod
    def backward(ctx, g_vals, g_idx):
        Q, X, idx = ctx.saved_tensors
        dQ, dX = backward(g_vals.contiguous().float(), idx, Q.detach(), X.detach(), ctx.metric,
                          need_dX=ctx.needs_input_grad[1])
        dQ = dQ.to(Q.dtype) if ctx.needs_input_grad[0] else None
        dX = dX.to(X.dtype) if (dX is not None and ctx.needs_input_grad[1]) else None
        return dQ, dX, None, None, None, None


def knn(Q, X, k, L=None, metric="mips", db: Database | None = None):
    """Autograd entry: (values, indices) with gradients to Q and X through the values."""
    if db is None:
        db = Database(X.detach(), metric, "bf16" if X.dtype == torch.bfloat16 else "fp32")
    L = int(L or bins_for_recall(k, 0.95, X.shape[0]))
    return KNN.apply(Q, X, k, L, metric, db)
