"""Python binding of libboba.so: argument marshalling only.

Every function here has the name of the C entry point it calls (include/boba.h)
and takes torch tensors that live on the current HIP device; all work runs in
the library's kernels on the current torch stream (or ``stream``).  PyTorch
provides device memory and streams, nothing else.  If libboba.so is missing the
first call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libboba.so")

BOBA_OK, BOBA_ERR_ARG, BOBA_ERR_RANGE, BOBA_ERR_OVERFLOW, BOBA_ERR_WORKSPACE, BOBA_ERR_HIP, BOBA_ERR_TIMEOUT = range(7)
BOBA_FLAG_INTERLEAVED = 0x1
BOBA_FLAG_RACY = 0x2  # non-atomic scatter (Sec. 4.4): a valid, not unique, result
BOBA_FLAG_FORCE_GENERAL = 0x4  # small graphs through the many-workgroup path (same results)
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_RANGE", 3: "ERR_OVERFLOW", 4: "ERR_WORKSPACE", 5: "ERR_HIP",
           6: "ERR_TIMEOUT"}

# name -> (restype, argtypes); the exact C prototypes of include/boba.h
_P, _I64, _U32, _I32, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_size_t
PROTOTYPES = {
    "boba_last_error": (ctypes.c_char_p, []),
    "boba_check_device_error": (_I32, [_P, _P]),
    "boba_reorder_workspace": (_SZ, [_I64, _I64]),
    "boba_reorder": (_I32, [_P, _P, _I64, _I64, _P, _P, _P, _SZ, _U32, _P]),
    "boba_reorder_noalloc": (_I32, [_P, _P, _I64, _I64, _P, _P, _U32, _P]),
    "boba_relabel": (_I32, [_P, _P, _I64, _P, _I64, _P, _P, _P]),
    "boba_relabel_bucketed_workspace": (_SZ, [_I64, _I64]),
    "boba_relabel_bucketed": (_I32, [_P, _P, _I64, _P, _I64, _P, _P, _P, _SZ, _P]),
    "boba_reorder_relabel_workspace": (_SZ, [_I64, _I64]),
    "boba_reorder_relabel": (_I32, [_P, _P, _I64, _I64, _P, _P, _P, _P, _P, _SZ, _U32, _P]),
    "boba_bin_by_dst_workspace": (_SZ, [_I64, _I64]),
    "boba_bin_by_dst": (_I32, [_P, _P, _I64, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "coo_to_csr_workspace": (_SZ, [_I64, _I64]),
    "coo_to_csr": (_I32, [_P, _P, _P, _I64, _I64, _P, _P, _P, _P, _SZ, _P]),
    "spmv_csr_workspace": (_SZ, [_I64, _I64]),
    "spmv_csr": (_I32, [_P, _P, _P, _I64, _I64, _I64, _P, _P, _P, _SZ, _P]),
    "boba_pagerank_workspace": (_SZ, [_I64, _I64]),
    "boba_pagerank": (_I32, [_P, _P, _P, _I64, _I64, ctypes.c_float, _I32, ctypes.c_double, _P, _P, _P, _P, _SZ,
                             _P]),
    "boba_nbr_workspace": (_SZ, [_I64, _I64]),
    "boba_nbr": (_I32, [_P, _P, _I64, _I64, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "boba_batch_workspace": (_SZ, [_I32, _P, _P, _P]),
    "boba_batch_plan_create": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P, _P, _P]),
    "boba_batch_plan_launch": (_I32, [_P, _P]),
    "boba_batch_plan_info": (_I32, [_P, _P]),
    "boba_batch_plan_destroy": (_I32, [_P]),
    "boba_graph_features_workspace": (_SZ, []),
    "boba_graph_features": (_I32, [_P, _P, _I64, _I64, _P, _P, _SZ, _P]),
    "boba_mlp_param_count": (_I32, []),
    "boba_mlp_forward": (_I32, [_P, _P, _I32, _P, _P]),
    "boba_mlp_backward_workspace": (_SZ, [_I32]),
    "boba_mlp_backward": (_I32, [_P, _P, _P, _I32, _P, _P, _P, _SZ, _P]),
    "boba_mlp_adam": (_I32, [_P, _P, _P, _P, _I32, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, _P]),
    "boba_timing_enable": (_I32, [_I32]),
    "boba_timing_collect": (_I32, [_P, _SZ, _P, _P, _I32]),
}

_lib = None


class BobaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libboba.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2306_10410_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != BOBA_OK:
        raise BobaError(status, load().boba_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_i32(t, name):
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int32 device tensor")
    return t


def _workspace(nbytes: int, device, ws=None):
    if ws is not None and ws.numel() >= nbytes:
        return ws
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def boba_reorder_workspace(n: int, m: int) -> int:
    return int(load().boba_reorder_workspace(n, m))


def boba_reorder(src, dst, n: int, *, with_order: bool = True, flags: int = 0, ws=None, perm=None,
                 order=None, stream=None):
    """Returns (perm, order) as int32 device tensors: perm[old] = new,
    order[new] = old (order is None unless with_order)."""
    _dev_i32(src, "src")
    _dev_i32(dst, "dst")
    m = src.numel()
    if dst.numel() != m:
        raise ValueError("src and dst differ in length")
    dev = src.device
    perm = torch.empty(n, dtype=torch.int32, device=dev) if perm is None else perm
    if with_order and order is None:
        order = torch.empty(n, dtype=torch.int32, device=dev)
    need = boba_reorder_workspace(n, m)
    ws = _workspace(need, dev, ws)
    _check(load().boba_reorder(_ptr(src), _ptr(dst), m, n, _ptr(perm), _ptr(order) if with_order else None,
                               _ptr(ws), ws.numel(), flags, _stream(stream)))
    return perm, (order if with_order else None)


BOBA_REORDER_NOALLOC_MAX_BYTES = 64 << 20  # include/boba.h


def boba_reorder_noalloc(src, dst, n: int, perm, order=None, *, flags: int = 0, stream=None):
    """boba_reorder with the library's static scratch as workspace: writes
    perm (and order, if given) and allocates nothing, so the caller passes
    both outputs."""
    _dev_i32(src, "src")
    _dev_i32(dst, "dst")
    _dev_i32(perm, "perm")
    if order is not None:
        _dev_i32(order, "order")
    m = src.numel()
    if dst.numel() != m:
        raise ValueError("src and dst differ in length")
    if perm.numel() < n or (order is not None and order.numel() < n):
        raise ValueError("perm/order hold fewer than n entries")
    _check(load().boba_reorder_noalloc(_ptr(src), _ptr(dst), m, n, _ptr(perm), _ptr(order), flags,
                                       _stream(stream)))
    return perm, order


def boba_relabel(src, dst, perm, *, src_out=None, dst_out=None, stream=None):
    _dev_i32(src, "src")
    _dev_i32(dst, "dst")
    _dev_i32(perm, "perm")
    src_out = torch.empty_like(src) if src_out is None else src_out
    dst_out = torch.empty_like(dst) if dst_out is None else dst_out
    _check(load().boba_relabel(_ptr(src), _ptr(dst), src.numel(), _ptr(perm), perm.numel(), _ptr(src_out),
                               _ptr(dst_out), _stream(stream)))
    return src_out, dst_out


def boba_relabel_bucketed_workspace(n: int, m: int) -> int:
    return int(load().boba_relabel_bucketed_workspace(n, m))


def boba_relabel_bucketed(src, dst, perm, *, src_out=None, dst_out=None, ws=None, stream=None):
    """boba_relabel through vertex buckets (no random perm reads); same results."""
    _dev_i32(src, "src")
    _dev_i32(dst, "dst")
    _dev_i32(perm, "perm")
    m, n = src.numel(), perm.numel()
    if dst.numel() != m:
        raise ValueError("src and dst differ in length")
    src_out = torch.empty_like(src) if src_out is None else src_out
    dst_out = torch.empty_like(dst) if dst_out is None else dst_out
    ws = _workspace(boba_relabel_bucketed_workspace(n, m), src.device, ws)
    _check(load().boba_relabel_bucketed(_ptr(src), _ptr(dst), m, _ptr(perm), n, _ptr(src_out), _ptr(dst_out),
                                        _ptr(ws), ws.numel(), _stream(stream)))
    return src_out, dst_out


def boba_reorder_relabel_workspace(n: int, m: int) -> int:
    return int(load().boba_reorder_relabel_workspace(n, m))


def boba_reorder_relabel(src, dst, n: int, *, with_order: bool = True, flags: int = 0, ws=None, perm=None,
                         order=None, src_out=None, dst_out=None, stream=None):
    """Returns (perm, order, src_out, dst_out)."""
    _dev_i32(src, "src")
    _dev_i32(dst, "dst")
    m = src.numel()
    if dst.numel() != m:
        raise ValueError("src and dst differ in length")
    dev = src.device
    perm = torch.empty(n, dtype=torch.int32, device=dev) if perm is None else perm
    if with_order and order is None:
        order = torch.empty(n, dtype=torch.int32, device=dev)
    src_out = torch.empty_like(src) if src_out is None else src_out
    dst_out = torch.empty_like(dst) if dst_out is None else dst_out
    ws = _workspace(boba_reorder_relabel_workspace(n, m), dev, ws)
    _check(load().boba_reorder_relabel(_ptr(src), _ptr(dst), m, n, _ptr(perm), _ptr(order) if with_order else None,
                                       _ptr(src_out), _ptr(dst_out), _ptr(ws), ws.numel(), flags, _stream(stream)))
    return perm, (order if with_order else None), src_out, dst_out


def boba_bin_by_dst_workspace(n: int, m: int) -> int:
    return int(load().boba_bin_by_dst_workspace(n, m))


def boba_bin_by_dst(src, dst, n: int, bin_bits: int, *, ws=None, out=None, stream=None):
    """Edges stably binned by destination (dst >> shift).  Returns (src_out, dst_out)."""
    _dev_i32(src, "src")
    _dev_i32(dst, "dst")
    m = src.numel()
    if dst.numel() != m:
        raise ValueError("src and dst differ in length")
    so, do = (torch.empty_like(src), torch.empty_like(dst)) if out is None else out
    ws = _workspace(boba_bin_by_dst_workspace(n, m), src.device, ws)
    _check(load().boba_bin_by_dst(_ptr(src), _ptr(dst), m, n, bin_bits, _ptr(so), _ptr(do), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return so, do


def coo_to_csr_workspace(n_rows: int, m: int) -> int:
    return int(load().coo_to_csr_workspace(n_rows, m))


def coo_to_csr(row, col, val, n_rows: int, *, ws=None, out=None, stream=None):
    """Returns (rowptr[n_rows+1], col_out, val_out or None)."""
    _dev_i32(row, "row")
    _dev_i32(col, "col")
    m = row.numel()
    dev = row.device
    if out is None:
        rowptr = torch.empty(n_rows + 1, dtype=torch.int32, device=dev)
        col_out = torch.empty(m, dtype=torch.int32, device=dev)
        val_out = None if val is None else torch.empty(m, dtype=torch.float32, device=dev)
    else:
        rowptr, col_out, val_out = out
    ws = _workspace(coo_to_csr_workspace(n_rows, m), dev, ws)
    _check(load().coo_to_csr(_ptr(row), _ptr(col), _ptr(val), m, n_rows, _ptr(rowptr), _ptr(col_out),
                             _ptr(val_out), _ptr(ws), ws.numel(), _stream(stream)))
    return rowptr, col_out, val_out


def spmv_csr_workspace(n_rows: int, nnz: int) -> int:
    return int(load().spmv_csr_workspace(n_rows, nnz))


def spmv_csr(rowptr, col, val, x, *, y=None, ws=None, stream=None):
    _dev_i32(rowptr, "rowptr")
    _dev_i32(col, "col")
    n_rows = rowptr.numel() - 1
    y = torch.empty(n_rows, dtype=torch.float32, device=x.device) if y is None else y
    ws = _workspace(spmv_csr_workspace(n_rows, col.numel()), x.device, ws)
    _check(load().spmv_csr(_ptr(rowptr), _ptr(col), _ptr(val), n_rows, x.numel(), col.numel(), _ptr(x), _ptr(y),
                           _ptr(ws), ws.numel(), _stream(stream)))
    return y


def boba_pagerank_workspace(n: int, nnz: int) -> int:
    return int(load().boba_pagerank_workspace(n, nnz))


def boba_pagerank(rowptr, col, damping: float = 0.85, max_iter: int = 20, tol: float = 0.0, *, out_rowptr=None,
                  rank=None, ws=None, stream=None):
    """PageRank over the transposed CSR (row v lists the sources of the edges
    into v); out_rowptr, the forward CSR's row pointer, gives the out-degrees
    without atomics.  Returns (rank float32[n], residual float64[max_iter],
    iters int32[1]), all device tensors; residual entries past iters are unset."""
    _dev_i32(rowptr, "rowptr")
    _dev_i32(col, "col")
    if out_rowptr is not None:
        _dev_i32(out_rowptr, "out_rowptr")
        if out_rowptr.numel() != rowptr.numel():
            raise ValueError("out_rowptr and rowptr differ in length")
    n = rowptr.numel() - 1
    dev = rowptr.device
    rank = torch.empty(max(n, 0), dtype=torch.float32, device=dev) if rank is None else rank
    residual = torch.full((max(max_iter, 0),), float("nan"), dtype=torch.float64, device=dev)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = _workspace(boba_pagerank_workspace(n, col.numel()), dev, ws)
    _check(load().boba_pagerank(_ptr(rowptr), _ptr(col), _ptr(out_rowptr), n, col.numel(), damping, max_iter, tol,
                                _ptr(rank), _ptr(residual) if max_iter > 0 else None, _ptr(iters), _ptr(ws),
                                ws.numel(), _stream(stream)))
    return rank, residual, iters


def boba_nbr_workspace(n_rows: int, nnz: int) -> int:
    return int(load().boba_nbr_workspace(n_rows, nnz))


def boba_nbr(rowptr, col, n_cols: int, line_ids: int = 32, *, per_row=False, ws=None, stream=None):
    """NBR of the CSR rows (Sec. 5.2).  Returns (mean over all rows, mean over
    non-empty rows), plus the distinct lines per row when per_row is set.
    Waits for the stream (the two means come back to the host)."""
    _dev_i32(rowptr, "rowptr")
    _dev_i32(col, "col")
    n_rows = rowptr.numel() - 1
    dev = rowptr.device
    lines = torch.empty(max(n_rows, 0), dtype=torch.int32, device=dev) if per_row else None
    result = torch.empty(4, dtype=torch.float64, device=dev)
    ws = _workspace(boba_nbr_workspace(n_rows, col.numel()), dev, ws)
    _check(load().boba_nbr(_ptr(rowptr), _ptr(col), n_rows, n_cols, col.numel(), line_ids, _ptr(lines),
                           _ptr(result), _ptr(ws), ws.numel(), _stream(stream)))
    if stream is not None:
        stream.synchronize()
    means = tuple(result[2:].tolist())  # computed by the library's final kernel
    return (*means, lines) if per_row else means


def boba_check_device_error(stream=None) -> int:
    code = ctypes.c_int32(0)
    _check(load().boba_check_device_error(_stream(stream), ctypes.byref(code)))
    return int(code.value)


def boba_timing_enable(on: bool = True):
    _check(load().boba_timing_enable(1 if on else 0))


def boba_timing_collect(max_entries: int = 64):
    """Returns {kernel name: (total ms, launches)} since the last collect."""
    buf = ctypes.create_string_buffer(64 * max_entries)
    ms = (ctypes.c_double * max_entries)()
    cnt = (ctypes.c_int64 * max_entries)()
    k = load().boba_timing_collect(buf, len(buf), ms, cnt, max_entries)
    names = buf.raw.split(b"\0")[:k]
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(k)}


class boba_tuning(ctypes.Structure):
    """Mirror of struct boba_tuning (0 = library default)."""
    _fields_ = [("small_max_n", ctypes.c_int32), ("scatter_tile", ctypes.c_int32),
                ("vertex_tile", ctypes.c_int32), ("relabel_tile", ctypes.c_int32),
                ("queues", ctypes.c_int32), ("spin_limit", ctypes.c_int32),
                ("scatter_atomic", ctypes.c_int32)]


def _host_i64(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def boba_batch_workspace(edge_off, vert_off, tuning=None) -> int:
    eo, peo = _host_i64(edge_off)
    vo, pvo = _host_i64(vert_off)
    return int(load().boba_batch_workspace(len(eo) - 1, peo, pvo, ctypes.byref(tuning) if tuning else None))


class BatchPlan:
    """A captured batched reorder (+relabel).  Keeps the tensors it was built
    on alive; launch() replays it on the current (or given) stream."""

    def __init__(self, edge_off, vert_off, src, dst, *, relabel=True, with_order=True, tuning=None,
                 stream=None):
        _dev_i32(src, "src")
        _dev_i32(dst, "dst")
        eo, peo = _host_i64(edge_off)
        vo, pvo = _host_i64(vert_off)
        G = len(eo) - 1
        dev = src.device
        self.src, self.dst = src, dst
        self.perm = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
        self.order = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev) if with_order else None
        self.src_out = torch.empty_like(src) if relabel else None
        self.dst_out = torch.empty_like(dst) if relabel else None
        tp = ctypes.byref(tuning) if tuning else None
        need = int(load().boba_batch_workspace(G, peo, pvo, tp))
        if need == 0 and G > 0:
            raise BobaError(BOBA_ERR_ARG, "invalid batch description")
        self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        self._plan = ctypes.c_void_p()
        _check(load().boba_batch_plan_create(G, peo, pvo, _ptr(src), _ptr(dst), _ptr(self.perm), _ptr(self.order),
                                             _ptr(self.src_out), _ptr(self.dst_out), _ptr(self.ws), self.ws.numel(),
                                             tp, _stream(stream), ctypes.byref(self._plan)))

    def launch(self, stream=None):
        _check(load().boba_batch_plan_launch(self._plan, _stream(stream)))
        return self

    def info(self):
        out = (ctypes.c_int64 * 4)()
        _check(load().boba_batch_plan_info(self._plan, out))
        return {"items": out[0], "whole_graph_items": out[1], "r_words": out[2], "bitmap_words": out[3]}

    def destroy(self):
        if self._plan:
            _check(load().boba_batch_plan_destroy(self._plan))
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _dev_f32(t, name):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 device tensor")
    return t


def boba_graph_features(src, dst, n: int, *, out=None, ws=None, stream=None):
    """16 FP32 features (device tensor) of an edge list."""
    _dev_i32(src, "src")
    _dev_i32(dst, "dst")
    out = torch.empty(16, dtype=torch.float32, device=src.device) if out is None else out
    ws = _workspace(int(load().boba_graph_features_workspace()), src.device, ws)
    _check(load().boba_graph_features(_ptr(src), _ptr(dst), src.numel(), n, _ptr(out), _ptr(ws), ws.numel(),
                                      _stream(stream)))
    return out


def boba_mlp_param_count() -> int:
    return int(load().boba_mlp_param_count())


def boba_mlp_forward(params, X, *, out=None, stream=None):
    _dev_f32(params, "params")
    _dev_f32(X, "X")
    B = X.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=X.device) if out is None else out
    _check(load().boba_mlp_forward(_ptr(params), _ptr(X), B, _ptr(out), _stream(stream)))
    return out


def boba_mlp_backward(params, X, y, *, grad=None, loss=None, ws=None, stream=None):
    _dev_f32(params, "params")
    _dev_f32(X, "X")
    _dev_f32(y, "y")
    B = X.shape[0]
    grad = torch.empty_like(params) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=X.device) if loss is None else loss
    ws = _workspace(int(load().boba_mlp_backward_workspace(B)), X.device, ws)
    _check(load().boba_mlp_backward(_ptr(params), _ptr(X), _ptr(y), B, _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return grad, loss


def boba_mlp_adam(params, m1, m2, grad, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    for a, nm in ((params, "params"), (m1, "m1"), (m2, "m2"), (grad, "grad")):
        _dev_f32(a, nm)
    _check(load().boba_mlp_adam(_ptr(params), _ptr(m1), _ptr(m2), _ptr(grad), params.numel(), t, lr, b1, b2, eps,
                                _stream(stream)))
