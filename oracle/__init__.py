"""CPU oracle for the BOBA hot path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2306_10410_amd``) and never imports it.

The arithmetic lives in ``boba_oracle.c`` (plain sequential C, FP64 where
floating point is involved); this module only compiles it with gcc, loads it
with ctypes and marshals numpy arrays.  ``features.py`` holds the plain numpy
definition of the selector's graph features, and ``pagerank`` below is plain
numpy in FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "boba_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MLP_IN, MLP_H = 16, 64
MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1  # 5313


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile boba_oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        L.oracle_boba.argtypes = [P, P, I64, I64, ctypes.c_int, P, P]
        L.oracle_relabel.argtypes = [P, P, I64, P, I64, P, P]
        L.oracle_coo_to_csr.argtypes = [P, P, P, I64, I64, P, P, P]
        L.oracle_spmv64.argtypes = [P, P, P, I64, I64, P, P]
        L.oracle_mlp_forward.argtypes = [P, P, I64, P]
        L.oracle_mlp_backward.argtypes = [P, P, P, I64, P, P]
        L.oracle_adam.argtypes = [P, P, P, P, I64, I64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double]
        L.oracle_nbr.argtypes = [P, P, I64, I64, P, P, P]
        L.oracle_bin_by_dst.argtypes = [P, P, I64, I64, ctypes.c_int, P, P]
        L.oracle_mlp_nparam.restype = I64
        for f in ("oracle_boba", "oracle_relabel", "oracle_coo_to_csr", "oracle_spmv64",
                  "oracle_mlp_forward", "oracle_mlp_backward", "oracle_adam", "oracle_nbr",
                  "oracle_bin_by_dst"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what}: oracle status {rc} ({'argument' if rc == 1 else 'vertex id out of range'})")


def boba(src, dst, n, interleaved=False):
    """Sequential BOBA (Algorithm 1 + isolated-vertex tail).  Returns
    (perm, order): perm[old] = new, order[new] = old."""
    src, dst = _i32(src), _i32(dst)
    perm = np.empty(n, np.int32)
    order = np.empty(n, np.int32)
    _check(lib().oracle_boba(_p(src), _p(dst), src.size, n, int(bool(interleaved)),
                             _p(perm), _p(order)), "boba")
    return perm, order


def relabel(src, dst, perm):
    src, dst, perm = _i32(src), _i32(dst), _i32(perm)
    s2 = np.empty_like(src)
    d2 = np.empty_like(dst)
    _check(lib().oracle_relabel(_p(src), _p(dst), src.size, _p(perm), perm.size,
                                _p(s2), _p(d2)), "relabel")
    return s2, d2


def coo_to_csr(row, col, val, n_rows):
    row, col = _i32(row), _i32(col)
    v = None if val is None else np.ascontiguousarray(val, dtype=np.float32)
    rowptr = np.empty(n_rows + 1, np.int32)
    col_out = np.empty_like(col)
    val_out = None if v is None else np.empty_like(v)
    _check(lib().oracle_coo_to_csr(_p(row), _p(col), _p(v), row.size, n_rows, _p(rowptr),
                                   _p(col_out), _p(val_out)), "coo_to_csr")
    return rowptr, col_out, val_out


def bin_by_dst(src, dst, n, bin_bits):
    """Edges stably sorted by dst >> shift (Sec. 5.6's binning by destination)."""
    src, dst = _i32(src), _i32(dst)
    so, do = np.empty_like(src), np.empty_like(dst)
    _check(lib().oracle_bin_by_dst(_p(src), _p(dst), src.size, n, int(bin_bits), _p(so), _p(do)), "bin_by_dst")
    return so, do


def spmv64(rowptr, col, val, x, n_rows=None):
    rowptr, col = _i32(rowptr), _i32(col)
    x = np.ascontiguousarray(x, dtype=np.float32)
    v = None if val is None else np.ascontiguousarray(val, dtype=np.float32)
    n_rows = rowptr.size - 1 if n_rows is None else n_rows
    y = np.empty(n_rows, np.float64)
    _check(lib().oracle_spmv64(_p(rowptr), _p(col), _p(v), n_rows, x.size, _p(x), _p(y)), "spmv")
    return y


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mlp_forward(params, X):
    params, X = _f64(params), _f64(X).reshape(-1, MLP_IN)
    y = np.empty(X.shape[0], np.float64)
    _check(lib().oracle_mlp_forward(_p(params), _p(X), X.shape[0], _p(y)), "mlp_forward")
    return y


def mlp_backward(params, X, y):
    params, X, y = _f64(params), _f64(X).reshape(-1, MLP_IN), _f64(y)
    g = np.empty(MLP_NPARAM, np.float64)
    loss = np.zeros(1, np.float64)
    _check(lib().oracle_mlp_backward(_p(params), _p(X), _p(y), X.shape[0], _p(g), _p(loss)),
           "mlp_backward")
    return g, float(loss[0])


def adam(params, m1, m2, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step, in place on float64 arrays params/m1/m2."""
    for a in (params, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    grad = _f64(grad)
    _check(lib().oracle_adam(_p(params), _p(m1), _p(m2), _p(grad), params.size, t,
                             lr, b1, b2, eps), "adam")


def nbr(rowptr, col, n, line_ids=32, per_row=False):
    """NBR (Sec. 5.2) over CSR rows.  Returns (mean over all n, mean over
    vertices with a non-empty neighbourhood), and with per_row also the
    distinct lines of every row."""
    rowptr, col = _i32(rowptr), _i32(col)
    s = np.zeros(1, np.float64)
    c = np.zeros(1, np.int64)
    d = np.zeros(n, np.int32) if per_row else None
    _check(lib().oracle_nbr(_p(rowptr), _p(col), n, line_ids, _p(s), _p(c), _p(d) if per_row else None), "nbr")
    means = (s[0] / n if n else 0.0), (s[0] / c[0] if c[0] else 0.0)
    return (*means, d) if per_row else means


def pagerank(src, dst, n, damping=0.85, iters=20, tol=0.0):
    """PageRank by power iteration (the PR application of Sec. 5.1), in FP64,
    straight from its definition over the edge list:
        r_0 = 1/n
        r_{k+1}[v] = (1 - d)/n + d * (sum over edges u->v of r_k[u]/outdeg(u) + D_k/n)
    with D_k the rank on vertices without out-edges.  Stops after the first
    iteration whose L1 change is below tol (tol > 0).  Returns (r, the L1
    change of every iteration run)."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    outdeg = np.bincount(src, minlength=n).astype(np.float64)
    r = np.full(n, 1.0 / n)
    changes = []
    for _ in range(iters):
        share = np.zeros(n)
        np.divide(r, outdeg, out=share, where=outdeg > 0)
        y = np.zeros(n)
        np.add.at(y, dst, share[src])  # every edge u->v carries r[u]/outdeg(u) to v
        dangling = r[outdeg == 0].sum()
        new = (1.0 - damping) / n + damping * (y + dangling / n)
        changes.append(float(np.abs(new - r).sum()))
        r = new
        if tol > 0 and changes[-1] < tol:
            break
    return r, changes