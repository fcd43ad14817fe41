"""Shared helpers for the GPU parity tests (not collected by pytest)."""
import numpy as np
import pytest
import torch

import oracle

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no HIP device visible")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(y, ref):
    y = np.asarray(y, np.float64)
    ref = np.asarray(ref, np.float64)
    nr = np.linalg.norm(ref)
    if nr == 0.0:
        return float(np.linalg.norm(y))
    return float(np.linalg.norm(y - ref) / nr)


SPMV_TOL = 1e-5  # relative L2 of FP32 SpMV against the FP64 oracle


def bits_equal(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint32), b.view(np.uint32))


def full_path_check(g, boba, interleaved=False, check_spmv=True, general=False):
    """Run reorder -> relabel -> CSR -> SpMV on the GPU and compare every
    element with the oracle on the same inputs.  general: small graphs through
    the many-workgroup reorder path instead of the one-launch path."""
    flags = (boba.BOBA_FLAG_INTERLEAVED if interleaved else 0) | (boba.BOBA_FLAG_FORCE_GENERAL if general else 0)
    s, d = dev(g.src), dev(g.dst)
    perm, order = boba.boba_reorder(s, d, g.n, flags=flags)
    p_ref, o_ref = oracle.boba(g.src, g.dst, g.n, interleaved=interleaved)
    assert np.array_equal(host(perm), p_ref), "perm differs from the oracle"
    assert np.array_equal(host(order), o_ref), "order differs from the oracle"
    s2, d2 = boba.boba_relabel(s, d, perm)
    s2_ref, d2_ref = oracle.relabel(g.src, g.dst, p_ref)
    assert np.array_equal(host(s2), s2_ref) and np.array_equal(host(d2), d2_ref), "relabel differs"
    # fused reorder + relabel gives the same four arrays
    fp, fo, fs, fd = boba.boba_reorder_relabel(s, d, g.n, flags=flags)
    assert np.array_equal(host(fp), p_ref) and np.array_equal(host(fo), o_ref), "fused perm/order differ"
    assert np.array_equal(host(fs), s2_ref) and np.array_equal(host(fd), d2_ref), "fused relabel differs"
    val = dev(g.val) if g.val is not None else None
    rowptr, col, v = boba.coo_to_csr(s2, d2, val, g.n)
    rp_ref, col_ref, v_ref = oracle.coo_to_csr(s2_ref, d2_ref, g.val, g.n)
    assert np.array_equal(host(rowptr), rp_ref), "rowptr differs"
    assert np.array_equal(host(col), col_ref), "CSR col differs"
    if g.val is not None:
        assert bits_equal(host(v), v_ref), "CSR val differs"
    if check_spmv and g.x is not None:
        y = boba.spmv_csr(rowptr, col, v, dev(g.x))
        y_ref = oracle.spmv64(rp_ref, col_ref, v_ref, g.x)
        err = rel_l2(host(y), y_ref)
        assert err <= SPMV_TOL, f"SpMV relative L2 {err:.3e} > {SPMV_TOL}"
    assert boba.boba_check_device_error() == boba.BOBA_OK


def nbr_check(rowptr, col, n_cols, line_ids=32):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    n_rows = rowptr.size - 1
    from paper_2306_10410_amd import boba
    over_n, over_ne, lines = boba.boba_nbr(dev(rowptr), dev(col), n_cols, line_ids, per_row=True)
    r_n, r_ne, r_lines = oracle.nbr(rowptr, col, n_rows, line_ids, per_row=True)
    assert np.array_equal(host(lines), r_lines), "distinct lines per row differ"
    # both sums add the same non-negative per-row ratios (each the same IEEE
    # quotient) in different orders: each is within (rows - 1) * 2^-53 of the
    # exact sum, relative
    tol = 2.0 * max(n_rows, 1) * 2.0 ** -53
    assert abs(over_n - r_n) <= tol * abs(r_n), (over_n, r_n)
    assert abs(over_ne - r_ne) <= tol * abs(r_ne), (over_ne, r_ne)
    nonempty = int(np.count_nonzero(np.diff(rowptr)))
    if nonempty:
        assert round(over_n * n_rows / over_ne) == nonempty
    assert boba.boba_check_device_error() == boba.BOBA_OK
    return over_n, over_ne
