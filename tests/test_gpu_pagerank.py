"""GPU parity of PageRank as repeated SpMV (the PR application of Sec. 5.1)
through the C ABI against the FP64 oracle.

Tolerance: ranks sum to 1.  One FP32 iteration rounds each pulled sum over at
most 64 sequential terms, a 6-level shuffle tree and the chunk carries, about
80 roundings of 2^-24 relative, so it adds at most ~5e-6 of L1 error; the
iteration contracts earlier errors by the damping a, so after k iterations the
error is below 5e-6 * (1 + a + ... + a^(k-1)) (3.3e-5 for a = 0.85 and any k).
The tests allow 1.5 times that bound, twice it for each iteration's L1
change."""
import numpy as np
import pytest
import torch

import oracle
from paper_2306_10410_amd import boba, graphgen
from gpu_util import dev, host, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

L1_TOL = 5e-5


def l1_bound(damping, iters):
    return 1.5 * 5e-6 * sum(damping ** k for k in range(iters))


def transposed_csr(src, dst, n):
    rowptr, col, _ = oracle.coo_to_csr(dst, src, None, n)  # row v: the sources of the edges into v
    return rowptr, col


def pr_check(src, dst, n, damping=0.85, iters=20):
    rowptr, col = transposed_csr(src, dst, n)
    rank, res, it = boba.boba_pagerank(dev(rowptr), dev(col), damping, iters)
    # out-degrees from the forward CSR's row pointer instead of atomics: the same bits
    fwd_rowptr, _, _ = oracle.coo_to_csr(src, dst, None, n)
    rank2, _, _ = boba.boba_pagerank(dev(rowptr), dev(col), damping, iters, out_rowptr=dev(fwd_rowptr))
    assert np.array_equal(host(rank2).view(np.uint32), host(rank).view(np.uint32))
    r_ref, ch_ref = oracle.pagerank(src, dst, n, damping, iters)
    rank_h = host(rank).astype(np.float64)
    bound = l1_bound(damping, max(iters, 1))
    err = np.abs(rank_h - r_ref).sum()
    assert err <= bound, (err, bound)
    assert int(host(it)[0]) == iters
    assert np.all(np.abs(host(res) - np.array(ch_ref)) <= 2 * bound)
    assert abs(rank_h.sum() - 1.0) <= bound
    assert boba.boba_check_device_error() == boba.BOBA_OK
    return rank


@pytest.mark.parametrize("kind,n,m", [("uniform", 16384, 131072), ("rmat", 1 << 16, (1 << 20) + 3),
                                      ("grid", 40000, 0), ("rgg", 30000, 300000)])
def test_graphs_fixed_iterations(kind, n, m):
    g = graphgen.small_workload(kind, n, m, 101 + n % 5)
    pr_check(g.src, g.dst, g.n)


@pytest.mark.parametrize("damping", [0.0, 0.5, 0.85, 1.0])
def test_damping_factors(damping):
    g = graphgen.small_workload("rmat", 1 << 14, 1 << 17, 102)
    pr_check(g.src, g.dst, g.n, damping, iters=12)


def test_stop_at_tolerance():
    g = graphgen.small_workload("rmat", 1 << 15, 1 << 19, 103)
    rowptr, col = transposed_csr(g.src, g.dst, g.n)
    tol = 1e-5
    rank, res, it = boba.boba_pagerank(dev(rowptr), dev(col), 0.85, 200, tol)
    k = int(host(it)[0])
    res_h = host(res)
    assert 0 < k < 200
    # the device stopped at the first iteration below the tolerance (its own residuals)
    assert res_h[k - 1] < tol and np.all(res_h[: k - 1] >= tol) and np.all(np.isnan(res_h[k:]))
    r_ref, _ = oracle.pagerank(g.src, g.dst, g.n, 0.85, k)
    assert np.abs(host(rank).astype(np.float64) - r_ref).sum() <= L1_TOL


def test_reordering_permutes_the_ranks():
    g = graphgen.small_workload("rmat", 1 << 16, 1 << 20, 104)
    perm, _, s2, d2 = boba.boba_reorder_relabel(dev(g.src), dev(g.dst), g.n)
    r1 = pr_check(g.src, g.dst, g.n)
    r2 = pr_check(host(s2), host(d2), g.n)
    p = host(perm)
    assert np.abs(host(r2)[p].astype(np.float64) - host(r1)).sum() <= 2 * L1_TOL


def test_degenerate_graphs():
    pr_check(np.zeros(0, np.int32), np.zeros(0, np.int32), 7)         # no edges: every vertex dangling
    pr_check(np.zeros(3, np.int32), np.zeros(3, np.int32), 1)         # one vertex, self-loops
    cyc = np.arange(1000, dtype=np.int32)
    rank = pr_check(cyc, np.roll(cyc, -1), 1000)                      # a cycle stays uniform
    assert np.abs(host(rank) - 1e-3).max() <= 1e-9
    rowptr, col = transposed_csr(cyc, np.roll(cyc, -1), 1000)
    rank, res, it = boba.boba_pagerank(dev(rowptr), dev(col), 0.85, 0)  # no iteration: r_0
    assert int(host(it)[0]) == 0 and np.all(host(rank) == np.float32(1.0) / np.float32(1000))


def test_out_of_range_sources_set_the_device_flag():
    assert boba.boba_check_device_error() == boba.BOBA_OK
    rowptr = dev(np.array([0, 2, 3, 3], np.int32))
    col = dev(np.array([1, 2, 7], np.int32))  # 7 >= n = 3
    boba.boba_pagerank(rowptr, col, 0.85, 3)
    assert boba.boba_check_device_error() == boba.BOBA_ERR_RANGE


def test_repeatable_bits():
    g = graphgen.small_workload("rmat", 1 << 15, 1 << 19, 105)
    rowptr, col = transposed_csr(g.src, g.dst, g.n)
    rp, cl = dev(rowptr), dev(col)
    first = host(boba.boba_pagerank(rp, cl, 0.85, 15)[0])
    for _ in range(3):
        assert np.array_equal(host(boba.boba_pagerank(rp, cl, 0.85, 15)[0]).view(np.uint32), first.view(np.uint32))
    torch.cuda.synchronize()
