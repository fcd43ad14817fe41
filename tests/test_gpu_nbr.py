"""GPU parity of the NBR metric (Sec. 5.2) through the C ABI: distinct lines
per row bit-exact against the oracle, the ratio sum within the rounding bound
of two summation orders, the number of non-empty rows exact."""
import numpy as np
import pytest

import oracle
from paper_2306_10410_amd import boba, graphgen
from gpu_util import dev, nbr_check, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def csr_of(src, dst, n):
    rowptr, col, _ = oracle.coo_to_csr(src, dst, None, n)
    return rowptr, col


@pytest.mark.parametrize("kind,n,m", [("uniform", 16384, 131072), ("rmat", 1 << 16, (1 << 20) + 3),
                                      ("rmat", 70001, 900007)])
def test_random_graphs_before_and_after_boba(kind, n, m):
    g = graphgen.small_workload(kind, n, m, 95 + n % 7)
    before = nbr_check(*csr_of(g.src, g.dst, g.n), g.n)
    p, _ = oracle.boba(g.src, g.dst, g.n)
    s2, d2 = oracle.relabel(g.src, g.dst, p)
    after = nbr_check(*csr_of(s2, d2, g.n), g.n)
    if kind == "rmat":
        assert after[1] < before[1]  # the reordering buys locality


@pytest.mark.parametrize("line_ids", [1, 2, 32, 1024, 1 << 30])
def test_line_widths(line_ids):
    g = graphgen.small_workload("rmat", 1 << 15, 1 << 19, 96)
    nbr_check(*csr_of(g.src, g.dst, g.n), g.n, line_ids)


def test_rows_around_the_wavefront_limit_and_chunk_edges():
    # degrees 255..258 straddle the longest row a wavefront counts; a run of
    # 250-entry rows puts row starts at every offset of the 1024-item chunks;
    # empty rows in between and at the end
    rng = np.random.default_rng(97)
    deg = np.concatenate([[255, 256, 257, 258, 0, 1, 64, 65, 0], np.full(40, 250), rng.integers(0, 300, 400),
                          [0, 0, 0]])
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    n = 5000
    col = rng.integers(0, n, rowptr[-1]).astype(np.int32)
    col[: 255 + 256] = rng.integers(0, 300, 511)  # dense lines: many repeats
    nbr_check(rowptr, col, n)
    nbr_check(rowptr, col, n, line_ids=1)


def test_rows_around_the_hash_set_limit():
    # rows of 2047..2050 entries straddle the longest row counted with a hash
    # set (longer ones take the bitmap); one draws from ~125 lines, one gives
    # about a line per entry, and 257 and 3000 entries sit inside each class
    rng = np.random.default_rng(101)
    deg = np.array([2047, 2048, 2049, 2050, 300, 1000, 5, 0, 3000, 257])
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    n = 1 << 20
    col = rng.integers(0, n, rowptr[-1]).astype(np.int32)
    col[rowptr[0]:rowptr[1]] = rng.integers(0, 4000, deg[0])
    col[rowptr[2]:rowptr[3]] = rng.integers(0, 70000, deg[2])
    nbr_check(rowptr, col, n)
    nbr_check(rowptr, col, n, line_ids=1)
    # an out-of-range column inside a row counted with the bitmap
    col[rowptr[8] + 100] = n + 5
    assert boba.boba_check_device_error() == boba.BOBA_OK
    boba.boba_nbr(dev(rowptr), dev(col), n)
    assert boba.boba_check_device_error() == boba.BOBA_ERR_RANGE


def test_long_runs_of_empty_rows():
    # chunks count rows as well as entries: 100,000 empty rows in the middle
    # and 200,000 at the end (where BOBA puts isolated vertices) are shared
    # out over many chunks
    rng = np.random.default_rng(100)
    deg = np.concatenate([rng.integers(0, 40, 3000), np.zeros(100000, np.int64), rng.integers(0, 400, 2000),
                          np.zeros(200000, np.int64)])
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    n = deg.size
    col = rng.integers(0, n, rowptr[-1]).astype(np.int32)
    nbr_check(rowptr, col, n)


def test_hub_rows_with_several_bitmap_passes():
    # one ID per line and 2^22 columns: a hub row spanning all of them takes
    # four passes of the 2^20-line bitmap; a second hub covers a narrow span
    rng = np.random.default_rng(98)
    n = 1 << 22
    hub1 = rng.integers(0, n, 1 << 20)
    hub1[:2] = (0, n - 1)
    hub2 = rng.integers(5000, 7000, 100000)
    small = rng.integers(0, n, 3000)
    col = np.concatenate([small[:1000], hub1, small[1000:2000], hub2, small[2000:]]).astype(np.int32)
    deg = [1000, hub1.size, 1000, hub2.size, 1000]
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    nbr_check(rowptr, col, n, line_ids=1)
    nbr_check(rowptr, col, n, line_ids=32)


def test_degenerate_inputs():
    nbr_check(np.zeros(6, np.int32), np.zeros(0, np.int32), 5)           # no entries
    nbr_check(np.zeros(1, np.int32), np.zeros(0, np.int32), 0)           # no rows
    nbr_check(np.array([0, 1], np.int32), np.array([0], np.int32), 1)    # one entry
    # a star: the hub's leaves fill consecutive lines, every leaf row one entry
    n = 10000
    s = np.concatenate([np.zeros(n - 1), np.arange(1, n)]).astype(np.int32)
    d = np.concatenate([np.arange(1, n), np.zeros(n - 1)]).astype(np.int32)
    over_n, over_ne = nbr_check(*csr_of(s, d, n), n)
    hub = ((n - 1) // 32 + 1) / (n - 1)  # IDs 1..9999 lie in lines 0..312
    assert abs(over_ne - (hub + n - 1) / n) < 1e-12


def test_out_of_range_columns_set_the_device_flag():
    assert boba.boba_check_device_error() == boba.BOBA_OK
    rowptr = dev(np.array([0, 2, 300], np.int32))
    col = dev(np.concatenate([[1, 7], np.arange(298) % 5]).astype(np.int32))  # 7 >= n_cols = 5
    boba.boba_nbr(rowptr, col, 5)
    assert boba.boba_check_device_error() == boba.BOBA_ERR_RANGE
    col = dev(np.concatenate([[1, 2], np.arange(298) % 5]).astype(np.int32))
    col[100] = 9  # inside the listed (longer than 256 entries) row
    boba.boba_nbr(rowptr, col, 5)
    assert boba.boba_check_device_error() == boba.BOBA_ERR_RANGE


def test_malformed_row_pointers_stay_in_bounds():
    # rowptr decreasing, negative and past nnz: offsets are clamped, so the
    # counts are unspecified but every access stays in bounds; a valid call
    # afterwards is exact again
    rng = np.random.default_rng(102)
    col = rng.integers(0, 50, 10).astype(np.int32)
    rowptr = np.array([0, 5, 3, 100000, 2, -7, 10], np.int32)
    over_n, over_ne = boba.boba_nbr(dev(rowptr), dev(col), 50)
    assert np.isfinite(over_n) and np.isfinite(over_ne)
    nnz = 5000
    col = rng.integers(0, 3000, nnz).astype(np.int32)
    rowptr = rng.integers(-5, nnz + 600, 20001).astype(np.int32)
    rowptr[::7] = np.sort(rowptr[::7])  # stretches that look well formed, long rows among them
    boba.boba_nbr(dev(rowptr), dev(col), 3000)
    assert boba.boba_check_device_error() == boba.BOBA_OK
    g = graphgen.small_workload("rmat", 1 << 14, 1 << 17, 103)
    nbr_check(*csr_of(g.src, g.dst, g.n), g.n)


def test_repeatable_bits():
    g = graphgen.small_workload("rmat", 1 << 16, 1 << 20, 99)
    rp, col = csr_of(g.src, g.dst, g.n)
    rp_d, col_d = dev(rp), dev(col)
    first = boba.boba_nbr(rp_d, col_d, g.n)
    for _ in range(3):
        assert boba.boba_nbr(rp_d, col_d, g.n) == first
