"""boba_reorder_noalloc, the reorder for callers that cannot allocate, against
boba_reorder (the entry point with a caller workspace) through the C ABI:
bit-identical perm and order on consecutive calls that share the library's
static scratch, the second on a smaller graph, and on unaligned inputs
(element-wise loads in the split).  Both are also checked against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2306_10410_amd import boba, graphgen
from gpu_util import dev, host, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def both(g, flags=0, shift=0):
    """perm/order from boba_reorder and from boba_reorder_noalloc on the same
    device arrays; shift > 0 starts src/dst that many int32 into their buffers
    (not 16-byte aligned: the split loads element by element)."""
    s_buf = dev(np.concatenate([np.zeros(shift, np.int32), g.src]))
    d_buf = dev(np.concatenate([np.zeros(shift, np.int32), g.dst]))
    s, d = s_buf[shift:], d_buf[shift:]
    p_ref, o_ref = boba.boba_reorder(s, d, g.n, flags=flags)
    # outputs prefilled with garbage: every entry must be written
    perm = torch.full((g.n,), -7, dtype=torch.int32, device=s.device)
    order = torch.full((g.n,), -7, dtype=torch.int32, device=s.device)
    print(f"noalloc: n={g.n} m={g.m} flags={flags} shift={shift}", flush=True)
    boba.boba_reorder_noalloc(s, d, g.n, perm, order, flags=flags)
    assert boba.boba_check_device_error() == boba.BOBA_OK
    return host(p_ref), host(o_ref), host(perm), host(order)


def check(g, flags=0, shift=0):
    p_ref, o_ref, p, o = both(g, flags, shift)
    assert np.array_equal(p, p_ref), "perm differs from boba_reorder"
    assert np.array_equal(o, o_ref), "order differs from boba_reorder"
    po, oo = oracle.boba(g.src, g.dst, g.n, interleaved=bool(flags & boba.BOBA_FLAG_INTERLEAVED))
    assert np.array_equal(p, po) and np.array_equal(o, oo), "differs from the oracle"


def test_two_calls_in_a_row_second_smaller():
    big = graphgen.small_workload("rmat", 1 << 16, (1 << 20) - 3, 71)
    assert boba.boba_reorder_workspace(big.n, big.m) <= boba.BOBA_REORDER_NOALLOC_MAX_BYTES
    check(big)
    small = graphgen.small_workload("uniform", 5000, 30001, 72)
    check(small)


def test_interleaved_and_unaligned():
    g = graphgen.small_workload("rgg", 20000, 150000, 73)
    check(g, flags=boba.BOBA_FLAG_INTERLEAVED)
    check(g, shift=1)
    h = graphgen.small_workload("uniform", 1 << 14, 1 << 17, 74)
    check(h)


def test_oversized_graph_is_refused_before_any_launch():
    n, m = 1 << 20, 1 << 23
    s = torch.zeros(m, dtype=torch.int32, device="cuda")
    perm = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(boba.BobaError) as e:
        boba.boba_reorder_noalloc(s, s, n, perm)
    assert e.value.status == boba.BOBA_ERR_WORKSPACE
    assert bool((perm == -7).all())
