"""Batched persistent reorder (+relabel) against the oracle, graph by graph,
over replays of the captured hipGraph and over tuning choices."""
import numpy as np
import pytest
import torch

import oracle
from paper_2306_10410_amd import boba, graphgen
from gpu_util import dev, host, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def mixed_batch(seed=5):
    specs = graphgen.batch_specs(24, seed=seed, log2_lo=4.0, log2_hi=17.2)
    graphs = [graphgen.make_batch_graph(s) for s in specs]
    ns = [s.n for s in specs]
    # degenerate members: no edges, one vertex with self-loops, isolated tail
    graphs += [(np.zeros(0, np.int32), np.zeros(0, np.int32)), (np.zeros(5, np.int32), np.zeros(5, np.int32)),
               (np.array([3, 3], np.int32), np.array([1, 0], np.int32))]
    ns += [17, 1, 40000]
    m = np.array([g[0].size for g in graphs], np.int64)
    eo = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    vo = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    return eo, vo, np.concatenate([g[0] for g in graphs]), np.concatenate([g[1] for g in graphs])


def check_against_oracle(eo, vo, src, dst, perm, order, so, do):
    for g in range(len(eo) - 1):
        a, b = eo[g], eo[g + 1]
        n = int(vo[g + 1] - vo[g])
        p_ref, o_ref = oracle.boba(src[a:b], dst[a:b], n)
        assert np.array_equal(perm[vo[g]:vo[g + 1]], p_ref), f"perm of graph {g} (n={n}, m={b - a})"
        if order is not None:
            assert np.array_equal(order[vo[g]:vo[g + 1]], o_ref), f"order of graph {g}"
        if so is not None:
            s_ref, d_ref = oracle.relabel(src[a:b], dst[a:b], p_ref)
            assert np.array_equal(so[a:b], s_ref) and np.array_equal(do[a:b], d_ref), f"relabel of graph {g}"


@pytest.fixture(scope="module")
def batch():
    return mixed_batch()


def test_batched_equals_per_graph_over_replays(batch):
    eo, vo, src, dst = batch
    s, d = dev(src), dev(dst)
    plan = boba.BatchPlan(eo, vo, s, d)
    info = plan.info()
    assert info["whole_graph_items"] > 0 and info["items"] > info["whole_graph_items"]  # both paths used
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                             host(plan.dst_out))
        # eager work between replays: clobber the outputs
        plan.perm.fill_(-7)
        plan.src_out.fill_(-7)
        plan.order.zero_()
        torch.cuda.synchronize()
    assert boba.boba_check_device_error() == boba.BOBA_OK
    plan.destroy()


@pytest.mark.parametrize("tuning", [(1024, 4096, 1024, 8192), (32768, 1 << 20, 1 << 20, 1 << 20), (1, 1000, 777, 5000)])
def test_tuning_never_changes_results(batch, tuning):
    eo, vo, src, dst = batch
    tu = boba.boba_tuning(*tuning)
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst), tuning=tu)
    plan.launch()
    check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                         host(plan.dst_out))
    assert boba.boba_check_device_error() == boba.BOBA_OK
    plan.destroy()


def test_reorder_only_plan(batch):
    eo, vo, src, dst = batch
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst), relabel=False, with_order=False)
    plan.launch()
    check_against_oracle(eo, vo, src, dst, host(plan.perm), None, None, None)
    plan.destroy()


def test_batched_matches_single_graph_entry_point(batch):
    eo, vo, src, dst = batch
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst))
    plan.launch()
    perm_b = host(plan.perm)
    for g in [0, 3, 7, len(eo) - 2]:
        a, b = eo[g], eo[g + 1]
        n = int(vo[g + 1] - vo[g])
        p, _ = boba.boba_reorder(dev(src[a:b]), dev(dst[a:b]), n)
        assert np.array_equal(host(p), perm_b[vo[g]:vo[g + 1]])
    plan.destroy()


def test_every_item_in_one_queue_is_run_by_all_xcds(batch):
    # queues=1 puts every item in the first queue: the workgroups of the
    # other XCDs run them by helping, so a graph's stages hand data from one
    # XCD to another (the coherence the cross-workgroup handoff relies on)
    eo, vo, src, dst = batch
    for rep in range(2):
        plan = boba.BatchPlan(eo, vo, dev(src), dev(dst), tuning=boba.boba_tuning(0, 65536, 16384, 65536, 1, 0))
        plan.launch()
        check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                             host(plan.dst_out))
        assert boba.boba_check_device_error() == boba.BOBA_OK
        plan.destroy()


def test_atomic_scatter_path(batch):
    # large graphs through device-wide atomic minima (the path of graphs with
    # more than 2^26 vertices) instead of SPLIT + FOLD
    eo, vo, src, dst = batch
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst), tuning=boba.boba_tuning(0, 0, 0, 0, 0, 0, 1))
    for rep in range(2):
        plan.launch()
        check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                             host(plan.dst_out))
    assert boba.boba_check_device_error() == boba.BOBA_OK
    plan.destroy()


@pytest.mark.parametrize("scatter_tile", [0, 4096])
def test_many_buckets_and_slices(scatter_tile):
    # SPLIT / FOLD at the bucket limit (2^26 vertices: 2048 buckets of 2^15),
    # a 129-bucket graph, a graph whose edges all hit one bucket, and small
    # members; scatter_tile 4096 gives the two smaller large graphs four slices
    rng = np.random.default_rng(41)
    graphs, ns = [], []
    n = 1 << 26
    graphs.append((rng.integers(0, n, 1 << 20, dtype=np.int32), rng.integers(0, n, 1 << 20, dtype=np.int32)))
    ns.append(n)
    n = (1 << 22) + 5
    g = graphgen.small_workload("rmat", n, 3000001, 42)
    graphs.append((g.src, g.dst))
    ns.append(n)
    n = 200003
    graphs.append((rng.integers(65536, 98304, 500001, dtype=np.int32), rng.integers(65536, 98304, 500001, dtype=np.int32)))
    ns.append(n)
    graphs.append((np.array([2, 0, 1], np.int32), np.array([1, 1, 0], np.int32)))
    ns.append(3)
    m = np.array([a.size for a, _ in graphs], np.int64)
    eo = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    vo = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    src = np.concatenate([a for a, _ in graphs])
    dst = np.concatenate([b for _, b in graphs])
    print(f"batch: n={int(vo[-1])} m={int(eo[-1])} scatter_tile={scatter_tile}", flush=True)
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst), tuning=boba.boba_tuning(0, scatter_tile, 0, 0))
    plan.launch()
    check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                         host(plan.dst_out))
    assert boba.boba_check_device_error() == boba.BOBA_OK
    plan.destroy()


def test_split_bucket_count_boundaries():
    # SPLIT's packed-count path takes graphs of at most 8 buckets: 1 bucket
    # (a graph above small_max_n = 1000 but below 2^15 vertices), 8 (2^18
    # vertices) and 9 (2^18 + 1), next to the per-element path
    rng = np.random.default_rng(43)
    ns = [2000, 1 << 18, (1 << 18) + 1, 5000]
    ms = [30001, 1000003, 999999, 77]
    graphs = [(rng.integers(0, n, m, dtype=np.int32), rng.integers(0, n, m, dtype=np.int32)) for n, m in zip(ns, ms)]
    m = np.array(ms, np.int64)
    eo = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    vo = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    src = np.concatenate([a for a, _ in graphs])
    dst = np.concatenate([b for _, b in graphs])
    for atomic in (0, 1):
        plan = boba.BatchPlan(eo, vo, dev(src), dev(dst), tuning=boba.boba_tuning(1000, 0, 0, 0, 0, 0, atomic))
        plan.launch()
        check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                             host(plan.dst_out))
        assert boba.boba_check_device_error() == boba.BOBA_OK
        plan.destroy()


def test_a_wait_that_gives_up_is_reported_as_a_timeout():
    # a spin limit of one sleep: waits for other workgroups' stages give up
    # almost at once (every kernel still runs to its end); the launch then
    # reports BOBA_ERR_TIMEOUT, or, if no wait had to give up, exact results
    rng = np.random.default_rng(31)
    n, m = 1 << 18, 1 << 21
    src = rng.integers(0, n, m, dtype=np.int32)
    dst = rng.integers(0, n, m, dtype=np.int32)
    eo = np.array([0, m], np.int64)
    vo = np.array([0, n], np.int64)
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst), tuning=boba.boba_tuning(0, 4096, 4096, 4096, 0, 1))
    plan.launch()
    torch.cuda.synchronize()
    code = boba.boba_check_device_error()
    assert code in (boba.BOBA_ERR_TIMEOUT, boba.BOBA_OK)
    if code == boba.BOBA_OK:
        check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                             host(plan.dst_out))
    plan.destroy()
    # the flag was cleared: a default plan afterwards is exact and reports OK
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst))
    plan.launch()
    check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out), host(plan.dst_out))
    assert boba.boba_check_device_error() == boba.BOBA_OK
    plan.destroy()


@pytest.mark.timeout(900)
def test_full_batch_config_against_the_oracle():
    # the benchmark's batch: 512 graphs, n = 2^U(10,18), edge factor U{4..32},
    # half RMAT half geometric (about 493M edges), default tuning, two replays;
    # every graph checked against the oracle (generated with threads: this
    # process already uses the GPU)
    from concurrent.futures import ThreadPoolExecutor
    specs = graphgen.batch_specs(512)
    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(graphgen.make_batch_graph, specs))
    m = np.array([p[0].size for p in parts], np.int64)
    eo = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    vo = np.concatenate([[0], np.cumsum([s.n for s in specs])]).astype(np.int64)
    src = np.concatenate([p[0] for p in parts])
    dst = np.concatenate([p[1] for p in parts])
    del parts
    print(f"batch: {len(specs)} graphs, m={int(eo[-1])} n={int(vo[-1])}", flush=True)
    plan = boba.BatchPlan(eo, vo, dev(src), dev(dst))
    plan.launch()
    plan.launch()
    check_against_oracle(eo, vo, src, dst, host(plan.perm), host(plan.order), host(plan.src_out),
                         host(plan.dst_out))
    assert boba.boba_check_device_error() == boba.BOBA_OK
    plan.destroy()
