"""Pins for the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle (oracle/boba_oracle.c) against something other
than its own formula: values printed in the paper's worked examples, closed
forms, invariants that characterise the BOBA labelling uniquely, brute force
over every edge order of tiny graphs, library routines (stable argsort,
scipy.sparse) and finite differences.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2306_10410_amd import graphgen


# ----------------------------------------------------------------- helpers
def encode(tokens, code):
    return np.array([code[t] for t in tokens], np.int32)


def brute_force_boba(I, J, n, interleaved=False):
    """F2: first(v) by linear search over the flattened sequence (plus the
    tail 0..n-1), new ID = number of vertices with a smaller first position."""
    m = len(I)
    if interleaved:
        S = [x for k in range(m) for x in (int(I[k]), int(J[k]))]
    else:
        S = [int(x) for x in I] + [int(x) for x in J]
    S += list(range(n))
    first = []
    for v in range(n):
        for i, s in enumerate(S):
            if s == v:
                first.append(i)
                break
    return np.array([sum(1 for u in range(n) if first[u] < first[v]) for v in range(n)], np.int32)


def parallel_formulation(I, J, n):
    """F3: Algorithm 2 with AtomicMin (np.minimum.at) over I++J, then a
    stable ParMapKeys of p = (0..n-1) by the keys r (stable argsort)."""
    m = len(I)
    S = np.concatenate([np.asarray(I, np.int64), np.asarray(J, np.int64)])
    r = np.full(n, np.iinfo(np.int64).max, np.int64)
    np.minimum.at(r, S, np.arange(2 * m, dtype=np.int64))
    order = np.argsort(r, kind="stable")
    perm = np.empty(n, np.int64)
    perm[order] = np.arange(n)
    return perm.astype(np.int32), order.astype(np.int32)


def restricted_growth_ok(I, J, perm):
    """T = perm o S over I++J must satisfy T[0] = 0 and T[i] <= 1 + max(T[<i]);
    together with perm being a bijection this characterises BOBA uniquely
    (on the vertices that occur; the tail is checked separately)."""
    T = perm[np.concatenate([I, J]).astype(np.int64)].astype(np.int64)
    if T.size == 0:
        return True
    run = np.maximum.accumulate(T)
    prev = np.concatenate([[-1], run[:-1]])
    return bool(T[0] == 0 and np.all(T <= prev + 1))


# ------------------------------------------------------- P1/P2 worked examples
@pytest.mark.parametrize("seed", [None, 0, 1, 2, 3])
@pytest.mark.parametrize("interleaved", [False, True])
def test_fig2_roads_printed_order(golden, seed, interleaved):
    g = golden("fig2_roads.txt")
    names = sorted(set(g["I"]) | set(g["J"]))
    assert len(names) == 13
    ids = np.arange(13) if seed is None else np.random.default_rng(seed).permutation(13)
    code = {name: int(ids[k]) for k, name in enumerate(names)}
    I, J = encode(g["I"], code), encode(g["J"], code)
    perm, order = oracle.boba(I, J, 13, interleaved=interleaved)
    assert [names[list(ids).index(v)] for v in order] == g["order"]
    assert np.array_equal(perm[order], np.arange(13))


def test_fig1_star_interleaved_printed_row(golden):
    g = golden("fig1_star.txt")
    names = sorted(set(g["I"]) | set(g["J"]), key=lambda s: (len(s), s))
    code = {nm: k for k, nm in enumerate(names)}
    I, J = encode(g["I"], code), encode(g["J"], code)
    _, order = oracle.boba(I, J, len(names), interleaved=True)
    assert [names[v] for v in order] == g["order_interleaved"]


def test_fig1_star_concatenated_follows_algorithm1(golden):
    # With I++J (Algorithm 1), every source comes first: 1 2 3 4 b 5 .. 10, then a.
    g = golden("fig1_star.txt")
    names = sorted(set(g["I"]) | set(g["J"]), key=lambda s: (len(s), s))
    code = {nm: k for k, nm in enumerate(names)}
    I, J = encode(g["I"], code), encode(g["J"], code)
    _, order = oracle.boba(I, J, len(names))
    assert [names[v] for v in order] == g["I"][:11] + ["a"]


# ------------------------------------------------------------ P3 closed forms
def test_empty_edge_list_gives_identity():
    for n in (0, 1, 7):
        perm, order = oracle.boba(np.zeros(0, np.int32), np.zeros(0, np.int32), n)
        assert np.array_equal(perm, np.arange(n)) and np.array_equal(order, np.arange(n))


def test_sorted_sources_covering_all_vertices_give_identity():
    rng = np.random.default_rng(5)
    n = 500
    I = np.sort(np.concatenate([np.arange(n), rng.integers(0, n, 1500)])).astype(np.int32)
    J = rng.integers(0, n, I.size).astype(np.int32)
    perm, _ = oracle.boba(I, J, n)
    assert np.array_equal(perm, np.arange(n))


def test_sources_forming_a_permutation():
    rng = np.random.default_rng(6)
    n = 1000
    I = rng.permutation(n).astype(np.int32)
    J = rng.integers(0, n, n).astype(np.int32)
    perm, _ = oracle.boba(I, J, n)
    assert np.array_equal(perm[I], np.arange(n))


def test_star_center_first_then_leaves_in_destination_order():
    rng = np.random.default_rng(7)
    n = 50
    c = 17
    leaves = rng.permutation([v for v in range(n) if v != c]).astype(np.int32)
    I = np.full(leaves.size, c, np.int32)
    perm, order = oracle.boba(I, leaves, n)
    assert perm[c] == 0
    assert np.array_equal(order[1:], leaves)


def test_isolated_vertices_follow_in_increasing_old_id():
    I = np.array([9, 3, 9], np.int32)
    J = np.array([3, 5, 5], np.int32)
    perm, order = oracle.boba(I, J, 12)
    assert list(order[:3]) == [9, 3, 5]
    assert list(order[3:]) == [0, 1, 2, 4, 6, 7, 8, 10, 11]


def test_self_loops_and_duplicates_are_ordinary_occurrences():
    I = np.array([4, 4, 2, 2], np.int32)
    J = np.array([4, 4, 0, 4], np.int32)
    _, order = oracle.boba(I, J, 5)
    assert list(order) == [4, 2, 0, 1, 3]


def test_out_of_range_vertex_is_an_error():
    with pytest.raises(oracle.OracleError):
        oracle.boba(np.array([0, 5], np.int32), np.array([1, 1], np.int32), 5)
    with pytest.raises(oracle.OracleError):
        oracle.boba(np.array([0, -1], np.int32), np.array([1, 1], np.int32), 5)


# ------------------------------------------------------------ P3 invariants
def _random_graphs():
    yield graphgen.small_workload("uniform", 300, 900, 11)
    yield graphgen.small_workload("rmat", 1024, 8192, 12)
    yield graphgen.small_workload("rgg", 800, 4000, 13)
    yield graphgen.small_workload("grid", 900, 0, 14)


@pytest.mark.parametrize("g", list(_random_graphs()), ids=lambda g: g.name)
def test_invariants_characterise_the_labelling(g):
    perm, order = oracle.boba(g.src, g.dst, g.n)
    # bijection
    assert np.array_equal(np.sort(perm), np.arange(g.n))
    assert np.array_equal(order[perm], np.arange(g.n))
    # restricted growth over I++J
    assert restricted_growth_ok(g.src, g.dst, perm)
    # tail: vertices that never occur come last, in increasing old ID
    occurs = np.zeros(g.n, bool)
    occurs[g.src] = True
    occurs[g.dst] = True
    k = int(occurs.sum())
    assert np.array_equal(order[k:], np.nonzero(~occurs)[0])
    # isomorphism: relabelled edges map back through order
    s2, d2 = oracle.relabel(g.src, g.dst, perm)
    assert np.array_equal(order[s2], g.src) and np.array_equal(order[d2], g.dst)
    # idempotence: BOBA of the BOBA-relabelled graph is the identity
    perm2, _ = oracle.boba(s2, d2, g.n)
    assert np.array_equal(perm2, np.arange(g.n))
    # Algorithm 2 with AtomicMin + stable ParMapKeys agrees
    p3, o3 = parallel_formulation(g.src, g.dst, g.n)
    assert np.array_equal(perm, p3) and np.array_equal(order, o3)


def test_label_invariance():
    g = graphgen.small_workload("rmat", 2048, 16384, 21)
    occurs = np.zeros(g.n, bool)
    occurs[g.src] = True
    occurs[g.dst] = True
    keep = np.nonzero(occurs)[0]
    remap = np.full(g.n, -1, np.int64)
    remap[keep] = np.arange(keep.size)
    src, dst, n = remap[g.src].astype(np.int32), remap[g.dst].astype(np.int32), keep.size
    perm, _ = oracle.boba(src, dst, n)
    base = oracle.relabel(src, dst, perm)
    for seed in range(3):
        sigma = np.random.default_rng(100 + seed).permutation(n).astype(np.int32)
        s, d = sigma[src], sigma[dst]
        p, _ = oracle.boba(s, d, n)
        again = oracle.relabel(s, d, p)
        assert np.array_equal(again[0], base[0]) and np.array_equal(again[1], base[1])


def test_grid_closed_form_restores_row_major_ids():
    side = 48
    src, dst = graphgen.grid(side, side)
    sigma = graphgen.random_labels(side * side, 31)
    s, d = graphgen.apply_labels(src, dst, sigma)
    perm, _ = oracle.boba(s, d, side * side)
    assert np.array_equal(perm[sigma], np.arange(side * side))


# ------------------------------------------------------------- P4 brute force
def test_brute_force_every_edge_order_tiny_multigraphs():
    rng = np.random.default_rng(41)
    checked = 0
    for trial in range(6):
        n = int(rng.integers(1, 6))
        m = int(rng.integers(1, 7))
        I0 = rng.integers(0, n, m)
        J0 = rng.integers(0, n, m)
        if trial == 0:
            J0[:] = I0  # only self-loops
        for p in itertools.permutations(range(m)):
            I = I0[list(p)].astype(np.int32)
            J = J0[list(p)].astype(np.int32)
            for inter in (False, True):
                perm, order = oracle.boba(I, J, n, interleaved=inter)
                assert np.array_equal(perm, brute_force_boba(I, J, n, inter))
                assert np.array_equal(order[perm], np.arange(n))
            checked += 1
    assert checked > 100


# ----------------------------------------------------------- relabel / CSR
def test_relabel_matches_fancy_indexing():
    g = graphgen.small_workload("uniform", 1000, 5000, 51)
    perm = np.random.default_rng(52).permutation(g.n).astype(np.int32)
    s2, d2 = oracle.relabel(g.src, g.dst, perm)
    assert np.array_equal(s2, perm[g.src]) and np.array_equal(d2, perm[g.dst])


@pytest.mark.parametrize("kind", ["uniform", "rmat", "grid"])
def test_csr_matches_stable_argsort(kind):
    g = graphgen.small_workload(kind, 1024, 6000, 61)
    rowptr, col, val = oracle.coo_to_csr(g.src, g.dst, g.val, g.n)
    o = np.argsort(g.src, kind="stable")
    assert np.array_equal(col, g.dst[o])
    assert np.array_equal(val.view(np.uint32), g.val[o].view(np.uint32))
    assert rowptr[0] == 0 and rowptr[-1] == g.m and np.all(np.diff(rowptr) >= 0)
    assert np.array_equal(np.diff(rowptr), np.bincount(g.src, minlength=g.n))


def test_csr_empty_and_no_values():
    rowptr, col, val = oracle.coo_to_csr(np.zeros(0, np.int32), np.zeros(0, np.int32), None, 4)
    assert list(rowptr) == [0] * 5 and col.size == 0 and val is None


# ------------------------------------------------------------------- SpMV
def test_spmv_matches_scipy_fp64():
    g = graphgen.small_workload("rmat", 2048, 20000, 71)
    rowptr, col, val = oracle.coo_to_csr(g.src, g.dst, g.val, g.n)
    y = oracle.spmv64(rowptr, col, val, g.x)
    A = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(g.n, g.n))
    ref = A @ g.x.astype(np.float64)
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_spmv_identity_and_degree():
    n = 300
    x = graphgen.uniform_values(n, 72)
    rp = np.arange(n + 1, dtype=np.int32)
    y = oracle.spmv64(rp, np.arange(n, dtype=np.int32), np.ones(n, np.float32), x)
    assert np.array_equal(y, x.astype(np.float64))
    g = graphgen.small_workload("uniform", n, 3000, 73)
    rowptr, col, _ = oracle.coo_to_csr(g.src, g.dst, None, n)
    y = oracle.spmv64(rowptr, col, None, np.ones(n, np.float32))
    assert np.array_equal(y, np.bincount(g.src, minlength=n).astype(np.float64))


# -------------------------------------------------------------------- MLP
def _mlp_params(seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.3, oracle.MLP_NPARAM)


def _split(P):
    k = 0
    out = []
    for shape in ((64, 16), (64,), (64, 64), (64,), (1, 64), (1,)):
        size = int(np.prod(shape))
        out.append(P[k:k + size].reshape(shape))
        k += size
    assert k == P.size
    return out


def test_mlp_forward_matches_matrix_form():
    P = _mlp_params(1)
    X = np.random.default_rng(2).normal(size=(33, 16))
    W1, b1, W2, b2, W3, b3 = _split(P)
    h1 = np.maximum(X @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    ref = (h2 @ W3.T + b3)[:, 0]
    assert np.allclose(oracle.mlp_forward(P, X), ref, rtol=1e-12, atol=1e-12)


def test_mlp_backward_matches_central_differences():
    P = _mlp_params(3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(9, 16))
    y = rng.normal(size=9)
    g, loss = oracle.mlp_backward(P, X, y)
    assert math.isclose(loss, float(np.mean((oracle.mlp_forward(P, X) - y) ** 2)), rel_tol=1e-12)
    h = 1e-6
    idx = np.concatenate([np.arange(0, oracle.MLP_NPARAM, 37), [oracle.MLP_NPARAM - 1]])
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (oracle.mlp_backward(Pp, X, y)[1] - oracle.mlp_backward(Pm, X, y)[1]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-7, (k, fd, g[k])


def test_adam_first_step_is_signed_learning_rate():
    P = np.zeros(5)
    m1, m2 = np.zeros(5), np.zeros(5)
    grad = np.array([0.5, -2.0, 1e-3, -7.0, 3.0])
    oracle.adam(P, m1, m2, grad, 1, lr=0.01, eps=0.0)
    assert np.allclose(P, -0.01 * np.sign(grad), rtol=1e-12)


@pytest.mark.parametrize("b1,b2", [(0.9, 0.999), (0.5, 0.75)])
def test_adam_constant_gradient_moves_by_the_learning_rate_every_step(b1, b2):
    # With the same gradient g at every step, m1_t = (1 - b1^t) g and
    # m2_t = (1 - b2^t) g^2, so the bias-corrected moments are exactly g and
    # g^2 at every t and each step moves a parameter by -lr * sign(g).  A
    # wrong exponent in the bias correction breaks this from t = 2 on.
    grad = np.array([0.5, -2.0, 1e-3, -7.0, 3.0])
    P = np.zeros(5)
    m1, m2 = np.zeros(5), np.zeros(5)
    for t in (1, 2, 3, 4):
        oracle.adam(P, m1, m2, grad, t, lr=0.01, b1=b1, b2=b2, eps=0.0)
        assert np.allclose(P, -0.01 * t * np.sign(grad), rtol=1e-12, atol=0.0), t
        assert np.allclose(m1, (1 - b1 ** t) * grad, rtol=1e-12)
        assert np.allclose(m2, (1 - b2 ** t) * grad * grad, rtol=1e-12)


def test_adam_second_step_after_a_zero_gradient():
    # g_1 = 0, g_2 = g: m1 = (1 - b1) g and m2 = (1 - b2) g^2, corrected by
    # 1 - b1^2 and 1 - b2^2, so the second step is
    # -lr * sign(g) * sqrt(1 + b2) / (1 + b1) (and the first step is zero).
    b1, b2, lr = 0.9, 0.999, 0.01
    grad = np.array([0.5, -2.0, 4.0])
    P = np.zeros(3)
    m1, m2 = np.zeros(3), np.zeros(3)
    oracle.adam(P, m1, m2, np.zeros(3), 1, lr=lr, b1=b1, b2=b2, eps=1e-300)
    assert np.all(P == 0.0)
    oracle.adam(P, m1, m2, grad, 2, lr=lr, b1=b1, b2=b2, eps=0.0)
    expect = -lr * np.sign(grad) * math.sqrt(1 + b2) / (1 + b1)
    assert np.allclose(P, expect, rtol=1e-12, atol=0.0)


# -------------------------------------------------------------------- NBR
def test_nbr_closed_forms():
    # vertex 0: 4 neighbours in one 32-ID line -> 1/4; vertex 1: 3 in 3 lines -> 1
    rowptr = np.array([0, 4, 7, 7], np.int32)
    col = np.array([0, 1, 2, 31, 0, 32, 64], np.int32)
    over_n, over_nonempty = oracle.nbr(rowptr, col, 3)
    assert math.isclose(over_nonempty, (0.25 + 1.0) / 2)
    assert math.isclose(over_n, (0.25 + 1.0) / 3)
    *_, per_row = oracle.nbr(rowptr, col, 3, per_row=True)
    assert list(per_row) == [1, 3, 0]


def test_nbr_line_width_extremes():
    # one ID per line: distinct neighbours / degree (duplicates lower it);
    # a line wider than every ID: one line per row, so the ratio is 1/degree
    rowptr = np.array([0, 3, 3, 8, 9], np.int32)
    col = np.array([5, 5, 5, 0, 1, 2, 1, 0, 7], np.int32)
    over_n, over_nonempty, per_row = oracle.nbr(rowptr, col, 4, line_ids=1, per_row=True)
    assert list(per_row) == [1, 0, 3, 1]
    assert math.isclose(over_nonempty, (1 / 3 + 3 / 5 + 1) / 3) and math.isclose(over_n, (1 / 3 + 3 / 5 + 1) / 4)
    _, over_nonempty, per_row = oracle.nbr(rowptr, col, 4, line_ids=1 << 20, per_row=True)
    assert list(per_row) == [1, 0, 1, 1]
    assert math.isclose(over_nonempty, (1 / 3 + 1 / 5 + 1) / 3)


def test_nbr_ignores_order_inside_rows():
    rng = np.random.default_rng(33)
    n = 3000
    deg = rng.integers(0, 40, n)
    rowptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    col = rng.integers(0, n, rowptr[-1]).astype(np.int32)
    ref = oracle.nbr(rowptr, col, n, per_row=True)
    shuffled = col.copy()
    for v in range(n):
        rng.shuffle(shuffled[rowptr[v]:rowptr[v + 1]])
    got = oracle.nbr(rowptr, shuffled, n, per_row=True)
    assert got[0] == ref[0] and np.array_equal(got[2], ref[2])


def test_nbr_grid_counted_geometrically():
    # W x H mesh in natural order with W a multiple of 32: ID r*W + c lies in
    # line (r, c // 32), so up and down neighbours are lines of their own and
    # left and right share a line unless c sits at a line edge (c % 32 in {0, 31})
    W, H = 96, 7
    s, d = graphgen.grid(H, W)
    rowptr, col, _ = oracle.coo_to_csr(s, d, None, W * H)
    total, lines = 0.0, []
    for r in range(H):
        for c in range(W):
            nb = [(r + dr, c + dc) for dr, dc in ((-1, 0), (0, -1), (0, 1), (1, 0))
                  if 0 <= r + dr < H and 0 <= c + dc < W]
            k = len({(rr, cc // 32) for rr, cc in nb})
            lines.append(k)
            total += k / len(nb)
    over_n, over_nonempty, per_row = oracle.nbr(rowptr, col, W * H, per_row=True)
    assert list(per_row) == lines
    assert math.isclose(over_n, total / (W * H), rel_tol=1e-12) and over_n == over_nonempty


def test_bin_by_dst_pins():
    rng = np.random.default_rng(31)
    for n, m in [(1, 5), (2, 9), (37, 200), (1000, 5000), (1 << 12, 1 << 14)]:
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        bits = int(np.ceil(np.log2(n))) if n > 1 else 0
        for bb in (1, 3, 8, 16, 31):
            so, do = oracle.bin_by_dst(src, dst, n, bb)
            shift = max(0, bits - bb)
            order = np.argsort(dst >> shift, kind="stable")  # a library routine, not the oracle's counting sort
            assert np.array_equal(so, src[order]) and np.array_equal(do, dst[order]), (n, m, bb)
            assert np.all(np.diff(do >> shift) >= 0)
        # enough bins: a full stable sort by destination
        so, do = oracle.bin_by_dst(src, dst, n, 31)
        assert np.array_equal(do, np.sort(dst)) and sorted(zip(so, do)) == sorted(zip(src, dst))
    # one bit, worked by hand: n = 4 (2-bit IDs), bins {0,1} | {2,3}, input order kept inside
    src = np.array([10, 11, 12, 13, 14], np.int32)
    dst = np.array([3, 0, 2, 1, 0], np.int32)
    so, do = oracle.bin_by_dst(src, dst, 4, 1)
    assert list(do) == [0, 1, 0, 3, 2] and list(so) == [11, 13, 14, 10, 12]
    with pytest.raises(Exception):
        oracle.bin_by_dst(src, np.array([0, 1, 2, 3, 4], np.int32), 4, 2)  # out of range


# -------------------------------------------------------------- PageRank
def test_pagerank_directed_cycle_stays_uniform():
    n = 7
    src = np.arange(n, dtype=np.int32)
    dst = np.roll(src, -1)
    r, changes = oracle.pagerank(src, dst, n, 0.85, 5)
    assert np.allclose(r, 1 / n, rtol=0, atol=1e-15) and max(changes) < 1e-15


def test_pagerank_star_closed_form():
    # undirected star, k leaves: at the fixed point r_c = (1 + a k) / (n (1 + a))
    # and r_leaf = (1 - a)/n + a r_c / k
    k, a = 9, 0.85
    n = k + 1
    leaves = np.arange(1, n, dtype=np.int32)
    src = np.concatenate([np.zeros(k, np.int32), leaves])
    dst = np.concatenate([leaves, np.zeros(k, np.int32)])
    r, changes = oracle.pagerank(src, dst, n, a, 500, tol=1e-13)
    rc = (1 + a * k) / (n * (1 + a))
    assert math.isclose(r[0], rc, rel_tol=1e-12)
    assert np.allclose(r[1:], (1 - a) / n + a * rc / k, rtol=1e-12, atol=0)
    assert changes[-1] < 1e-13 and all(c >= 1e-13 for c in changes[:-1])  # stopped at the first one below


def test_pagerank_is_the_google_matrix_eigenvector():
    # directed multigraph with dangling vertices: the fixed point is the
    # eigenvector of eigenvalue 1 of G = a (P + dangling spread) + (1 - a)/n
    rng = np.random.default_rng(34)
    n, m, a = 12, 30, 0.8
    src = rng.integers(0, 8, m).astype(np.int32)   # vertices 8..11 have no out-edges
    dst = rng.integers(0, n, m).astype(np.int32)
    G = np.full((n, n), (1 - a) / n)
    outdeg = np.bincount(src, minlength=n)
    for u, v in zip(src, dst):
        G[v, u] += a / outdeg[u]
    for u in range(n):
        if outdeg[u] == 0:
            G[:, u] += a / n
    w, V = np.linalg.eig(G)
    vec = np.real(V[:, np.argmin(np.abs(w - 1))])
    vec /= vec.sum()
    r, _ = oracle.pagerank(src, dst, n, a, 400)
    assert np.allclose(r, vec, rtol=1e-10, atol=1e-13)
    assert math.isclose(r.sum(), 1.0, rel_tol=1e-12)


def test_pagerank_without_damping_or_edges():
    rng = np.random.default_rng(35)
    src = rng.integers(0, 50, 200).astype(np.int32)
    dst = rng.integers(0, 50, 200).astype(np.int32)
    r, _ = oracle.pagerank(src, dst, 50, 0.0, 3)          # damping 0: uniform
    assert np.allclose(r, 1 / 50, rtol=1e-14, atol=0)
    r, _ = oracle.pagerank(np.zeros(0, np.int32), np.zeros(0, np.int32), 5, 0.85, 4)  # all dangling
    assert np.allclose(r, 0.2, rtol=1e-14, atol=0)
