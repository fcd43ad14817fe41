"""Seeded synthetic graph generators shared by the tests, the benchmark and the
CPU oracle's callers.

This module holds input generation only: random graphs, random label
permutations, random edge orders and random values.  It contains none of the
reordering, relabelling, CSR or SpMV arithmetic, and it imports neither the GPU
library nor the oracle.

The graph families stand in for the paper's datasets (Sec. 5, Table 2), which
are not available offline:

* ``rmat``     Kronecker/RMAT graphs with (a, b, c, d) = (0.57, 0.19, 0.19, 0.05),
               the generator behind the kron_g500-logn20/21 sets.
* ``grid``     a 2-D 4-neighbour mesh, the regular, road/delaunay-like regime of
               Fig. 2 and the uniform-degree discussion of Sec. 1.2.
* ``rgg``      random geometric graphs in the unit square, like rgg_n_2_*.
* ``uniform``  i.i.d. uniform endpoints: the case BOBA cannot help (Sec. 1.2).

All randomness comes from ``numpy.random.Generator(PCG64)`` streams derived from
an integer seed with ``SeedSequence``, so every array is reproducible on any
machine.  Large RMAT graphs are generated in fixed chunks, each with its own
child stream, on a thread pool; the result does not depend on the thread count.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

RMAT_ABC = (0.57, 0.19, 0.19)
_CHUNK = 1 << 22  # edges per RMAT chunk (fixed: part of the stream definition)


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


# --------------------------------------------------------------------------- RMAT
def _rmat_chunk(args):
    child, count, scale, a, b, c = args
    rng = np.random.Generator(np.random.PCG64(child))
    src = np.zeros(count, np.int32)
    dst = np.zeros(count, np.int32)
    fa, fab, fabc = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    for bit in range(scale):
        u = rng.random(count, dtype=np.float32)
        # quadrant a: (0,0)  b: (0,1)  c: (1,0)  d: (1,1)
        row_bit = u >= fab
        col_bit = ((u >= fa) & (u < fab)) | (u >= fabc)
        src |= row_bit.astype(np.int32) << bit
        dst |= col_bit.astype(np.int32) << bit
    return src, dst


def rmat(scale: int, m: int, seed: int, abc=RMAT_ABC, n: int | None = None):
    """``m`` i.i.d. RMAT edges over ``2**scale`` IDs (no noise; self-loops and
    duplicates kept).  With ``n`` < 2**scale, edges with an endpoint >= n are
    redrawn from a continuation of the same stream until all fit."""
    a, b, c = abc
    seq = np.random.SeedSequence(seed)
    nchunks = max(1, -(-m // _CHUNK))
    kids = seq.spawn(nchunks)
    jobs = [(kids[i], min(_CHUNK, m - i * _CHUNK), scale, a, b, c) for i in range(nchunks)]
    if m == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    with ThreadPoolExecutor(_threads()) as ex:
        parts = list(ex.map(_rmat_chunk, jobs))
    src = np.concatenate([p[0] for p in parts])
    dst = np.concatenate([p[1] for p in parts])
    if n is not None and n < (1 << scale):
        extra = seq.spawn(1)[0]
        rounds = 0
        while True:
            bad = np.nonzero((src >= n) | (dst >= n))[0]
            if bad.size == 0:
                break
            child = extra.spawn(1)[0]
            s2, d2 = _rmat_chunk((child, bad.size, scale, a, b, c))
            src[bad] = s2
            dst[bad] = d2
            rounds += 1
            if rounds > 10000:
                raise RuntimeError("rmat redraw did not converge")
    return src, dst


# --------------------------------------------------------------------------- grid
def grid(rows: int, cols: int):
    """4-neighbour mesh, vertex (r, c) has ID r*cols + c.  For each vertex in
    row-major order, emit its edges to up, left, right, down (those inside the
    grid), so sources appear in increasing ID order."""
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    r = ids // cols
    c = ids % cols
    cand = []
    for dr, dc in ((-1, 0), (0, -1), (0, 1), (1, 0)):  # up, left, right, down
        ok = (r + dr >= 0) & (r + dr < rows) & (c + dc >= 0) & (c + dc < cols)
        cand.append(np.where(ok, ids + dr * cols + dc, -1))
    nb = np.stack(cand, axis=-1).reshape(-1, 4)  # [vertex, 4] in emission order
    src = np.repeat(np.arange(rows * cols, dtype=np.int64), 4)
    dst = nb.reshape(-1)
    keep = dst >= 0
    return src[keep].astype(np.int32), dst[keep].astype(np.int32)


# --------------------------------------------------------------------------- RGG
def rgg(n: int, radius: float, seed: int):
    """Random geometric graph: n points U[0,1)^2; every ordered pair (u, v),
    u != v, at distance < radius is an edge.  Points get IDs in cell-major
    order (cells of side >= radius, row-major over cells; by x inside a
    cell) and edges are emitted grouped by source in increasing ID."""
    rng = _rng(seed)
    pts = rng.random((n, 2))
    if n == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    g = max(1, int(math.floor(1.0 / radius)))
    cell = np.minimum((pts * g).astype(np.int64), g - 1)
    cid = cell[:, 1] * g + cell[:, 0]
    order = np.lexsort((pts[:, 0], cid))
    pts = pts[order]
    cid = cid[order]
    cell = cell[order]
    start = np.searchsorted(cid, np.arange(g * g + 1))
    srcs, dsts = [], []
    r2 = radius * radius
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            cx = cell[:, 0] + dx
            cy = cell[:, 1] + dy
            ok = (cx >= 0) & (cx < g) & (cy >= 0) & (cy < g)
            nc = np.where(ok, cy * g + cx, 0)
            lo = np.where(ok, start[nc], 0)
            hi = np.where(ok, start[nc + 1], 0)
            cnt = hi - lo
            tot = int(cnt.sum())
            if tot == 0:
                continue
            u = np.repeat(np.arange(n, dtype=np.int64), cnt)
            base = np.repeat(lo - np.concatenate(([0], np.cumsum(cnt)[:-1])), cnt)
            v = np.arange(tot, dtype=np.int64) + base
            d = pts[u] - pts[v]
            keep = (d[:, 0] ** 2 + d[:, 1] ** 2 < r2) & (u != v)
            srcs.append(u[keep])
            dsts.append(v[keep])
    src = np.concatenate(srcs) if srcs else np.zeros(0, np.int64)
    dst = np.concatenate(dsts) if dsts else np.zeros(0, np.int64)
    o = np.lexsort((dst, src))  # grouped by source, neighbours by ID
    return src[o].astype(np.int32), dst[o].astype(np.int32)


# ------------------------------------------------------------------ label / order
def _gather_threaded(table: np.ndarray, idx: np.ndarray) -> np.ndarray:
    out = np.empty(idx.shape, table.dtype)
    step = max(1, -(-idx.size // (4 * _threads())))

    def job(s):
        np.take(table, idx[s:s + step], out=out[s:s + step])

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(job, range(0, idx.size, step)))
    return out


def random_labels(n: int, seed: int) -> np.ndarray:
    """A uniformly random label permutation sigma of [0, n) (int32)."""
    return _rng(seed).permutation(n).astype(np.int32)


def apply_labels(src: np.ndarray, dst: np.ndarray, sigma: np.ndarray):
    """Rename every endpoint v as sigma[v] (the random input labelling)."""
    return _gather_threaded(sigma, src), _gather_threaded(sigma, dst)


def shuffle_edges(src: np.ndarray, dst: np.ndarray, seed: int):
    """Uniformly random edge order."""
    p = _rng(seed).permutation(src.size)
    return _gather_threaded(src, p), _gather_threaded(dst, p)


def uniform_values(count: int, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    return _rng(seed).uniform(lo, hi, size=count).astype(np.float32)


def uniform_edges(n: int, m: int, seed: int):
    rng = _rng(seed)
    return (rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32),
            rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32))


# --------------------------------------------------------------------- workloads
@dataclass
class Graph:
    name: str
    n: int
    src: np.ndarray
    dst: np.ndarray
    val: np.ndarray | None = None
    x: np.ndarray | None = None

    @property
    def m(self) -> int:
        return int(self.src.size)


BASE_SEED = 0xB0BA0000


def make_workload(name: str, with_values: bool = True) -> Graph:
    """Named single-graph workloads.  Seeds: base = 0xB0BA0000 + id; labels
    base+1, edge order base+2, values base+3, x base+4.

    uniform14  n = 16,384, m = 131,072 i.i.d. uniform endpoints, random labels.
    rmat20     RMAT scale 20, edge factor 16, random labels.
    rmat24     RMAT scale 24, edge factor 16, random labels.
    grid4096   4096 x 4096 mesh (m = 67,092,480), random labels, edge order kept.
    RMAT edges are i.i.d., so their generated order is already a uniformly
    random order and no separate shuffle is applied.
    """
    ids = {"uniform14": 1, "rmat20": 2, "rmat24": 3, "grid4096": 4}
    if name.startswith("rmat") and name[4:].isdigit() and name not in ids:
        ids[name] = 100 + int(name[4:])
    if name not in ids:
        raise ValueError(f"unknown workload {name!r}")
    base = BASE_SEED + ids[name]
    if name == "uniform14":
        n, m = 16384, 131072
        src, dst = uniform_edges(n, m, base)
    elif name.startswith("rmat"):
        scale = int(name[4:])
        n, m = 1 << scale, 16 << scale
        src, dst = rmat(scale, m, base)
    else:
        side = 4096
        n = side * side
        src, dst = grid(side, side)
    sigma = random_labels(n, base + 1)
    src, dst = apply_labels(src, dst, sigma)
    g = Graph(name, n, src, dst)
    if with_values:
        g.val = uniform_values(g.m, base + 3)
        g.x = uniform_values(n, base + 4)
    return g


def small_workload(kind: str, n: int, m: int, seed: int) -> Graph:
    """Small graphs for parity tests (kind: uniform | rmat | grid | rgg)."""
    if kind == "uniform":
        src, dst = uniform_edges(n, m, seed)
    elif kind == "rmat":
        scale = max(1, int(math.ceil(math.log2(max(n, 2)))))
        src, dst = rmat(scale, m, seed, n=n)
    elif kind == "grid":
        side = max(1, int(math.isqrt(n)))
        n = side * side
        src, dst = grid(side, side)
    elif kind == "rgg":
        deg = max(1.0, m / max(n, 1))
        src, dst = rgg(n, math.sqrt(deg / (math.pi * n)), seed)
    else:
        raise ValueError(kind)
    sigma = random_labels(n, seed + 1)
    src, dst = apply_labels(src, dst, sigma)
    g = Graph(f"{kind}_{n}_{src.size}", n, src, dst)
    g.val = uniform_values(g.m, seed + 3)
    g.x = uniform_values(n, seed + 4)
    return g


# ----------------------------------------------------------------- batch (many)
@dataclass
class BatchSpec:
    kind: str  # "rmat" | "rgg"
    n: int
    edge_factor: int
    seed: int


def batch_specs(count: int = 512, seed: int = BASE_SEED + 5,
                log2_lo: float = 10.0, log2_hi: float = 18.0):
    """Graph g: n_g = floor(2**U(log2_lo, log2_hi)), edge factor U{4..32};
    even g RMAT (scale ceil(log2 n_g), out-of-range endpoints redrawn,
    m_g = n_g * ef_g), odd g RGG with radius sqrt(ef_g / (pi n_g))."""
    rng = _rng(seed)
    u = rng.uniform(log2_lo, log2_hi, size=count)
    ef = rng.integers(4, 33, size=count)
    return [BatchSpec("rmat" if g % 2 == 0 else "rgg", int(math.floor(2.0 ** u[g])),
                      int(ef[g]), seed * 1000 + 7 * g) for g in range(count)]


def make_batch_graph(spec: BatchSpec):
    n = spec.n
    if spec.kind == "rmat":
        scale = max(1, int(math.ceil(math.log2(n))))
        src, dst = rmat(scale, n * spec.edge_factor, spec.seed, n=n)
    else:
        src, dst = rgg(n, math.sqrt(spec.edge_factor / (math.pi * n)), spec.seed)
    sigma = random_labels(n, spec.seed + 1)
    return apply_labels(src, dst, sigma)


def _batch_job(spec):
    return make_batch_graph(spec)


def make_batch(specs, workers: int = 0):
    """Generate the graphs of `specs` and concatenate them.  Returns
    (edge_off[G+1], vert_off[G+1], src, dst) with local vertex IDs per graph.
    workers > 1 uses forked worker processes: call it before the parent
    process touches the GPU."""
    if workers > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            parts = list(ex.map(_batch_job, specs, chunksize=4))
    else:
        parts = [make_batch_graph(s) for s in specs]
    m = np.array([p[0].size for p in parts], np.int64)
    n = np.array([s.n for s in specs], np.int64)
    edge_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    vert_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    src = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.int32)
    dst = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.int32)
    return edge_off, vert_off, src, dst
