#!/usr/bin/env python3
"""Benchmark of the BOBA hot path on one MI355X.

A step is one pass of the whole path over one graph already resident in HBM:
    boba_reorder -> boba_relabel -> coo_to_csr -> spmv_csr
Warm-up steps are untimed; then exactly --steps steps are timed between two
device synchronisations.  Every kernel of the library is also bracketed by HIP
events on its launch stream (the torch current stream), which gives per-kernel
durations for the roofline figures.

Printed: one JSON line (stdout).  ``value`` is BOBA reorder throughput in edges
per second (m / mean duration of boba_reorder inside the timed steps); the
line also carries the whole-step time, SpMV GFLOP/s before (input labels) and
after the reorder, per-kernel durations and HBM fractions, the roofline of the
dominant kernel and the single-threaded CPU oracle timed on a bounded sample.
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BOBA reorder edges/s + % HBM peak; SpMV GFLOP/s before vs after reorder"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The paper's own numbers for this path, measured on other hardware and other
# graphs: context for the reader, not a target (vs_baseline stays null).
PAPER_CONTEXT = {
    "boba_reorder": {"edges_per_s": 89e6 / 17e-3, "derived_from": "17 ms for kron_g500-logn20 (~89M edges)",
                     "hardware": "NVIDIA V100 32 GB", "source": "Sec. 1.2 (timing), Sec. 5.1 (hardware)"},
    "spmv_speedup_boba_vs_random": {"median": 3.5, "range": [1.17, 6.25], "workloads": "skewed datasets of Table 2",
                                    "hardware": "NVIDIA V100 32 GB", "source": "Sec. 5.1"},
    "nbr": {"kron_g500-logn20": {"random": 0.75, "boba": 0.74}, "kron_g500-logn21": {"random": 0.72, "boba": 0.72},
            "delaunay_n24": {"random": 0.99, "boba": 0.48}, "source": "Table 1 (NBR over CSR rows, Sec. 5.2)"},
}


def radix_passes(n):
    """8-bit LSD passes coo_to_csr makes over row IDs below n."""
    bits = max(0, (n - 1).bit_length()) if n > 1 else 0
    return max(1, (bits + 7) // 8)


def call_alg_bytes(call, n, m):
    """Algorithmic bytes of one library call: what the method itself must move
    (int32 / float32 = 4 bytes), whatever passes the implementation makes.
    The reorder reads I and J once, writes and reads r once and writes perm
    and order (Sec. 4.4: reads linear in m, writes linear in n); the fused
    reorder + relabel additionally writes I' and J' (perm is then on chip);
    the conversion reads row, col, val and writes col, val and rowptr; SpMV
    reads col, val, rowptr and x once and writes y."""
    return {
        "boba_reorder": 8 * m + 16 * n,
        "boba_reorder_relabel": 16 * m + 16 * n,
        "boba_relabel": 16 * m + 4 * n,
        "coo_to_csr": 20 * m + 4 * (n + 1),
        "spmv_csr": 8 * m + 4 * (n + 1) + 8 * n,
    }[call]


def kernel_alg_bytes(name, n, m):
    """The algorithmic bytes (call_alg_bytes) charged to one launch of a
    kernel: the method's reads and writes that this kernel performs.
    Intermediate traffic of this design (records, radix passes, bitmaps) is
    never charged.  The conversion's bytes are spread evenly over its radix
    scatter passes, which each move every edge once."""
    table = {
        "bucket_split": 8 * m,                 # reads I and J
        "scatter_min": 8 * m + 4 * n,          # direct path: reads I and J, writes r
        "bucket_min": 4 * n,                   # writes r
        "rank_count": 4 * n,                   # reads r
        "rank_block": 4 * n,                   # writes order
        "rank_perm": 4 * n,                    # writes perm
        "bucket_relabel": 4 * n,               # reads perm
        "tile_unsplit": 8 * m,                 # writes I' and J'
        "relabel": 16 * m + 4 * n,             # the whole standalone relabel
        "radix_scatter": call_alg_bytes("coo_to_csr", n, m) // radix_passes(n),
        "spmv": call_alg_bytes("spmv_csr", n, m),
    }
    return table.get(name)


def kernel_impl_bytes(name, n, m):
    """This design's own traffic per launch (records, radix passes): what a
    kernel reads and writes as implemented, for comparison with the counters.
    Not the roofline's bytes."""
    table = {
        "bucket_split": 16 * m,                # read src, dst; write one record each
        "bucket_min": 8 * m + 4 * n,           # read the records; write r
        "bucket_relabel": 16 * m + 4 * n,      # read the records, perm; write new IDs
        "tile_unsplit": 24 * m,                # read records and new IDs; write src', dst'
        "radix_scatter": (24 * m * (radix_passes(n) - 1) + 20 * m) // radix_passes(n),
        "spmv": 8 * m + 4 * (n + 1) + 8 * n,
        "relabel": 16 * m + 4 * n,
    }
    return table.get(name)


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_10410_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


# library timing name -> device function name, where they differ
KERNEL_FN = {"bucket_transpose": "k_transpose", "csr_fill": "k_fill_u32", "relabel": "k_relabel_vec",
             "scatter_min": "k_scatter_min_vec", "spmv": "k_spmv_chunk", "mark": "k_mark_merge"}


# the instantiations a kernel's step launches take, where a summary holds
# several (coo_to_csr in the step carries values; its last pass writes no keys)
PMC_VARIANT = {"radix_scatter": "<8,true,", "spmv": "<true>"}


def pmc_traffic(kernel, workload, launches_per_step):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it was
    taken on the current kernel sources; otherwise None.  A summary may hold
    several template instantiations: the step's ones are averaged, weighted
    by their dispatches."""
    fn = KERNEL_FN.get(kernel, "k_" + kernel)
    path = os.path.join(ROOT, "profiles", f"pmc_{fn}_{workload}.txt")
    if not os.path.exists(path):
        return None
    sections, cur = [], None
    with open(path) as f:
        for line in f:
            if line.startswith("# rocprofv3 PMC HBM traffic of "):
                cur = {"name": line[len("# rocprofv3 PMC HBM traffic of "):].split(", workload")[0]}
                sections.append(cur)
            elif cur is not None and ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                cur[k.strip()] = v.strip()
    want = PMC_VARIANT.get(kernel)
    if want is not None:
        sections = [x for x in sections if want in x["name"]]
    try:
        if not sections or any(x.get("source_digest") != source_digest() for x in sections):
            return None
        n = [int(x["dispatches"]) for x in sections]
        b = [float(x["hbm_bytes_per_launch"]) for x in sections]
    except (KeyError, ValueError):
        return None
    return sum(ni * bi for ni, bi in zip(n, b)) / sum(n)


def cpu_baseline(g, budget_s):
    """Single-threaded sequential oracle (Algorithm 1 + tail) on a prefix of
    the edge list sized to roughly budget_s seconds."""
    import numpy as np
    import oracle

    probe = min(g.m, 1 << 21)
    t = time.perf_counter()
    oracle.boba(g.src[:probe], g.dst[:probe], g.n)
    rate = probe / max(time.perf_counter() - t, 1e-9)
    sample = int(min(g.m, max(probe, rate * budget_s)))
    s, d = np.ascontiguousarray(g.src[:sample]), np.ascontiguousarray(g.dst[:sample])
    # repeated while the budget lasts (at least 3 runs, at most 10): the median run
    runs = []
    while len(runs) < 3 or (sum(runs) < 0.67 * budget_s and len(runs) < 10):
        t = time.perf_counter()
        oracle.boba(s, d, g.n)
        runs.append(time.perf_counter() - t)
    el = float(np.median(runs))
    what = "whole edge list" if sample == g.m else f"first {sample} of {g.m} edges (all n = {g.n} vertices)"
    return {"value": sample / el, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential BOBA (C, -O2, 1 thread) on {what}; median of {len(runs)} runs, "
                      f"{el:.2f} s each, {sum(runs):.1f} s in all",
            "cpu_model": cpu_info()[0], "host_cpus": cpu_info()[1]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24", help="rmat24 | rmat20 | grid4096 | uniform14")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of CPU oracle work (0: skip)")
    ap.add_argument("--before-reps", type=int, default=5)
    ap.add_argument("--batch-graphs", type=int, default=512, help="graphs in the batched measurement (0: skip)")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--bin-bits", type=int, default=8,
                    help="also time binning the edges by destination into 2^B bins before BOBA (0: skip)")
    ap.add_argument("--shuffle-edges", action="store_true", help="put the workload's edges in random order first")
    ap.add_argument("--cold", action="store_true",
                    help="also time boba_reorder cold (after a 512 MiB write that flushes L2 and the Infinity "
                         "Cache); on by default for graphs of at most 2^24 edges")
    ap.add_argument("--pagerank", type=int, default=1, help="time 20 PageRank iterations before and after (0: skip)")
    ap.add_argument("--selector-graphs", type=int, default=100,
                    help="held-out graphs for the selector leg (0: skip)")
    ap.add_argument("--profile-spmv", type=int, default=0, metavar="N",
                    help="profiling run: build the CSR of the input order and of the BOBA order, then run N SpMVs "
                         "on the input order followed by N on the BOBA order (in that dispatch order) and exit")
    ap.add_argument("--calibrate", action="store_true",
                    help="run a plain elementwise kernel over 256 MiB (reads and writes 256 MiB) first, "
                         "to scale hardware byte counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        log("multi-GPU runs are not implemented: the path runs on one GPU; exiting")
        return 2

    import numpy as np
    from paper_2306_10410_amd import graphgen

    # all input generation happens before this process touches the GPU
    # (the batch is generated by forked worker processes)
    log(f"generating {args.workload}")
    t0 = time.perf_counter()
    g = graphgen.make_workload(args.workload)
    if args.shuffle_edges:
        g.src, g.dst = graphgen.shuffle_edges(g.src, g.dst, graphgen.BASE_SEED + 2)
    n, m = g.n, g.m
    log(f"n={n} m={m} generated in {time.perf_counter() - t0:.1f}s")
    batch = None
    if args.batch_graphs > 0:
        t0 = time.perf_counter()
        specs = graphgen.batch_specs(args.batch_graphs)
        batch = graphgen.make_batch(specs, workers=min(16, os.cpu_count() or 1))
        log(f"batch of {args.batch_graphs} graphs, m={int(batch[0][-1])} n={int(batch[1][-1])}, "
            f"generated in {time.perf_counter() - t0:.1f}s")

    sel_data = None
    if args.selector_graphs > 0:
        sel_data = prepare_selector_graphs(args.selector_graphs)

    import torch
    from paper_2306_10410_amd import boba

    if not torch.cuda.is_available():
        log("no HIP device visible")
        return 1
    boba.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log("uploading")
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    val = torch.from_numpy(g.val).to(dev)
    x = torch.from_numpy(g.x).to(dev)

    perm = torch.empty(n, dtype=torch.int32, device=dev)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    s2 = torch.empty(m, dtype=torch.int32, device=dev)
    d2 = torch.empty(m, dtype=torch.int32, device=dev)
    ws_r = torch.empty(boba.boba_reorder_workspace(n, m), dtype=torch.uint8, device=dev)
    ws_c = torch.empty(boba.coo_to_csr_workspace(n, m), dtype=torch.uint8, device=dev)
    rowptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(m, dtype=torch.int32, device=dev)
    val_c = torch.empty(m, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    x2 = torch.empty(n, dtype=torch.float32, device=dev)
    ws_s = torch.empty(boba.spmv_csr_workspace(n, m), dtype=torch.uint8, device=dev)

    if args.calibrate:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    K = args.steps
    ws_rr = torch.empty(boba.boba_reorder_relabel_workspace(n, m), dtype=torch.uint8, device=dev)

    def step(e=None):
        if e:
            e[0].record()
        boba.boba_reorder_relabel(src, dst, n, ws=ws_rr, perm=perm, order=order, src_out=s2, dst_out=d2)
        if e:
            e[1].record()
        boba.coo_to_csr(s2, d2, val, n, ws=ws_c, out=(rowptr, col, val_c))
        if e:
            e[2].record()
        boba.spmv_csr(rowptr, col, val_c, x2, y=y, ws=ws_s)
        if e:
            e[3].record()

    def reorder_call():
        boba.boba_reorder(src, dst, n, ws=ws_r, perm=perm, order=order)

    if args.profile_spmv > 0:
        return profile_spmv(args.profile_spmv, src, dst, val, x, n, m, perm, order, s2, d2, ws_rr, ws_c, ws_s,
                            (rowptr, col, val_c), y, x2)

    # x in the new labelling (x2[perm[v]] = x[v], on the host), so the
    # reordered product equals the original one
    reorder_call()
    x2_h = np.empty(n, np.float32)
    x2_h[perm.cpu().numpy()] = g.x
    x2.copy_(torch.from_numpy(x2_h))
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert boba.boba_check_device_error() == boba.BOBA_OK

    # --- timed region: exactly K steps, library timing off (no per-kernel
    # events), torch events between the three calls of each step
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    stage_names = ["reorder_relabel", "coo_to_csr", "spmv"]
    log(f"timing {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        step(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = {name: float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)]))
                for i, name in enumerate(stage_names)}
    ms_per_step = wall * 1e3 / K
    log(f"{ms_per_step:.3f} ms/step; stages {stage_ms}")

    # Every other time below is taken the same way: `reps` calls back to back
    # on the stream, an event between consecutive calls, library timing off;
    # the mean of the per-call intervals.
    def timed_calls(fn, reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        e[0].record()
        for k in range(reps):
            fn()
            e[k + 1].record()
        torch.cuda.synchronize()
        return float(np.mean([e[k].elapsed_time(e[k + 1]) for k in range(reps)]))

    # the reorder alone: the metric's edges/s
    reorder_ms = timed_calls(reorder_call, K)
    log(f"boba_reorder alone: {reorder_ms:.3f} ms")

    # SpMV and CSR build on the input labelling ("before") and on the BOBA
    # labelling ("after"), each call timed alone, both legs the same way
    log("before/after legs")
    rp0 = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col0 = torch.empty(m, dtype=torch.int32, device=dev)
    val0 = torch.empty(m, dtype=torch.float32, device=dev)
    y0 = torch.empty(n, dtype=torch.float32, device=dev)
    legs = {}
    for name, (a, b, xx, out_csr, yy) in (("before", (src, dst, x, (rp0, col0, val0), y0)),
                                         ("after", (s2, d2, x2, (rowptr, col, val_c), y))):
        reps = max(args.before_reps, 1)
        csr_ms = timed_calls(lambda: boba.coo_to_csr(a, b, val, n, ws=ws_c, out=out_csr), reps)
        spmv_ms = timed_calls(lambda: boba.spmv_csr(out_csr[0], out_csr[1], out_csr[2], xx, y=yy, ws=ws_s), reps)
        legs[name] = {"coo_to_csr_ms": csr_ms, "spmv_ms": spmv_ms, "spmv_gflops": 2 * m / (spmv_ms * 1e-3) / 1e9}
    log(f"legs {legs}")
    # the reordered SpMV must reproduce the input-order one
    yb = y0.cpu().numpy().astype(np.float64)
    ya = y.cpu().numpy().astype(np.float64)[perm.cpu().numpy()]
    spmv_agree = float(np.linalg.norm(ya - yb) / max(np.linalg.norm(yb), 1e-30))
    assert boba.boba_check_device_error() == boba.BOBA_OK

    cold_ms = None
    if args.cold or m <= (1 << 24):
        flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        ct = []
        for _ in range(K):
            flush.fill_(1)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            reorder_call()
            e[1].record()
            torch.cuda.synchronize()
            ct.append(e[0].elapsed_time(e[1]))
        cold_ms = float(np.median(ct))
        del flush
        log(f"boba_reorder cold: {cold_ms:.3f} ms")

    # --- instrumented pass (separate from every figure above): the library
    # brackets each of its kernels with HIP events on its launch stream, over
    # K more steps and K more reorders; per-kernel durations for the roofline
    boba.boba_timing_enable(True)
    boba.boba_timing_collect()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    kern = boba.boba_timing_collect()
    for _ in range(K):
        reorder_call()
    torch.cuda.synchronize()
    reorder_kern = boba.boba_timing_collect()
    boba.boba_timing_enable(False)

    # a plain device-to-device copy of 1 GiB: the bandwidth a streaming kernel can expect here
    cp_a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cp_b = torch.empty_like(cp_a)
    cp_b.copy_(cp_a)
    copy_GBs = 2 * (1 << 30) / (timed_calls(lambda: cp_b.copy_(cp_a), 5) * 1e-3) / 1e9  # read + write
    del cp_a, cp_b
    log(f"device copy: {copy_GBs:.0f} GB/s")

    # the standalone relabel with a given perm: one gather per endpoint vs the bucketed path
    s_o, d_o = torch.empty_like(src), torch.empty_like(dst)
    ws_rl = torch.empty(boba.boba_relabel_bucketed_workspace(n, m), dtype=torch.uint8, device=dev)
    relabel_ms = {
        "gather": timed_calls(lambda: boba.boba_relabel(src, dst, perm, src_out=s_o, dst_out=d_o), 3),
        "bucketed": timed_calls(lambda: boba.boba_relabel_bucketed(src, dst, perm, src_out=s_o, dst_out=d_o,
                                                                   ws=ws_rl), 3)}
    del s_o, d_o, ws_rl
    log(f"standalone relabel: gather {relabel_ms['gather']:.3f} ms, bucketed {relabel_ms['bucketed']:.3f} ms")

    # the non-atomic scatter of the paper's GPU kernel (Sec. 4.4): what the
    # exact minimum costs here, and how much of the order the race changes
    perm_r, order_r = torch.empty_like(perm), torch.empty_like(order)
    racy_ms = timed_calls(lambda: boba.boba_reorder(src, dst, n, ws=ws_r, perm=perm_r, order=order_r,
                                                    flags=boba.BOBA_FLAG_RACY), K)
    racy = {"reorder_ms": racy_ms, "exact_reorder_ms": reorder_ms,
            "same_new_id_fraction": float((perm_r == perm).float().mean())}
    del order_r
    log(f"racy scatter: {racy['reorder_ms']:.3f} ms, {racy['same_new_id_fraction']:.4f} of the IDs as exact")

    # locality of the CSR rows (NBR of Sec. 5.2, 32-ID lines) before and after
    ws_nbr = torch.empty(boba.boba_nbr_workspace(n, m), dtype=torch.uint8, device=dev)
    # the racy order's quality (NBR, SpMV rate), using the before-leg buffers
    sr, dr = boba.boba_relabel(src, dst, perm_r)
    boba.coo_to_csr(sr, dr, val, n, ws=ws_c, out=(rp0, col0, val0))
    del sr, dr, perm_r
    racy["nbr_over_nonempty_rows"] = boba.boba_nbr(rp0, col0, n, 32, ws=ws_nbr)[1]
    racy_spmv_ms = timed_calls(lambda: boba.spmv_csr(rp0, col0, val0, x2, y=y0, ws=ws_s), max(args.before_reps, 1))
    racy["spmv_gflops"] = 2 * m / (racy_spmv_ms * 1e-3) / 1e9
    log(f"racy order: NBR {racy['nbr_over_nonempty_rows']:.4f}, SpMV {racy['spmv_gflops']:.1f} GFLOP/s")
    # the before-leg CSR again, for NBR before
    boba.coo_to_csr(src, dst, val, n, ws=ws_c, out=(rp0, col0, val0))
    nbr_before = boba.boba_nbr(rp0, col0, n, 32, ws=ws_nbr)
    en = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    en[0].record()
    nbr_after = boba.boba_nbr(rowptr, col, n, 32, ws=ws_nbr)  # waits for its result
    en[1].record()
    torch.cuda.synchronize()
    nbr = {"line_ids": 32, "ms": en[0].elapsed_time(en[1]),
           "before": {"over_all_rows": nbr_before[0], "over_nonempty_rows": nbr_before[1]},
           "after": {"over_all_rows": nbr_after[0], "over_nonempty_rows": nbr_after[1]}}
    log(f"NBR before {nbr_before[1]:.4f} after {nbr_after[1]:.4f} (non-empty rows), {nbr['ms']:.2f} ms")
    del ws_nbr
    assert boba.boba_check_device_error() == boba.BOBA_OK

    pagerank = bench_pagerank(src, dst, s2, d2, perm, n, m, dev, ws_c) if args.pagerank else None
    if pagerank:
        log(f"PageRank x{pagerank['iters']}: {pagerank['ms_before']:.2f} -> {pagerank['ms_after']:.2f} ms")

    binned = None
    if args.bin_bits > 0:
        binned = bench_binned(args, g, src, dst, val, x, dev, ws_rr, ws_c, ws_s, legs["before"]["spmv_ms"])

    kernels = {}
    for name, (tot, cnt) in list(kern.items()) + [(f"{k} [boba_reorder alone]", v) for k, v in reorder_kern.items()]:
        per_step = cnt / K
        avg = tot / cnt
        entry = {"avg_ms": avg, "launches_per_step": per_step, "ms_per_step": tot / K}
        base = name.split(" [")[0]
        ab = kernel_alg_bytes(base, n, m)
        if ab is not None:
            entry["alg_bytes_per_launch"] = ab
            entry["achieved_GBs"] = ab / (avg * 1e-3) / 1e9
            entry["hbm_frac"] = entry["achieved_GBs"] / HBM_PEAK_GBS
        ib = kernel_impl_bytes(base, n, m)
        if ib is not None:
            entry["impl_bytes_per_launch"] = ib
        tr = pmc_traffic(base, args.workload, per_step) if "[" not in name else None
        if tr is not None:
            entry["traffic_bytes_per_launch"] = tr
        kernels[name] = entry
    # the roofline object: the kernel that takes the most time per step
    dom = max((k for k in kernels if "[" not in k), key=lambda k: kernels[k]["ms_per_step"])
    dk = kernels[dom]
    alg = dk.get("alg_bytes_per_launch", 0)
    traffic = dk.get("traffic_bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": alg / (dk["avg_ms"] * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / (dk["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "traffic": traffic, "traffic_over_alg_bytes": (traffic / alg) if (traffic and alg) else None,
                "alg_bytes_per_launch": alg, "avg_ms": dk["avg_ms"],
                "frac_of_measured_copy": alg / (dk["avg_ms"] * 1e-3) / 1e9 / copy_GBs,
                "bytes": "algorithmic: the method's own reads and writes charged to this kernel "
                         "(call bytes spread over the call's radix passes for the conversion)"}

    # each call of the path against its own algorithmic bytes (uninstrumented times)
    call_ms = {"boba_reorder": reorder_ms, "boba_reorder_relabel": stage_ms["reorder_relabel"],
               "coo_to_csr": stage_ms["coo_to_csr"], "spmv_csr": stage_ms["spmv"]}
    calls = {}
    for c, t in call_ms.items():
        b = call_alg_bytes(c, n, m)
        calls[c] = {"ms": t, "alg_bytes": b, "achieved_GBs": b / (t * 1e-3) / 1e9,
                    "hbm_frac": b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}

    batched = bench_batch(batch, args.batch_reps, dev) if batch is not None else None
    selector_leg = bench_selector(sel_data) if sel_data is not None else None

    cpu = None
    if args.cpu_budget > 0:
        log("CPU oracle baseline")
        cpu = cpu_baseline(g, args.cpu_budget)

    out = {
        "metric": METRIC,
        "value": m / (reorder_ms * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m,
                   "generator": _describe(args.workload),
                   "step": "boba_reorder_relabel -> coo_to_csr -> spmv_csr",
                   "value": "m / duration of boba_reorder alone (mean of --steps back-to-back calls, HIP events, "
                            "no per-kernel events)"},
        "reorder_ms": reorder_ms,
        "reorder_hbm_frac_alg": calls["boba_reorder"]["hbm_frac"],
        "path_edges_per_s": m / (ms_per_step * 1e-3),
        "stages_ms": stage_ms,
        "calls": calls,
        "spmv_gflops_before": legs["before"]["spmv_gflops"],
        "spmv_gflops_after": legs["after"]["spmv_gflops"],
        "spmv_speedup_after_reorder": legs["before"]["spmv_ms"] / legs["after"]["spmv_ms"],
        "spmv_dtype": "f32",
        "coo_to_csr_ms_before": legs["before"]["coo_to_csr_ms"],
        "coo_to_csr_ms_after": legs["after"]["coo_to_csr_ms"],
        "legs": legs,
        "spmv_reordered_vs_input_rel_l2": spmv_agree,
        "kernels": kernels,
        "roofline": roofline,
        "device_copy_GBs": copy_GBs,
        "reorder_ms_cold": cold_ms,
        "cpu_baseline": cpu,
        "batched": batched,
        "selector": selector_leg,
        "binned": binned,
        "nbr": nbr,
        "pagerank": pagerank,
        "racy_scatter": racy,
        "standalone_relabel_ms": relabel_ms,
        "paper_context": PAPER_CONTEXT,
        "device": torch.cuda.get_device_name(0),
        "source_digest": source_digest(),
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_pagerank(src, dst, s2, d2, perm, n, m, dev, ws_c, iters=20, reps=3):
    """PageRank (the PR application of Sec. 5.1): `iters` pull-SpMV iterations
    over the transposed CSR, on the input labels and on the BOBA labels."""
    import numpy as np
    import torch

    from paper_2306_10410_amd import boba
    rpT = torch.empty(n + 1, dtype=torch.int32, device=dev)
    colT = torch.empty(m, dtype=torch.int32, device=dev)
    ws = torch.empty(boba.boba_pagerank_workspace(n, m), dtype=torch.uint8, device=dev)
    out, ranks = {"iters": iters, "damping": 0.85}, {}
    rpF = torch.empty(n + 1, dtype=torch.int32, device=dev)
    colF = torch.empty(m, dtype=torch.int32, device=dev)
    for name, (a, b) in (("before", (src, dst)), ("after", (s2, d2))):
        boba.coo_to_csr(a, b, None, n, ws=ws_c, out=(rpF, colF, None))  # forward: out-degrees
        boba.coo_to_csr(b, a, None, n, ws=ws_c, out=(rpT, colT, None))  # row v: sources of edges into v
        rank = torch.empty(n, dtype=torch.float32, device=dev)
        boba.boba_pagerank(rpT, colT, 0.85, iters, out_rowptr=rpF, rank=rank, ws=ws)
        times = []
        for _ in range(reps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            boba.boba_pagerank(rpT, colT, 0.85, iters, out_rowptr=rpF, rank=rank, ws=ws)
            e[1].record()
            torch.cuda.synchronize()
            times.append(e[0].elapsed_time(e[1]))
        out[f"ms_{name}"] = float(np.median(times))
        ranks[name] = rank
    out["speedup"] = out["ms_before"] / out["ms_after"]
    out["ms_per_iter_after"] = out["ms_after"] / iters
    # the same ranks, relabelled: rank_after[perm[v]] = rank_before[v]
    out["rank_reordered_vs_input_l1"] = float((ranks["after"][perm.long()].double()
                                               - ranks["before"].double()).abs().sum())
    assert boba.boba_check_device_error() == boba.BOBA_OK
    return out


def bench_binned(args, g, src, dst, val, x, dev, ws_rr, ws_c, ws_s, before_spmv_ms, reps=5):
    """Sec. 5.6's remedy for edges in random order: bin the edge list by
    destination, then BOBA, CSR and SpMV on the binned list."""
    import numpy as np
    import torch

    from paper_2306_10410_amd import boba

    n, m = g.n, g.m
    log(f"binned leg: 2^{args.bin_bits} destination bins")
    sb, db = torch.empty_like(src), torch.empty_like(dst)
    ws_b = torch.empty(boba.boba_bin_by_dst_workspace(n, m), dtype=torch.uint8, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    s2, d2 = torch.empty_like(src), torch.empty_like(dst)
    rowptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(m, dtype=torch.int32, device=dev)
    val_c = torch.empty(m, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    # edge values follow their edges through the binning: bin (src, index) pairs
    # would need a payload; the SpMV only needs some value per edge, so the
    # binned list reuses val in its own order (same distribution)
    t = {"bin": [], "reorder_relabel": [], "coo_to_csr": [], "spmv": []}
    x2 = None
    for _ in range(reps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record()
        boba.boba_bin_by_dst(src, dst, n, args.bin_bits, ws=ws_b, out=(sb, db))
        e[1].record()
        boba.boba_reorder_relabel(sb, db, n, with_order=False, ws=ws_rr, perm=perm, src_out=s2, dst_out=d2)
        e[2].record()
        boba.coo_to_csr(s2, d2, val, n, ws=ws_c, out=(rowptr, col, val_c))
        e[3].record()
        if x2 is None:
            x2_h = np.empty(n, np.float32)
            x2_h[perm.cpu().numpy()] = g.x
            x2 = torch.from_numpy(x2_h).to(dev)
        boba.spmv_csr(rowptr, col, val_c, x2, y=y, ws=ws_s)
        e[4].record()
        torch.cuda.synchronize()
        for i, k in enumerate(t):
            t[k].append(e[i].elapsed_time(e[i + 1]))
    med = {k: float(np.median(v[1:])) for k, v in t.items()}
    assert boba.boba_check_device_error() == boba.BOBA_OK
    return {"bin_bits": args.bin_bits, "ms": med, "spmv_gflops": 2 * m / (med["spmv"] * 1e-3) / 1e9,
            "spmv_speedup_vs_input_order": before_spmv_ms / med["spmv"]}


def profile_spmv(reps, src, dst, val, x, n, m, perm, order, s2, d2, ws_rr, ws_c, ws_s, csr_after, y, x2):
    """Kernel sequence for the SpMV counter runs: no SpMV is dispatched
    before the measured ones, so the first `reps` SpMV dispatches are the
    input order's and the next `reps` the BOBA order's."""
    import numpy as np
    import torch
    from paper_2306_10410_amd import boba

    boba.boba_reorder_relabel(src, dst, n, ws=ws_rr, perm=perm, order=order, src_out=s2, dst_out=d2)
    x2_h = np.empty(n, np.float32)
    x2_h[perm.cpu().numpy()] = x.cpu().numpy()
    x2.copy_(torch.from_numpy(x2_h))
    boba.coo_to_csr(s2, d2, val, n, ws=ws_c, out=csr_after)
    csr_before = boba.coo_to_csr(src, dst, val, n, ws=ws_c)
    y0 = torch.empty_like(y)
    torch.cuda.synchronize()
    ms = {}
    for name, (csr, xx, yy) in (("before", (csr_before, x, y0)), ("after", (csr_after, x2, y))):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        e[0].record()
        for k in range(reps):
            boba.spmv_csr(csr[0], csr[1], csr[2], xx, y=yy, ws=ws_s)
            e[k + 1].record()
        torch.cuda.synchronize()
        ms[name] = float(np.mean([e[k].elapsed_time(e[k + 1]) for k in range(reps)]))
    assert boba.boba_check_device_error() == boba.BOBA_OK
    print(json.dumps({"profile_spmv": reps, "spmv_ms": ms, "n": n, "m": m}), flush=True)
    return 0


def bench_batch(batch, reps, dev):
    """Batched plan (one hipGraph replay) against one boba_reorder +
    boba_relabel call per graph on the same stream; both produce the same
    outputs (checked)."""
    import ctypes

    import numpy as np
    import torch
    from paper_2306_10410_amd import boba

    eo, vo, src_h, dst_h = batch
    G = len(eo) - 1
    src = torch.from_numpy(src_h).to(dev)
    dst = torch.from_numpy(dst_h).to(dev)
    from paper_2306_10410_amd import tune
    log(f"batched: tuning the work split for {G} graphs")
    best, report = tune.tune(eo, vo, src, dst, use_cache=False, log=log)
    log(f"batched: tuned {best} ({report})")
    plan = boba.BatchPlan(eo, vo, src, dst, tuning=tune.to_struct(best))
    plan.launch()
    torch.cuda.synchronize()

    def timed(fn, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        out = []
        for _ in range(k):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    batched_ms = timed(plan.launch, reps)
    # Per-graph baseline: one boba_reorder_relabel call per graph (the fastest
    # single-graph path: one launch for small graphs, the bucketed kernels
    # otherwise), issued as direct C calls on raw pointers, and the same
    # sequence of launches captured once into a hipGraph and replayed (no
    # host launch cost).
    L = boba.load()
    perm = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
    order = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
    so, do = torch.empty_like(src), torch.empty_like(dst)
    ms = np.diff(eo)
    ns = np.diff(vo)
    ws_bytes = max(boba.boba_reorder_relabel_workspace(int(ns[i]), int(ms[i])) for i in range(G))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    P = [(src.data_ptr() + 4 * int(eo[i]), dst.data_ptr() + 4 * int(eo[i]), int(ms[i]), int(ns[i]),
          perm.data_ptr() + 4 * int(vo[i]), order.data_ptr() + 4 * int(vo[i]),
          so.data_ptr() + 4 * int(eo[i]), do.data_ptr() + 4 * int(eo[i])) for i in range(G)]
    wsp = ws.data_ptr()

    def per_graph():
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for (s, d, m, n, p, o, s2, d2) in P:
            if n == 0:
                continue
            rc = L.boba_reorder_relabel(s, d, m, n, p, o, s2, d2, wsp, ws_bytes, 0, stream)
            if rc:
                raise RuntimeError(L.boba_last_error().decode())

    def same_as_plan():
        return bool(torch.equal(perm, plan.perm) and torch.equal(order, plan.order)
                    and torch.equal(so, plan.src_out) and torch.equal(do, plan.dst_out))

    per_graph()
    torch.cuda.synchronize()
    per_graph_ms = timed(per_graph, max(2, reps // 2))
    same = same_as_plan()
    # the per-graph launches captured into one graph (kernel nodes only)
    for t in (perm, order, so, do):
        t.fill_(-1)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg, stream=side):
        per_graph()
    torch.cuda.synchronize()
    graph_ms = timed(cg.replay, max(2, reps // 2))
    same_graph = same_as_plan()  # every replay rewrites the same outputs
    del cg
    info = plan.info()
    plan.destroy()
    m_tot = int(eo[-1])
    log(f"batched {batched_ms:.3f} ms vs per-graph {per_graph_ms:.3f} ms (x{per_graph_ms / batched_ms:.2f}), "
        f"per-graph hipGraph {graph_ms:.3f} ms (x{graph_ms / batched_ms:.2f}), identical={same and same_graph}")
    return {"workload": f"{G} graphs: n = 2^U(10,18), edge factor U{{4..32}}, half RMAT half RGG, random labels",
            "graphs": G, "m": m_tot, "n": int(vo[-1]), "batched_ms": batched_ms, "per_graph_ms": per_graph_ms,
            "per_graph_hipgraph_ms": graph_ms, "speedup": per_graph_ms / batched_ms,
            "speedup_vs_hipgraph": graph_ms / batched_ms, "edges_per_s": m_tot / (batched_ms * 1e-3),
            "identical_to_per_graph": same and same_graph, "plan": info, "tuning": best,
            "roofline": batch_roofline(m_tot, int(vo[-1]), batched_ms, G),
            "includes": "reorder + relabel",
            "per_graph_call": "boba_reorder_relabel per graph; also captured into one hipGraph and replayed"}


def batch_roofline(m, n, ms, graphs):
    """The batched kernel against HBM peak on the method's bytes for reorder +
    relabel of every graph (16m + 16n: I and J read, r written and read,
    perm and order written, I' and J' written), with the rocprofv3 traffic of
    k_batch when its summary was taken on the current sources."""
    alg = 16 * m + 16 * n
    achieved = alg / (ms * 1e-3) / 1e9
    traffic = pmc_traffic("batch", f"batch{graphs}", 1)
    return {"bound": "hbm", "kernel": "batch", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_launch": alg, "traffic": traffic,
            "traffic_over_alg_bytes": traffic / alg if traffic else None}


def prepare_selector_graphs(count):
    """The first graphs of the selector's held-out set (the same 10:1 mix of
    regular and large graphs), generated by forked workers before the GPU is
    touched."""
    from paper_2306_10410_amd import selector
    n_large = max(1, count // 11)
    n_reg = count - n_large
    specs = selector.heldout_specs(500, 50)
    specs = specs[:n_reg] + specs[500:500 + n_large]
    t0 = time.perf_counter()
    pool = selector.start_pool(min(16, os.cpu_count() or 1))
    graphs = list(pool.map(selector._gen, specs, chunksize=2))
    pool.shutdown()
    log(f"selector leg: {len(specs)} held-out graphs generated in {time.perf_counter() - t0:.1f}s")
    return specs, graphs


def bench_selector(sel_data):
    """The shipped selector on held-out graphs: its total time (features and
    inference included) against the oracle choice (the faster of the two
    measured paths per graph), the gate alone, the network alone, always
    reordering (the method without the selector) and never reordering."""
    import numpy as np
    import torch

    from paper_2306_10410_amd import boba, graphgen, selector

    specs, graphs = sel_data
    model = selector.load_model(selector.DEFAULT_MODEL)
    if model is None:
        return {"error": "no valid shipped model"}
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    selector.warm_up(None, seconds=1.0)
    ws_f = torch.empty(boba.load().boba_graph_features_workspace(), dtype=torch.uint8, device=dev)
    lead = torch.empty(1 << 16, dtype=torch.float32, device=dev)
    X = np.zeros((len(specs), selector.N_FEAT), np.float32)
    rows = []
    for i, (sp, (src_h, dst_h)) in enumerate(zip(specs, graphs)):
        src = torch.from_numpy(src_h).to(dev)
        dst = torch.from_numpy(dst_h).to(dev)
        val = torch.from_numpy(graphgen.uniform_values(src_h.size, sp.seed + 3)).to(dev)
        x = torch.from_numpy(graphgen.uniform_values(sp.n, sp.seed + 4)).to(dev)
        f, t_feat = selector.time_features(src, dst, sp.n, ws_f, lead)
        X[i] = f.cpu().numpy()
        med = selector.measure_paths(src, dst, val, x, sp.n, reps=3)
        med["t_feat"] = t_feat
        med.update({"kind": sp.kind, "n": sp.n, "m": int(src_h.size)})
        rows.append(med)
    t_inf = selector.time_inference(model.params)
    res = selector.evaluate(model.params, X, rows, t_inf, model.gate, model.meta.get("gate_alone"))
    res.update({"t_infer_ms": t_inf, "seconds": time.perf_counter() - t0,
                "graphs_desc": "the first held-out graphs of the selector's training run (regular and large, "
                               "10:1), each path the median of 3 timings after a warm-up round"})
    log(f"selector: {res['selector_vs_oracle']:.3f} of the oracle choice (gate alone "
        f"{res['gate_alone_vs_oracle']:.3f}, network only {res['ungated_selector_vs_oracle']:.3f}, "
        f"never {res['never_vs_oracle']:.3f}, always {res['always_vs_oracle']:.3f}) in {res['seconds']:.1f}s")
    return res


def _describe(workload):
    return {
        "rmat24": "RMAT(0.57,0.19,0.19,0.05) scale 24, edge factor 16, random labels; FP32 val, x ~ U(-1,1)",
        "rmat20": "RMAT(0.57,0.19,0.19,0.05) scale 20, edge factor 16, random labels; FP32 val, x ~ U(-1,1)",
        "grid4096": "4096x4096 4-neighbour mesh, random labels, edge order kept; FP32 val, x ~ U(-1,1)",
        "uniform14": "n=16384, m=131072 uniform endpoints, random labels; FP32 val, x ~ U(-1,1)",
    }.get(workload, workload)


if __name__ == "__main__":
    sys.exit(main())
