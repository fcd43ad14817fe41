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


def kernel_alg_bytes(name, n, m):
    """Algorithmic bytes per launch: what the kernel must read and write at
    minimum given its inputs and outputs (int32 / float32 = 4 bytes)."""
    table = {
        "scatter_min": 8 * m + 4 * n,          # read src, dst; write r once
        "relabel": 16 * m + 4 * n,             # read src, dst, perm once; write both
        # read key, col, val; write them (the last pass writes no keys):
        # the mean over the ceil(bits(n - 1) / 8) passes
        "radix_scatter": (24 * m * (radix_passes(n) - 1) + 20 * m) // radix_passes(n),
        "spmv": 8 * m + 4 * (n + 1) + 8 * n,   # val, col, rowptr, x once, y
        "bucket_split": 16 * m,                # read src, dst; write one record each
        "bucket_min": 8 * m + 4 * n,           # read the records; write r
        "bucket_relabel": 16 * m + 4 * n,      # read the records, perm; write new IDs
        "tile_unsplit": 24 * m,                # read records and new IDs; write src', dst'
        "rank": 12 * n,                        # read r, write perm, order
        "mark": 4 * n,                         # read r (bitmap writes are ours)
        "rank_count": 4 * n,                   # read r
        "rank_scatter": 12 * n,                # read r; write {r, v} per occurring vertex (<= n)
        "rank_block": 16 * n,                  # read the entries; write ranks and order
        "rank_perm": 16 * n,                   # read entries and ranks; write perm
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

    stage_names = ["reorder_relabel", "coo_to_csr", "spmv"]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
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

    # x in the new labelling (x2[perm[v]] = x[v], on the host), so the
    # reordered product equals the original one
    boba.boba_reorder(src, dst, n, ws=ws_r, perm=perm, order=order)
    x2_h = np.empty(n, np.float32)
    x2_h[perm.cpu().numpy()] = g.x
    x2.copy_(torch.from_numpy(x2_h))
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert boba.boba_check_device_error() == boba.BOBA_OK

    boba.boba_timing_enable(True)
    boba.boba_timing_collect()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = boba.boba_timing_collect()
    stage_ms = {name: float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(args.steps)]))
                for i, name in enumerate(stage_names)}
    ms_per_step = wall * 1e3 / args.steps
    log(f"{ms_per_step:.3f} ms/step; stages {stage_ms}")

    # the reorder alone (the metric's edges/s): boba_reorder timed the same number of times
    er = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for k in range(args.steps):
        er[k][0].record()
        boba.boba_reorder(src, dst, n, ws=ws_r, perm=perm, order=order)
        er[k][1].record()
    torch.cuda.synchronize()
    reorder_kern = boba.boba_timing_collect()
    boba.boba_timing_enable(False)
    stage_ms["reorder"] = float(np.mean([er[k][0].elapsed_time(er[k][1]) for k in range(args.steps)]))
    cold_ms = None
    if args.cold or m <= (1 << 24):
        flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        ct = []
        for _ in range(args.steps):
            flush.fill_(1)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            boba.boba_reorder(src, dst, n, ws=ws_r, perm=perm, order=order)
            e[1].record()
            torch.cuda.synchronize()
            ct.append(e[0].elapsed_time(e[1]))
        cold_ms = float(np.median(ct))
        del flush
        log(f"boba_reorder cold: {cold_ms:.3f} ms")
    # a plain device-to-device copy of 1 GiB: the bandwidth a streaming kernel can expect here
    cp_a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cp_b = torch.empty_like(cp_a)
    cp_b.copy_(cp_a)
    cpt = []
    for _ in range(5):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        cp_b.copy_(cp_a)
        e[1].record()
        torch.cuda.synchronize()
        cpt.append(e[0].elapsed_time(e[1]))
    copy_GBs = 2 * (1 << 30) / (float(np.median(cpt)) * 1e-3) / 1e9  # read + write
    del cp_a, cp_b
    log(f"device copy: {copy_GBs:.0f} GB/s")
    log(f"boba_reorder alone: {stage_ms['reorder']:.3f} ms")

    # the standalone relabel with a given perm: one gather per endpoint vs the bucketed path
    s_o, d_o = torch.empty_like(src), torch.empty_like(dst)
    ws_rl = torch.empty(boba.boba_relabel_bucketed_workspace(n, m), dtype=torch.uint8, device=dev)
    relabel_ms = {}
    for name, fn in (("gather", lambda: boba.boba_relabel(src, dst, perm, src_out=s_o, dst_out=d_o)),
                     ("bucketed", lambda: boba.boba_relabel_bucketed(src, dst, perm, src_out=s_o, dst_out=d_o,
                                                                     ws=ws_rl))):
        fn()
        rt = []
        for _ in range(3):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record()
            fn()
            e[1].record()
            torch.cuda.synchronize()
            rt.append(e[0].elapsed_time(e[1]))
        relabel_ms[name] = float(np.median(rt))
    del s_o, d_o, ws_rl
    log(f"standalone relabel: gather {relabel_ms['gather']:.3f} ms, bucketed {relabel_ms['bucketed']:.3f} ms")

    # the non-atomic scatter of the paper's GPU kernel (Sec. 4.4): what the
    # exact minimum costs here, and how much of the order the race changes
    perm_r, order_r = torch.empty_like(perm), torch.empty_like(order)
    boba.boba_reorder(src, dst, n, ws=ws_r, perm=perm_r, order=order_r, flags=boba.BOBA_FLAG_RACY)
    racy_t = []
    for _ in range(args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        boba.boba_reorder(src, dst, n, ws=ws_r, perm=perm_r, order=order_r, flags=boba.BOBA_FLAG_RACY)
        e[1].record()
        torch.cuda.synchronize()
        racy_t.append(e[0].elapsed_time(e[1]))
    racy = {"reorder_ms": float(np.mean(racy_t)), "exact_reorder_ms": stage_ms["reorder"],
            "same_new_id_fraction": float((perm_r == perm).float().mean())}
    del order_r
    log(f"racy scatter: {racy['reorder_ms']:.3f} ms, {racy['same_new_id_fraction']:.4f} of the IDs as exact")

    # SpMV and CSR build on the input labelling ("before")
    log("before-reorder leg")
    rp0 = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col0 = torch.empty(m, dtype=torch.int32, device=dev)
    val0 = torch.empty(m, dtype=torch.float32, device=dev)
    y0 = torch.empty(n, dtype=torch.float32, device=dev)
    b_csr, b_spmv = [], []
    for _ in range(args.before_reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        boba.coo_to_csr(src, dst, val, n, ws=ws_c, out=(rp0, col0, val0))
        e[1].record()
        boba.spmv_csr(rp0, col0, val0, x, y=y0, ws=ws_s)
        e[2].record()
        torch.cuda.synchronize()
        b_csr.append(e[0].elapsed_time(e[1]))
        b_spmv.append(e[1].elapsed_time(e[2]))
    before_csr_ms, before_spmv_ms = float(np.median(b_csr)), float(np.median(b_spmv))
    # the reordered SpMV must reproduce the input-order one
    yb = y0.cpu().numpy().astype(np.float64)
    ya = y.cpu().numpy().astype(np.float64)[perm.cpu().numpy()]
    spmv_agree = float(np.linalg.norm(ya - yb) / max(np.linalg.norm(yb), 1e-30))
    assert boba.boba_check_device_error() == boba.BOBA_OK

    # locality of the CSR rows (NBR of Sec. 5.2, 32-ID lines) before and after
    ws_nbr = torch.empty(boba.boba_nbr_workspace(n, m), dtype=torch.uint8, device=dev)
    # the racy order's quality (NBR, SpMV rate), using the before-leg buffers
    sr, dr = boba.boba_relabel(src, dst, perm_r)
    boba.coo_to_csr(sr, dr, val, n, ws=ws_c, out=(rp0, col0, val0))
    del sr, dr, perm_r
    racy["nbr_over_nonempty_rows"] = boba.boba_nbr(rp0, col0, n, 32, ws=ws_nbr)[1]
    rt = []
    for _ in range(args.before_reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        boba.spmv_csr(rp0, col0, val0, x2, y=y0, ws=ws_s)
        e[1].record()
        torch.cuda.synchronize()
        rt.append(e[0].elapsed_time(e[1]))
    racy["spmv_gflops"] = 2 * m / (float(np.median(rt)) * 1e-3) / 1e9
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

    pagerank = bench_pagerank(src, dst, s2, d2, perm, n, m, dev, ws_c)
    log(f"PageRank x{pagerank['iters']}: {pagerank['ms_before']:.2f} -> {pagerank['ms_after']:.2f} ms")

    binned = None
    if args.bin_bits > 0:
        binned = bench_binned(args, g, src, dst, val, x, dev, ws_rr, ws_c, ws_s, before_spmv_ms)

    kernels = {}
    for name, (tot, cnt) in list(kern.items()) + [(f"{k} [boba_reorder alone]", v) for k, v in reorder_kern.items()]:
        per_step = cnt / args.steps
        avg = tot / cnt
        entry = {"avg_ms": avg, "launches_per_step": per_step, "ms_per_step": tot / args.steps}
        ab = kernel_alg_bytes(name.split(" [")[0], n, m)
        if ab is not None:
            entry["alg_bytes_per_launch"] = ab
            entry["achieved_GBs"] = ab / (avg * 1e-3) / 1e9
            entry["hbm_frac"] = entry["achieved_GBs"] / HBM_PEAK_GBS
        kernels[name] = entry
    dom = max((k for k in kernels if "alg_bytes_per_launch" in kernels[k] and "[" not in k),
              key=lambda k: kernels[k]["ms_per_step"])
    dk = kernels[dom]
    traffic = pmc_traffic(dom, args.workload, dk["launches_per_step"])
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["achieved_GBs"], "peak": HBM_PEAK_GBS,
                "frac_of_measured_copy": dk["achieved_GBs"] / copy_GBs,
                "unit": "GB/s", "frac": dk["achieved_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                "alg_bytes_per_launch": dk["alg_bytes_per_launch"], "avg_ms": dk["avg_ms"]}

    batched = bench_batch(batch, args.batch_reps, dev) if batch is not None else None

    reorder_ms = stage_ms["reorder"]
    reorder_alg = 8 * m + 16 * n  # read I, J; write and read r; write perm and order
    cpu = None
    if args.cpu_budget > 0:
        log("CPU oracle baseline")
        cpu = cpu_baseline(g, args.cpu_budget)

    out = {
        "metric": METRIC,
        "value": m / (reorder_ms * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
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
                   "value": "m / duration of boba_reorder alone (mean of --steps calls, HIP events)"},
        "reorder_ms": reorder_ms,
        "reorder_hbm_frac_alg": reorder_alg / (reorder_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "path_edges_per_s": m / (ms_per_step * 1e-3),
        "stages_ms": stage_ms,
        "spmv_gflops_before": 2 * m / (before_spmv_ms * 1e-3) / 1e9,
        "spmv_gflops_after": 2 * m / (stage_ms["spmv"] * 1e-3) / 1e9,
        "spmv_speedup_after_reorder": before_spmv_ms / stage_ms["spmv"],
        "spmv_dtype": "f32",
        "coo_to_csr_ms_before": before_csr_ms,
        "coo_to_csr_ms_after": stage_ms["coo_to_csr"],
        "spmv_reordered_vs_input_rel_l2": spmv_agree,
        "kernels": kernels,
        "roofline": roofline,
        "device_copy_GBs": copy_GBs,
        "reorder_ms_cold": cold_ms,
        "cpu_baseline": cpu,
        "batched": batched,
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
    # per-graph launches: direct C calls on raw pointers (no per-call Python tensor work)
    L = boba.load()
    perm = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
    order = torch.empty(int(vo[-1]), dtype=torch.int32, device=dev)
    so, do = torch.empty_like(src), torch.empty_like(dst)
    ms = np.diff(eo)
    ns = np.diff(vo)
    ws_bytes = max(boba.boba_reorder_workspace(int(ns[i]), int(ms[i])) for i in range(G))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = [(src.data_ptr() + 4 * int(eo[i]), dst.data_ptr() + 4 * int(eo[i]), int(ms[i]), int(ns[i]),
          perm.data_ptr() + 4 * int(vo[i]), order.data_ptr() + 4 * int(vo[i]),
          so.data_ptr() + 4 * int(eo[i]), do.data_ptr() + 4 * int(eo[i])) for i in range(G)]
    wsp = ws.data_ptr()

    def per_graph():
        for (s, d, m, n, p, o, s2, d2) in P:
            if n == 0:
                continue
            rc = L.boba_reorder(s, d, m, n, p, o, wsp, ws_bytes, 0, stream)
            rc |= L.boba_relabel(s, d, m, p, n, s2, d2, stream)
            if rc:
                raise RuntimeError(L.boba_last_error().decode())

    per_graph()
    torch.cuda.synchronize()
    per_graph_ms = timed(per_graph, max(2, reps // 2))
    same = bool(torch.equal(perm, plan.perm) and torch.equal(order, plan.order) and torch.equal(so, plan.src_out)
                and torch.equal(do, plan.dst_out))
    info = plan.info()
    plan.destroy()
    m_tot = int(eo[-1])
    log(f"batched {batched_ms:.3f} ms vs per-graph {per_graph_ms:.3f} ms (x{per_graph_ms / batched_ms:.2f}), "
        f"identical={same}")
    return {"workload": f"{G} graphs: n = 2^U(10,18), edge factor U{{4..32}}, half RMAT half RGG, random labels",
            "graphs": G, "m": m_tot, "n": int(vo[-1]), "batched_ms": batched_ms, "per_graph_ms": per_graph_ms,
            "speedup": per_graph_ms / batched_ms, "edges_per_s": m_tot / (batched_ms * 1e-3),
            "identical_to_per_graph": same, "plan": info, "tuning": best, "includes": "reorder + relabel"}


def _describe(workload):
    return {
        "rmat24": "RMAT(0.57,0.19,0.19,0.05) scale 24, edge factor 16, random labels; FP32 val, x ~ U(-1,1)",
        "rmat20": "RMAT(0.57,0.19,0.19,0.05) scale 20, edge factor 16, random labels; FP32 val, x ~ U(-1,1)",
        "grid4096": "4096x4096 4-neighbour mesh, random labels, edge order kept; FP32 val, x ~ U(-1,1)",
        "uniform14": "n=16384, m=131072 uniform endpoints, random labels; FP32 val, x ~ U(-1,1)",
    }.get(workload, workload)


if __name__ == "__main__":
    sys.exit(main())
