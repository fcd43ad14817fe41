"""Autotuner for the batched plan's work split (struct boba_tuning).

The batched kernel's results never depend on the tuning (the tests check
this); only its speed does.  The tuner times candidate tunings on the actual
batch by coordinate descent over a small grid, one parameter at a time, and
caches the winner in a JSON file keyed by the device architecture and a coarse
description of the batch (graph count and total edges, rounded to powers of
two).  The cache path is $BOBA_TUNE_CACHE, else ~/.cache/boba_tune.json.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import boba

GRID = {
    "small_max_n": [8192, 16384, 32768],
    # records per (vertex bucket, slice) item: 4M gives one slice per bucket
    # for graphs of up to 2^24 edges, 64K four
    "scatter_tile": [65536, 262144, 1048576, 4194304],
    "vertex_tile": [16384, 65536],
    "relabel_tile": [16384, 65536, 262144],
}
DEFAULT = {"small_max_n": 32768, "scatter_tile": 262144, "vertex_tile": 16384, "relabel_tile": 16384}


def cache_path() -> str:
    return os.environ.get("BOBA_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "boba_tune.json"))


def batch_key(edge_off, vert_off) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    G = len(edge_off) - 1
    m = int(edge_off[-1])
    n = int(vert_off[-1])
    b = lambda x: int(round(math.log2(max(x, 1))))
    return f"{arch}|G2^{b(G)}|m2^{b(m)}|n2^{b(n)}"


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p + ".tmp", "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(p + ".tmp", p)
    except OSError:
        pass


def to_struct(t: dict) -> boba.boba_tuning:
    return boba.boba_tuning(t["small_max_n"], t["scatter_tile"], t["vertex_tile"], t["relabel_tile"])


def time_plan(edge_off, vert_off, src, dst, tuning: dict, reps: int = 3, relabel: bool = True) -> float:
    plan = boba.BatchPlan(edge_off, vert_off, src, dst, relabel=relabel, tuning=to_struct(tuning))
    try:
        plan.launch()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.launch()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))
    finally:
        plan.destroy()


def tune(edge_off, vert_off, src, dst, *, relabel: bool = True, use_cache: bool = True, reps: int = 3,
         log=None) -> tuple[dict, dict]:
    """Returns (best tuning dict, report).  src/dst are the device tensors the
    plan will run on (the timing uses them; outputs are scratch)."""
    key = batch_key(edge_off, vert_off) + ("|relabel" if relabel else "|reorder")
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return dict(cache[key]["tuning"]), {"key": key, "cached": True, "ms": cache[key]["ms"]}
    best = dict(DEFAULT)
    best_ms = time_plan(edge_off, vert_off, src, dst, best, reps, relabel)
    trials = [(dict(best), best_ms)]
    for name, values in GRID.items():
        for v in values:
            if v == best[name]:
                continue
            cand = dict(best)
            cand[name] = v
            ms = time_plan(edge_off, vert_off, src, dst, cand, reps, relabel)
            trials.append((cand, ms))
            if log:
                log(f"tune {name}={v}: {ms:.3f} ms (best {best_ms:.3f})")
            if ms < best_ms:
                best, best_ms = cand, ms
    if use_cache:
        cache[key] = {"tuning": best, "ms": best_ms}
        _store_cache(cache)
    return best, {"key": key, "cached": False, "ms": best_ms, "trials": len(trials)}
