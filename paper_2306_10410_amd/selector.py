"""Learned reorder selector: will BOBA pay for itself on this graph?

Not part of the paper's method: it answers the net-speedup question of the
paper's Problem 2 (Sec. 1.1) per graph instead of reordering every graph.

Serving path (all on the GPU, through the C ABI):
    boba_graph_features (16 FP32 features) -> boba_mlp_forward -> one float
    prediction of log2(T_never / T_always) -> reorder iff it is > 0.
The feature standardisation used in training is folded into the first layer,
so the deployed network takes raw features.  Without a usable model, or when
a feature or the prediction is not finite, the policy falls back to always
reordering (the method itself).

Labels are measured by the method itself on the GPU:
    T_never  = t(coo_to_csr on input labels) + t(spmv_iters SpMVs on it)
    T_always = t(boba_reorder_relabel) + t(coo_to_csr on BOBA labels)
               + t(spmv_iters SpMVs on it)
each the median of `reps` HIP-event timings (the SpMVs run back to back; the
two paths alternate in going first, each after an untimed lead-in of small
kernels).  Training uses the library's own
backward and Adam kernels.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

from . import graphgen

N_FEAT = 16
SPMV_ITERS = 20
# Network trained on an MI355X by `python -m paper_2306_10410_amd.selector`
# (4000 + 400 graphs, see main); timings, and so the model, are device-specific.
DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_model.npz")


# --------------------------------------------------------------------- timing
def _events(torch, k):
    return [torch.cuda.Event(enable_timing=True) for _ in range(k)]


def measure_paths(src, dst, val, x, n, *, reps=5, spmv_iters=SPMV_ITERS, ws=None):
    """Times both paths on device tensors.  Returns a dict of median ms."""
    import torch

    from . import boba

    m = src.numel()
    dev = src.device
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(m, dtype=torch.int32, device=dev)
    vv = torch.empty(m, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    s2, d2 = torch.empty_like(src), torch.empty_like(dst)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    ws_r = torch.empty(max(1, boba.boba_reorder_relabel_workspace(n, m)), dtype=torch.uint8, device=dev)
    ws_c = torch.empty(max(1, boba.coo_to_csr_workspace(n, m)), dtype=torch.uint8, device=dev)
    ws_s = torch.empty(max(1, boba.spmv_csr_workspace(n, m)), dtype=torch.uint8, device=dev)
    # The SpMV iterations run back to back between two events, as a solver
    # would run them.  Each path is preceded by a short untimed burst of small
    # kernels, and the two paths take turns going first: the first kernels
    # after the host's synchronisation run slower (clocks, an idle queue),
    # which would otherwise count against whichever path always came first.
    lead = torch.empty(1 << 16, dtype=torch.float32, device=dev)

    def lead_in():
        for _ in range(4):
            lead.fill_(0.0)

    def never(e):
        lead_in()
        e[0].record()
        boba.coo_to_csr(src, dst, val, n, ws=ws_c, out=(rp, col, vv))
        e[1].record()
        for _ in range(spmv_iters):
            boba.spmv_csr(rp, col, vv, x, y=y, ws=ws_s)
        e[2].record()

    def always(e):
        lead_in()
        e[0].record()
        boba.boba_reorder_relabel(src, dst, n, ws=ws_r, perm=perm, order=order, src_out=s2, dst_out=d2)
        e[1].record()
        boba.coo_to_csr(s2, d2, val, n, ws=ws_c, out=(rp, col, vv))
        e[2].record()
        for _ in range(spmv_iters):
            boba.spmv_csr(rp, col, vv, x, y=y, ws=ws_s)  # x in any labelling: same access pattern cost
        e[3].record()

    t = {k: [] for k in ("csr_in", "spmv_in", "reorder_relabel", "csr_boba", "spmv_boba")}
    for rnd in range(reps + 1):  # first round warms up
        en, ea = _events(torch, 3), _events(torch, 4)
        if rnd % 2 == 0:
            never(en)
            always(ea)
        else:
            always(ea)
            never(en)
        torch.cuda.synchronize()
        for k, (a, b) in (("csr_in", (en[0], en[1])), ("spmv_in", (en[1], en[2])),
                          ("reorder_relabel", (ea[0], ea[1])), ("csr_boba", (ea[1], ea[2])),
                          ("spmv_boba", (ea[2], ea[3]))):
            t[k].append(a.elapsed_time(b))
    med = {k: float(np.median(v[1:])) for k, v in t.items()}
    med["never"] = med["csr_in"] + med["spmv_in"]
    med["always"] = med["reorder_relabel"] + med["csr_boba"] + med["spmv_boba"]
    return med


# ------------------------------------------------------------------- dataset
def selector_specs(count, seed, log2_lo=10.0, log2_hi=18.0):
    """Graphs from the batch families (RMAT / RGG, random labels)."""
    return graphgen.batch_specs(count, seed=seed, log2_lo=log2_lo, log2_hi=log2_hi)


def _gen(spec):
    return graphgen.make_batch_graph(spec)


def start_pool(workers):
    """A pool of generator processes.  Create it before this process touches
    the GPU: the workers are forked and never use the GPU themselves."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    return ProcessPoolExecutor(workers, mp_context=mp.get_context("fork"))


def warm_up(log=None, seconds=2.0):
    """Runs both paths on a mid-sized graph for a while, so that the timings
    that follow see the GPU at its working clocks."""
    import torch

    dev = torch.device("cuda:0")
    g = graphgen.small_workload("rmat", 1 << 18, 1 << 22, graphgen.BASE_SEED + 55)
    src, dst = torch.from_numpy(g.src).to(dev), torch.from_numpy(g.dst).to(dev)
    val, x = torch.from_numpy(g.val).to(dev), torch.from_numpy(g.x).to(dev)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        measure_paths(src, dst, val, x, g.n, reps=1)
    if log:
        log(f"warm-up {time.perf_counter() - t0:.1f}s")


def time_features(src, dst, n, ws, lead, reps=3):
    """The features of a graph and their cost, timed like the two paths: a
    warm-up call, then the median of `reps` calls, each after an untimed
    lead-in (the first touch of a new graph -- TLB and cache misses -- is paid
    by whatever runs first on it, whichever policy is used)."""
    import torch

    from . import boba

    f = boba.boba_graph_features(src, dst, n, ws=ws)
    ts = []
    for _ in range(reps):
        e = _events(torch, 2)
        for _ in range(4):
            lead.fill_(0.0)
        e[0].record()
        boba.boba_graph_features(src, dst, n, out=f, ws=ws)
        e[1].record()
        torch.cuda.synchronize()
        ts.append(e[0].elapsed_time(e[1]))
    return f, float(np.median(ts))


def build_dataset(specs, *, reps=5, log=None, pool=None):
    """Features (GPU kernel), both path timings and the label for every spec.
    Graphs come from `pool` (see start_pool) when given."""
    import torch

    from . import boba

    dev = torch.device("cuda:0")
    X = np.zeros((len(specs), N_FEAT), np.float32)
    rows = []
    ws_f = torch.empty(boba.load().boba_graph_features_workspace(), dtype=torch.uint8, device=dev)
    lead = torch.empty(1 << 16, dtype=torch.float32, device=dev)
    graphs = pool.map(_gen, specs, chunksize=4) if pool is not None else map(_gen, specs)
    for i, (s, (src_h, dst_h)) in enumerate(zip(specs, graphs)):
        src = torch.from_numpy(src_h).to(dev)
        dst = torch.from_numpy(dst_h).to(dev)
        val = torch.from_numpy(graphgen.uniform_values(src_h.size, s.seed + 3)).to(dev)
        x = torch.from_numpy(graphgen.uniform_values(s.n, s.seed + 4)).to(dev)
        f, t_feat = time_features(src, dst, s.n, ws_f, lead)
        X[i] = f.cpu().numpy()
        med = measure_paths(src, dst, val, x, s.n, reps=reps)
        med["t_feat"] = t_feat
        med.update({"kind": s.kind, "n": s.n, "m": int(src_h.size), "seed": s.seed})
        rows.append(med)
        if log and (i + 1) % 250 == 0:
            log(f"dataset {i + 1}/{len(specs)}")
    T_never = np.array([r["never"] for r in rows])
    T_always = np.array([r["always"] for r in rows])
    y = np.log2(T_never / T_always).astype(np.float32)
    return X, y, rows


# --------------------------------------------------------------------- model
def init_params(seed):
    """He-style initialisation of the 16-64-64-1 network (float32)."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, np.sqrt(2 / 16), (64, 16)), np.zeros(64),
             rng.normal(0, np.sqrt(2 / 64), (64, 64)), np.zeros(64),
             rng.normal(0, np.sqrt(1 / 64), (1, 64)), np.zeros(1)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def fold_standardisation(params, mu, sigma):
    """Returns parameters that take raw features: W1' = W1 / sigma,
    b1' = b1 - W1' mu."""
    p = params.astype(np.float64).copy()
    W1 = p[:1024].reshape(64, 16)
    b1 = p[1024:1088]
    W1n = W1 / sigma[None, :]
    p[1024:1088] = b1 - W1n @ mu
    p[:1024] = W1n.ravel()
    return p.astype(np.float32)


def train(X, y, *, epochs=200, batch=256, lr=1e-3, seed=0, log=None, weights=None):
    """Adam on mean squared error with the library's kernels.  Returns
    (deployable params on raw features, mu, sigma, loss history).

    weights (optional, one per graph): minibatch rows are drawn with
    probability proportional to them (with replacement, N draws per epoch)
    instead of a plain shuffle.  With weights = |T_never - T_always| the
    regression spends its capacity where a wrong decision costs time."""
    import torch

    from . import boba

    dev = torch.device("cuda:0")
    mu = X.mean(axis=0).astype(np.float64)
    sigma = X.std(axis=0).astype(np.float64)
    sigma[sigma < 1e-6] = 1.0
    Xs = ((X - mu) / sigma).astype(np.float32)
    ys = y.astype(np.float32)
    Xd = torch.from_numpy(Xs).to(dev)
    yd = torch.from_numpy(ys).to(dev)
    p = torch.from_numpy(init_params(seed)).to(dev)
    m1, m2 = torch.zeros_like(p), torch.zeros_like(p)
    grad = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed + 1)
    N = X.shape[0]
    step = 0
    hist = []
    prob = None
    if weights is not None:
        w = np.asarray(weights, np.float64)
        prob = w / w.sum()
    for ep in range(epochs):
        idx = rng.permutation(N) if prob is None else rng.choice(N, size=N, p=prob)
        for b0 in range(0, N, batch):
            sel = idx[b0:b0 + batch]  # minibatch rows assembled on the host, then copied
            xb = torch.from_numpy(np.ascontiguousarray(Xs[sel])).to(dev)
            yb = torch.from_numpy(np.ascontiguousarray(ys[sel])).to(dev)
            boba.boba_mlp_backward(p, xb, yb, grad=grad, loss=loss)
            step += 1
            boba.boba_mlp_adam(p, m1, m2, grad, step, lr=lr)
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            _, full = boba.boba_mlp_backward(p, Xd, yd)
            hist.append(float(full.cpu()[0]))
            if log:
                log(f"epoch {ep}: train mse {hist[-1]:.4f}")
    return fold_standardisation(p.cpu().numpy(), mu, sigma), mu, sigma, hist


# ----------------------------------------------------------------- selector
def _digest(arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


class Model:
    """A deployable selector: MLP parameters on raw features and the size gate
    (log2(1 + m) below which the graph is not reordered and no feature is
    computed)."""

    def __init__(self, params, gate=float("-inf"), meta=None):
        self.params = np.asarray(params, np.float32)
        self.gate = float(gate)
        self.meta = dict(meta or {})


def save_model(path, params, mu, sigma, meta=None, gate=float("-inf")):
    g = np.array([gate], np.float64)
    p32 = params.astype(np.float32)
    np.savez(path, params=p32, mu=mu, sigma=sigma, gate=g, version=np.array([2]),
             checksum=np.frombuffer(_digest([p32, mu, sigma, g]).encode(), np.uint8),
             meta=np.frombuffer(json.dumps(meta or {}).encode(), np.uint8))


def load_model(path):
    """Returns a Model, or None if the file is missing or invalid (then the
    policy falls back to always reordering)."""
    try:
        z = np.load(path, allow_pickle=False)
        params, mu, sigma, gate = z["params"], z["mu"], z["sigma"], z["gate"]
        ok = (int(z["version"][0]) == 2 and params.shape == (5313,) and params.dtype == np.float32
              and gate.shape == (1,) and not np.isnan(gate[0])
              and bytes(z["checksum"]).decode() == _digest([params, mu, sigma, gate])
              and np.all(np.isfinite(params)))
        if not ok:
            return None
        try:
            meta = json.loads(bytes(z["meta"]).decode()) if "meta" in z.files else {}
        except ValueError:
            meta = {}
        return Model(params, gate[0], meta if isinstance(meta, dict) else {})
    except Exception:
        return None


class Selector:
    """decide(src, dst, n) -> (reorder?, prediction).  Graphs below the size
    gate are not reordered (prediction -inf, no GPU work).  Falls back to
    always reordering when there is no usable model or the prediction is not
    finite."""

    def __init__(self, params=None, device="cuda:0", gate=float("-inf")):
        import torch

        from . import boba

        self.boba = boba
        self.dev = torch.device(device)
        self.params = None if params is None else torch.from_numpy(np.asarray(params, np.float32)).to(self.dev)
        self.gate = float(gate)
        self.ws = torch.empty(boba.load().boba_graph_features_workspace(), dtype=torch.uint8, device=self.dev)
        self.feat = torch.empty(1, N_FEAT, dtype=torch.float32, device=self.dev)
        self.out = torch.empty(1, dtype=torch.float32, device=self.dev)

    @classmethod
    def from_file(cls, path=DEFAULT_MODEL, device="cuda:0"):
        model = load_model(path)
        return cls(None, device) if model is None else cls(model.params, device, model.gate)

    def decide(self, src, dst, n):
        if self.params is None:
            return True, float("nan")
        if np.log2(1.0 + src.numel()) < self.gate:
            return False, float("-inf")
        self.boba.boba_graph_features(src, dst, n, out=self.feat.view(-1), ws=self.ws)
        self.boba.boba_mlp_forward(self.params, self.feat, out=self.out)
        pred = float(self.out.cpu()[0])
        if not np.isfinite(pred):
            return True, pred
        return pred > 0.0, pred


def _policy_totals(pred, rows, t_infer_ms, gate):
    """Per-graph time of the gated policy: below the gate the input order is
    kept (no feature work); above it features + inference + the MLP's choice
    (a non-finite prediction reorders)."""
    never = np.array([r["never"] for r in rows])
    always = np.array([r["always"] for r in rows])
    feat = np.array([r["t_feat"] for r in rows])
    lm = np.log2(1.0 + np.array([r["m"] for r in rows], np.float64))
    choose = np.where(np.isfinite(pred), pred > 0, True)
    gated = lm < gate
    t = np.where(gated, never, feat + t_infer_ms + np.where(choose, always, never))
    return t, choose & ~gated


def choose_gate(pred, rows, t_infer_ms):
    """The size gate that minimises the policy's total time on the given
    (training) graphs: every distinct log2(1 + m), and no gate."""
    lm = np.log2(1.0 + np.array([r["m"] for r in rows], np.float64))
    cands = np.concatenate([[-np.inf], np.unique(lm), [np.inf]])
    best = min(cands, key=lambda g: float(_policy_totals(pred, rows, t_infer_ms, g)[0].sum()))
    return float(best)


def best_gate_alone(rows):
    """The threshold that minimises the total time of the gate alone (below
    it keep the order, above it always reorder; no features) on the given
    (training) graphs."""
    never = np.array([r["never"] for r in rows])
    always = np.array([r["always"] for r in rows])
    lm = np.log2(1.0 + np.array([r["m"] for r in rows], np.float64))
    cands = np.concatenate([[-np.inf], np.unique(lm), [np.inf]])
    return float(min(cands, key=lambda g: float(np.where(lm >= g, always, never).sum())))


def evaluate(params, X, rows, t_infer_ms, gate=float("-inf"), gate_alone=None):
    """Held-out totals: the selector's choice (plus its feature and inference
    time above the gate) against the oracle choice, always-reorder,
    never-reorder, the gate alone at the selector's threshold and (if given)
    the gate alone at its own best threshold on the training graphs."""
    import torch

    from . import boba

    dev = torch.device("cuda:0")
    pred = boba.boba_mlp_forward(torch.from_numpy(params).to(dev), torch.from_numpy(X).to(dev)).cpu().numpy()
    never = np.array([r["never"] for r in rows])
    always = np.array([r["always"] for r in rows])
    t_sel, choose = _policy_totals(pred, rows, t_infer_ms, gate)
    t_nogate, choose_ng = _policy_totals(pred, rows, t_infer_ms, float("-inf"))
    # the gate alone: below it keep the input order, above it always reorder
    # (no features, no network)
    lm = np.log2(1.0 + np.array([r["m"] for r in rows], np.float64))
    above = lm >= gate
    t_gate = np.where(above, always, never)
    ga = gate if gate_alone is None else float(gate_alone)
    t_alone = np.where(lm >= ga, always, never)
    opt = np.minimum(never, always)
    sel_total = float(t_sel.sum())
    truth = always < never
    return {"graphs": len(rows), "gate_log2m": gate, "selector_ms": sel_total,
            "oracle_choice_ms": float(opt.sum()), "always_ms": float(always.sum()), "never_ms": float(never.sum()),
            "gate_only_ms": float(t_gate.sum()), "mlp_only_ms": float(t_nogate.sum()),
            "gate_alone_log2m": ga, "gate_alone_ms": float(t_alone.sum()),
            "gate_alone_vs_oracle": float(t_alone.sum()) / float(opt.sum()),
            "selector_vs_oracle": sel_total / float(opt.sum()),
            "selector_vs_always": sel_total / float(always.sum()),
            "selector_vs_never": sel_total / float(never.sum()),
            "gate_only_vs_oracle": float(t_gate.sum()) / float(opt.sum()),
            "ungated_selector_vs_oracle": float(t_nogate.sum()) / float(opt.sum()),
            "never_vs_oracle": float(never.sum()) / float(opt.sum()),
            "always_vs_oracle": float(always.sum()) / float(opt.sum()),
            "above_gate": int(above.sum()),
            "above_gate_oracle_reorder": int((truth & above).sum()),
            "above_gate_selector_reorder": int((choose & above).sum()),
            "above_gate_agreement": float(np.mean(choose[above] == truth[above])) if above.any() else None,
            "decisions_reorder": int(choose.sum()), "oracle_reorder": int(truth.sum()),
            "agreement": float(np.mean(choose == truth)),
            "mlp_agreement": float(np.mean(choose_ng == truth))}


def heldout_specs(count_regular=500, count_large=50, log2_hi=18.0, large_log2_hi=21.0):
    """The held-out graph specs of the training run (seeds disjoint from the
    training graphs): `count_regular` with log2 n in [10, log2_hi] and
    `count_large` in [log2_hi, large_log2_hi]."""
    specs = selector_specs(count_regular, graphgen.BASE_SEED + 51, log2_hi=log2_hi)
    if count_large:
        specs += selector_specs(count_large, graphgen.BASE_SEED + 53, log2_hi, large_log2_hi)
    return specs


def time_inference(params, reps=50):
    """Median ms of one MLP forward for one graph plus the host read-back."""
    import torch

    from . import boba

    dev = torch.device("cuda:0")
    p = torch.from_numpy(params).to(dev)
    f = torch.zeros(1, N_FEAT, dtype=torch.float32, device=dev)
    out = torch.empty(1, dtype=torch.float32, device=dev)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        boba.boba_mlp_forward(p, f, out=out)
        float(out.cpu()[0])
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts))


def main(argv=None):
    ap = argparse.ArgumentParser(description="train and evaluate the reorder selector on the GPU")
    ap.add_argument("--train", type=int, default=4000)
    ap.add_argument("--heldout", type=int, default=500)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--log2-hi", type=float, default=18.0)
    ap.add_argument("--large", type=int, default=0, help="extra graphs with log2 n in [log2-hi, large-log2-hi]")
    ap.add_argument("--large-log2-hi", type=float, default=22.0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default="selector_model.npz")
    ap.add_argument("--data-out", default="selector_data.npz")
    ap.add_argument("--weighted", type=int, default=1,
                    help="draw training minibatches in proportion to |T_never - T_always| (0: plain shuffle)")
    ap.add_argument("--from-data", default=None,
                    help="train on the features, timings and labels saved by an earlier run (--data-out) "
                         "instead of measuring the graphs again")
    ap.add_argument("--eval-model", default=None,
                    help="measure the held-out graphs only and evaluate this saved model (no training)")
    args = ap.parse_args(argv)
    log = lambda s: print(f"[selector] {s}", file=sys.stderr, flush=True)
    tr_specs = selector_specs(args.train, graphgen.BASE_SEED + 50, log2_hi=args.log2_hi)
    ho_specs = selector_specs(args.heldout, graphgen.BASE_SEED + 51, log2_hi=args.log2_hi)
    if args.large:
        k = args.large
        tr_specs += selector_specs(k, graphgen.BASE_SEED + 52, args.log2_hi, args.large_log2_hi)
        ho_specs += selector_specs(max(1, k // 8), graphgen.BASE_SEED + 53, args.log2_hi, args.large_log2_hi)
    if args.from_data:
        return train_and_report(args, log, *load_data(args.from_data))
    pool = start_pool(args.workers) if args.workers > 1 else None  # before the GPU is touched
    t0 = time.perf_counter()
    warm_up(log)
    if args.eval_model:
        model = load_model(args.eval_model)
        if model is None:
            raise SystemExit(f"{args.eval_model}: not a valid selector model")
        Xho, _, rho = build_dataset(ho_specs, reps=args.reps, log=log, pool=pool)
        if pool is not None:
            pool.shutdown()
        t_inf = time_inference(model.params)
        res = evaluate(model.params, Xho, rho, t_inf, model.gate, model.meta.get("gate_alone"))
        res.update({"model": args.eval_model, "t_infer_ms": t_inf,
                    "t_feat_ms_median": float(np.median([r["t_feat"] for r in rho]))})
        print(json.dumps(res), flush=True)
        return 0
    # training and held-out graphs are measured interleaved, so that slow
    # drifts of the machine do not separate the two sets
    specs = tr_specs + ho_specs
    order = np.random.default_rng(graphgen.BASE_SEED + 54).permutation(len(specs))
    X, y, rows = build_dataset([specs[i] for i in order], reps=args.reps, log=log, pool=pool)
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    X, y, rows = X[inv], y[inv], [rows[i] for i in inv]
    ntr = len(tr_specs)
    Xtr, ytr, rtr = X[:ntr], y[:ntr], rows[:ntr]
    Xho, yho, rho = X[ntr:], y[ntr:], rows[ntr:]
    if pool is not None:
        pool.shutdown()
    log(f"datasets in {time.perf_counter() - t0:.1f}s; train labels: {np.mean(ytr > 0):.3f} reorder-pays")
    np.savez(args.data_out, Xtr=Xtr, ytr=ytr, Xho=Xho, yho=yho,
             rows_tr=np.frombuffer(json.dumps(rtr).encode(), np.uint8),
             rows_ho=np.frombuffer(json.dumps(rho).encode(), np.uint8))
    return train_and_report(args, log, Xtr, ytr, rtr, Xho, yho, rho)


def load_data(path):
    z = np.load(path)
    return (z["Xtr"], z["ytr"], json.loads(bytes(z["rows_tr"]).decode()), z["Xho"], z["yho"],
            json.loads(bytes(z["rows_ho"]).decode()))


def train_and_report(args, log, Xtr, ytr, rtr, Xho, yho, rho):
    """Trains on the training graphs, picks the size gate on them, saves the
    model and prints the held-out evaluation."""
    # a graph's weight is what the wrong choice would cost on it, with a floor
    # so that no graph is never seen
    gap = np.abs(np.array([r["never"] - r["always"] for r in rtr]))
    weights = gap + 0.05 * float(np.median(gap)) if args.weighted else None
    params, mu, sigma, hist = train(Xtr, ytr, epochs=args.epochs, log=log, weights=weights)
    t_inf = time_inference(params)
    import torch

    from . import boba
    pred_tr = boba.boba_mlp_forward(torch.from_numpy(params).cuda(), torch.from_numpy(Xtr).cuda()).cpu().numpy()
    gate = choose_gate(pred_tr, rtr, t_inf)
    alone = best_gate_alone(rtr)
    log(f"size gate: log2(1 + m) >= {gate:.3f} (the gate alone would take {alone:.3f})")
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    save_model(args.out, params, mu, sigma, {"train": len(rtr), "epochs": args.epochs,
                                             "weighted": bool(args.weighted), "gate_alone": alone}, gate=gate)
    res = evaluate(params, Xho, rho, t_inf, gate, alone)
    res.update({"train_graphs": len(rtr), "train_mse": hist[-1], "t_infer_ms": t_inf, "weighted": bool(args.weighted),
                "t_feat_ms_median": float(np.median([r["t_feat"] for r in rho]))})
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
