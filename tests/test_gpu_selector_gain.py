"""What the trained selector gains over the method without it.

The shipped network (trained on an MI355X by the library's own kernels) picks,
per graph, between keeping the input order and BOBA.  On a mix of small graphs
(where reordering costs more than the 20 SpMVs win back) and one large random
geometric graph (where it wins), the selector's total time -- including its
own feature and inference time -- must beat both fixed policies: always
reordering (the method alone) and never reordering."""
import time

import numpy as np
import pytest
import torch

from paper_2306_10410_amd import graphgen, selector
from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

SPECS = [graphgen.BatchSpec("rmat", 1 << 14, 16, 9101), graphgen.BatchSpec("rgg", 1 << 14, 12, 9102),
         graphgen.BatchSpec("rmat", 1 << 16, 24, 9103), graphgen.BatchSpec("rgg", 3 << 15, 20, 9104),
         graphgen.BatchSpec("rgg", 1 << 20, 26, 9105)]


def test_trained_selector_beats_fixed_policies():
    model = selector.load_model(selector.DEFAULT_MODEL)
    assert model is not None, "shipped model missing or corrupt"
    sel = selector.Selector(model.params, gate=model.gate)
    dev = torch.device("cuda:0")
    tot = {"selector": 0.0, "always": 0.0, "never": 0.0}
    decisions = []
    for spec in SPECS:
        s_h, d_h = graphgen.make_batch_graph(spec)
        src, dst = torch.from_numpy(s_h).to(dev), torch.from_numpy(d_h).to(dev)
        val = torch.from_numpy(graphgen.uniform_values(s_h.size, spec.seed + 3)).to(dev)
        x = torch.from_numpy(graphgen.uniform_values(spec.n, spec.seed + 4)).to(dev)
        med = selector.measure_paths(src, dst, val, x, spec.n, reps=5)
        sel.decide(src, dst, spec.n)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        choice, _ = sel.decide(src, dst, spec.n)  # returns after reading the prediction back
        t_decide = (time.perf_counter() - t0) * 1e3
        decisions.append(choice)
        tot["selector"] += t_decide + (med["always"] if choice else med["never"])
        tot["always"] += med["always"]
        tot["never"] += med["never"]
    print("totals (ms):", {k: round(v, 3) for k, v in tot.items()}, "decisions:", decisions)
    assert decisions[-1] is True  # the large geometric graph is reordered
    assert not any(decisions[:-1])  # the small graphs keep their order
    assert tot["selector"] < 0.95 * min(tot["always"], tot["never"])
