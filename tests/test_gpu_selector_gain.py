"""What the trained selector gains over the method without it.

The shipped selector (a size gate, then the network trained on an MI355X by
the library's own kernels) picks, per graph, between keeping the input order
and BOBA.  The graphs: small ones below the gate (reordering costs more than
the 20 SpMVs win back), two large random geometric graphs above it (BOBA wins
back several times its cost) and a large RMAT graph above it (close to break
even at this size).  The selector's total time, including its own feature and
inference time, must beat both fixed policies: always reordering (the method
alone) and never reordering.  Its choices above the gate are also compared
with the gate alone (always reordering there); that comparison is printed,
not asserted: on the large RMAT graph the two paths are within a few percent,
so either choice is a good one."""
import time

import numpy as np
import pytest
import torch

from paper_2306_10410_amd import graphgen, selector
from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

SPECS = [graphgen.BatchSpec("rmat", 1 << 14, 16, 9101), graphgen.BatchSpec("rgg", 1 << 14, 12, 9102),
         graphgen.BatchSpec("rmat", 1 << 16, 24, 9103), graphgen.BatchSpec("rgg", 3 << 15, 20, 9104),
         graphgen.BatchSpec("rgg", 1 << 20, 26, 9105), graphgen.BatchSpec("rgg", 3 << 19, 16, 9106),
         graphgen.BatchSpec("rmat", 1 << 20, 24, 9107)]
LARGE_RGG = (4, 5)   # indices of the large geometric graphs


def test_trained_selector_beats_fixed_policies():
    model = selector.load_model(selector.DEFAULT_MODEL)
    assert model is not None, "shipped model missing or corrupt"
    sel = selector.Selector(model.params, gate=model.gate)
    dev = torch.device("cuda:0")
    tot = {"selector": 0.0, "always": 0.0, "never": 0.0, "gate_only": 0.0}
    decisions, above = [], []
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
        above.append(bool(np.log2(1.0 + s_h.size) >= model.gate))
        tot["selector"] += t_decide + (med["always"] if choice else med["never"])
        tot["always"] += med["always"]
        tot["never"] += med["never"]
        tot["gate_only"] += med["always"] if above[-1] else med["never"]
    print("totals (ms):", {k: round(v, 3) for k, v in tot.items()}, "decisions:", decisions, "above gate:", above)
    assert all(decisions[i] for i in LARGE_RGG)  # the large geometric graphs are reordered
    assert not any(decisions[:4]) and not any(above[:4])  # the small graphs keep their order (gate)
    assert all(above[4:])
    assert tot["selector"] < 0.95 * min(tot["always"], tot["never"])
