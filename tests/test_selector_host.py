"""Selector host logic on the CPU: folding the feature standardisation into the
first layer, checkpoint round trip and the fallback on missing or corrupt models."""
import numpy as np

import oracle
from paper_2306_10410_amd import selector


def test_fold_standardisation_equals_standardised_forward():
    rng = np.random.default_rng(1)
    p = selector.init_params(3)
    X = rng.normal(5, 3, size=(40, 16))
    mu, sigma = X.mean(0), X.std(0)
    ref = oracle.mlp_forward(p.astype(np.float64), (X - mu) / sigma)
    folded = selector.fold_standardisation(p, mu, sigma)
    got = oracle.mlp_forward(folded.astype(np.float64), X)
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-5)


def test_checkpoint_round_trip_and_corruption(tmp_path):
    p = selector.init_params(4)
    mu, sigma = np.arange(16.0), np.ones(16)
    path = str(tmp_path / "m.npz")
    selector.save_model(path, p, mu, sigma, {"x": 1}, gate=12.5)
    model = selector.load_model(path)
    assert np.array_equal(model.params, p) and model.gate == 12.5
    # corrupt one parameter: checksum fails -> no model (fallback: always reorder)
    z = dict(np.load(path))
    z["params"] = z["params"].copy()
    z["params"][7] += 1.0
    np.savez(path, **z)
    assert selector.load_model(path) is None
    assert selector.load_model(str(tmp_path / "missing.npz")) is None
    # non-finite parameters are refused too
    bad = p.copy()
    bad[0] = np.nan
    selector.save_model(path, bad, mu, sigma)
    assert selector.load_model(path) is None


def test_size_gate_minimises_training_total():
    # small graphs: reordering never pays and features cost more than any gain;
    # large graphs: reordering pays and the MLP says so
    rows, pred = [], []
    for m, never, always, p in [(100, 0.5, 0.6, -1.0), (1000, 0.5, 0.7, 1.0), (10 ** 6, 5.0, 3.0, 2.0),
                                (10 ** 7, 9.0, 4.0, 1.5)]:
        rows.append({"m": m, "never": never, "always": always, "t_feat": 0.2})
        pred.append(p)
    pred = np.array(pred)
    gate = selector.choose_gate(pred, rows, 0.05)
    assert np.log2(1 + 1000) < gate <= np.log2(1 + 10 ** 6)
    t, choose = selector._policy_totals(pred, rows, 0.05, gate)
    assert np.allclose(t, [0.5, 0.5, 3.25, 4.25]) and list(choose) == [False, False, True, True]
    # without a gate every graph pays the feature and inference time
    t0, _ = selector._policy_totals(pred, rows, 0.05, float("-inf"))
    assert np.allclose(t0, [0.75, 0.95, 3.25, 4.25])
    # a non-finite prediction reorders (fallback)
    _, ch = selector._policy_totals(np.array([np.nan] * 4), rows, 0.05, float("-inf"))
    assert ch.all()


def test_gate_is_covered_by_the_checksum(tmp_path):
    p = selector.init_params(6)
    path = str(tmp_path / "g.npz")
    selector.save_model(path, p, np.zeros(16), np.ones(16), gate=10.0)
    z = dict(np.load(path))
    z["gate"] = np.array([3.0])
    np.savez(path, **z)
    assert selector.load_model(path) is None
