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
    selector.save_model(path, p, mu, sigma, {"x": 1})
    assert np.array_equal(selector.load_model(path), p)
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
