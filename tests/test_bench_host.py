"""Host-side pieces of the benchmark and the tuner (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_algorithmic_bytes_tables():
    n, m = 1 << 24, 1 << 28
    # the method's bytes per call: reads of I and J linear in m, writes linear in n
    assert bench.call_alg_bytes("boba_reorder", n, m) == 8 * m + 16 * n
    assert bench.call_alg_bytes("coo_to_csr", n, m) == 20 * m + 4 * (n + 1)
    assert bench.call_alg_bytes("spmv_csr", n, m) == 8 * m + 4 * (n + 1) + 8 * n
    # charged to kernels: only the method's own reads and writes
    assert bench.kernel_alg_bytes("bucket_split", n, m) == 8 * m
    assert bench.kernel_alg_bytes("bucket_min", n, m) == 4 * n
    # the conversion's bytes spread over its passes
    assert bench.radix_passes(n) == 3 and bench.radix_passes(256) == 1 and bench.radix_passes(257) == 2
    assert bench.kernel_alg_bytes("radix_scatter", n, m) == (20 * m + 4 * (n + 1)) // 3
    assert bench.kernel_alg_bytes("spmv", n, m) == 8 * m + 4 * (n + 1) + 8 * n
    assert bench.kernel_alg_bytes("no_such_kernel", n, m) is None
    # the design's own traffic stays a separate table
    assert bench.kernel_impl_bytes("bucket_split", n, m) == 16 * m
    assert bench.kernel_impl_bytes("radix_scatter", n, m) == (2 * 24 * m + 20 * m) // 3
    # every kernel's charge is at most its implementation's traffic
    for k in ("bucket_split", "bucket_min", "bucket_relabel", "tile_unsplit", "radix_scatter", "spmv", "relabel"):
        assert bench.kernel_alg_bytes(k, n, m) <= bench.kernel_impl_bytes(k, n, m), k


def test_pmc_traffic_requires_a_matching_source_digest(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: "abc123")

    def section(name, digest, dispatches, hbm):
        return (f"# rocprofv3 PMC HBM traffic of {name}, workload w\nsource_digest: {digest}\n"
                f"dispatches: {dispatches}\nhbm_bytes_per_launch: {hbm}\n")

    f = prof / "pmc_k_radix_scatter_w.txt"
    # the step's instantiations, weighted by dispatches; the others ignored
    f.write_text(section("k_radix_scatter<8,false,false>", "abc123", 8, 1000) +
                 section("k_radix_scatter<8,true,false>", "abc123", 12, 60) +
                 section("k_radix_scatter<8,true,true>", "abc123", 6, 30))
    assert bench.pmc_traffic("radix_scatter", "w", 3) == 50.0
    f.write_text(section("k_radix_scatter<8,true,false>", "stale", 12, 60) +
                 section("k_radix_scatter<8,true,true>", "abc123", 6, 30))
    assert bench.pmc_traffic("radix_scatter", "w", 3) is None   # a kernel changed since
    f.write_text(section("k_radix_scatter<8,false,false>", "abc123", 8, 1000))
    assert bench.pmc_traffic("radix_scatter", "w", 3) is None   # not the step's instantiation
    (prof / "pmc_k_bucket_split_w.txt").write_text(section("k_bucket_split", "abc123", 9, 42))
    assert bench.pmc_traffic("bucket_split", "w", 1) == 42.0
    assert bench.pmc_traffic("spmv", "w", 1) is None  # no summary


def test_committed_profiles_name_their_command():
    prof = os.path.join(ROOT, "profiles")
    files = [f for f in os.listdir(prof) if f.endswith(".txt")]
    assert files
    for f in files:
        text = open(os.path.join(prof, f)).read()
        assert "rocprofv3" in text and "bench.py" in text and "source_digest:" in text, f


def test_tuner_cache_key_and_struct(monkeypatch, tmp_path):
    pytest.importorskip("torch")
    from paper_2306_10410_amd import tune
    monkeypatch.setenv("BOBA_TUNE_CACHE", str(tmp_path / "c.json"))
    key = tune.batch_key([0, 1000, 3000], [0, 100, 300])
    assert key.endswith("|G2^1|m2^12|n2^8")
    tune._store_cache({"k": {"tuning": tune.DEFAULT, "ms": 1.0}})
    assert tune._load_cache()["k"]["tuning"] == tune.DEFAULT
    st = tune.to_struct(tune.DEFAULT)
    assert (st.small_max_n, st.scatter_tile) == (tune.DEFAULT["small_max_n"], tune.DEFAULT["scatter_tile"])
    for name, values in tune.GRID.items():
        assert tune.DEFAULT[name] in values, name


def test_batch_roofline_on_the_method_bytes():
    import bench
    r = bench.batch_roofline(m=1000, n=100, ms=1e-3, graphs=3)
    assert r["alg_bytes_per_launch"] == 16 * 1000 + 16 * 100
    assert abs(r["achieved"] - 17600 / 1e-6 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / bench.HBM_PEAK_GBS) < 1e-12
    assert r["traffic"] is None  # no summary for a 3-graph batch
