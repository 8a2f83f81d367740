"""Host-side pieces of the benchmark (no GPU): refusal of several GPUs,
the algorithmic byte count and the guard on recorded hardware counters."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_host_cpu_model_is_named():
    assert isinstance(bench.host_cpu_model(), str) and bench.host_cpu_model()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one MI355X" in r.stderr and not r.stdout.strip()


def test_algorithmic_bytes():
    # per row: rep 8 + stabilizer 2 + x_i + y_i; per off-diagonal element: x_j + rep_j
    assert bench.alg_bytes_of(10, 100, False) == 10 * 26 + 100 * 16
    assert bench.alg_bytes_of(10, 100, True) == 10 * 42 + 100 * 24


def test_recorded_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    rec = {"config": "square40", "sources_sha256": bench.kernel_sources_sha256(),
           "kernels": {"hash": {"dram_read_bytes": 10240.0, "dram_write_bytes": 3072.0}}}
    p = tmp_path / "k_apply_square40_counters.json"
    p.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.recorded_traffic("square40", 2) == 10240.0 + 3072.0
    assert bench.recorded_traffic("square40", 0) is None          # no record for this lookup
    assert bench.recorded_traffic("triangular36", 2) is None      # no record for another workload
    rec["sources_sha256"] = "0" * 64
    p.write_text(json.dumps(rec))
    assert bench.recorded_traffic("square40", 2) is None          # sources changed since the counters


def test_valu_bound_from_recorded_instructions(tmp_path, monkeypatch):
    rec = {"config": "square40", "sources_sha256": bench.kernel_sources_sha256(),
           "kernels": {"hash": {"dram_read_bytes": 1.0, "dram_write_bytes": 1.0,
                                "sq": {"SQ_INSTS_VALU": 0.5 * 256 * 2.4e9}}}}
    (tmp_path / "k_apply_square40_counters.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    v = bench.valu_bound("square40", 2, 1.0)          # half a second of issue in a one-second launch
    assert v["bound"] == "alu" and abs(v["frac"] - 0.5) < 1e-12
    assert bench.valu_bound("square40", 0, 1.0) is None
    assert bench.counters_path("square32_batch").endswith("k_batch_apply_square32_batch_counters.json")
