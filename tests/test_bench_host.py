"""Host logic of bench.py (no GPU): the algorithmic flop count behind
roofline.achieved and the separately reported model count, the traffic
record lookup keyed by workload and the kernel's source hash, the CPU model
string, and the refusal of more than one GPU."""

import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_flop_count(bench):
    # per sub-step: the two tent gathers (11) and the Boris and position
    # updates (34); per step of dt: the decision (10)
    assert bench.FLOPS_PER_SUBSTEP == 45 and bench.FLOPS_PER_DECISION == 10
    c = {"steps_by_k": [1000, 20, 3, 0, 0, 0, 0, 0, 0]}
    want = 1000 * (10 + 45) + 20 * (10 + 4 * 45) + 3 * (10 + 16 * 45)
    assert bench.algorithmic_flops(c) == want


def test_model_flop_count_is_reported_apart(bench):
    # the kernels' own per-particle formulation: grid coordinate 2, E tent
    # 4p+8, B tent 4p+7, Boris 26, position 10; decision 11
    for p in (1, 2, 3, 5):
        assert bench.model_flops_per_substep(p) == 2 + (4 * p + 8) + (4 * p + 7) + 26 + 10
    c = {"steps_by_k": [1000, 20, 3, 0, 0, 0, 0, 0, 0]}
    want = 1000 * (11 + 77) + 20 * (11 + 4 * 77) + 3 * (11 + 16 * 77)
    assert bench.model_flops(c, 3) == want


def test_traffic_record_needs_the_current_source_hash(bench, tmp_path, monkeypatch):
    key = "fp64fast/occ5"
    _, files = bench.KERNELS[key]
    rec = {f"{key}@predictor": {"source_hash": bench.source_hash(files), "launches_per_pass": 1,
                                "bytes_per_launch": 1.25e10}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic(key, 1, "predictor") == 1.25e10
    assert bench.measured_traffic(key, 1, "large") is None      # another workload
    assert bench.measured_traffic(key, 2, "predictor") is None  # another launch shape
    rec[f"{key}@predictor"]["source_hash"] = "0" * 16           # taken on another kernel
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(key, 1, "predictor") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(key, 1, "predictor") is None


def test_cpu_model_string(bench):
    s = bench.cpu_model()
    assert isinstance(s, str) and s


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
