"""The benchmark's output contract, on the CPU: one JSON line with the required keys, a refusal (with
a message) for more than one GPU, and the CPU-baseline object produced by the oracle sample."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synth import configs  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


@pytest.mark.parametrize("flags", [["--steps", "0"], ["--warmup", "-1"]])
def test_empty_timed_region_is_refused_with_a_message(flags):
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *flags],
                         capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert out.returncode == 2
    assert "--steps" in json.loads(out.stdout.strip().splitlines()[-1])["error"]


def test_every_workload_is_listed():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                         capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert out.returncode == 0
    for w in bench.WORKLOADS:
        assert w in out.stdout
    assert set(bench.DEFAULTS) == set(bench.WORKLOADS)


def test_md_line_carries_the_contract_keys():
    class A:
        steps, warmup = 10, 2
    roof = {"bound": "hbm", "achieved": 1.0, "peak": 8000.0, "unit": "GB/s", "frac": 1.25e-4, "traffic": None}
    line = bench.md_line(A, "kg_batched", 1e9, 0.5, 1000, {"cells": 1}, roof)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in line, k
    assert line["n_gpus"] == 1 and line["config"]["workload"] == "kg_batched"
    assert line["ms_per_step"] == 50.0 and line["vs_baseline"] is None
    json.dumps(line)


def test_cpu_baseline_is_the_oracle_on_a_bounded_sample():
    cells = [configs.kg_cell([20] * 10, 5)]
    p = configs.kg_params(precision="fp64")
    cb, s = bench.oracle_sample(p, cells, np.eye(3)[None], 10, "one small cell", seconds=0.2)
    assert cb["kind"] == "oracle" and cb["unit"] == "atom-steps/s" and cb["value"] > 0
    assert cb["cores"] >= 1 and "200 atoms" in cb["sample"]
    assert cb["single_core_value"] > 0 and cb["host_threads"] >= 1 and cb["cpu_model"]
    assert s.shape == (1, 6) and np.all(np.isfinite(s))


def test_traffic_records_belong_to_their_workload_and_source():
    # a workload without its own counter record reports null traffic, never another workload's
    assert not os.path.exists(os.path.join(ROOT, "profiles", "traffic_k_force_kg_kg_glassy.json"))
    assert bench.traffic_from_profiles("k_force_kg", "kg_glassy") is None
    for kernel, w in (("k_force_eam", "cu_element"), ("k_force_eam", "cu_batched"), ("k_force_kg", "kg_batched"),
                      ("k_force_kg", "fe_tet")):
        path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{w}.json")
        got = bench.traffic_from_profiles(kernel, w)
        if not os.path.exists(path):
            assert got is None
            continue
        rec = json.load(open(path))
        if rec["source_hash"] == bench.kernel_source_hash():
            assert got == rec["bytes_per_launch"] and got > 0
        else:                       # counters taken on other kernel sources are not reported
            assert got is None
