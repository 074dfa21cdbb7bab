"""bench.py's command-line contract: one GPU only, and one JSON line with the fields a run
reports (metric, throughput, timing, roofline of the dominant kernel); counter bytes are
reported only for the workload and kernel sources they were measured on."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_only_for_the_measured_workload_and_sources(monkeypatch):
    got = bench.measured_traffic("op_zinv_f32", (256, 256, 256))
    with open(os.path.join(ROOT, "profiles", "polycrystal256_hbm_traffic.json")) as f:
        d = json.load(f)
    if d["csrc_sha256_16"] == bench.csrc_hash():
        k = d["kernels"]["op_zinv_f32"]
        assert got == k["read_bytes"] + k["write_bytes"]
    else:
        assert got is None
    assert bench.measured_traffic("op_zinv_f32", (128, 128, 128)) is None
    monkeypatch.setattr(bench, "csrc_hash", lambda: "0000000000000000")
    assert bench.measured_traffic("op_zinv_f32", (256, 256, 256)) is None


@pytest.mark.gpu
def test_json_line_has_the_contract_fields():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--grid", "32", "--steps", "1", "--warmup", "1", "--no-cpu",
           "--no-batch"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    # the CG loops alone run faster than whole increments (which add the Newton level)
    assert d["cg_loop_voxel_iters_per_s"] > d["value"]
    assert d["vs_baseline"] is None and d["cpu_baseline"] is None  # --no-cpu
    assert d["config"]["workload"] == "polycrystal32_svk_stress" and d["config"]["grid"] == [32, 32, 32]
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert roof["traffic"] is None  # counters were taken on the 256^3 workload


def test_steady_launch_filter():
    """The roofline's launch average keeps the launches within 10% of the median (the steady
    CG iterations) and counts the no-op launches and the others apart."""
    ms = [0.008] * 3 + [0.50] * 2 + [0.586, 0.585, 0.587, 0.588, 0.584, 0.583, 0.59] * 3
    keep, noop, other = bench.steady_launches(ms)
    assert noop == 3 and other == 2 and len(keep) == 21
    assert abs(keep.mean() - np.mean([0.586, 0.585, 0.587, 0.588, 0.584, 0.583, 0.59])) < 1e-12


def test_cpu_baseline_samples_run_on_tiny_instances():
    from paper_1901_06531_amd import synth
    rate, its, dt = bench._oracle_cg_rate(synth.workload_polycrystal(n=8, ngrains=8), 0.01)
    assert rate > 0 and its >= 3
    t, nits = bench._oracle_newton_step(synth.workload_polycrystal(n=8, ngrains=8))
    assert t > 0 and nits >= 1
    assert bench._oracle_operator_s(synth.workload_polycrystal(n=8, ngrains=8)) > 0
