"""The autotuner's schedule report and its cache: a context reports the x- and y-pass
variants and radix splits it runs; with GHOM_TUNE_CACHE naming a file, the choices made at
creation are appended to it, and a later process takes its choices from it; forcing a variant
through an option is reported as set, not tuned; variants a grid does not have are refused."""

import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

from paper_1901_06531_amd import ghom  # noqa: E402

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
from paper_1901_06531_amd import ghom
with ghom.Solver((16, 16, 16), precision=ghom.FP32_SPLIT) as s:
    print(s.schedule())
    print(s.get_option(ghom.OPT_XPROJ_F64), s.get_option(ghom.OPT_XPROJ_F32))
"""


def _child(env):
    r = subprocess.run([sys.executable, "-c", CHILD % ROOT], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout.strip().splitlines()


def test_schedule_report_and_forced_variants():
    print("schedule report", flush=True)
    with ghom.Solver((256, 16, 8), precision=ghom.FP32_SPLIT) as s:
        text = s.schedule()
        assert text.startswith("256x16x8 (1 problem); f64: x ") and "; f32: x " in text and "(tuned)" in text
        s.set_option(ghom.OPT_XPROJ_F64, 4)
        assert "f64: x rows3 8x4x8 (set)" in s.schedule()
        s.set_option(ghom.OPT_XPROJ_F32, 1)
        assert "f32: x rows 16x16 (set)" in s.schedule()
        with pytest.raises(ghom.GhomError):
            s.set_option(ghom.OPT_YPASS_F64, 3)  # y length 16 has no three-stage schedule
        with pytest.raises(ghom.GhomError):
            s.set_option(ghom.OPT_YPASS_F32, 2)  # nor a narrow variant distinct from the wide one
        s.set_option(ghom.OPT_XPROJ_F64, 0)
        assert "f64: x " in s.schedule() and "(tuned)" in s.schedule().split(";")[1]
    with ghom.Solver((16, 16, 16)) as s:
        with pytest.raises(ghom.GhomError):
            s.set_option(ghom.OPT_XPROJ_F64, 4)  # x length 16 has no three-stage schedule


def test_tuning_cache_file(tmp_path):
    print("tuning cache file", flush=True)
    path = tmp_path / "tune.txt"
    env = dict(os.environ, GHOM_TUNE_CACHE=str(path))
    first = _child(env)
    lines = path.read_text().split("\n")
    keys = {l.split()[0]: int(l.split()[1]) for l in lines if l.strip()}
    xk = [k for k in keys if ":x:f64:16x16x16:p1:" in k]
    assert len(xk) == 1 and keys[xk[0]] in (1, 2, 3)
    assert any(":y:f32:16x16x16:p1:" in k for k in keys)
    # a later process takes its choice from the file: force x groups (2) for float64
    forced = [l if ":x:f64:16x16x16:p1:" not in l else "%s 2" % l.split()[0] for l in lines if l.strip()]
    path.write_text("\n".join(forced) + "\n")
    second = _child(env)
    assert second[1].split()[0] == "2"
    assert "f64: x groups 4x4 (tuned)" in second[0]
    assert first[0].split(";")[0] == second[0].split(";")[0]


def test_profiling_stride_times_every_kth_launch():
    """GHOM_OPT_PROFILE_EVERY = k brackets every k-th launch of a timed kernel name: the same
    increment (same iteration counts) yields about a third of the samples with k = 3 (the CG
    iterations queued after a solve has stopped, which exit at once, vary in number with the
    host's timing, so the launch totals differ by a few)."""
    from paper_1901_06531_amd import synth
    print("profiling stride", flush=True)
    w = synth.workload_polycrystal(n=32, ngrains=8)
    counts = {}
    for k in (1, 3):
        with ghom.Solver(w["shape"], precision=ghom.FP32_SPLIT) as s:
            s.setup(w)
            s.set_tolerances(1e-6, 1e-8, 1e-5)
            assert s.get_option(ghom.OPT_PROFILE_EVERY) == 1
            s.set_option(ghom.OPT_PROFILE_EVERY, k)
            assert s.get_option(ghom.OPT_PROFILE_EVERY) == k
            s.set_profiling_filter("op_zfwd_f32")
            s.set_profiling(True)
            info = s.step()
            prof = s.profile()
            counts[k] = (info["cg_iters_total"], prof["op_zfwd_f32"][0], len(s.profile_samples("op_zfwd_f32")))
            with pytest.raises(ghom.GhomError):
                s.set_option(ghom.OPT_PROFILE_EVERY, 0)
    print("  counts", counts, flush=True)
    (cg1, n1, m1), (cg3, n3, m3) = counts[1], counts[3]
    assert cg1 == cg3 and n1 == m1 and n3 == m3
    assert n1 >= cg1 and 3 * n3 >= cg3 and n3 < n1
    assert abs(n3 - n1 / 3) <= 4
