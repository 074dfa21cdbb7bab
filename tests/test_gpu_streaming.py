"""The transform passes built with nontemporal (streaming) loads and stores give the same bits
as their cached builds: the hint only changes where the data is kept.  Small problems (each
material law), whose contexts pick the cached builds, are run both ways in both precisions; a
context whose CG iteration touches more than 256 MB picks streaming at creation."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1901_06531_amd import ghom, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(w, prec, nt):
    with ghom.Solver(w["shape"], precision=prec) as s:
        s.setup(w)
        s.set_tolerances(1e-10, 1e-11, 1e-5 if prec == ghom.FP32_SPLIT else 0.0)
        assert s.get_option(ghom.OPT_STREAM_NT) == 0  # fits in the last-level cache
        s.set_option(ghom.OPT_STREAM_NT, nt)
        assert s.get_option(ghom.OPT_STREAM_NT) == nt
        recs = []
        for _ in range(len(w["target"])):
            info = s.step()
            recs.append((info["newton_iters"], info["cg_iters_total"]) + s.averages())
        return recs, s.field(ghom.FIELD_F)


def _workload(law):
    if law == "nh":
        w = synth.workload_particles(n=32, count=8)
    elif law == "svk":
        w = synth.workload_polycrystal(n=32, ngrains=16)
    else:
        from test_gpu_visco import _workload as visco_workload
        w = visco_workload((16, 16, 16), "mixed")
    w["target"] = w["target"][:2]
    return w


@pytest.mark.parametrize("law", ["nh", "svk", "visco"])
@pytest.mark.parametrize("prec", [ghom.FP64, ghom.FP32_SPLIT])
def test_streaming_builds_give_the_same_bits(prec, law):
    w = _workload(law)
    ref, Fr = _run(w, prec, 0)
    got, Fg = _run(w, prec, 1)
    for a, b in zip(ref, got):
        assert a[0] == b[0] and a[1] == b[1]
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    assert np.array_equal(Fr, Fg)


def test_streaming_is_chosen_by_working_set():
    shape = (96, 96, 96)
    # float32 CG vectors: about 184 B per voxel, 163 MB; float64: about 362 B, 320 MB
    with ghom.Solver(shape, precision=ghom.FP32_SPLIT) as s:
        assert s.get_option(ghom.OPT_STREAM_NT) == 0
    with ghom.Solver(shape, precision=ghom.FP64) as s:
        assert s.get_option(ghom.OPT_STREAM_NT) == 1
        with pytest.raises(ghom.GhomError) as e:
            s.set_option(ghom.OPT_STREAM_NT, 2)
        assert e.value.name == "EINVAL"
