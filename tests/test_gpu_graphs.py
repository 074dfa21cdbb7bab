"""CG iterations replayed from captured HIP graphs give the same bits as launched one by one.

Each increment replays the captured graphs many times, with the library's own eager work
(residuals, re-projections, Newton updates, host reads of the stop flags) between the replays;
every increment's averages and the final fields are compared with an eager run of the same
problem, bit for bit (every kernel and every reduction runs in a fixed order).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1901_06531_amd import ghom, synth  # noqa: E402

from test_gpu_batch import _problems  # noqa: E402

pytestmark = pytest.mark.gpu


def _single(w, prec, graphs):
    with ghom.Solver(w["shape"], precision=prec) as s:
        s.setup(w)
        s.set_tolerances(1e-10, 1e-11, 1e-5 if prec == ghom.FP32_SPLIT else 0.0)
        s.set_option(ghom.OPT_GRAPHS, graphs)
        assert s.get_option(ghom.OPT_GRAPHS) == graphs
        recs = []
        for _ in range(len(w["target"])):
            info = s.step()
            recs.append((info["newton_iters"], info["cg_iters_total"]) + s.averages())
        return recs, s.field(ghom.FIELD_F)


@pytest.mark.parametrize("prec", [ghom.FP64, ghom.FP32_SPLIT])
def test_single_problem_graph_replays_match_eager(prec):
    w = synth.workload_particles(n=32, count=8)
    w["target"] = w["target"][:3]
    ref, Fr = _single(w, prec, 0)
    got, Fg = _single(w, prec, 1)
    for a, b in zip(ref, got):
        assert a[0] == b[0] and a[1] == b[1]
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    assert np.array_equal(Fr, Fg)


def _batch(ws, graphs):
    with ghom.Batch(ws, precision=ghom.FP32_SPLIT) as b:
        b.set_tolerances(1e-10, 1e-11, 1e-5)
        b.set_option(ghom.OPT_GRAPHS, graphs)
        out = []
        for _ in range(3):
            infos = b.step()
            out.append([(i["newton_iters"], i["cg_iters_total"]) + b.averages(k) for k, i in enumerate(infos)])
        return out, [b.field(k) for k in range(len(ws))]


def test_batch_graph_replays_match_eager():
    ws = _problems()
    ref, Fr = _batch(ws, 0)
    got, Fg = _batch(ws, 1)
    for inc_a, inc_b in zip(ref, got):
        for a, b in zip(inc_a, inc_b):
            assert a[0] == b[0] and a[1] == b[1]
            assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    for a, b in zip(Fr, Fg):
        assert np.array_equal(a, b)


def test_large_solves_queued_in_two_parts_match_graph_replays():
    """From 2^21 voxels on, CG steps launched one by one are queued in two parts (the forward
    z pass ahead of the host's look at the stop flags, the other passes after it); graph
    replays queue whole steps.  Both give the same bits."""
    w = synth.workload_polycrystal(n=128, ngrains=64)
    w["target"] = w["target"][:2]
    ref, Fr = _single(w, ghom.FP32_SPLIT, 0)
    got, Fg = _single(w, ghom.FP32_SPLIT, 1)
    for a, b in zip(ref, got):
        print("  newton %d cg %d" % (a[0], a[1]), flush=True)
        assert a[0] == b[0] and a[1] == b[1]
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    assert np.array_equal(Fr, Fg)
