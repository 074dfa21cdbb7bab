"""The allocation-free entry point ghom_apply_projection_static (G* of eq. 22 in a static
device array, no context): two calls in a row, the second on a smaller grid, each against
ghom_apply_projection of a context on the same input (bit for bit with the same x-pass
variant, else to 1e-12 of the largest entry) and against the oracle; a grid beyond the
array's capacity is refused."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ghom_oracle as go  # noqa: E402
from paper_1901_06531_amd import ghom, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _field(shape, seed):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.standard_normal((9,) + shape)).to("cuda")


@pytest.mark.parametrize("mask", ["mixed", "stress"])
def test_static_projection_matches_the_context_entry_point(mask):
    m = synth.mask_uniaxial(0) if mask == "mixed" else synth.mask_full_stress()
    for shape, lengths in (((64, 48, 32), (1.0, 1.5, 0.75)), ((12, 16, 9), (1.0, 1.0, 1.0))):
        say("static projection", shape, mask)
        v = _field(shape, 7)
        out = torch.empty_like(v)
        ghom.apply_projection_static(v, out, m, lengths)
        with ghom.Solver(shape, lengths) as s:
            s.set_option(ghom.OPT_XPROJ_F64, 1)  # the static path's x-pass variant
            s.set_control(m)
            ref = s.apply_projection(v)
            same = torch.equal(out, ref)
            s.set_option(ghom.OPT_XPROJ_F64, 0)
            tuned = s.apply_projection(v)
        assert same
        scale = float(tuned.abs().max())
        assert float((out - tuned).abs().max()) <= 1e-12 * scale
        o = go.apply_projection(v.cpu().numpy(), m, lengths)
        assert np.max(np.abs(out.cpu().numpy() - o)) <= 1e-12 * np.max(np.abs(o))


def test_static_projection_in_place_and_refusals():
    shape = (16, 16, 16)
    v = _field(shape, 3)
    keep = v.clone()
    out = torch.empty_like(v)
    ghom.apply_projection_static(v, out, synth.mask_full_strain())
    ghom.apply_projection_static(v, v, synth.mask_full_strain())  # in place
    assert torch.equal(v, out)
    # idempotent: G*(G*(a)) = G*(a)
    twice = torch.empty_like(v)
    ghom.apply_projection_static(out, twice, synth.mask_full_strain())
    assert float((twice - out).abs().max()) <= 1e-12 * float(keep.abs().max())
    big = torch.zeros((9, 96, 96, 96), dtype=torch.float64, device="cuda")
    with pytest.raises(ghom.GhomError, match="static scratch holds"):
        ghom.apply_projection_static(big, big, synth.mask_full_strain())
    with pytest.raises(ghom.GhomError, match="grid lengths"):
        ghom.apply_projection_static(torch.zeros((9, 10, 16, 16), dtype=torch.float64, device="cuda"),
                                     torch.zeros((9, 10, 16, 16), dtype=torch.float64, device="cuda"),
                                     synth.mask_full_strain())
