"""torch.autograd wrapper of the solver (HomogenizedResponse) against the oracle.

Forward: <F>, <P> at the end of the history equal the oracle's; backward: the gradient of a
loss on <F> with respect to the per-voxel stiffness scale equals the oracle's adjoint
gradient (itself pinned to finite differences in the CPU tests), and its directional value
matches central differences of the wrapped forward map.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ghom_oracle as go  # noqa: E402
from paper_1901_06531_amd import ghom, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _workload():
    shape = (12, 8, 16)
    g = np.random.default_rng(21)
    phase = (g.uniform(size=shape) < 0.3).astype(np.uint16)
    mask = synth.mask_uniaxial(0)
    F_end = np.eye(3)
    F_end[0, 0] = 1.04
    return dict(shape=shape, kind="nh", phase=phase, mu=[1.0, 8.0], lam=[2.0, 16.0], mask=mask,
                target=synth.history_mixed(mask, F_end.reshape(9), 2), newton_tol=1e-12, cg_tol=1e-13)


def test_homogenized_response_forward_and_gradient():
    w = _workload()
    s0 = synth.smooth_scale_field(w["shape"], 12, ell=0.2, lo=1.0, hi=2.5)
    o = go.Oracle(w["shape"])
    o.set_material_neohookean(w["phase"], w["mu"], w["lam"])
    o.set_stiffness_scale(s0)
    o.set_control(w["mask"])
    o.set_history(w["target"])
    o.set_tolerances(w["newton_tol"], w["cg_tol"])
    go.run_history(o, len(w["target"]))
    Fo, Po = o.averages(o.F)
    gF = np.array([0.3, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, -0.5])  # cotangent of <F>
    ref_grad = o.adjoint_grad_scale(gF)

    with ghom.Solver(w["shape"]) as solver:
        solver.setup(w)
        s = torch.tensor(s0, dtype=torch.float64, device="cuda", requires_grad=True)
        Fbar, Pbar = ghom.HomogenizedResponse.apply(s, solver)
        np.testing.assert_allclose(Fbar.detach().cpu().numpy(), Fo, rtol=0, atol=1e-11)
        np.testing.assert_allclose(Pbar.detach().cpu().numpy(), Po, rtol=0, atol=1e-11)
        # the <P> cotangent on the stress-controlled components contributes nothing
        fixed = torch.tensor(w["mask"].astype(np.float64), device="cuda")
        loss = (Fbar * torch.tensor(gF, device="cuda")).sum() + 7.0 * (Pbar * fixed).sum()
        loss.backward()
        got = s.grad.detach().cpu().numpy()
        assert got.shape == w["shape"]
        err = np.max(np.abs(got - ref_grad)) / np.max(np.abs(ref_grad))
        assert err < 1e-8, err

        # directional check through the forward map itself
        d = synth.smooth_scale_field(w["shape"], 13, ell=0.15, lo=-1.0, hi=1.0)
        eps = 1e-5
        with torch.no_grad():
            Jp = float(ghom.HomogenizedResponse.apply(torch.tensor(s0 * (1 + eps * d), device="cuda"), solver)[0]
                       .cpu().numpy() @ gF)
            Jm = float(ghom.HomogenizedResponse.apply(torch.tensor(s0 * (1 - eps * d), device="cuda"), solver)[0]
                       .cpu().numpy() @ gF)
        fd = (Jp - Jm) / 2.0
        ad = float(np.sum(got * eps * d * s0))
        assert abs(fd - ad) <= 1e-5 * abs(ad), (fd, ad)

        # a cotangent of <P> on a deformation-controlled component is refused
        s2 = torch.tensor(s0, dtype=torch.float64, device="cuda", requires_grad=True)
        Fb2, Pb2 = ghom.HomogenizedResponse.apply(s2, solver)
        free = int(np.flatnonzero(w["mask"] == 0)[0])
        with pytest.raises(NotImplementedError):
            Pb2[free].backward()
