"""Pins of the oracle's rotation gauge under full stress control (Sec. 2.2, eq. 19-20).

Under full stress control F is fixed only up to the rigid rotations that leave the
prescribed stress unchanged; at a stress-free state the tangent annihilates all three of
them.  The gauge holds three deformation-gradient entries instead of three stress
components for uniaxial histories.  Pins: the rule and its components; the identity it
rests on (<P F^T> = <P> <F>^T at equilibrium, symmetric); the 40-increment triangle history
of the polycrystal through both stress-free crossings with a bounded Newton count and every
one of the nine prescribed stress components met; the rotation invariants of the gauged and
ungauged solutions agree where the ungauged one converges; loading along y and z.
"""

import numpy as np
import pytest

from oracle import ghom_oracle as go
from paper_1901_06531_amd import synth


def _poly(shape, ngrains, mask, target, ntol, ctol, gauge=True):
    w = synth.workload_polycrystal(n=shape[0], ngrains=ngrains)
    o = go.Oracle(w["shape"])
    o.set_material_svk(w["phase"], w["C"])
    o.set_rotation_gauge(gauge)
    o.set_control(mask)
    o.set_history(target)
    o.set_tolerances(ntol, ctol, 0.0, 60, 5000)
    return o


def _mat(v):
    return np.asarray(v, float).reshape(3, 3)


# ---------------------------------------------------------------- the rule -------------

def test_gauge_rule_and_components():
    full = synth.mask_full_stress()
    for a in range(3):
        T = synth.history_stress_triangle(0.02, 8, comp=4 * a)
        assert go.rotation_gauge_axis(full, T) == a
        comps = go.rotation_gauge_components(a)
        # strict lower triangle in the cyclic order (a, b, c), each off the diagonal
        b, c = (a + 1) % 3, (a + 2) % 3
        assert comps == [3 * b + a, 3 * c + a, 3 * c + b]
        m = go.effective_mask(full, T)
        assert list(np.flatnonzero(m == 0)) == sorted(comps)
    assert go.rotation_gauge_components(0) == [3, 6, 7]
    # the zero history takes axis 0
    assert go.rotation_gauge_axis(full, np.zeros((3, 9))) == 0
    # no gauge: a mixed mask, a stress with two normal components, a shear, a skew stress
    two = np.zeros((2, 9))
    two[:, 0], two[:, 4] = 0.01, 0.02
    shear = np.zeros((2, 9))
    shear[:, 1] = shear[:, 3] = 0.01
    for mask, T in [(synth.mask_uniaxial(0), synth.history_stress_triangle(0.02, 8)),
                    (full, two), (full, shear)]:
        assert go.rotation_gauge_axis(mask, T) is None
        np.testing.assert_array_equal(go.effective_mask(mask, T), np.asarray(mask, float))
    # off: the mask as set
    np.testing.assert_array_equal(go.effective_mask(full, synth.history_stress_triangle(0.02, 8), gauge=False),
                                  np.ones(9))


def test_oracle_applies_the_rule_in_any_set_up_order():
    T = synth.history_stress_triangle(0.02, 8, comp=8)
    o = go.Oracle((4, 4, 4))
    o.set_history(T)
    o.set_control(synth.mask_full_stress())
    assert o.gauge_axis == 2 and list(np.flatnonzero(o.mask == 0)) == sorted(go.rotation_gauge_components(2))
    o.set_rotation_gauge(False)
    assert o.gauge_axis is None and np.all(o.mask == 1)
    o.set_rotation_gauge(True)
    o.set_control(synth.mask_uniaxial(0))
    assert o.gauge_axis is None and np.array_equal(o.mask, synth.mask_uniaxial(0).astype(float))


# ---------------------------------------------------------------- the identity ---------

def test_mean_of_P_Ft_is_product_of_means_at_equilibrium():
    """<P F^T> = <P> <F>^T for a converged state (compatible F, divergence-free P), and it
    is symmetric because P F^T is symmetric at every voxel; the gauge's argument rests on
    both.  Checked on a mixed-control state (no gauge involved) and a gauged one."""
    shape = (8, 8, 8)
    T = synth.history_stress_triangle(0.02, 4)
    for mask in (synth.mask_uniaxial(0), synth.mask_full_stress()):
        target = T if mask.sum() == 9 else synth.history_mixed(mask, np.diag([1.02, 1, 1]).reshape(9), 4)
        o = _poly(shape, 16, mask, target, 1e-11, 1e-13)
        go.run_history(o, 2)
        P = o.stress().reshape(3, 3, -1)
        F = o.F.reshape(3, 3, -1)
        PFt = np.einsum("ikn,jkn->ij", P, F) / o.N
        Pm, Fm = P.mean(axis=2), F.mean(axis=2)
        np.testing.assert_allclose(PFt, Pm @ Fm.T, atol=1e-12)
        np.testing.assert_allclose(PFt, PFt.T, atol=1e-12)
        # and pointwise symmetry, the objectivity of the law
        pv = np.einsum("ikn,jkn->nij", P, F)
        assert np.max(np.abs(pv - pv.transpose(0, 2, 1))) < 1e-13


# ---------------------------------------------------------------- the history ----------

@pytest.mark.slow
def test_polycrystal_triangle_history_through_both_stress_free_crossings():
    """16^3, 64 grains, the benchmark's 40-increment history 0 -> +0.02 -> 0 -> -0.02 -> 0
    at the paper's tolerances (Sec. 4).  Without the gauge the first compressive increment
    after the stress-free state needs tens of Newton iterations, about a thousand CG
    iterations and several CG breakdowns, and ends rotated by about 8 degrees about x."""
    w = synth.workload_polycrystal(n=16, ngrains=64)
    o = _poly((16, 16, 16), 64, w["mask"], w["target"], 1e-6, 1e-8)
    assert o.gauge_axis == 0
    for k in range(40):
        b0 = o.cg_breakdowns
        rec = o.step()
        assert rec.newton_iters <= 4, (k + 1, rec.newton_iters)
        assert rec.cg_iters <= 120, (k + 1, rec.cg_iters)
        assert o.cg_breakdowns == b0
        # all nine prescribed components, the three released by the gauge included
        assert np.max(np.abs(rec.P_avg - w["target"][k])) < 2e-9, (k + 1, rec.P_avg - w["target"][k])
        F = _mat(rec.F_avg)
        assert F[1, 0] == 0.0 or abs(F[1, 0]) < 1e-15
        assert abs(F[2, 0]) < 1e-15 and abs(F[2, 1]) < 1e-15
        PF = _mat(rec.P_avg) @ F.T
        assert np.max(np.abs(PF - PF.T)) < 2e-9
    # back at zero stress: a rotation-free undeformed cell
    assert np.max(np.abs(o.F - go.EYE9[:, None, None, None])) < 1e-7


@pytest.mark.slow
def test_gauged_and_ungauged_solutions_share_their_rotation_invariants():
    """Increments 1-20 (the ungauged solve converges there): <P>, <F>^T <F> and F^T F per
    voxel agree; the ungauged solution drifts by a rotation."""
    w = synth.workload_polycrystal(n=16, ngrains=64)
    g = _poly((16, 16, 16), 64, w["mask"], w["target"], 1e-10, 1e-12, gauge=True)
    u = _poly((16, 16, 16), 64, w["mask"], w["target"], 1e-10, 1e-12, gauge=False)
    assert u.gauge_axis is None
    drift = 0.0
    for k in range(20):
        rg, ru = g.step(), u.step()
        np.testing.assert_allclose(rg.P_avg, ru.P_avg, rtol=0, atol=2e-12)
        Fg, Fu = _mat(rg.F_avg), _mat(ru.F_avg)
        np.testing.assert_allclose(Fg.T @ Fg, Fu.T @ Fu, rtol=0, atol=2e-12)
        Cg = np.einsum("kin,kjn->ijn", g.F.reshape(3, 3, -1), g.F.reshape(3, 3, -1))
        Cu = np.einsum("kin,kjn->ijn", u.F.reshape(3, 3, -1), u.F.reshape(3, 3, -1))
        assert np.max(np.abs(Cg - Cu)) < 5e-11
        drift = max(drift, abs(Fu[2, 1]))
    assert drift > 1e-6  # the ungauged solution is rotated about the load axis


@pytest.mark.parametrize("axis", [1, 2])
def test_gauge_along_y_and_z(axis):
    """8^3 polycrystal, triangle wave of P_aa over 8 increments (through zero twice): every
    prescribed component met, the gauge entries zero; the first increments agree with the
    ungauged solve on the rotation invariants."""
    T = synth.history_stress_triangle(0.02, 8, comp=4 * axis)
    mask = synth.mask_full_stress()
    g = _poly((8, 8, 8), 16, mask, T, 1e-10, 1e-12)
    u = _poly((8, 8, 8), 16, mask, T, 1e-10, 1e-12, gauge=False)
    assert g.gauge_axis == axis
    comps = go.rotation_gauge_components(axis)
    for k in range(8):
        rg = g.step()
        assert rg.newton_iters <= 5
        assert np.max(np.abs(rg.P_avg - T[k])) < 1e-11
        assert np.max(np.abs(rg.F_avg[comps])) < 1e-15
        if k < 3:
            ru = u.step()
            np.testing.assert_allclose(rg.P_avg, ru.P_avg, atol=1e-12)
            Fg, Fu = _mat(rg.F_avg), _mat(ru.F_avg)
            np.testing.assert_allclose(Fg.T @ Fg, Fu.T @ Fu, atol=1e-12)
