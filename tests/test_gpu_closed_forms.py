"""The HIP path against solutions that do not come from the oracle: the 0-D material point of a
homogeneous cell under uniaxial stress (two scalar equations solved by fsolve) and the exact
rank-one laminate (layer gradients a (x) e1 with traction continuity, fsolve), under strain and
mixed control, in FP64 and FP32-split.

Tolerances: FP64 within 1e-11 of the closed forms (the Newton tolerance 1e-11 and CG tolerance
1e-13 of the runs); FP32-split within 1e-9 (the float64 residual drives the solution to the
Newton tolerance; the float32 solves add a relative 1e-9 to the last correction)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1901_06531_amd import ghom, synth  # noqa: E402

from test_oracle_solver import CASE1, _laminate, _laminate_exact, _uniaxial_0d  # noqa: E402

pytestmark = pytest.mark.gpu

PRECS = [(ghom.FP64, 1e-11), (ghom.FP32_SPLIT, 1e-9)]


def _solver(shape, phase, mu, lam, mask, target, prec):
    s = ghom.Solver(shape, precision=prec)
    s.set_material_neohookean(phase, np.asarray(mu, float), np.asarray(lam, float))
    s.set_control(mask)
    s.set_history(target)
    s.set_tolerances(1e-11, 1e-13, 0.0 if prec == ghom.FP64 else 1e-5)
    return s


@pytest.mark.parametrize("prec,tol", PRECS)
def test_homogeneous_uniaxial_stress_matches_material_point(prec, tol):
    print("homogeneous cell, uniaxial P11 = 0.1, precision", prec, flush=True)
    a, b = _uniaxial_0d(1.0, 2.0, 0.1)
    shape = (4, 4, 4)
    P_end = np.zeros(9)
    P_end[0] = 0.1
    with _solver(shape, np.zeros(shape, np.uint16), [1.0], [2.0], synth.mask_full_stress(),
                 synth.history_stress_ramp(P_end, 2), prec) as s:
        for _ in range(2):
            s.step()
        F, P = s.averages()
        Ff = s.field(ghom.FIELD_F)
    np.testing.assert_allclose(F, [a, 0, 0, 0, b, 0, 0, 0, b], rtol=0, atol=tol)
    np.testing.assert_allclose(P, P_end, rtol=0, atol=tol)
    assert np.max(np.abs(Ff - F[:, None, None, None])) < tol  # the field stays uniform


@pytest.mark.parametrize("prec,tol", PRECS)
@pytest.mark.parametrize("thick", [2, 6])
def test_laminate_strain_control_matches_exact_solution(prec, tol, thick):
    print("laminate, strain control, thickness", thick, "precision", prec, flush=True)
    nx = 8
    g = np.random.default_rng(thick)
    Fbar = np.eye(3) + 0.08 * g.standard_normal((3, 3))
    with _solver((nx, 4, 4), _laminate(nx, thick), [1.0, 10.0], [2.0, 20.0], synth.mask_full_strain(),
                 Fbar.reshape(1, 9), prec) as s:
        s.step()
        F = s.field(ghom.FIELD_F).reshape(3, 3, nx, 4, 4)
    FA, FB = _laminate_exact(Fbar, thick / nx, [(10.0, 20.0), (1.0, 2.0)])
    assert np.max(np.abs(F[:, :, :thick] - FA[:, :, None, None, None])) < tol
    assert np.max(np.abs(F[:, :, thick:] - FB[:, :, None, None, None])) < tol


@pytest.mark.parametrize("prec,tol", PRECS)
def test_laminate_mixed_control_matches_exact_solution(prec, tol):
    print("laminate, mixed control (paper case 1), precision", prec, flush=True)
    nx, thick = 8, 2
    F_end = np.eye(3)
    F_end[0, 0] = 1.1
    target = synth.history_mixed(CASE1, F_end.reshape(9), 2)
    with _solver((nx, 4, 4), _laminate(nx, thick), [1.0, 10.0], [2.0, 20.0], CASE1, target, prec) as s:
        for _ in range(2):
            s.step()
        F = s.field(ghom.FIELD_F).reshape(3, 3, nx, 4, 4)
        Fa, Pa = s.averages()
    FA, FB = _laminate_exact(F_end, thick / nx, [(10.0, 20.0), (1.0, 2.0)], mask=CASE1, Pbar=np.zeros(9))
    assert np.max(np.abs(F[:, :, :thick] - FA[:, :, None, None, None])) < tol
    assert np.max(np.abs(F[:, :, thick:] - FB[:, :, None, None, None])) < tol
    assert np.max(np.abs(Pa[CASE1 > 0])) < tol  # the stress-controlled components are met


@pytest.mark.parametrize("prec,tol", PRECS)
def test_homogeneous_cubic_svk_uniaxial_stress_matches_material_point(prec, tol):
    """Unrotated cubic Saint Venant-Kirchhoff cell under P11 = p, every other P component 0:
    F = diag(a, b, b) with S22 = 0 (E22 = -C12 E11 / (C11 + C12)) and a S11 = p, i.e.
    a (a^2 - 1) / 2 (C11 - 2 C12^2 / (C11 + C12)) = p, solved as a scalar cubic."""
    print("homogeneous cubic SVK cell, uniaxial P11 = 0.05, precision", prec, flush=True)
    C11, C12, C44, p = 1.7, 1.2, 0.75, 0.05
    Y = C11 - 2 * C12 ** 2 / (C11 + C12)
    roots = np.roots([Y / 2, 0.0, -Y / 2, -p])
    a = float(min((r.real for r in roots if abs(r.imag) < 1e-12 and r.real > 0), key=lambda r: abs(r - 1)))
    E11 = (a * a - 1) / 2
    b = np.sqrt(1 + 2 * (-C12 * E11 / (C11 + C12)))
    shape = (4, 4, 4)
    P_end = np.zeros(9)
    P_end[0] = p
    with ghom.Solver(shape, precision=prec) as s:
        s.set_material_svk(np.zeros(shape, np.uint16), synth.cubic_C(C11, C12, C44).reshape(1, 81))
        s.set_control(synth.mask_full_stress())
        s.set_history(synth.history_stress_ramp(P_end, 2))
        s.set_tolerances(1e-11, 1e-13, 0.0 if prec == ghom.FP64 else 1e-5)
        for _ in range(2):
            s.step()
        F, P = s.averages()
    np.testing.assert_allclose(F, [a, 0, 0, 0, b, 0, 0, 0, b], rtol=0, atol=tol)
    np.testing.assert_allclose(P, P_end, rtol=0, atol=tol)
