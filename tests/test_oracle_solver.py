"""Pins of the oracle's Newton / conjugate-gradient solver under strain, stress and mixed
control (Sec. 2.1-2.3, Sec. 3.1, Sec. 4).

Pins: the 0-D material point (homogeneous cell), the exact rank-one laminate, Hill-Mandel,
prescribed components met, the paper's claim that the three control types of Sec. 3.1
reach the same end point, the symmetry of a centred inclusion, the adjoint gradient against
finite differences, and the failure modes.
"""

import numpy as np
import pytest
from scipy.optimize import fsolve

from oracle import ghom_oracle as go
from paper_1901_06531_amd import synth

CASE1 = synth.mask_uniaxial(0)  # the paper's case (1), eq. (23)


def _nh(shape, phase, mu, lam, mask, target, ntol=1e-11, ctol=1e-13, scale=None):
    o = go.Oracle(shape)
    o.set_material_neohookean(phase, mu, lam)
    if scale is not None:
        o.set_stiffness_scale(scale)
    o.set_control(mask)
    o.set_history(target)
    o.set_tolerances(ntol, ctol)
    return o


def _nh_P(F, mu, lam):
    FiT = np.linalg.inv(F).T
    return mu * (F - FiT) + lam * np.log(np.linalg.det(F)) * FiT


# ---------------------------------------------------------------- homogeneous cell ----

def _uniaxial_0d(mu, lam, p):
    """F = diag(a, b, b) with P11 = p, P22 = P33 = 0 for the neo-Hookean law (scalar
    equations solved by fsolve, independent of the field solver)."""
    def eqs(v):
        a, b = v
        lnJ = np.log(a * b * b)
        return [mu * (a - 1 / a) + lam * lnJ / a - p, mu * (b - 1 / b) + lam * lnJ / b]
    a, b = fsolve(eqs, [1.0, 1.0], xtol=1e-14)
    return a, b


@pytest.mark.parametrize("mu,lam,a_ref,b_ref", [
    (1.0, 2.0, 1.038651158152040, 0.987385999756615),
    (10.0, 20.0, 1.003761346734352, 0.998748831153567),
])
def test_homogeneous_uniaxial_stress_matches_material_point(mu, lam, a_ref, b_ref):
    a, b = _uniaxial_0d(mu, lam, 0.1)
    assert abs(a - a_ref) < 1e-13 and abs(b - b_ref) < 1e-13
    shape = (4, 4, 4)
    P_end = np.zeros(9)
    P_end[0] = 0.1
    o = _nh(shape, np.zeros(shape, np.uint16), [mu], [lam], synth.mask_full_stress(),
            synth.history_stress_ramp(P_end, 2))
    recs = go.run_history(o)
    np.testing.assert_allclose(recs[-1].F_avg, [a, 0, 0, 0, b, 0, 0, 0, b], atol=1e-12)
    # the field stays uniform
    assert np.max(np.abs(o.F - recs[-1].F_avg[:, None, None, None])) < 1e-14


def test_homogeneous_strain_control_needs_no_cg():
    shape = (4, 4, 4)
    F_end = np.eye(3) + 0.05 * np.random.default_rng(0).standard_normal((3, 3))
    o = _nh(shape, np.zeros(shape, np.uint16), [1.0], [2.0], synth.mask_full_strain(),
            synth.history_strain_ramp(F_end.reshape(9), 3))
    for rec in go.run_history(o):
        assert rec.cg_iters == 0 and rec.newton_iters == 1
    np.testing.assert_allclose(o.averages()[1], _nh_P(F_end, 1.0, 2.0).reshape(9), atol=1e-14)


# ---------------------------------------------------------------- rank-one laminate ----

def _laminate(nx, thick):
    phase = np.zeros((nx, 4, 4), np.uint16)
    phase[:thick] = 1
    return phase


def _laminate_exact(Fbar, f, mats, mask=None, Pbar=None):
    """Layers normal to e1 with volume fractions (f, 1-f):
    F_A = Fbar + (1-f) a (x) e1, F_B = Fbar - f a (x) e1, traction continuity P_A e1 = P_B e1.
    With a mask, the mask-1 entries of Fbar are unknown too and <P> = Pbar there."""
    (muA, lamA), (muB, lamB) = mats
    free = np.zeros(9, bool) if mask is None else np.asarray(mask) > 0

    def split(v):
        Fb = Fbar.reshape(9).copy()
        Fb[free] = v[3:]
        Fb = Fb.reshape(3, 3)
        a = v[:3]
        FA = Fb + (1 - f) * np.outer(a, [1, 0, 0])
        FB = Fb - f * np.outer(a, [1, 0, 0])
        return FA, FB

    def eqs(v):
        FA, FB = split(v)
        PA, PB = _nh_P(FA, muA, lamA), _nh_P(FB, muB, lamB)
        res = list(PA[:, 0] - PB[:, 0])
        if free.any():
            Pm = (f * PA + (1 - f) * PB).reshape(9)
            res += list(Pm[free] - np.asarray(Pbar).reshape(9)[free])
        return res

    v0 = np.concatenate([np.zeros(3), Fbar.reshape(9)[free]])
    v = fsolve(eqs, v0, xtol=1e-14)
    assert np.max(np.abs(eqs(v))) < 1e-13
    return split(v)


@pytest.mark.parametrize("thick", [2, 4, 6])
def test_laminate_strain_control_matches_exact_solution(thick):
    nx = 8
    mats = [(10.0, 20.0), (1.0, 2.0)]  # phase 1 (layer A) stiff, phase 0 soft
    g = np.random.default_rng(thick)
    Fbar = np.eye(3) + 0.08 * g.standard_normal((3, 3))
    o = _nh((nx, 4, 4), _laminate(nx, thick), [1.0, 10.0], [2.0, 20.0],
            synth.mask_full_strain(), Fbar.reshape(1, 9))
    o.step()
    FA, FB = _laminate_exact(Fbar, thick / nx, mats)
    F = o.F.reshape(3, 3, nx, 4, 4)
    np.testing.assert_allclose(F[:, :, :thick], FA[:, :, None, None, None] * np.ones((1, 1, thick, 4, 4)), atol=1e-11)
    np.testing.assert_allclose(F[:, :, thick:], FB[:, :, None, None, None] * np.ones((1, 1, nx - thick, 4, 4)), atol=1e-11)


def test_laminate_mixed_control_matches_exact_solution():
    nx, thick = 8, 2
    mats = [(10.0, 20.0), (1.0, 2.0)]
    F_end = np.eye(3)
    F_end[0, 0] = 1.1
    target = synth.history_mixed(CASE1, F_end.reshape(9), 2)
    o = _nh((nx, 4, 4), _laminate(nx, thick), [1.0, 10.0], [2.0, 20.0], CASE1, target)
    go.run_history(o)
    FA, FB = _laminate_exact(F_end, thick / nx, mats, mask=CASE1, Pbar=np.zeros(9))
    F = o.F.reshape(3, 3, nx, 4, 4)
    np.testing.assert_allclose(F[:, :, 0, 0, 0], FA, atol=1e-11)
    np.testing.assert_allclose(F[:, :, -1, 0, 0], FB, atol=1e-11)


def test_laminate_small_strain_harmonic_mean():
    """Small strain along the lamination normal: the effective normal modulus is the
    harmonic mean of (lam + 2 mu) (Reuss bound is exact for a laminate)."""
    nx, thick = 8, 4
    eps = 1e-7
    F_end = np.eye(3)
    F_end[0, 0] += eps
    o = _nh((nx, 4, 4), _laminate(nx, thick), [1.0, 10.0], [2.0, 20.0],
            synth.mask_full_strain(), F_end.reshape(1, 9))
    o.step()
    M = 1.0 / (0.5 / 4.0 + 0.5 / 40.0)
    assert abs(o.averages()[1][0] / eps - M) / M < 1e-5


# ---------------------------------------------------------------- equilibrium pins -----

def _two_phase(shape, seed):
    g = np.random.default_rng(seed)
    return (g.uniform(size=shape) < 0.3).astype(np.uint16)


def test_hill_mandel_and_prescribed_components():
    shape = (8, 8, 8)
    F_end = np.eye(3)
    F_end[0, 0] = 1.08
    target = synth.history_mixed(CASE1, F_end.reshape(9), 2)
    o = _nh(shape, _two_phase(shape, 7), [1.0, 10.0], [2.0, 20.0], CASE1, target)
    go.run_history(o)
    Favg, Pavg = o.averages()
    P = o.stress()
    hm = np.mean(np.sum(P * o.F, axis=0))
    assert abs(hm - Pavg @ Favg) < 1e-10
    np.testing.assert_allclose(Favg[CASE1 == 0], F_end.reshape(9)[CASE1 == 0], atol=1e-14)
    np.testing.assert_allclose(Pavg[CASE1 == 1], 0.0, atol=1e-11)


def test_centred_sphere_symmetry():
    shape = (8, 8, 8)
    P_end = np.zeros(9)
    P_end[0] = 0.1
    o = _nh(shape, synth.centered_sphere(shape, 0.25), [1.0, 10.0], [2.0, 20.0],
            synth.mask_full_stress(), synth.history_stress_ramp(P_end, 2))
    go.run_history(o)
    Favg, Pavg = o.averages()
    off = [1, 2, 3, 5, 6, 7]
    assert np.max(np.abs(Favg[off])) < 1e-12
    assert abs(Favg[4] - Favg[8]) < 1e-12
    np.testing.assert_allclose(Pavg, P_end, atol=1e-11)


def test_three_control_types_reach_the_same_end_point():
    """Sec. 3.1: case (1) mixed, case (2) full stress ramp to P_end(1) and case (3) full
    strain ramp to F_end(1) end at the same macroscopic and microscopic state; only case
    (3) develops transverse stress along the way."""
    shape = (8, 8, 8)
    phase = synth.centered_sphere(shape, 0.3)
    mu, lam = [1.0, 10.0], [2.0, 20.0]
    F_end = np.eye(3)
    F_end[0, 0] = 1.06
    n = 3
    o1 = _nh(shape, phase, mu, lam, CASE1, synth.history_mixed(CASE1, F_end.reshape(9), n))
    r1 = go.run_history(o1)
    F1, P1 = o1.averages()
    o2 = _nh(shape, phase, mu, lam, synth.mask_full_stress(), synth.history_stress_ramp(P1, n))
    go.run_history(o2)
    o3 = _nh(shape, phase, mu, lam, synth.mask_full_strain(), synth.history_strain_ramp(F1, n))
    r3 = go.run_history(o3)
    for o in (o2, o3):
        F, P = o.averages()
        np.testing.assert_allclose(F, F1, atol=1e-10)
        np.testing.assert_allclose(P, P1, atol=1e-10)
        np.testing.assert_allclose(o.F, o1.F, atol=1e-9)
    # transverse stress: zero under mixed control at every increment, nonzero under strain
    assert max(abs(r.P_avg[4]) for r in r1) < 1e-11
    assert abs(r3[0].P_avg[4]) > 1e-4


# ---------------------------------------------------------------- adjoint --------------

@pytest.mark.parametrize("stress_control", [False, True])
def test_adjoint_gradient_matches_finite_differences(stress_control):
    """dJ/ds(x) from the adjoint solve against central differences of re-solved states
    (J = <F>_22 under the paper's case (1) mask, J = <F>_11 under full stress control)."""
    shape = (6, 6, 6)
    g = np.random.default_rng(8)
    phase = _two_phase(shape, 9)
    s = synth.smooth_scale_field(shape, 10, ell=0.2, lo=1.0, hi=3.0)
    a = np.zeros(9)
    if stress_control:
        mask = synth.mask_full_stress()
        P_end = np.zeros(9)
        P_end[0] = 0.05
        target = synth.history_stress_ramp(P_end, 2)
        a[0] = 1.0
        tol, ctol, rel = 1e-12, 1e-12, 1e-4
    else:
        mask = CASE1
        F_end = np.eye(3)
        F_end[0, 0] = 1.05
        target = synth.history_mixed(mask, F_end.reshape(9), 2)
        a[4] = 1.0
        tol, ctol, rel = 1e-13, 1e-14, 1e-6
    o = _nh(shape, phase, [1.0, 10.0], [2.0, 20.0], mask, target, tol, ctol, s)
    go.run_history(o)
    grad = o.adjoint_grad_scale(a).reshape(-1)
    F0 = o.F.copy()
    Pbar = o.target_stress()
    for v in g.choice(o.N, 5, replace=False):
        h = 1e-4 * s.reshape(-1)[v]
        J = []
        for sign in (+1, -1):
            sp = s.reshape(-1).copy()
            sp[v] += sign * h
            o2 = _nh(shape, phase, [1.0, 10.0], [2.0, 20.0], mask, o.target, tol, ctol, sp)
            o2.set_state(F0, o.k)
            o2.newton(Pbar)
            J.append(o2.averages()[0] @ a)
        fd = (J[0] - J[1]) / (2 * h)
        assert abs(fd - grad[v]) <= rel * abs(grad[v]) + 1e-12


def test_adjoint_scale_identity_and_controlled_components():
    """sum_x s(x) dJ/ds(x) equals the derivative of J under a uniform scaling s -> c s at
    c = 1 (chain rule); and J on a deformation-controlled component has zero gradient."""
    shape = (6, 6, 6)
    phase = _two_phase(shape, 3)
    s = synth.smooth_scale_field(shape, 4, ell=0.2, lo=1.0, hi=2.0)
    F_end = np.eye(3)
    F_end[0, 0] = 1.05
    o = _nh(shape, phase, [1.0, 10.0], [2.0, 20.0], CASE1,
            synth.history_mixed(CASE1, F_end.reshape(9), 1), 1e-13, 1e-15, s)
    go.run_history(o)
    a = np.zeros(9)
    a[0] = 1.0  # F11 is prescribed: J cannot depend on s
    assert np.max(np.abs(o.adjoint_grad_scale(a))) < 1e-14
    a = np.zeros(9)
    a[4] = 1.0  # F22 is free
    grad = o.adjoint_grad_scale(a)
    J = []
    for c in (1 + 1e-4, 1 - 1e-4):
        o2 = _nh(shape, phase, [1.0, 10.0], [2.0, 20.0], CASE1, o.target, 1e-13, 1e-15, c * s)
        o2.set_state(o.F, o.k)
        o2.newton(o.target_stress())
        J.append(o2.averages()[0][4])
    fd = (J[0] - J[1]) / 2e-4
    assert abs(np.sum(s * grad) - fd) < 1e-7 * abs(fd) + 1e-12


# ---------------------------------------------------------------- failure modes --------

def test_cg_iteration_cap():
    shape = (6, 6, 6)
    P_end = np.zeros(9)
    P_end[0] = 0.1
    o = _nh(shape, _two_phase(shape, 1), [1.0, 10.0], [2.0, 20.0], synth.mask_full_stress(),
            synth.history_stress_ramp(P_end, 1))
    o.max_cg = 1
    with pytest.raises(go.NotConvergedError):
        o.step()


def test_indefinite_tangent_breaks_cg():
    shape = (4, 4, 4)
    P_end = np.zeros(9)
    P_end[0] = 0.1
    o = _nh(shape, np.zeros(shape, np.uint16), [-1.0], [0.0], synth.mask_full_stress(),
            synth.history_stress_ramp(P_end, 1))
    with pytest.raises(go.BreakdownError):
        o.step()


def test_nonsymmetric_stress_at_identity_breaks_cg():
    """At F = I the tangent only sees sym(dF); a skew part in P-bar cannot be met."""
    shape = (4, 4, 4)
    P_end = np.zeros(9)
    P_end[1] = 0.01
    o = _nh(shape, np.zeros(shape, np.uint16), [1.0], [2.0], synth.mask_full_stress(),
            synth.history_stress_ramp(P_end, 1))
    o.max_newton = 8
    with pytest.raises(go.OracleError):
        o.step()
    assert o.cg_breakdowns >= 1


def test_inverted_deformation_is_a_domain_error():
    shape = (4, 4, 4)
    F_end = np.eye(3)
    F_end[0, 0] = -0.5
    o = _nh(shape, np.zeros(shape, np.uint16), [1.0], [2.0], synth.mask_full_strain(),
            F_end.reshape(1, 9))
    with pytest.raises(go.DomainError):
        o.step()


# ---------------------------------------------------------------- stop rules (Sec. 4) --

def test_voxel_averaged_l2_norm():
    """rms is the voxel-averaged L2 norm of Sec. 4: sqrt of the mean over voxels of the
    squared Frobenius norm.  A uniform field of norm a gives a; a single voxel of norm a
    gives a / sqrt(N) (the mean of the norms would give a / N, the plain 2-norm a)."""
    shape = (4, 6, 5)
    N = 120
    o = go.Oracle(shape)
    rng = np.random.default_rng(7)
    t = rng.standard_normal(9)
    a = 0.37
    t *= a / np.linalg.norm(t)
    uniform = np.broadcast_to(t[:, None, None, None], (9,) + shape).copy()
    assert abs(o.rms(uniform) - a) < 1e-15
    single = np.zeros((9,) + shape)
    single[:, 2, 3, 1] = t
    assert abs(o.rms(single) - a / np.sqrt(N)) < 1e-16
    # two voxels of norms 3 and 4: sqrt((9 + 16) / N)
    two = np.zeros((9,) + shape)
    two[0, 0, 0, 0], two[4, 1, 2, 3] = 3.0, 4.0
    assert abs(o.rms(two) - 5.0 / np.sqrt(N)) < 1e-15


def test_newton_criterion():
    """max over voxels of |dF(x)| divided by |<F>| (Frobenius norms, Sec. 4)."""
    shape = (3, 4, 5)
    dF = np.zeros((9,) + shape)
    dF[1, 2, 3, 4] = 3.0
    dF[5, 2, 3, 4] = 4.0       # that voxel has norm 5
    dF[0, 0, 0, 0] = 4.5       # a smaller one elsewhere
    I9 = go.EYE9
    assert abs(go.Oracle.newton_criterion(dF, I9) - 5.0 / np.sqrt(3.0)) < 1e-15
    assert abs(go.Oracle.newton_criterion(dF, 2.0 * I9) - 2.5 / np.sqrt(3.0)) < 1e-15
    Fbar = np.array([1.1, 0.2, 0, 0, 0.9, 0, 0.3, 0, 1.0])
    assert abs(go.Oracle.newton_criterion(dF, Fbar) - 5.0 / np.linalg.norm(Fbar)) < 1e-15
    # a uniform correction: its norm over |<F>|
    u = np.broadcast_to(np.arange(9.0)[:, None, None, None], (9,) + shape)
    assert abs(go.Oracle.newton_criterion(u, I9) - np.sqrt(204.0) / np.sqrt(3.0)) < 1e-13


def test_cg_stops_on_the_voxel_averaged_residual():
    """The CG solve returns once rms(b - A x) is below the threshold and not before: the
    true residual of the returned iterate is below cg_tol, the iterate of one iteration
    less is above it."""
    shape = (8, 8, 8)
    # mixed control (the paper's case (1)): the rotations are fixed, A is positive definite
    o = _nh(shape, _two_phase(shape, 3), [1.0, 10.0], [2.0, 20.0], CASE1,
            synth.history_mixed(CASE1, np.diag([1.05, 1, 1]).reshape(9), 1))
    o.F = o.F + 0.02 * np.random.default_rng(1).standard_normal(o.F.shape)
    b = o.residual(o.stress(), np.zeros(9))
    o.cg_tol = 1e-3 * o.rms(b)
    x, its = o.conjugate_gradient(b)
    assert its >= 2 and o.cg_breakdowns == 0
    assert o.rms(b - o.apply_operator(x)) <= o.cg_tol * (1 + 1e-8)
    o.max_cg = its - 1
    with pytest.raises(go.NotConvergedError):
        o.conjugate_gradient(b)


def test_newton_records_the_criterion_of_its_last_correction():
    shape = (8, 8, 8)
    o = _nh(shape, _two_phase(shape, 4), [1.0, 10.0], [2.0, 20.0], synth.mask_full_stress(),
            synth.history_stress_ramp(np.diag([0.05, 0, 0]).reshape(9), 1), ntol=1e-6, ctol=1e-9)
    F0 = o.F.copy()
    o.max_newton = 1
    with pytest.raises(go.NotConvergedError):
        o.step()
    dF = o.F - F0
    expect = go.Oracle.newton_criterion(dF, o.F.reshape(9, -1).mean(axis=1))
    o2 = _nh(shape, _two_phase(shape, 4), [1.0, 10.0], [2.0, 20.0], synth.mask_full_stress(),
             synth.history_stress_ramp(np.diag([0.05, 0, 0]).reshape(9), 1), ntol=expect * 1.0000001, ctol=1e-9)
    rec = o2.step()
    assert rec.newton_iters == 1 and abs(rec.crit - expect) < 1e-15 * max(1.0, expect)


def test_cg_stall_returns_the_iterate():
    """An operator whose output carries a relative error of 1e-6 (a residual floor) with a
    threshold far below that floor: the solve stops after the stall window instead of
    running to max_cg, returns its iterate and counts the stall."""
    shape = (6, 6, 6)
    o = _nh(shape, _two_phase(shape, 5), [1.0, 10.0], [2.0, 20.0], CASE1,
            synth.history_mixed(CASE1, np.diag([1.05, 1, 1]).reshape(9), 1))
    exact = o.apply_operator
    rng = np.random.default_rng(11)

    def noisy(v, F9=None):
        out = exact(v, F9)
        return out + 1e-6 * np.linalg.norm(out) / np.sqrt(out.size) * rng.standard_normal(out.shape)

    o.apply_operator = noisy
    b = o.residual(o.stress(), np.zeros(9)) + go.apply_projection(
        0.01 * np.random.default_rng(2).standard_normal(o.F.shape), o.mask)
    o.cg_tol = 1e-12 * o.rms(b)
    o.max_cg = 1000
    x, its = o.conjugate_gradient(b)
    assert o.cg_stalls == 1 and o.cg_breakdowns == 0
    assert o.cg_stall_window < its < 200
    # the iterate is a useful one: the true residual is down by two orders at least (the
    # noise of every operator output accumulates in the recursive residual)
    assert o.rms(b - exact(x)) < 1e-2 * o.rms(b)
