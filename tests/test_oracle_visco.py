"""Pins of the oracle's viscoelastic law (path- and rate-dependent, internal variables).

The law (oracle.visco_update): S = Cinf : E + Q with dQ/dt + Q/tau = C1 : dE/dt, integrated
exactly over increments in which E is linear in time.  Pinned by
  * the relaxation of a homogeneous cell after a strain ramp against the convolution
    integral Q(t) = int_0^t exp(-(t-s)/tau) C1 : dE/ds ds evaluated by quadrature;
  * its limits: tau -> infinity is Saint Venant-Kirchhoff with Cinf + C1, tau -> 0 is
    Saint Venant-Kirchhoff with Cinf (both on a heterogeneous cell under mixed control,
    against the oracle's own SVK law);
  * central differences of P for the algorithmic tangent;
  * Hill-Mandel along a heterogeneous relaxation history, and the long-time limit of
    creep under a held stress (the relaxed, Cinf-only equilibrium).
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import ghom_oracle as go
from paper_1901_06531_amd import synth


def _iso(mu, lam):
    return synth.isotropic_C(mu, lam).reshape(81)


def _two_phase(shape, seed=3):
    centers, radii = synth.rsa_spheres(2, 0.15, 0.2, seed, target_vf=0.15)
    return synth.spheres_phase(shape, centers, radii)


def test_relaxation_after_strain_ramp_matches_convolution_integral():
    shape = (4, 4, 4)
    mu_inf, lam_inf, mu1, lam1, tau, dt = 1.0, 1.5, 2.0, 3.0, 0.7, 0.25
    o = go.Oracle(shape)
    o.set_material_visco(np.zeros(shape, np.uint16), [_iso(mu_inf, lam_inf)], [_iso(mu1, lam1)], [tau])
    o.set_time_step(dt)
    o.set_control(synth.mask_full_strain())
    F1 = np.array([[1.05, 0.02, 0.0], [0.01, 0.98, 0.0], [0.0, 0.0, 1.01]])
    n = 6
    o.set_history(np.stack([F1.reshape(9)] * n))  # ramp over increment 1, then held
    o.set_tolerances(1e-12, 1e-13)
    recs = go.run_history(o)
    E1 = 0.5 * (F1.T @ F1 - np.eye(3))
    C1 = synth.isotropic_C(mu1, lam1)
    Cinf = synth.isotropic_C(mu_inf, lam_inf)
    C1E = np.einsum("ijkl,kl->ij", C1, E1)
    for k, rec in enumerate(recs, start=1):
        t = k * dt
        # dE/ds = E1 / dt on [0, dt], 0 afterwards
        q, _ = integrate.quad(lambda s_: math.exp(-(t - s_) / tau) / dt, 0.0, dt, epsabs=1e-14, epsrel=1e-13)
        S = np.einsum("ijkl,kl->ij", Cinf, E1) + q * C1E
        np.testing.assert_allclose(rec.P_avg, (F1 @ S).reshape(9), rtol=0, atol=1e-13)
        assert rec.cg_iters == 0  # homogeneous under strain control: nothing to solve


@pytest.mark.parametrize("limit", ["slow", "fast"])
def test_time_scale_limits_reduce_to_saint_venant_kirchhoff(limit):
    shape = (8, 8, 8)
    phase = _two_phase(shape)
    Cinf = np.stack([_iso(1.0, 2.0), _iso(8.0, 12.0)])
    C1 = np.stack([_iso(0.5, 0.7), _iso(3.0, 2.0)])
    mask = synth.mask_uniaxial(0)
    F_end = np.eye(3)
    F_end[0, 0] = 1.04
    target = synth.history_mixed(mask, F_end.reshape(9), 3)
    tau = [1e300, 1e300] if limit == "slow" else [1e-300, 1e-300]
    o = go.Oracle(shape)
    o.set_material_visco(phase, Cinf, C1, tau)
    o.set_control(mask)
    o.set_history(target)
    o.set_tolerances(1e-12, 1e-13)
    got = go.run_history(o)
    r = go.Oracle(shape)
    r.set_material_svk(phase, Cinf + C1 if limit == "slow" else Cinf)
    r.set_control(mask)
    r.set_history(target)
    r.set_tolerances(1e-12, 1e-13)
    ref = go.run_history(r)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a.P_avg, b.P_avg, rtol=0, atol=1e-12)
        np.testing.assert_allclose(a.F_avg, b.F_avg, rtol=0, atol=1e-12)


def test_algorithmic_tangent_matches_finite_differences():
    g = np.random.default_rng(4)
    n = 5
    F = np.eye(3) + 0.1 * g.standard_normal((n, 3, 3))
    E_n = 0.05 * g.standard_normal((n, 3, 3))
    E_n = 0.5 * (E_n + E_n.transpose(0, 2, 1))
    Q_n = 0.2 * g.standard_normal((n, 3, 3))
    Q_n = 0.5 * (Q_n + Q_n.transpose(0, 2, 1))
    Cinf = np.stack([synth.rotate_C(synth.cubic_C(1.7, 1.2, 0.75), synth.haar_rotations(1, i)[0]) for i in range(n)])
    C1 = np.stack([synth.isotropic_C(0.8 + 0.1 * i, 1.1) for i in range(n)])
    a, b = go.visco_factors(0.3, np.linspace(0.2, 2.0, n))
    dF = g.standard_normal((n, 3, 3))
    h = 1e-6
    fd = (go.visco_stress(F + h * dF, E_n, Q_n, Cinf, C1, a, b) -
          go.visco_stress(F - h * dF, E_n, Q_n, Cinf, C1, a, b)) / (2 * h)
    an = go.visco_tangent_apply(F, E_n, Q_n, Cinf, C1, a, b, dF)
    assert np.max(np.abs(fd - an)) < 1e-8 * np.max(np.abs(an))


def test_hill_mandel_along_relaxation_and_creep_to_the_relaxed_state():
    shape = (8, 8, 8)
    phase = _two_phase(shape, seed=5)
    Cinf = np.stack([_iso(1.0, 2.0), _iso(8.0, 12.0)])
    C1 = np.stack([_iso(1.0, 1.0), _iso(4.0, 4.0)])
    tau = [0.5, 2.0]
    mask = synth.mask_full_stress()
    P_end = np.zeros(9)
    P_end[0] = 0.05
    nramp, nhold = 2, 12
    target = np.concatenate([synth.history_stress_ramp(P_end, nramp), np.stack([P_end] * nhold)])
    o = go.Oracle(shape)
    o.set_material_visco(phase, Cinf, C1, tau)
    o.set_time_step(1.0)
    o.set_control(mask)
    o.set_history(target)
    o.set_tolerances(1e-12, 1e-13)
    recs = []
    F11 = []
    for _ in range(len(target)):
        rec = o.step()
        recs.append(rec)
        hm = float(np.mean(np.sum(o.P_last * o.F, axis=0)))
        assert abs(hm - float(rec.P_avg @ rec.F_avg)) < 1e-11
        F11.append(rec.F_avg[0])
    # creep under the held stress: <F>_11 grows monotonically toward the relaxed value
    hold = np.array(F11[nramp - 1:])
    assert np.all(np.diff(hold) > 0)
    # long hold (dt >> tau): the overstress has decayed; the state is the Cinf equilibrium
    o.set_time_step(1e6)
    o.set_history(np.concatenate([target, np.stack([P_end] * 2)]))
    o.step()
    last = o.step()
    r = go.Oracle(shape)
    r.set_material_svk(phase, Cinf)
    r.set_control(mask)
    r.set_history(synth.history_stress_ramp(P_end, 4))
    r.set_tolerances(1e-12, 1e-13)
    ref = go.run_history(r)[-1]
    np.testing.assert_allclose(last.P_avg, ref.P_avg, rtol=0, atol=1e-11)
    C_last = last.F_avg.reshape(3, 3).T @ last.F_avg.reshape(3, 3)
    C_ref = ref.F_avg.reshape(3, 3).T @ ref.F_avg.reshape(3, 3)
    np.testing.assert_allclose(C_last, C_ref, rtol=0, atol=1e-9)


def _visco_oracle(shape, phase, Cinf, C1, tau, mask, target, s=None, dt=0.5):
    o = go.Oracle(shape)
    o.set_material_visco(phase, Cinf, C1, tau)
    o.set_time_step(dt)
    if s is not None:
        o.set_stiffness_scale(s)
    o.set_control(mask)
    o.set_history(target)
    o.set_tolerances(1e-13, 1e-14)
    go.run_history(o)
    return o


def _adjoint_case(seed=7):
    shape = (6, 6, 6)
    phase = _two_phase(shape, seed=seed)
    Cinf = np.stack([_iso(1.0, 2.0), _iso(6.0, 8.0)])
    C1 = np.stack([_iso(1.5, 1.0), _iso(3.0, 2.0)])
    tau = [0.4, 1.5]
    mask = synth.mask_uniaxial(0)
    F_end = np.eye(3)
    F_end[0, 0] = 1.04
    ramp = synth.history_mixed(mask, F_end.reshape(9), 2)
    target = np.concatenate([ramp, ramp[-1:], ramp[-1:]])
    s = synth.smooth_scale_field(shape, 9, ell=0.3, lo=1.0, hi=2.0).reshape(-1)
    a = np.zeros(9)
    a[4] = 1.0   # <F>_22 and <F>_33 are free under this control
    a[8] = 0.5
    return shape, phase, Cinf, C1, tau, mask, target, s, a


def test_history_adjoint_matches_finite_differences():
    shape, phase, Cinf, C1, tau, mask, target, s, a = _adjoint_case()
    o = _visco_oracle(shape, phase, Cinf, C1, tau, mask, target, s)
    grad = o.adjoint_grad_scale_history(a).reshape(-1)

    def J(sv):
        return float(_visco_oracle(shape, phase, Cinf, C1, tau, mask, target, sv).averages()[0] @ a)

    g = np.random.default_rng(2)
    for v in g.choice(s.size, 4, replace=False):
        h = 1e-4 * s[v]
        sp, sm = s.copy(), s.copy()
        sp[v] += h
        sm[v] -= h
        fd = (J(sp) - J(sm)) / (2 * h)
        assert abs(fd - grad[v]) <= 1e-6 * np.max(np.abs(grad)), (v, fd, grad[v])
    d = synth.smooth_scale_field(shape, 10, ell=0.3, lo=-1.0, hi=1.0).reshape(-1)
    eps = 1e-5
    fd = (J(s * (1 + eps * d)) - J(s * (1 - eps * d))) / 2
    ad = float(np.dot(grad, eps * d * s))
    assert abs(fd - ad) <= 1e-6 * abs(ad)


@pytest.mark.parametrize("limit", ["slow", "no_branch"])
def test_history_adjoint_limits_match_the_hyperelastic_adjoint(limit):
    shape, phase, Cinf, C1, tau, mask, target, s, a = _adjoint_case(seed=8)
    if limit == "slow":
        tau, C_el = [1e300, 1e300], Cinf + C1
    else:
        C1, C_el = 0.0 * C1, Cinf
    o = _visco_oracle(shape, phase, Cinf, C1, tau, mask, target, s)
    got = o.adjoint_grad_scale_history(a)
    r = go.Oracle(shape)
    r.set_material_svk(phase, C_el)
    r.set_stiffness_scale(s)
    r.set_control(mask)
    r.set_history(target)
    r.set_tolerances(1e-13, 1e-14)
    go.run_history(r)
    ref = r.adjoint_grad_scale(a)
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))
