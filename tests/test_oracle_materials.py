"""Pins of the oracle's hyperelastic laws: P = dW/dF and K:dF = dP[dF] by central finite
differences of the energies, major symmetry of K, small-strain limit, objectivity."""

import numpy as np
import pytest

from oracle import ghom_oracle as go
from paper_1901_06531_amd import synth


def _random_F(g, m, amp=0.2):
    return np.eye(3) + amp * g.standard_normal((m, 3, 3))


def _fd_stress(energy, F, h=1e-6):
    P = np.zeros_like(F)
    for i in range(3):
        for j in range(3):
            E = np.zeros((3, 3))
            E[i, j] = h
            P[:, i, j] = (energy(F + E) - energy(F - E)) / (2 * h)
    return P


def _laws(g, m):
    mu = g.uniform(0.5, 3.0, m)
    lam = g.uniform(0.5, 5.0, m)
    R = synth.haar_rotations(m, 11)
    C = synth.rotate_C(synth.cubic_C(1.7, 1.2, 0.75), R)
    return {
        "nh": (lambda F: go.nh_energy(F, mu, lam), lambda F: go.nh_stress(F, mu, lam),
               lambda F, d: go.nh_tangent_apply(F, mu, lam, d)),
        "svk": (lambda F: go.svk_energy(F, C), lambda F: go.svk_stress(F, C),
                lambda F, d: go.svk_tangent_apply(F, C, d)),
    }


@pytest.mark.parametrize("law", ["nh", "svk"])
def test_stress_is_energy_derivative(law):
    g = np.random.default_rng(0)
    F = _random_F(g, 16)
    W, P, _ = _laws(g, 16)[law]
    np.testing.assert_allclose(P(F), _fd_stress(W, F), rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("law", ["nh", "svk"])
def test_tangent_is_stress_derivative(law):
    g = np.random.default_rng(1)
    F = _random_F(g, 16)
    dF = g.standard_normal((16, 3, 3))
    _, P, K = _laws(g, 16)[law]
    h = 1e-6
    fd = (P(F + h * dF) - P(F - h * dF)) / (2 * h)
    np.testing.assert_allclose(K(F, dF), fd, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("law", ["nh", "svk"])
def test_tangent_major_symmetry(law):
    g = np.random.default_rng(2)
    F = _random_F(g, 16)
    A, B = g.standard_normal((2, 16, 3, 3))
    _, _, K = _laws(g, 16)[law]
    lhs = np.einsum("nij,nij->n", A, K(F, B))
    rhs = np.einsum("nij,nij->n", K(F, A), B)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_small_strain_limit_is_isotropic_hooke():
    """At F = I both laws give P = 0 and K:dF = 2 mu sym(dF) + lam tr(dF) I for isotropic
    moduli (SVK with the isotropic C; neo-Hookean with the same mu, lam)."""
    g = np.random.default_rng(3)
    m = 8
    mu = g.uniform(0.5, 3.0, m)
    lam = g.uniform(0.5, 5.0, m)
    F = np.broadcast_to(np.eye(3), (m, 3, 3)).copy()
    dF = g.standard_normal((m, 3, 3))
    hooke = (mu[:, None, None] * (dF + dF.transpose(0, 2, 1))
             + (lam * np.trace(dF, axis1=1, axis2=2))[:, None, None] * np.eye(3))
    C = np.stack([synth.isotropic_C(a, b) for a, b in zip(mu, lam)])
    assert np.max(np.abs(go.nh_stress(F, mu, lam))) < 1e-15
    assert np.max(np.abs(go.svk_stress(F, C))) < 1e-15
    np.testing.assert_allclose(go.nh_tangent_apply(F, mu, lam, dF), hooke, atol=1e-13)
    np.testing.assert_allclose(go.svk_tangent_apply(F, C, dF), hooke, atol=1e-13)


@pytest.mark.parametrize("law", ["nh", "svk"])
def test_objectivity(law):
    """P(Q F) = Q P(F) for any rotation Q."""
    g = np.random.default_rng(4)
    F = _random_F(g, 8)
    Q = synth.haar_rotations(8, 12)
    _, P, _ = _laws(g, 8)[law]
    np.testing.assert_allclose(P(Q @ F), Q @ P(F), atol=1e-12)


def test_cubic_stiffness_has_cubic_symmetry_and_rotates():
    C = synth.cubic_C(1.7, 1.2, 0.75)
    # Voigt entries
    assert C[0, 0, 0, 0] == 1.7 and C[0, 0, 1, 1] == 1.2 and C[0, 1, 0, 1] == 0.75
    # invariant under a 90 degree rotation about z
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    np.testing.assert_allclose(synth.rotate_C(C, Rz), C, atol=1e-15)
    # rotating the crystal rotates the response: S(R E R^T) = R S(E) R^T
    R = synth.haar_rotations(1, 3)[0]
    Cr = synth.rotate_C(C, R)
    E = np.random.default_rng(5).standard_normal((3, 3))
    E = E + E.T
    S = np.einsum("ijkl,kl->ij", C, E)
    Sr = np.einsum("ijkl,kl->ij", Cr, R @ E @ R.T)
    np.testing.assert_allclose(Sr, R @ S @ R.T, atol=1e-13)


def test_domain_error_on_inverted_voxel():
    F = np.eye(3)[None].repeat(2, 0)
    F[1, 0, 0] = -0.5
    with pytest.raises(go.DomainError):
        go.nh_stress(F, np.ones(2), np.ones(2))
