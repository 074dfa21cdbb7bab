"""Pins of the oracle's Fourier transform and modified projection G* (Sec. 2.1-2.3).

Each test checks the oracle against something other than itself: a brute-force DFT sum,
the Helmholtz decomposition of eq. (6)-(8) on explicit plane waves, and the algebraic
properties the paper states or implies (projector, major symmetry, real output, the
null-frequency control of eq. (19)/(22), the Nyquist rule of eq. (10)).
"""

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import ghom_oracle as go

SHAPES = [(4, 4, 4), (6, 4, 5), (3, 5, 8)]
LENGTHS = [(1.0, 1.0, 1.0), (1.0, 2.0, 0.5), (0.7, 1.3, 1.0)]
MIXED = np.array([0, 0, 0, 1, 1, 0, 1, 1, 1], dtype=float)  # the paper's case (1), eq. (23)


def _brute_dft(a):
    """Plain O(N^2) sum X(k) = sum_x a(x) exp(-2 pi i k.x / n)."""
    mats = [np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n) for n in a.shape]
    return np.einsum("ax,by,cz,xyz->abc", *mats, a)


def _grid_phase(shape, k):
    """2 pi k.x/n on the voxel grid (x_d = i_d / n_d in cell units)."""
    idx = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    return 2 * np.pi * sum(kd * X for kd, X in zip(k, idx))


@pytest.mark.parametrize("shape", SHAPES)
def test_library_fft_matches_brute_force_dft(shape):
    g = np.random.default_rng(0)
    a = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    np.testing.assert_allclose(sfft.fftn(a), _brute_dft(a), rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape,lengths", list(zip(SHAPES, LENGTHS)))
def test_gradient_fields_are_preserved(shape, lengths):
    """A compatible field (the gradient of a periodic displacement, eq. 8) is left
    unchanged: for a plane wave u = a cos(2 pi k.x), grad u is proportional to a (x) xi."""
    g = np.random.default_rng(1)
    field = np.zeros((3, 3) + shape)
    for k in [(1, 0, 0), (0, 1, 1), (1, -1, 2), (-1, 2, 1)]:
        k = tuple(kd % n if n > 2 * abs(kd) else 0 for kd, n in zip(k, shape))
        ks = [(kd if kd <= (n - 1) // 2 else kd - n) for kd, n in zip(k, shape)]
        if all(v == 0 for v in ks):
            continue
        xi = np.array([kd / L for kd, L in zip(ks, lengths)])
        a = g.standard_normal(3)
        ph = _grid_phase(shape, k)
        field += np.einsum("i,j,...->ij...", a, xi, -np.sin(ph))
    B = go.apply_projection(field.reshape((9,) + shape), np.ones(9), lengths)
    np.testing.assert_allclose(B, field.reshape((9,) + shape), atol=1e-12)


@pytest.mark.parametrize("shape,lengths", list(zip(SHAPES, LENGTHS)))
def test_row_orthogonal_fields_are_annihilated(shape, lengths):
    """Fields whose rows are orthogonal to xi (B xi = 0, the complement of a (x) xi in
    the Frobenius product) are removed: eq. (9) projects each row on xi/|xi|."""
    g = np.random.default_rng(2)
    field = np.zeros((3, 3) + shape)
    for k in [(1, 0, 0), (0, 1, 1), (1, 1, 1)]:
        ks = [(kd if kd <= (n - 1) // 2 else kd - n) for kd, n in zip(k, shape)]
        xi = np.array([kd / L for kd, L in zip(ks, lengths)])
        t = np.cross(xi, g.standard_normal(3))
        s = np.cross(xi, t)
        ph = _grid_phase(shape, k)
        for _ in range(2):
            a, b = g.standard_normal(3), g.standard_normal(3)
            field += np.einsum("i,j,...->ij...", a, t, np.cos(ph))
            field += np.einsum("i,j,...->ij...", b, s, np.sin(ph))
    B = go.apply_projection(field.reshape((9,) + shape), np.ones(9), lengths)
    assert np.max(np.abs(B)) < 1e-12


@pytest.mark.parametrize("shape,lengths", list(zip(SHAPES, LENGTHS)))
@pytest.mark.parametrize("mask", [np.zeros(9), np.ones(9), MIXED])
def test_projector_properties(shape, lengths, mask):
    """Idempotent, self-adjoint in sum_x A:B, real in / real out."""
    g = np.random.default_rng(3)
    A = g.standard_normal((9,) + shape)
    C = g.standard_normal((9,) + shape)
    GA = go.apply_projection(A, mask, lengths)
    GC = go.apply_projection(C, mask, lengths)
    np.testing.assert_allclose(go.apply_projection(GA, mask, lengths), GA, atol=1e-12)
    assert abs(np.vdot(GA, C) - np.vdot(A, GC)) < 1e-11 * np.abs(A).sum()
    # the complex transform of the projected field has no imaginary residue
    Ahat = sfft.fftn(A.reshape((3, 3) + shape), axes=(2, 3, 4))
    Bc = sfft.ifftn(go.project_spectrum(Ahat, mask, lengths), axes=(2, 3, 4))
    assert np.max(np.abs(Bc.imag)) < 1e-13


@pytest.mark.parametrize("shape", SHAPES)
def test_null_frequency_follows_the_mask(shape):
    """eq. (22): at xi = 0 stress-controlled components pass (eq. 19), deformation-controlled
    ones vanish (eq. 10).  A uniform field has only xi = 0 content."""
    g = np.random.default_rng(4)
    u = g.standard_normal(9)
    field = np.broadcast_to(u[:, None, None, None], (9,) + shape).copy()
    for mask in (np.zeros(9), np.ones(9), MIXED):
        B = go.apply_projection(field, mask, (1, 1, 1))
        np.testing.assert_allclose(B, field * mask[:, None, None, None], atol=1e-13)
    # and for a general field the mean of every deformation-controlled component is zero
    A = g.standard_normal((9,) + shape)
    B = go.apply_projection(A, MIXED, (1, 1, 1))
    means = B.reshape(9, -1).mean(axis=1)
    np.testing.assert_allclose(means[MIXED == 0], 0.0, atol=1e-14)
    np.testing.assert_allclose(means[MIXED == 1], A.reshape(9, -1).mean(axis=1)[MIXED == 1], atol=1e-13)


def test_nyquist_content_is_removed():
    """eq. (10): on even axes the highest frequency is dropped; a wave (-1)^i along any
    even axis, times anything along the others, vanishes."""
    shape = (4, 6, 5)
    g = np.random.default_rng(5)
    i, j, k = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    for alt in ((-1.0) ** i, (-1.0) ** j):
        field = g.standard_normal((9, 1, 1, 1)) * alt * np.cos(2 * np.pi * k / 5)
        assert np.max(np.abs(go.apply_projection(field, np.ones(9)))) < 1e-13
    # odd axis: no Nyquist, a wave at the top frequency survives if it is compatible
    xi = np.array([0.0, 0.0, 2.0])
    field = np.einsum("i,j,...->ij...", np.ones(3), xi, np.cos(2 * np.pi * 2 * k / 5)).reshape((9,) + shape)
    np.testing.assert_allclose(go.apply_projection(field, np.ones(9)), field, atol=1e-12)


@pytest.mark.parametrize("shape,lengths", list(zip(SHAPES, LENGTHS)))
def test_projected_spectrum_is_compatible(shape, lengths):
    """Curl-free output: B_ij xi_k = B_ik xi_j at every xi != 0."""
    g = np.random.default_rng(6)
    A = g.standard_normal((3, 3) + shape)
    Bh = go.project_spectrum(sfft.fftn(A, axes=(2, 3, 4)), MIXED, lengths)
    xi = go.frequency_vectors(shape, lengths)
    lhs = np.einsum("ij...,k...->ijk...", Bh, xi)
    assert np.max(np.abs(lhs - lhs.transpose(0, 2, 1, 3, 4, 5))) < 1e-11
