"""The seeded generators reproduce the paper's load patterns and the stated workloads."""

import json
import os

import numpy as np

from paper_1901_06531_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_load_cases.json")


def test_case1_mask_is_the_papers_eq23_pattern():
    pat = json.load(open(GOLD))["case1_uniaxial_mixed"]["pattern"]
    want = np.array([[1 if c == "P" else 0 for c in row] for row in pat]).reshape(9)
    np.testing.assert_array_equal(synth.mask_uniaxial(0), want)
    # cyclic permutation keeps the number of prescribed stresses
    for ax in range(3):
        assert synth.mask_uniaxial(ax).sum() == 5


def test_pseudo_uniaxial_endpoint_is_isochoric():
    g = json.load(open(GOLD))["case4_pseudo_uniaxial"]
    lam = g["lambda_end"]
    t = np.sqrt(1.0 / (1.0 + lam))
    F = np.diag([1 + lam, t, t])
    np.testing.assert_allclose(np.diag(F), g["final_F_diag"], rtol=0, atol=1e-15)
    assert abs(np.linalg.det(F) - g["final_det"]) < 1e-15


def test_centered_sphere_voxel_count():
    # voxel centres strictly inside r = 0.25 on 16^3: 280 voxels (no centre lies on the sphere)
    assert int(synth.centered_sphere((16, 16, 16), 0.25).sum()) == 280


def test_rsa_spheres_do_not_overlap_and_hit_volume_fraction():
    c, r = synth.rsa_spheres(40, 0.05, 0.10, 1, target_vf=0.25)
    assert abs((4 / 3) * np.pi * np.sum(r ** 3) - 0.25) < 1e-12
    d = np.abs(c[:, None, :] - c[None, :, :])
    d = np.sqrt(np.sum(np.minimum(d, 1 - d) ** 2, axis=-1))
    iu = np.triu_indices(40, 1)
    assert np.all(d[iu] >= (r[:, None] + r[None, :])[iu])
    ph = synth.spheres_phase((64, 64, 64), c, r)
    assert abs(ph.mean() - 0.25) < 0.01


def test_rotations_are_proper_orthogonal():
    R = synth.haar_rotations(64, 3)
    np.testing.assert_allclose(R @ R.transpose(0, 2, 1), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)


def test_histories():
    h = synth.history_stress_triangle(0.02, 40)
    assert h.shape == (40, 9)
    assert abs(h[9, 0] - 0.02) < 1e-15 and abs(h[29, 0] + 0.02) < 1e-15 and abs(h[39, 0]) < 1e-15
    assert np.all(h[:, 1:] == 0)
    m = synth.mask_uniaxial(0)
    F_end = np.eye(3)
    F_end[0, 0] = 1.2
    hm = synth.history_mixed(m, F_end.reshape(9), 4)
    assert abs(hm[-1, 0] - 1.2) < 1e-15 and np.all(hm[:, m == 1] == 0)


def test_voronoi_and_scale_field():
    g = synth.voronoi_grains((16, 16, 16), 8, 2)
    assert g.dtype == np.uint16 and set(np.unique(g)) <= set(range(8))
    s = synth.smooth_scale_field((16, 16, 16), 5)
    assert abs(s.min() - 1.0) < 1e-12 and abs(s.max() - 10.0) < 1e-12
