"""Seeded synthetic inputs: microstructures, material tables and macroscopic load histories.

These generators hold none of the homogenization arithmetic; they only build the inputs
(phase maps, per-phase moduli, stiffness scale fields, control masks and target histories)
that both the HIP library and the CPU checker receive.

Layout conventions shared with the library:
  * phase maps are uint16 arrays of shape (nx, ny, nz), C order (z fastest);
  * voxel (i, j, k) has its centre at ((i + 1/2)/nx, (j + 1/2)/ny, (k + 1/2)/nz) of the
    unit periodic cell;
  * a control mask is 9 bytes, component c = 3*i + j, 1 = first Piola-Kirchhoff stress
    prescribed (IJ), 0 = deformation gradient prescribed (ij);
  * a history is an (nsteps, 9) float64 array: row k-1 gives, for increment k, the target
    stress on mask-1 components and the target deformation gradient on mask-0 ones.
"""

from __future__ import annotations

import math

import numpy as np

IDENTITY9 = np.eye(3).reshape(9)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ------------------------------------------------------------------ geometry -----------

def voxel_centers(shape):
    """Three (nx, ny, nz) arrays with the voxel-centre coordinates in [0, 1)."""
    axes = [(np.arange(n) + 0.5) / n for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def _periodic_sq_dist(X, Y, Z, c):
    d2 = 0.0
    for A, ci in zip((X, Y, Z), c):
        d = np.abs(A - ci)
        d = np.minimum(d, 1.0 - d)
        d2 = d2 + d * d
    return d2


def spheres_phase(shape, centers, radii) -> np.ndarray:
    """Phase 1 where a voxel centre lies strictly inside some sphere (periodic), else 0."""
    X, Y, Z = voxel_centers(shape)
    phase = np.zeros(shape, dtype=np.uint16)
    for c, r in zip(centers, radii):
        inside = _periodic_sq_dist(X, Y, Z, c) < r * r
        phase[inside] = 1
    return phase


def centered_sphere(shape, radius=0.25) -> np.ndarray:
    """One sphere at the cell centre."""
    return spheres_phase(shape, [(0.5, 0.5, 0.5)], [radius])


def rsa_spheres(count, rmin, rmax, seed, target_vf=None, gap=0.0, max_tries=200000):
    """Non-overlapping periodic spheres by random sequential addition.

    Radii are drawn uniformly in [rmin, rmax]; if ``target_vf`` is given they are all scaled
    by one common factor so that the analytic volume fraction equals it.  Spheres are placed
    largest first; a candidate centre is accepted when its periodic distance to every placed
    centre is at least r_i + r_j + gap.  Returns (centers (count, 3), radii (count,)).
    """
    g = rng(seed)
    radii = g.uniform(rmin, rmax, size=count)
    if target_vf is not None:
        vol = (4.0 / 3.0) * math.pi * np.sum(radii ** 3)
        radii = radii * (target_vf / vol) ** (1.0 / 3.0)
    order = np.argsort(-radii, kind="stable")
    radii = radii[order]
    centers = np.zeros((count, 3))
    placed = 0
    tries = 0
    while placed < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition failed to place %d spheres" % count)
        c = g.uniform(0.0, 1.0, size=3)
        if placed:
            d = np.abs(centers[:placed] - c)
            d = np.minimum(d, 1.0 - d)
            dist = np.sqrt(np.sum(d * d, axis=1))
            if np.any(dist < radii[:placed] + radii[placed] + gap):
                continue
        centers[placed] = c
        placed += 1
    return centers, radii


def voronoi_grains(shape, ngrains, seed) -> np.ndarray:
    """Periodic Voronoi tessellation: each voxel takes the index of its nearest seed
    (minimum image); seeds are uniform in the unit cell."""
    from scipy.spatial import cKDTree

    g = rng(seed)
    seeds = g.uniform(0.0, 1.0, size=(ngrains, 3))
    tree = cKDTree(seeds, boxsize=1.0)
    X, Y, Z = voxel_centers(shape)
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) % 1.0
    _, idx = tree.query(pts, k=1, workers=-1)
    return idx.astype(np.uint16).reshape(shape)


def haar_rotations(count, seed) -> np.ndarray:
    """Uniformly random rotations from uniform unit quaternions (Shoemake, Graphics Gems
    III, 1992).  Returns (count, 3, 3)."""
    g = rng(seed)
    u1, u2, u3 = g.uniform(0.0, 1.0, size=(3, count))
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    w, x, y, z = (a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3))
    R = np.empty((count, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def smooth_scale_field(shape, seed, ell=0.1, lo=1.0, hi=10.0) -> np.ndarray:
    """Smooth random field in [lo, hi]: white noise filtered by a Gaussian of length ell
    (in cell units), then mapped affinely onto [lo, hi].  Shape (nx, ny, nz), float64."""
    g = rng(seed)
    w = g.standard_normal(shape)
    k = [np.fft.fftfreq(n, d=1.0 / n) for n in shape]
    KX, KY, KZ = np.meshgrid(*k, indexing="ij")
    filt = np.exp(-(KX ** 2 + KY ** 2 + KZ ** 2) * (ell ** 2) * (2 * np.pi) ** 2 / 2.0)
    phi = np.fft.ifftn(np.fft.fftn(w) * filt).real
    phi = (phi - phi.min()) / (phi.max() - phi.min())
    return lo + (hi - lo) * phi


# ------------------------------------------------------------------ materials ----------

def isotropic_C(mu, lam) -> np.ndarray:
    """Isotropic stiffness C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk), (3,3,3,3)."""
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def cubic_C(C11, C12, C44) -> np.ndarray:
    """Cubic stiffness in the crystal frame (Voigt C11, C12, C44; C_1212 = C44)."""
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            C[i, i, j, j] = C11 if i == j else C12
    for i in range(3):
        for j in range(3):
            if i != j:
                C[i, j, i, j] = C44
                C[i, j, j, i] = C44
    return C


def rotate_C(C, R) -> np.ndarray:
    """C'_ijkl = R_ia R_jb R_kc R_ld C_abcd for each rotation in R (..., 3, 3)."""
    return np.einsum("...ia,...jb,...kc,...ld,abcd->...ijkl", R, R, R, R, C)


# ------------------------------------------------------------------ load histories -----

def mask_full_stress():
    return np.ones(9, dtype=np.uint8)


def mask_full_strain():
    return np.zeros(9, dtype=np.uint8)


def mask_uniaxial(axis=0):
    """The paper's case (1) (Sec. 3.1): F prescribed on 11, 12, 13, 23 (F_11 the ramp,
    the others 0) and P prescribed (zero) on 21, 22, 31, 32, 33 -- with the axes permuted
    cyclically so that ``axis`` is the loading direction."""
    base = np.array([[0, 0, 0], [1, 1, 0], [1, 1, 1]], dtype=np.uint8)
    perm = [(axis + d) % 3 for d in range(3)]
    m = np.zeros((3, 3), dtype=np.uint8)
    for a in range(3):
        for b in range(3):
            m[perm[a], perm[b]] = base[a, b]
    return m.reshape(9)


def mask_transverse_free(axis=0):
    """F prescribed on every component except the two transverse normal ones, which are
    stress free (the 128^3 particle workload's mixed control)."""
    m = np.zeros(9, dtype=np.uint8)
    for d in range(3):
        if d != axis:
            m[4 * d] = 1
    return m


def history_stress_ramp(P_end9, nsteps):
    """Full stress control: P-bar = P_end * k / nsteps."""
    P_end9 = np.asarray(P_end9, float).reshape(9)
    return np.stack([P_end9 * (k / nsteps) for k in range(1, nsteps + 1)])


def history_strain_ramp(F_end9, nsteps):
    """Full strain control: F-bar = I + (F_end - I) k / nsteps (the paper's case (3), with
    the identity restored)."""
    F_end9 = np.asarray(F_end9, float).reshape(9)
    return np.stack([IDENTITY9 + (F_end9 - IDENTITY9) * (k / nsteps) for k in range(1, nsteps + 1)])


def history_mixed(mask, F_end9, nsteps, P_end9=None):
    """Mixed control: mask-0 components ramp linearly from I to F_end, mask-1 components
    ramp from 0 to P_end (default 0)."""
    mask = np.asarray(mask).reshape(9)
    Fh = history_strain_ramp(F_end9, nsteps)
    Ph = history_stress_ramp(np.zeros(9) if P_end9 is None else P_end9, nsteps)
    return np.where(mask[None, :] > 0, Ph, Fh)


def history_stress_triangle(amp, nsteps, comp=0):
    """P_comp follows a triangle wave 0 -> +amp -> 0 -> -amp -> 0 over nsteps increments
    (nsteps divisible by 4), every other stress component 0."""
    q = nsteps // 4
    vals = []
    for k in range(1, nsteps + 1):
        if k <= q:
            v = amp * k / q
        elif k <= 3 * q:
            v = amp * (2 * q - k) / q
        else:
            v = amp * (k - 4 * q) / q
        vals.append(v)
    out = np.zeros((nsteps, 9))
    out[:, comp] = vals
    return out


# ------------------------------------------------------------------ workloads ----------

def workload_sphere16():
    """16^3 cell, one centred sphere of radius 0.25; neo-Hookean matrix (mu, lam) = (1, 2),
    inclusion (10, 20); full stress control with P11 ramped to 0.1 in 5 increments."""
    shape = (16, 16, 16)
    P_end = np.zeros(9)
    P_end[0] = 0.1
    return dict(
        name="sphere16_nh_stress", shape=shape, kind="nh",
        phase=centered_sphere(shape, 0.25), mu=np.array([1.0, 10.0]), lam=np.array([2.0, 20.0]),
        mask=mask_full_stress(), target=history_stress_ramp(P_end, 5),
        newton_tol=1e-10, cg_tol=1e-12)


def workload_particles(n=128, seed=1, count=40, vf=0.25, nsteps=20):
    """n^3 cell with ``count`` non-overlapping random spheres (radii U[0.05, 0.10] scaled to
    volume fraction ``vf``); neo-Hookean contrast 10; F11 -> 1.2 over ``nsteps`` increments
    with P22 = P33 = 0 and every other F component prescribed (off-diagonal 0)."""
    shape = (n, n, n)
    centers, radii = rsa_spheres(count, 0.05, 0.10, seed, target_vf=vf)
    mask = mask_transverse_free(0)
    F_end = np.eye(3)
    F_end[0, 0] = 1.2
    return dict(
        name="particles%d_nh_mixed" % n, shape=shape, kind="nh",
        phase=spheres_phase(shape, centers, radii), mu=np.array([1.0, 10.0]),
        lam=np.array([2.0, 20.0]), mask=mask,
        target=history_mixed(mask, F_end.reshape(9), nsteps), newton_tol=1e-6, cg_tol=1e-8)


def workload_polycrystal(n=256, ngrains=512, seed_grains=2, seed_rot=3, nsteps=40):
    """n^3 periodic Voronoi polycrystal with ``ngrains`` grains, each a Saint
    Venant-Kirchhoff cubic crystal (C11, C12, C44) = (1.7, 1.2, 0.75) under a uniformly
    random rotation; full stress control, P11 cycled 0 -> 0.02 -> 0 -> -0.02 -> 0."""
    shape = (n, n, n)
    grains = voronoi_grains(shape, ngrains, seed_grains)
    R = haar_rotations(ngrains, seed_rot)
    C = rotate_C(cubic_C(1.7, 1.2, 0.75), R)
    return dict(
        name="polycrystal%d_svk_stress" % n, shape=shape, kind="svk", phase=grains,
        C=C.reshape(ngrains, 81), mask=mask_full_stress(),
        target=history_stress_triangle(0.02, nsteps, comp=0), newton_tol=1e-6, cg_tol=1e-8)


def workload_adjoint(n=128, seed_geo=1, seed_s=5, nsteps=10):
    """Two-phase neo-Hookean cell (as the particle workload) with a smooth per-voxel
    stiffness scale s(x) in [1, 10]; full stress control P11 -> 0.05 over ``nsteps``."""
    base = workload_particles(n, seed_geo)
    P_end = np.zeros(9)
    P_end[0] = 0.05
    base.update(
        name="adjoint%d_nh_stress" % n, scale=smooth_scale_field(base["shape"], seed_s),
        mask=mask_full_stress(), target=history_stress_ramp(P_end, nsteps),
        newton_tol=1e-10, cg_tol=1e-12)
    return base


def workload_paper_particles(n=64, nsteps=100):
    """The particle-reinforced example of Sec. 3.1 with a synthetic geometry: 4 equal spheres
    at volume fraction 0.2 on the sites of a face-centred cubic cell shifted by (1/4, 1/4,
    1/4), an isotropic SVK matrix with shear modulus 28 and bulk modulus 46.67 (so
    lambda = 28) and particles ten times stiffer in both moduli.  The case-(1) control: F11
    ramps to 1.2 over ``nsteps`` increments, F12 = F13 = F23 = 0 prescribed, every other
    stress component zero.  Cases (2) and (3) are built from case (1)'s end state
    (history_stress_ramp, history_strain_ramp).

    The voxelized cell is symmetric under the reflections x -> 1/2 - x (and likewise in y, z)
    for even n, so case (1) ends with a diagonal stress: a stress target with a skew part
    cannot be reached from F = I, where the tangent annihilates uniform rotations."""
    a, b = 0.25, 0.75
    centers = np.array([[a, a, a], [b, b, a], [b, a, b], [a, b, b]])
    radii = np.full(4, (0.20 * 3.0 / (16.0 * math.pi)) ** (1.0 / 3.0))
    shape = (n, n, n)
    phase = spheres_phase(shape, centers, radii)
    mu, bulk = 28.0, 46.67
    lam = bulk - 2.0 * mu / 3.0
    C = np.stack([isotropic_C(mu, lam), isotropic_C(10 * mu, 10 * lam)])
    mask = mask_uniaxial(0)
    F_end = np.eye(3)
    F_end[0, 0] = 1.2
    return dict(name="paper_particles%d" % n, shape=shape, kind="svk", phase=phase, C=C, mask=mask,
                target=history_mixed(mask, F_end.reshape(9), nsteps), newton_tol=1e-6, cg_tol=1e-8)


def mask_normal_stress_free():
    """Every off-diagonal F component prescribed, the three normal stresses free (P_ii = 0):
    the simple-shear control (the sheared plane is set by the F history)."""
    m = np.zeros(9, dtype=np.uint8)
    for d in range(3):
        m[4 * d] = 1
    return m


def workload_batch(sizes=(32, 48, 64, 96), per_size=16, nsteps=10, seed0=100):
    """Batch of RVEs under six load cases each.

    Each RVE (per_size of every size, seeds seed0 + index) holds U{4..12} random
    non-overlapping spheres scaled to volume fraction 0.20, neo-Hookean matrix (1, 2) and
    inclusions c (1, 2) with contrast c ~ U[5, 20].  Load cases: uniaxial along x, y, z
    (the paper's case-(1) pattern permuted, F_aa -> 1.10) and simple shear in xy, yz, zx
    (F_ab -> 0.20), each over ``nsteps`` increments.  Returns a list of workload dicts (the
    phase map is shared by the six cases of an RVE)."""
    out = []
    idx = 0
    for n in sizes:
        for _ in range(per_size):
            g = rng(seed0 + idx)
            count = int(g.integers(4, 13))
            c = float(g.uniform(5.0, 20.0))
            centers, radii = rsa_spheres(count, 0.05, 0.10, seed0 + idx, target_vf=0.20)
            shape = (n, n, n)
            phase = spheres_phase(shape, centers, radii)
            mu = np.array([1.0, c])
            lam = np.array([2.0, 2.0 * c])
            cases = []
            for a in range(3):
                mask = mask_uniaxial(a)
                F_end = np.eye(3)
                F_end[a, a] = 1.10
                cases.append(("uniaxial_%s" % "xyz"[a], mask, history_mixed(mask, F_end.reshape(9), nsteps)))
            for a, b in ((0, 1), (1, 2), (2, 0)):
                mask = mask_normal_stress_free()
                F_end = np.eye(3)
                F_end[a, b] = 0.20
                cases.append(("shear_%s%s" % ("xyz"[a], "xyz"[b]), mask, history_mixed(mask, F_end.reshape(9), nsteps)))
            for name, mask, target in cases:
                out.append(dict(name="rve%d_%d_%s" % (idx, n, name), shape=shape, kind="nh", phase=phase, mu=mu,
                                lam=lam, mask=mask, target=target, newton_tol=1e-6, cg_tol=1e-8))
            idx += 1
    return out
