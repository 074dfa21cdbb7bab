"""FP64 CPU oracle for Galerkin-FFT homogenization with stress and mixed control.

Method: Lucarini & Segurado, "An algorithm for stress and mixed control in Galerkin
based FFT homogenization" (arXiv:1901.06531).

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference the HIP path is
checked against.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product library never calls it and shares no code with it.

Everything is computed in float64 with plain NumPy array arithmetic.  The 3-D discrete
Fourier transform is taken from ``scipy.fft`` (a library primitive); the projection, the
materials, the conjugate-gradient solve and the Newton loop are written out below in the
order and notation of the paper.

Conventions (the paper leaves them open; the reading taken is stated where it is used):

* A tensor field is an array of shape ``(9, nx, ny, nz)``; component ``c = 3*i + j`` holds
  the tensor entry ``(i, j)``.  Internally fields are viewed as ``(3, 3, nx, ny, nz)``.
* The cell is periodic with edge lengths ``(Lx, Ly, Lz)``; the frequency vector of the
  integer wave numbers ``(kx, ky, kz)`` is ``xi = (kx/Lx, ky/Ly, kz/Lz)`` (Sec. 2.1,
  "Projection operator": xi has the dimension of an inverse length; a factor 2*pi would
  cancel in xi_j xi_l / xi.xi).
* ``mask[c] = 1`` marks a stress-controlled component IJ (the macroscopic first
  Piola-Kirchhoff stress is prescribed), ``mask[c] = 0`` a deformation-gradient
  controlled component ij (Sec. 2.3).

Parity pins: every function here is checked in ``tests/test_oracle_*.py`` against
brute-force transforms, closed forms, finite differences and invariants.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

WORKERS = max(1, os.cpu_count() or 1)

EYE9 = np.eye(3).reshape(9)


class OracleError(RuntimeError):
    """Base class of the oracle's failure modes."""


class DomainError(OracleError):
    """det F <= 0 somewhere: the hyperelastic laws are undefined."""


class BreakdownError(OracleError):
    """Conjugate gradients met p.Ap <= 0 or a non-finite value."""


class NotConvergedError(OracleError):
    """An iteration cap was reached."""


# --------------------------------------------------------------------------------------
# Fourier grid and the projection operator (Sec. 2.1 eq. 9-10, Sec. 2.2 eq. 19,
# Sec. 2.3 eq. 22)
# --------------------------------------------------------------------------------------

def wave_numbers(n: int) -> np.ndarray:
    """Signed integer wave numbers of an axis of n points, in DFT output order.

    Index k < n/2 is the wave number k, index k > n/2 the wave number k - n; for even n the
    index n/2 is the Nyquist frequency (kept as -n/2 here; it is zeroed by the projection).
    """
    k = np.arange(n)
    return np.where(k <= (n - 1) // 2, k, k - n)


def nyquist_mask(shape) -> np.ndarray:
    """True at every frequency where some even-length axis sits at its Nyquist index n/2.

    Reading of the paper's "Nyquist frequencies" (eq. 10, 19, 22): the operator is zero
    wherever ANY even axis is at its highest frequency.  This keeps the projected spectrum
    Hermitian (real fields map to real fields) and the operator an orthogonal projector.
    """
    nx, ny, nz = shape
    out = np.zeros(shape, dtype=bool)
    if nx % 2 == 0:
        out[nx // 2, :, :] = True
    if ny % 2 == 0:
        out[:, ny // 2, :] = True
    if nz % 2 == 0:
        out[:, :, nz // 2] = True
    return out


def frequency_vectors(shape, lengths=(1.0, 1.0, 1.0)) -> np.ndarray:
    """xi at every frequency, shape (3, nx, ny, nz): xi_d = k_d / L_d."""
    ks = [wave_numbers(n) / float(L) for n, L in zip(shape, lengths)]
    return np.stack(np.meshgrid(*ks, indexing="ij"))


def project_spectrum(A_hat: np.ndarray, mask, lengths=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Apply the modified projection G* of eq. (22) to a spectrum, frequency by frequency.

    ``A_hat`` has shape (3, 3, nx, ny, nz).  At xi != 0 (and off the Nyquist set) the
    compatible part of eq. (8)/(9) is returned: B_ij = delta_ik xi_j xi_l / (xi.xi) A_kl,
    i.e. each tensor row projected on xi/|xi|.  At Nyquist frequencies B = 0 (eq. 10).  At
    xi = 0 a stress-controlled component is passed through unchanged (the fourth-order
    identity of eq. 19) and a deformation-controlled one is set to zero (eq. 10), which is
    eq. (22).  Full strain control is mask == 0 everywhere, full stress control mask == 1.
    """
    shape = A_hat.shape[2:]
    xi = frequency_vectors(shape, lengths)
    xi2 = np.einsum("d...,d...->...", xi, xi)
    null = xi2 == 0.0
    safe = np.where(null, 1.0, xi2)
    # row i of A contracted with xi, divided by xi.xi, then outer product with xi
    row_dot = np.einsum("il...,l...->i...", A_hat, xi) / safe
    B = np.einsum("i...,j...->ij...", row_dot, xi)
    B[:, :, nyquist_mask(shape)] = 0.0
    m = np.asarray(mask, dtype=float).reshape(3, 3)
    B[:, :, null] = (m[:, :, None] * A_hat[:, :, null])
    return B


def apply_projection(field9: np.ndarray, mask, lengths=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Real-space G*(A) = F^-1{ G*_hat : F{A} } of a real tensor field (eq. 2 with G*)."""
    shape = field9.shape[1:]
    A = field9.reshape((3, 3) + shape)
    A_hat = sfft.fftn(A, axes=(2, 3, 4), workers=WORKERS)
    B_hat = project_spectrum(A_hat, mask, lengths)
    B = sfft.ifftn(B_hat, axes=(2, 3, 4), workers=WORKERS)
    return np.ascontiguousarray(B.real.reshape((9,) + shape))


# --------------------------------------------------------------------------------------
# Rotation gauge under full stress control (Sec. 2.2; a reading, the paper is silent)
# --------------------------------------------------------------------------------------

def rotation_gauge_axis(mask, target):
    """Axis a of the rotation gauge, or None when the gauge does not apply.

    Under full stress control (every component stress-controlled, eq. 19) F is fixed only
    up to the rigid rotations Q with Q P-bar = P-bar: all three rotations when P-bar = 0,
    the rotation about a when P-bar = p e_a (x) e_a.  The gauge applies when the mask is
    all ones and every target row of the history is a multiple of e_a (x) e_a for one axis
    a (the zero history takes a = 0).
    """
    m = np.asarray(mask).reshape(9)
    if not np.all(m == 1):
        return None
    T = np.asarray(target, dtype=float).reshape(-1, 9)
    for a in range(3):
        off = [c for c in range(9) if c != 4 * a]
        if np.all(T[:, off] == 0.0):
            return a
    return None


def rotation_gauge_components(a):
    """Components held fixed by the gauge of axis a: with (a, b, c) in cyclic order, the
    entries F_ba, F_ca and F_cb (the strict lower triangle in the order a, b, c).

    Why this is the same problem: for periodic compatible F and divergence-free P the mean
    of P F^T equals <P> <F>^T (the fluctuation term integrates to zero), and P F^T is
    symmetric at every voxel for an objective law, so <P> <F>^T is symmetric at
    equilibrium.  With <F>_ba = <F>_ca = <F>_cb = 0 and the six other stress components at
    p e_a (x) e_a, that symmetry forces <P>_ba = <P>_ca = <P>_cb = 0: the released
    components still meet the target.  Among the rotated solutions Q F (Q P-bar = P-bar)
    exactly one has the three entries zero, so the gauge removes the null space of the
    rotations without changing the rotation invariants (<P>, <F>^T <F>, F^T F per voxel).
    """
    b, c = (a + 1) % 3, (a + 2) % 3
    return [3 * b + a, 3 * c + a, 3 * c + b]


def effective_mask(mask, target, gauge=True):
    """The control mask the solver uses: ``mask`` with the rotation gauge applied (its
    three components become deformation-controlled, held at their current value because
    their target entries are zero)."""
    m = np.asarray(mask, dtype=float).reshape(9).copy()
    if not gauge or target is None:
        return m
    a = rotation_gauge_axis(m, target)
    if a is not None:
        m[rotation_gauge_components(a)] = 0.0
    return m


# --------------------------------------------------------------------------------------
# Hyperelastic materials (Sec. 3.1 Saint Venant-Kirchhoff; compressible neo-Hookean)
# All functions act on voxel-first arrays of 3x3 matrices, shape (M, 3, 3).
# --------------------------------------------------------------------------------------

def _voxels(field9: np.ndarray) -> np.ndarray:
    """(9, nx, ny, nz) -> (N, 3, 3) view-copy, voxel first."""
    return np.ascontiguousarray(field9.reshape(9, -1).T).reshape(-1, 3, 3)


def _field(vox: np.ndarray, shape) -> np.ndarray:
    """(N, 3, 3) -> (9, nx, ny, nz)."""
    return np.ascontiguousarray(vox.reshape(-1, 9).T).reshape((9,) + tuple(shape))


def _check_det(J):
    if not np.all(J > 0.0):
        raise DomainError("det F <= 0 at %d voxel(s)" % int(np.sum(~(J > 0.0))))


def nh_energy(F, mu, lam):
    """Compressible neo-Hookean energy W = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2."""
    J = np.linalg.det(F)
    _check_det(J)
    lnJ = np.log(J)
    I1 = np.einsum("nij,nij->n", F, F)
    return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2


def nh_stress(F, mu, lam):
    """First Piola-Kirchhoff stress P = dW/dF = mu (F - F^-T) + lam ln J F^-T."""
    J = np.linalg.det(F)
    _check_det(J)
    FiT = np.linalg.inv(F).transpose(0, 2, 1)
    lnJ = np.log(J)
    return mu[:, None, None] * (F - FiT) + (lam * lnJ)[:, None, None] * FiT


def nh_tangent_apply(F, mu, lam, dF):
    """K : dF with K = dP/dF (eq. 4) for the neo-Hookean law.

    dP = mu dF + lam tr(F^-1 dF) F^-T + (mu - lam ln J) F^-T dF^T F^-T.
    """
    J = np.linalg.det(F)
    _check_det(J)
    Finv = np.linalg.inv(F)
    FiT = Finv.transpose(0, 2, 1)
    lnJ = np.log(J)
    tr = np.einsum("nij,nji->n", Finv, dF)
    back = FiT @ dF.transpose(0, 2, 1) @ FiT
    return (mu[:, None, None] * dF + (lam * tr)[:, None, None] * FiT
            + (mu - lam * lnJ)[:, None, None] * back)


def _green_lagrange(F):
    return 0.5 * (F.transpose(0, 2, 1) @ F - np.eye(3))


def svk_energy(F, C):
    """Saint Venant-Kirchhoff energy W = 1/2 E : C : E, E = (F^T F - I)/2; C shape (M,3,3,3,3)."""
    E = _green_lagrange(F)
    return 0.5 * np.einsum("nij,nijkl,nkl->n", E, C, E)


def svk_stress(F, C):
    """P = F S with S = C : E (Saint Venant-Kirchhoff)."""
    E = _green_lagrange(F)
    S = np.einsum("nijkl,nkl->nij", C, E)
    return F @ S


def svk_tangent_apply(F, C, dF):
    """K : dF = dF S + F (C : sym(F^T dF)) for Saint Venant-Kirchhoff."""
    E = _green_lagrange(F)
    S = np.einsum("nijkl,nkl->nij", C, E)
    FtdF = F.transpose(0, 2, 1) @ dF
    dE = 0.5 * (FtdF + FtdF.transpose(0, 2, 1))
    dS = np.einsum("nijkl,nkl->nij", C, dE)
    return dF @ S + F @ dS


# Finite-strain viscoelasticity (a path- and rate-dependent law with internal variables,
# eq. 1 of the paper's general setting; the paper's own crystal-plasticity model is not
# given).  Saint Venant-Kirchhoff form with one relaxing branch: S = Cinf : E + Q, where the
# overstress Q (symmetric, internal variable) obeys dQ/dt + Q / tau = C1 : dE/dt.  Over an
# increment of length dt with E linear in time the equation integrates exactly to
#   Q_{n+1} = a Q_n + b C1 : (E_{n+1} - E_n),  a = exp(-dt/tau),  b = tau (1 - a) / dt,
# and the algorithmic tangent of S is Cinf + b C1.  E_n and Q_n are the values committed at
# the end of the previous increment.
def visco_factors(dt, tau):
    """a = exp(-dt/tau) and b = tau (1 - a) / dt per voxel (b -> 1 as dt/tau -> 0)."""
    x = dt / np.asarray(tau, float)
    a = np.exp(-x)
    b = np.where(x > 0, -np.expm1(-x) / np.where(x > 0, x, 1.0), 1.0)
    return a, b


def visco_update(F, E_n, Q_n, Cinf, C1, a, b):
    """E, Q and S at the end of the increment for deformation gradient F."""
    E = _green_lagrange(F)
    Q = a[:, None, None] * Q_n + b[:, None, None] * np.einsum("nijkl,nkl->nij", C1, E - E_n)
    S = np.einsum("nijkl,nkl->nij", Cinf, E) + Q
    return E, Q, S


def visco_stress(F, E_n, Q_n, Cinf, C1, a, b):
    """P = F S of the viscoelastic law at the end of the increment."""
    return F @ visco_update(F, E_n, Q_n, Cinf, C1, a, b)[2]


def visco_tangent_apply(F, E_n, Q_n, Cinf, C1, a, b, dF):
    """K : dF = dF S + F ((Cinf + b C1) : sym(F^T dF)), the derivative of visco_stress in F
    at fixed E_n, Q_n and dt."""
    S = visco_update(F, E_n, Q_n, Cinf, C1, a, b)[2]
    FtdF = F.transpose(0, 2, 1) @ dF
    dE = 0.5 * (FtdF + FtdF.transpose(0, 2, 1))
    dS = np.einsum("nijkl,nkl->nij", Cinf, dE) + b[:, None, None] * np.einsum("nijkl,nkl->nij", C1, dE)
    return dF @ S + F @ dS


# --------------------------------------------------------------------------------------
# The solver: Newton (eq. 4, 20) with conjugate gradients on G*(K : dF) (Sec. 2.2-2.3)
# --------------------------------------------------------------------------------------

@dataclass
class StepRecord:
    """Outcome of one load increment."""
    F_avg: np.ndarray
    P_avg: np.ndarray
    newton_iters: int
    cg_iters: int
    cg_per_newton: list = field(default_factory=list)
    crit: float = float("nan")


class Oracle:
    """Plain FP64 Galerkin-FFT solver with per-component stress / deformation control.

    Usage mirrors the C library: set the grid, the material, the control mask and the
    load history, then call :meth:`step` once per increment.
    """

    CHUNK = 1 << 18  # voxels per material evaluation chunk (bounds temporary memory)

    def __init__(self, shape, lengths=(1.0, 1.0, 1.0)):
        self.shape = tuple(int(n) for n in shape)
        self.lengths = tuple(float(L) for L in lengths)
        self.N = int(np.prod(self.shape))
        self.kind = None
        self.phase = None
        self.scale = np.ones(self.N)
        self.mask = np.zeros(9)       # the mask the solver uses (rotation gauge applied)
        self.user_mask = np.zeros(9)  # the mask as set
        self.gauge = True
        self.target = None
        self.newton_tol = 1e-6
        self.cg_tol = 1e-8
        self.cg_forcing = 0.0
        self.max_newton = 50
        self.max_cg = 5000
        self.k = 0
        self.dt = 1.0
        self.cg_breakdowns = 0
        self.cg_stalls = 0
        self.cg_stall_window = 20
        self.F = np.tile(EYE9[:, None], (1, self.N)).reshape((9,) + self.shape)
        self.history: list[StepRecord] = []

    @property
    def gauge_axis(self):
        """Axis of the rotation gauge in use, or None (see rotation_gauge_axis)."""
        if not self.gauge or self.target is None:
            return None
        return rotation_gauge_axis(self.user_mask, self.target)

    # ---- set-up ---------------------------------------------------------------------
    def set_material_neohookean(self, phase, mu, lam):
        self.kind = "nh"
        self.phase = np.asarray(phase).reshape(-1).astype(np.int64)
        self.mu_tab = np.asarray(mu, dtype=float).reshape(-1)
        self.lam_tab = np.asarray(lam, dtype=float).reshape(-1)

    def set_material_svk(self, phase, C):
        """C: per-phase stiffness, shape (nphase, 3, 3, 3, 3) or (nphase, 81)."""
        self.kind = "svk"
        self.phase = np.asarray(phase).reshape(-1).astype(np.int64)
        self.C_tab = np.asarray(C, dtype=float).reshape(-1, 3, 3, 3, 3)

    def set_material_visco(self, phase, Cinf, C1, tau):
        """Viscoelastic law (see visco_update): per-phase equilibrium stiffness Cinf, branch
        stiffness C1 (each (nphase, 3, 3, 3, 3) or (nphase, 81)) and relaxation time tau.
        The internal variables start at E_n = Q_n = 0."""
        self.kind = "visco"
        self.phase = np.asarray(phase).reshape(-1).astype(np.int64)
        self.Cinf_tab = np.asarray(Cinf, dtype=float).reshape(-1, 3, 3, 3, 3)
        self.C1_tab = np.asarray(C1, dtype=float).reshape(-1, 3, 3, 3, 3)
        self.tau_tab = np.asarray(tau, dtype=float).reshape(-1)
        self.E_n = np.zeros((self.N, 3, 3))
        self.Q_n = np.zeros((self.N, 3, 3))
        self.checkpoints = []  # per increment: F at convergence, E_n, Q_n before the commit

    def set_time_step(self, dt):
        """Length of every load increment (rate-dependent laws only)."""
        self.dt = float(dt)

    def set_stiffness_scale(self, s):
        """Per-voxel factor s(x) > 0 multiplying every modulus of the voxel's phase."""
        self.scale = np.ones(self.N) if s is None else np.asarray(s, float).reshape(-1).copy()

    def set_control(self, mask):
        self.user_mask = np.asarray(mask, dtype=float).reshape(9).copy()
        self.mask = effective_mask(self.user_mask, self.target, self.gauge)

    def set_history(self, target):
        """target[k-1] holds, for increment k, P-bar on stress-controlled and F-bar on
        deformation-controlled components (Sec. 2.3, eq. 21)."""
        self.target = np.asarray(target, dtype=float).reshape(-1, 9).copy()
        self.mask = effective_mask(self.user_mask, self.target, self.gauge)

    def set_rotation_gauge(self, on):
        """Turn the rotation gauge of full stress control on (default) or off."""
        self.gauge = bool(on)
        self.mask = effective_mask(self.user_mask, self.target, self.gauge)

    def set_tolerances(self, newton_tol, cg_tol, cg_forcing=0.0, max_newton=50, max_cg=5000):
        self.newton_tol, self.cg_tol, self.cg_forcing = float(newton_tol), float(cg_tol), float(cg_forcing)
        self.max_newton, self.max_cg = int(max_newton), int(max_cg)

    def set_state(self, F9, k=None):
        self.F = np.array(F9, dtype=float).reshape((9,) + self.shape)
        if k is not None:
            self.k = int(k)

    # ---- material evaluation ---------------------------------------------------------
    def _chunks(self):
        for lo in range(0, self.N, self.CHUNK):
            yield slice(lo, min(self.N, lo + self.CHUNK))

    def _mat_args(self, sl):
        ph = self.phase[sl]
        s = self.scale[sl]
        if self.kind == "nh":
            return self.mu_tab[ph] * s, self.lam_tab[ph] * s
        if self.kind == "visco":
            a, b = visco_factors(self.dt, self.tau_tab[ph])
            return (self.E_n[sl], self.Q_n[sl], self.Cinf_tab[ph] * s[:, None, None, None, None],
                    self.C1_tab[ph] * s[:, None, None, None, None], a, b)
        return (self.C_tab[ph] * s[:, None, None, None, None],)

    def stress(self, F9=None) -> np.ndarray:
        """P(F) at every voxel, (9, nx, ny, nz)."""
        Fv = _voxels(self.F if F9 is None else F9)
        out = np.empty_like(Fv)
        for sl in self._chunks():
            args = self._mat_args(sl)
            if self.kind == "nh":
                out[sl] = nh_stress(Fv[sl], *args)
            elif self.kind == "visco":
                out[sl] = visco_stress(Fv[sl], *args)
            else:
                out[sl] = svk_stress(Fv[sl], *args)
        return _field(out, self.shape)

    def tangent_apply(self, dF9, F9=None) -> np.ndarray:
        """K(F) : dF at every voxel (eq. 4)."""
        Fv = _voxels(self.F if F9 is None else F9)
        dv = _voxels(dF9)
        out = np.empty_like(Fv)
        for sl in self._chunks():
            args = self._mat_args(sl)
            if self.kind == "nh":
                out[sl] = nh_tangent_apply(Fv[sl], *args, dv[sl])
            elif self.kind == "visco":
                out[sl] = visco_tangent_apply(Fv[sl], *args, dv[sl])
            else:
                out[sl] = svk_tangent_apply(Fv[sl], *args, dv[sl])
        return _field(out, self.shape)

    # ---- linear algebra of one Newton iteration --------------------------------------
    def apply_operator(self, v9, F9=None) -> np.ndarray:
        """A(v) = G*(K : v), the left-hand side of eq. (20)."""
        return apply_projection(self.tangent_apply(v9, F9), self.mask, self.lengths)

    def residual(self, P9, Pbar9) -> np.ndarray:
        """b = -G*(P(F) - P-bar), the right-hand side of eq. (20).

        P-bar is uniform, so it only meets G* at xi = 0, where the mask keeps it on the
        stress-controlled components and drops it on the deformation-controlled ones.
        """
        diff = P9 - np.asarray(Pbar9, float).reshape(9, 1, 1, 1)
        return -apply_projection(diff, self.mask, self.lengths)

    def rms(self, v9) -> float:
        """Voxel-averaged L2 norm: sqrt( (1/N) sum_x |v(x)|^2 ) (Sec. 4)."""
        return math.sqrt(float(np.vdot(v9, v9)) / self.N)

    @staticmethod
    def newton_criterion(dF9, Favg9) -> float:
        """Newton stop quantity of Sec. 4: the largest correction of the deformation gradient
        over the voxels relative to the averaged one, max_x |dF(x)| / |<F>| (Frobenius
        norms)."""
        per_voxel = np.sqrt(np.sum(np.asarray(dF9, float).reshape(9, -1) ** 2, axis=0))
        return float(np.max(per_voxel)) / float(np.linalg.norm(np.asarray(Favg9, float).reshape(9)))

    def conjugate_gradient(self, b9, F9=None):
        """Solve A dF = b by plain conjugate gradients from dF = 0 (Sec. 2.1).

        Stop when rms(r) <= max(cg_tol, cg_forcing * rms(b)) (absolute voxel-averaged L2
        norm of the residual, Sec. 4).  Returns (dF, iterations).

        Breakdown (p.Ap <= 0 or not finite): at the first iteration nothing can be done and
        BreakdownError is raised; later, the iterate reached so far is returned and the
        count ``self.cg_breakdowns`` is raised by one.  Under full stress control without
        the rotation gauge the rigid rotations that leave P-bar unchanged make A singular
        (slightly indefinite away from equilibrium); CG then stalls at round-off level and
        the Newton loop carries on.

        Stall (a reading; the paper names no safeguard): when r.r has not gone below its
        smallest value in the solve for ``cg_stall_window`` iterations in a row, the
        residual has a floor above the threshold (a right-hand side the operator cannot
        reach); the iterate is returned and ``self.cg_stalls`` is raised by one.
        """
        x = np.zeros_like(b9)
        r = b9.copy()
        p = r.copy()
        rr = float(np.vdot(r, r))
        tol = max(self.cg_tol, self.cg_forcing * math.sqrt(rr / self.N))
        best, since = rr, 0
        it = 0
        while math.sqrt(rr / self.N) > tol:
            if it >= self.max_cg:
                raise NotConvergedError("CG reached max_cg=%d" % self.max_cg)
            if since >= self.cg_stall_window:
                self.cg_stalls += 1
                break
            Ap = self.apply_operator(p, F9)
            pAp = float(np.vdot(p, Ap))
            if not (pAp > 0.0 and math.isfinite(pAp)):
                if it == 0 or not math.isfinite(pAp):
                    raise BreakdownError("CG breakdown: p.Ap = %r at iteration %d" % (pAp, it))
                self.cg_breakdowns += 1
                break
            alpha = rr / pAp
            x += alpha * p
            r -= alpha * Ap
            rr_new = float(np.vdot(r, r))
            beta = rr_new / rr
            p = r + beta * p
            rr = rr_new
            it += 1
            if rr < best:
                best, since = rr, 0
            else:
                since += 1
        return x, it

    def averages(self, F9=None, P9=None):
        F9 = self.F if F9 is None else F9
        P9 = self.stress(F9) if P9 is None else P9
        return F9.reshape(9, -1).mean(axis=1), P9.reshape(9, -1).mean(axis=1)

    # ---- one load increment ----------------------------------------------------------
    def step(self) -> StepRecord:
        """Advance one increment: shift the prescribed F means, then Newton (eq. 20/22)."""
        if self.kind is None or self.target is None:
            raise OracleError("material and history must be set before step()")
        k = self.k + 1
        if k > len(self.target):
            raise OracleError("history exhausted")
        fmask = self.mask == 0
        prev = EYE9 if k == 1 else self.target[k - 2]
        # deformation-controlled means move uniformly by the change of F-bar (eq. 3, 21)
        shift = np.where(fmask, self.target[k - 1] - prev, 0.0)
        Pbar = np.where(fmask, 0.0, self.target[k - 1])
        self.F = self.F + shift.reshape(9, 1, 1, 1)
        rec = self.newton(Pbar)
        self.k = k
        if self.kind == "visco":
            self.checkpoints.append((self.F.copy(), self.E_n.copy(), self.Q_n.copy(), self.dt))
            self.commit()
        self.history.append(rec)
        return rec

    def commit(self):
        """End of an increment of the viscoelastic law: E_n and Q_n take their values at
        the converged F."""
        Fv = _voxels(self.F)
        E_new = np.empty_like(self.E_n)
        Q_new = np.empty_like(self.Q_n)
        for sl in self._chunks():
            E_new[sl], Q_new[sl], _ = visco_update(Fv[sl], *self._mat_args(sl))
        self.E_n, self.Q_n = E_new, Q_new

    def target_stress(self, k=None):
        """P-bar of increment k (default: the current one) on the stress-controlled
        components, 0 elsewhere."""
        k = self.k if k is None else k
        return np.where(self.mask > 0, self.target[k - 1], 0.0)

    def newton(self, Pbar) -> StepRecord:
        """Newton iterations (eq. 4, 20) from the current F to equilibrium under P-bar.

        Each iteration evaluates P(F) and b = -G*(P - P-bar), stops at once if
        rms(b) <= cg_tol (nothing left to correct), else solves A dF = b by CG, sets
        F += dF and stops when max_x |dF(x)| / |<F>| < newton_tol (Sec. 4).
        """
        newton = 0
        cg_total = 0
        per = []
        crit = float("inf")
        converged = False
        for _ in range(self.max_newton):
            newton += 1
            P = self.stress()
            b = self.residual(P, Pbar)
            if self.rms(b) <= self.cg_tol:
                per.append(0)
                converged = True
                break
            dF, its = self.conjugate_gradient(b)
            per.append(its)
            cg_total += its
            self.F = self.F + dF
            crit = self.newton_criterion(dF, self.F.reshape(9, -1).mean(axis=1))
            if crit < self.newton_tol:
                converged = True
                break
        if not converged:
            raise NotConvergedError("Newton reached max_newton=%d (crit %.3e)" % (self.max_newton, crit))
        # P at the converged F (for a path-dependent law: before the internal variables are
        # committed at the end of the increment)
        self.P_last = self.stress()
        Favg, Pavg = self.averages(P9=self.P_last)
        return StepRecord(Favg, Pavg, newton, cg_total, per, crit)

    # ---- adjoint ---------------------------------------------------------------------
    def adjoint_grad_scale_history(self, a9) -> np.ndarray:
        """Gradient of J = a : <F> at the end of the history with respect to s(x), for the
        viscoelastic law (a backward sweep over the checkpointed increments).

        Increment n solves G*(P_n - P-bar_n) = 0 with P_n = F_n S_n,
        S_n = s Cinf:E_n + a Q_{n-1} + b s C1:(E_n - E_{n-1}), then commits E_n = E(F_n),
        Q_n = a Q_{n-1} + b s C1:(E_n - E_{n-1}).  Linearising in s and eliminating each
        increment's correction with an adjoint field lam_n (A_n lam_n = G*(h_n), A_n the
        increment's operator, symmetric on the range of G*), with L_n = sym(F_n^T lam_n):
          h_n = F_n (mE + b s C1:mQ)  (+ a/N uniform at the last increment),
          dJ/ds += b mQ:C1:(E_n - E_{n-1}) - L_n:(Cinf:E_n + b C1:(E_n - E_{n-1})),
          mQ <- a (mQ - L_n),  mE <- b s C1:(L_n - mQ)  (mQ, mE start at zero),
        from the last increment back to the first.  With C1 = 0 it reduces to
        adjoint_grad_scale (-lam : P / s).
        """
        if self.kind != "visco":
            raise OracleError("the history adjoint is for the viscoelastic law")
        if len(self.checkpoints) != self.k or self.k == 0:
            raise OracleError("the history adjoint needs every increment since the start")
        keep = (self.F, self.E_n, self.Q_n, self.dt)
        ph = self.phase
        s = self.scale
        Cinf = self.Cinf_tab[ph]
        C1 = self.C1_tab[ph]
        mQ = np.zeros((self.N, 3, 3))
        mE = np.zeros((self.N, 3, 3))
        grad = np.zeros(self.N)
        abar = np.broadcast_to(np.asarray(a9, float).reshape(9, 1, 1, 1) / self.N, (9,) + self.shape)
        try:
            for n in range(self.k, 0, -1):
                F9, E_prev, Q_prev, dt = self.checkpoints[n - 1]
                self.F, self.E_n, self.Q_n, self.dt = F9, E_prev, Q_prev, dt
                a, b = visco_factors(dt, self.tau_tab[ph])
                Fv = _voxels(F9)
                E = _green_lagrange(Fv)
                C1mQ = np.einsum("nijkl,nkl->nij", C1, mQ)
                M = mE + (b * s)[:, None, None] * C1mQ
                h = _field(Fv @ M, self.shape)
                if n == self.k:
                    h = h + abar
                lam, _ = self.conjugate_gradient(apply_projection(np.ascontiguousarray(h), self.mask, self.lengths))
                lv = _voxels(lam)
                FtL = Fv.transpose(0, 2, 1) @ lv
                L = 0.5 * (FtL + FtL.transpose(0, 2, 1))
                dE = E - E_prev
                C1dE = np.einsum("nijkl,nkl->nij", C1, dE)
                T = np.einsum("nijkl,nkl->nij", Cinf, E) + b[:, None, None] * C1dE
                grad += b * np.einsum("nij,nij->n", mQ, C1dE) - np.einsum("nij,nij->n", L, T)
                mE = (b * s)[:, None, None] * np.einsum("nijkl,nkl->nij", C1, L - mQ)
                mQ = a[:, None, None] * (mQ - L)
        finally:
            self.F, self.E_n, self.Q_n, self.dt = keep
        return grad.reshape(self.shape)

    def adjoint_grad_scale(self, a9) -> np.ndarray:
        """Gradient of J = a : <F> with respect to the per-voxel stiffness scale s(x).

        At a converged state G*(P(F, s) - P-bar) = 0 with the unknown part of F in the
        range of G*.  Differentiating, A dF/ds = -G*(dP/ds); J changes by
        <a/N, dF> = <G*(a/N), dF>.  With lam solving A lam = G*(a/N) (A is symmetric on
        the range of G*), dJ/ds(x) = -lam(x) : dP/ds(x) = -lam(x) : P(x) / s(x), because
        every modulus is proportional to s.
        """
        if self.kind == "visco":
            raise OracleError("the adjoint here is for path-independent (hyperelastic) laws")
        g = np.broadcast_to(np.asarray(a9, float).reshape(9, 1, 1, 1) / self.N, (9,) + self.shape)
        rhs = apply_projection(np.ascontiguousarray(g), self.mask, self.lengths)
        lam, _ = self.conjugate_gradient(rhs)
        P = self.stress()
        return -(np.sum(lam * P, axis=0) / self.scale.reshape(self.shape))


def run_history(oracle: Oracle, nsteps=None):
    """Run increments 1..nsteps (default: the whole history); returns the records."""
    n = len(oracle.target) if nsteps is None else int(nsteps)
    return [oracle.step() for _ in range(n)]
