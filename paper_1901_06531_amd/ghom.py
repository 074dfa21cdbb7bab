"""ctypes binding of libghom.so (include/ghom.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module converts NumPy
arrays to the C layouts, hands device pointers of torch tensors through, and turns status
codes into exceptions.  Importing it loads the library and raises if it is missing.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libghom.so")

FP64 = 0
FP32_SPLIT = 1
FIELD_F = 0
FIELD_P = 1
OPT_XPROJ_F64 = 1
OPT_XPROJ_F32 = 2
OPT_ZSLABS = 3
OPT_GRAPHS = 4
OPT_CHECKPOINTS = 5
OPT_STREAM_NT = 6
OPT_ROTATION_GAUGE = 7
OPT_YPASS_F64 = 8
OPT_YPASS_F32 = 9
OPT_PROFILE_EVERY = 10

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTCONVERGED", -5: "ESINGULAR",
          -6: "EDOMAIN", -7: "ESTATE"}
STATUS_CODE = {v: k for k, v in STATUS.items()}


class GhomError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code
        self.name = STATUS.get(code, "?")


class StepInfo(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int), ("cg_iters_total", ctypes.c_int),
                ("cg_breakdowns", ctypes.c_int), ("status", ctypes.c_int),
                ("crit", ctypes.c_double), ("res_rms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("t_cg_ms", ctypes.c_double),
                ("cg_stalls", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i = ctypes.c_int
MATERIAL_NEOHOOKEAN = 1
MATERIAL_SVK = 2


class Problem(ctypes.Structure):
    """ghom_problem: one problem of a batch."""
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("kind", ctypes.c_int),
                ("phase", ctypes.c_void_p), ("nphase", ctypes.c_int), ("mu", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("C", ctypes.c_void_p), ("mask", ctypes.c_uint8 * 9),
                ("nsteps", ctypes.c_int), ("target", ctypes.c_void_p)]
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "ghom_create": (_i, [ctypes.POINTER(_vp), _i, _i, _i, _d, _d, _d, _i, _i, _vp]),
    "ghom_destroy": (None, [_vp]),
    "ghom_last_error": (ctypes.c_char_p, [_vp]),
    "ghom_set_material_neohookean": (_i, [_vp, _vp, _i, _vp, _vp]),
    "ghom_set_material_svk": (_i, [_vp, _vp, _i, _vp]),
    "ghom_set_material_visco": (_i, [_vp, _vp, _i, _vp, _vp, _vp]),
    "ghom_set_time_step": (_i, [_vp, _d]),
    "ghom_set_stiffness_scale": (_i, [_vp, _vp]),
    "ghom_set_control": (_i, [_vp, _vp]),
    "ghom_get_control": (_i, [_vp, _vp, ctypes.POINTER(_i)]),
    "ghom_set_history": (_i, [_vp, _i, _vp]),
    "ghom_set_tolerances": (_i, [_vp, _d, _d, _d, _i, _i]),
    "ghom_step": (_i, [_vp, ctypes.POINTER(StepInfo)]),
    "ghom_step_adaptive": (_i, [_vp, _i, _i, ctypes.POINTER(StepInfo), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "ghom_resolve": (_i, [_vp, ctypes.POINTER(StepInfo)]),
    "ghom_get_averages": (_i, [_vp, _vp, _vp]),
    "ghom_get_field": (_i, [_vp, _i, _vp]),
    "ghom_get_field_device": (_i, [_vp, _i, _vp]),
    "ghom_save_state": (_i, [_vp, _vp, ctypes.POINTER(_i)]),
    "ghom_load_state": (_i, [_vp, _vp, _i]),
    "ghom_adjoint_grad_scale": (_i, [_vp, _vp, _vp]),
    "ghom_apply_operator": (_i, [_vp, _vp, _vp]),
    "ghom_apply_projection": (_i, [_vp, _vp, _vp]),
    "ghom_apply_projection_static": (_i, [_i, _i, _i, _d, _d, _d, _vp, _vp, _vp, _i, _vp]),
    "ghom_residual": (_i, [_vp, _vp, _vp]),
    "ghom_batch_create": (_i, [ctypes.POINTER(_vp), _vp, _i, _i, _i, _vp]),
    "ghom_batch_destroy": (None, [_vp]),
    "ghom_batch_last_error": (ctypes.c_char_p, [_vp]),
    "ghom_batch_set_tolerances": (_i, [_vp, _d, _d, _d, _i, _i]),
    "ghom_batch_step": (_i, [_vp, _vp]),
    "ghom_batch_get_averages": (_i, [_vp, _i, _vp, _vp]),
    "ghom_batch_get_field": (_i, [_vp, _i, _i, _vp]),
    "ghom_batch_set_option": (_i, [_vp, _i, _i]),
    "ghom_batch_num_classes": (_i, [_vp]),
    "ghom_set_option": (_i, [_vp, _i, _i]),
    "ghom_get_option": (_i, [_vp, _i, ctypes.POINTER(_i)]),
    "ghom_get_schedule": (_i, [_vp, ctypes.c_char_p, _i]),
    "ghom_batch_get_schedule": (_i, [_vp, _i, ctypes.c_char_p, _i]),
    "ghom_set_profiling": (_i, [_vp, _i]),
    "ghom_set_profiling_filter": (_i, [_vp, ctypes.c_char_p]),
    "ghom_profile_count": (_i, [_vp]),
    "ghom_profile_get": (_i, [_vp, _i, ctypes.c_char_p, _i, ctypes.POINTER(_i), _dp]),
    "ghom_profile_samples": (_i, [_vp, _i, _vp, _i]),
    "ghom_profile_reset": (_i, [_vp]),
}

_lib = None


def _bind_torch_runtime():
    """Load torch's HIP runtime before libghom.so so that the process holds one runtime.

    torch ships its own libamdhip64 / libhsa-runtime64 with the same sonames as the system
    ones libghom.so is linked against.  Loaded first, torch's copies satisfy libghom.so's
    dependencies; loaded second they would come in as a second runtime and torch would
    then find no device.
    """
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _bind_torch_runtime()
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libghom.so not built at %s: run paper_1901_06531_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t):
    """Device pointer of a contiguous torch CUDA tensor."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _field_ptr(t, numel, dtype, device, what):
    """Device pointer of a field tensor after checking what the C ABI cannot: a contiguous
    tensor of `numel` values of `dtype` on GPU `device`."""
    if not getattr(t, "is_cuda", False) or not t.is_contiguous():
        raise ValueError("%s: expected a contiguous device tensor" % what)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, not %s" % (what, dtype, t.dtype))
    if t.numel() != numel:
        raise ValueError("%s must hold 9 x N = %d values, not %d" % (what, numel, t.numel()))
    if t.device.index != device:
        raise ValueError("%s is on cuda:%s, the solver on cuda:%d" % (what, t.device.index, device))
    return ctypes.c_void_p(t.data_ptr())


def _torch_sync():
    import torch
    if torch.cuda.is_available():
        torch.cuda.synchronize()


def apply_projection_static(v, out, mask, lengths=(1.0, 1.0, 1.0), stream=None):
    """out = G*(v) without a context or any device allocation (ghom_apply_projection_static).

    v and out: float64 device tensors of shape (9, nx, ny, nz) on one GPU (they may be the
    same tensor), at most 64^3 voxels; mask: 9 entries, 1 = stress-controlled.  The caller
    provides `out`: nothing is allocated here or in the library."""
    import torch
    if v.dim() != 4 or v.shape[0] != 9:
        raise ValueError("expected a field of shape (9, nx, ny, nz)")
    nx, ny, nz = (int(n) for n in v.shape[1:])
    dev = v.device.index if v.device.index is not None else 0
    vp = _field_ptr(v, 9 * nx * ny * nz, torch.float64, dev, "projection input")
    op = _field_ptr(out, 9 * nx * ny * nz, torch.float64, dev, "projection output")
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(9)
    _torch_sync()
    rc = lib().ghom_apply_projection_static(nx, ny, nz, *[float(L) for L in lengths], _ptr(m), vp, op, dev, stream)
    if rc != 0:
        raise GhomError(rc, lib().ghom_last_error(None).decode())
    return out


class Solver:
    """One Galerkin-FFT problem on one GPU (a ghom_ctx)."""

    def __init__(self, shape, lengths=(1.0, 1.0, 1.0), precision=FP64, device=0, stream=None):
        self.shape = tuple(int(n) for n in shape)
        self.N = int(np.prod(self.shape))
        self.precision = precision
        self.device = int(device)
        self._c = ctypes.c_void_p()
        rc = lib().ghom_create(ctypes.byref(self._c), *self.shape, *[float(v) for v in lengths],
                               int(precision), int(device), stream)
        if rc != 0:
            raise GhomError(rc, "ghom_create failed for shape %s: %s" % (self.shape, lib().ghom_last_error(None).decode()))

    # -- plumbing ------------------------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise GhomError(rc, lib().ghom_last_error(self._c).decode())
        return rc

    def close(self):
        if self._c:
            lib().ghom_destroy(self._c)
            self._c = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- set-up --------------------------------------------------------------------------
    def set_material_neohookean(self, phase, mu, lam):
        ph = np.ascontiguousarray(np.asarray(phase).reshape(-1), dtype=np.uint16)
        mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(-1)
        lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
        self._check(lib().ghom_set_material_neohookean(self._c, _ptr(ph), len(mu), _ptr(mu), _ptr(lam)))

    def set_material_svk(self, phase, C):
        ph = np.ascontiguousarray(np.asarray(phase).reshape(-1), dtype=np.uint16)
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(-1, 81)
        self._check(lib().ghom_set_material_svk(self._c, _ptr(ph), C.shape[0], _ptr(C)))

    def set_material_visco(self, phase, Cinf, C1, tau):
        ph = np.ascontiguousarray(np.asarray(phase).reshape(-1), dtype=np.uint16)
        Ci = np.ascontiguousarray(Cinf, dtype=np.float64).reshape(-1, 81)
        C1 = np.ascontiguousarray(C1, dtype=np.float64).reshape(-1, 81)
        tau = np.ascontiguousarray(tau, dtype=np.float64).reshape(-1)
        if not (Ci.shape[0] == C1.shape[0] == tau.shape[0]):
            raise ValueError("Cinf, C1 and tau need one entry per phase")
        self._check(lib().ghom_set_material_visco(self._c, _ptr(ph), Ci.shape[0], _ptr(Ci), _ptr(C1), _ptr(tau)))

    def set_time_step(self, dt):
        self._check(lib().ghom_set_time_step(self._c, float(dt)))

    def set_stiffness_scale(self, s):
        if s is None:
            self._check(lib().ghom_set_stiffness_scale(self._c, None))
        else:
            s = np.ascontiguousarray(s, dtype=np.float64).reshape(-1)
            self._check(lib().ghom_set_stiffness_scale(self._c, _ptr(s)))

    def set_control(self, mask):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(9)
        self._check(lib().ghom_set_control(self._c, _ptr(m)))
        self.mask = m.copy()

    def set_history(self, target):
        t = np.ascontiguousarray(target, dtype=np.float64).reshape(-1, 9)
        self._check(lib().ghom_set_history(self._c, t.shape[0], _ptr(t)))
        self.nsteps = t.shape[0]

    def control(self):
        """(mask in use, rotation-gauge axis or -1): the mask as set with the rotation gauge
        of full stress control applied (ghom_get_control)."""
        m = np.zeros(9, dtype=np.uint8)
        a = ctypes.c_int()
        self._check(lib().ghom_get_control(self._c, _ptr(m), ctypes.byref(a)))
        return m, a.value

    def set_tolerances(self, newton_tol=1e-6, cg_tol=1e-8, cg_forcing=0.0, max_newton=50, max_cg=5000):
        self._check(lib().ghom_set_tolerances(self._c, newton_tol, cg_tol, cg_forcing, max_newton, max_cg))

    def setup(self, w, precision_tols=None):
        """Applies a workload dict of paper_1901_06531_amd.synth."""
        if w["kind"] == "nh":
            self.set_material_neohookean(w["phase"], w["mu"], w["lam"])
        elif w["kind"] == "visco":
            self.set_material_visco(w["phase"], w["Cinf"], w["C1"], w["tau"])
        else:
            self.set_material_svk(w["phase"], w["C"])
        if w.get("dt") is not None:
            self.set_time_step(w["dt"])
        if w.get("scale") is not None:
            self.set_stiffness_scale(w["scale"])
        self.set_control(w["mask"])
        self.set_history(w["target"])
        self.set_tolerances(w["newton_tol"], w["cg_tol"])
        return self

    # -- solve ---------------------------------------------------------------------------
    def step(self, check=True):
        """One load increment (ghom_step).  With check=False a failed increment returns its
        info dict (with 'status' and 'error') instead of raising."""
        info = StepInfo()
        rc = lib().ghom_step(self._c, ctypes.byref(info))
        if check or rc == 0:
            self._check(rc)
            return info.as_dict()
        d = info.as_dict()
        d.update(status=rc, error="%s: %s" % (STATUS.get(rc, "?"), lib().ghom_last_error(self._c).decode()))
        return d

    def step_adaptive(self, max_cuts=8, grow_below=2):
        """One load increment in sub-increments (ghom_step_adaptive); the info dict also
        holds 'substeps' and 'cuts'."""
        info = StepInfo()
        subs, cuts = ctypes.c_int(), ctypes.c_int()
        rc = lib().ghom_step_adaptive(self._c, int(max_cuts), int(grow_below), ctypes.byref(info),
                                      ctypes.byref(subs), ctypes.byref(cuts))
        self._check(rc)
        d = info.as_dict()
        d.update(substeps=subs.value, cuts=cuts.value)
        return d

    def resolve(self):
        info = StepInfo()
        self._check(lib().ghom_resolve(self._c, ctypes.byref(info)))
        return info.as_dict()

    def averages(self):
        F = np.zeros(9)
        P = np.zeros(9)
        self._check(lib().ghom_get_averages(self._c, _ptr(F), _ptr(P)))
        return F, P

    def field(self, which=FIELD_F):
        out = np.empty((9,) + self.shape)
        self._check(lib().ghom_get_field(self._c, int(which), _ptr(out)))
        return out

    def field_device(self, which=FIELD_F, out=None):
        """Field `which` into a float64 device tensor of shape (9, nx, ny, nz)
        (ghom_get_field_device)."""
        import torch
        if out is None:
            out = torch.empty((9,) + self.shape, dtype=torch.float64, device=torch.device("cuda", self.device))
        ptr = _field_ptr(out, 9 * self.N, torch.float64, self.device, "field output")
        _torch_sync()
        self._check(lib().ghom_get_field_device(self._c, int(which), ptr))
        return out

    def save_state(self):
        out = np.empty((9,) + self.shape)
        k = ctypes.c_int()
        self._check(lib().ghom_save_state(self._c, _ptr(out), ctypes.byref(k)))
        return out, k.value

    def load_state(self, F, k):
        F = np.ascontiguousarray(F, dtype=np.float64).reshape((9,) + self.shape)
        self._check(lib().ghom_load_state(self._c, _ptr(F), int(k)))

    def adjoint_grad_scale(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(9)
        out = np.empty(self.shape)
        self._check(lib().ghom_adjoint_grad_scale(self._c, _ptr(a), _ptr(out)))
        return out

    # -- device entry points (torch tensors as device memory) ----------------------------
    def apply_operator(self, v, out=None):
        import torch
        dt = torch.float64 if self.precision == FP64 else torch.float32
        vp = _field_ptr(v, 9 * self.N, dt, self.device, "operator input")
        out = torch.empty_like(v) if out is None else out
        op = _field_ptr(out, 9 * self.N, dt, self.device, "operator output")
        if op.value == vp.value:
            raise ValueError("operator input and output must not overlap")
        _torch_sync()
        self._check(lib().ghom_apply_operator(self._c, vp, op))
        return out

    def apply_projection(self, v, out=None):
        import torch
        vp = _field_ptr(v, 9 * self.N, torch.float64, self.device, "projection input")
        out = torch.empty_like(v) if out is None else out
        op = _field_ptr(out, 9 * self.N, torch.float64, self.device, "projection output")
        _torch_sync()
        self._check(lib().ghom_apply_projection(self._c, vp, op))
        return out

    def residual(self, Pbar):
        import torch
        out = torch.empty((9,) + self.shape, dtype=torch.float64, device=torch.device("cuda", self.device))
        Pb = np.ascontiguousarray(Pbar, dtype=np.float64).reshape(9)
        _torch_sync()
        self._check(lib().ghom_residual(self._c, _ptr(Pb), _dev_ptr(out)))
        return out

    # -- kernel options ------------------------------------------------------------------
    def set_option(self, key, value):
        self._check(lib().ghom_set_option(self._c, int(key), int(value)))

    def get_option(self, key):
        v = ctypes.c_int()
        self._check(lib().ghom_get_option(self._c, int(key), ctypes.byref(v)))
        return v.value

    def schedule(self):
        """The kernel schedule in use (ghom_get_schedule)."""
        buf = ctypes.create_string_buffer(512)
        n = lib().ghom_get_schedule(self._c, buf, 512)
        if n < 0:
            self._check(n)
        return buf.value.decode()

    # -- profiling -----------------------------------------------------------------------
    def set_profiling(self, on=True):
        self._check(lib().ghom_set_profiling(self._c, int(bool(on))))

    def set_profiling_filter(self, name=None):
        """Time only the launches recorded under `name` (None: all)."""
        self._check(lib().ghom_set_profiling_filter(self._c, None if name is None else name.encode()))

    def profile(self):
        n = lib().ghom_profile_count(self._c)
        out = {}
        buf = ctypes.create_string_buffer(128)
        for i in range(n):
            cnt = ctypes.c_int()
            ms = ctypes.c_double()
            self._check(lib().ghom_profile_get(self._c, i, buf, 128, ctypes.byref(cnt), ctypes.byref(ms)))
            out[buf.value.decode()] = (cnt.value, ms.value)
        return out

    def profile_samples(self, name):
        """Per-launch milliseconds of the record `name` (ghom_profile_samples)."""
        n = lib().ghom_profile_count(self._c)
        buf = ctypes.create_string_buffer(128)
        for i in range(n):
            self._check(lib().ghom_profile_get(self._c, i, buf, 128, None, None))
            if buf.value.decode() == name:
                cnt = lib().ghom_profile_samples(self._c, i, None, 0)
                if cnt < 0:
                    self._check(cnt)
                out = np.zeros(cnt, dtype=np.float32)
                got = lib().ghom_profile_samples(self._c, i, _ptr(out), cnt)
                if got < 0:
                    self._check(got)
                return out
        raise KeyError(name)

    def profile_reset(self):
        self._check(lib().ghom_profile_reset(self._c))


class Batch:
    """Many independent problems advanced together (a ghom_batch).

    ``workloads`` is a list of dicts as made by paper_1901_06531_amd.synth (shape, kind,
    phase, mu/lam or C, mask, target)."""

    def __init__(self, workloads, precision=FP32_SPLIT, device=0, stream=None):
        self.n = len(workloads)
        self.shapes = [tuple(int(v) for v in w["shape"]) for w in workloads]
        self._keep = []
        arr = (Problem * self.n)()
        for i, w in enumerate(workloads):
            pr = arr[i]
            pr.nx, pr.ny, pr.nz = self.shapes[i]
            ph = np.ascontiguousarray(np.asarray(w["phase"]).reshape(-1), dtype=np.uint16)
            tgt = np.ascontiguousarray(w["target"], dtype=np.float64).reshape(-1, 9)
            self._keep += [ph, tgt]
            pr.phase = ph.ctypes.data
            pr.target = tgt.ctypes.data
            pr.nsteps = tgt.shape[0]
            for c in range(9):
                pr.mask[c] = int(np.asarray(w["mask"]).reshape(9)[c])
            if w["kind"] == "nh":
                mu = np.ascontiguousarray(w["mu"], dtype=np.float64).reshape(-1)
                lam = np.ascontiguousarray(w["lam"], dtype=np.float64).reshape(-1)
                self._keep += [mu, lam]
                pr.kind = MATERIAL_NEOHOOKEAN
                pr.nphase = len(mu)
                pr.mu, pr.lam = mu.ctypes.data, lam.ctypes.data
            else:
                C = np.ascontiguousarray(w["C"], dtype=np.float64).reshape(-1, 81)
                self._keep.append(C)
                pr.kind = MATERIAL_SVK
                pr.nphase = C.shape[0]
                pr.C = C.ctypes.data
        self._b = ctypes.c_void_p()
        rc = lib().ghom_batch_create(ctypes.byref(self._b), ctypes.cast(arr, ctypes.c_void_p), self.n, int(precision),
                                     int(device), stream)
        self._keep = None
        if rc != 0:
            raise GhomError(rc, "ghom_batch_create failed: %s" % lib().ghom_batch_last_error(None).decode())

    def _check(self, rc):
        if rc != 0:
            raise GhomError(rc, lib().ghom_batch_last_error(self._b).decode())
        return rc

    def close(self):
        if self._b:
            lib().ghom_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_tolerances(self, newton_tol=1e-6, cg_tol=1e-8, cg_forcing=0.0, max_newton=50, max_cg=5000):
        self._check(lib().ghom_batch_set_tolerances(self._b, newton_tol, cg_tol, cg_forcing, max_newton, max_cg))

    def set_option(self, key, value):
        self._check(lib().ghom_batch_set_option(self._b, int(key), int(value)))

    def num_classes(self):
        return lib().ghom_batch_num_classes(self._b)

    def schedules(self):
        """The kernel schedule of every launch group (ghom_batch_get_schedule)."""
        out = []
        buf = ctypes.create_string_buffer(512)
        for i in range(self.num_classes()):
            n = lib().ghom_batch_get_schedule(self._b, i, buf, 512)
            if n < 0:
                self._check(n)
            out.append(buf.value.decode())
        return out

    def step(self, raise_on_error=True):
        infos = (StepInfo * self.n)()
        rc = lib().ghom_batch_step(self._b, ctypes.cast(infos, ctypes.c_void_p))
        if raise_on_error:
            self._check(rc)
        return [infos[i].as_dict() for i in range(self.n)]

    def averages(self, i):
        F = np.zeros(9)
        P = np.zeros(9)
        self._check(lib().ghom_batch_get_averages(self._b, int(i), _ptr(F), _ptr(P)))
        return F, P

    def field(self, i, which=FIELD_F):
        out = np.empty((9,) + self.shapes[i])
        self._check(lib().ghom_batch_get_field(self._b, int(i), int(which), _ptr(out)))
        return out


def _autograd_function():
    import torch

    class HomogenizedResponse(torch.autograd.Function):
        """Differentiable map s(x) -> (<F>, <P>) at the end of a solver's load history.

        ``HomogenizedResponse.apply(s, solver)``: ``solver`` is a set-up Solver (material,
        control, history, tolerances); s is the per-voxel stiffness scale (any torch tensor
        of N values).  Forward sets s, restarts from F = I and runs every increment; it
        returns <F> and <P> as float64 tensors of 9 values on the device of s.

        Backward evaluates dJ/ds for J = g_F : <F> by the adjoint solve of the library
        (ghom_adjoint_grad_scale with a = g_F) at the final state.  On stress-controlled
        components <P> equals the prescribed value for every s, so its cotangent adds
        nothing; a cotangent of <P> on a deformation-controlled component is rejected
        (that derivative needs another adjoint right-hand side, which is not provided).
        """

        @staticmethod
        def forward(ctx, s, solver):
            sv = s.detach().to("cpu", torch.float64).reshape(-1).numpy()
            if sv.size != solver.N:
                raise ValueError("s must hold one value per voxel (%d), got %d" % (solver.N, sv.size))
            solver.set_stiffness_scale(sv)
            eye = np.broadcast_to(np.eye(3).reshape(9, 1, 1, 1), (9,) + solver.shape)
            solver.load_state(eye, 0)
            for _ in range(solver.nsteps):
                solver.step()
            Fbar, Pbar = solver.averages()
            ctx.solver = solver
            ctx.sv = sv.copy()
            ctx.state = solver.save_state()
            ctx.shape_s = s.shape
            return (torch.as_tensor(Fbar, device=s.device), torch.as_tensor(Pbar, device=s.device))

        @staticmethod
        def backward(ctx, gF, gP):
            solver = ctx.solver
            if gP is not None:
                gp = gP.detach().to("cpu", torch.float64).numpy()
                fctl = np.asarray(solver.mask).reshape(9) == 0
                if np.any(gp[fctl] != 0.0):
                    raise NotImplementedError("gradient of <P> on deformation-controlled components")
            a = np.zeros(9) if gF is None else gF.detach().to("cpu", torch.float64).numpy()
            solver.set_stiffness_scale(ctx.sv)
            solver.load_state(*ctx.state)
            g = solver.adjoint_grad_scale(a)
            dev = gF.device if gF is not None else gP.device
            return torch.as_tensor(g, device=dev).reshape(ctx.shape_s), None

    return HomogenizedResponse


def __getattr__(name):
    if name == "HomogenizedResponse":
        fn = _autograd_function()
        globals()[name] = fn
        return fn
    raise AttributeError(name)
