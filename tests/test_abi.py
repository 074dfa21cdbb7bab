"""The C-ABI library loads on the CPU and exports every function ghom.h declares
(no compute call is made here: there is no GPU)."""

import ctypes
import os
import re

import pytest

from paper_1901_06531_amd import ghom

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ghom.h")


def declared():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ghom_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["ghom_create", "ghom_destroy", "ghom_set_material_neohookean", "ghom_set_material_svk",
                 "ghom_set_control", "ghom_set_history", "ghom_step", "ghom_get_averages",
                 "ghom_apply_operator", "ghom_adjoint_grad_scale"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(ghom.LIB_PATH), reason="libghom.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(ghom.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding's table covers the header exactly
    assert sorted(ghom._SIGS) == declared()


@pytest.mark.skipif(not os.path.exists(ghom.LIB_PATH), reason="libghom.so not built")
def test_argument_checks_need_no_gpu():
    L = ghom.lib()
    out = ctypes.c_void_p()
    # unsupported grid length and bad precision are rejected before any device call
    assert L.ghom_create(ctypes.byref(out), 10, 16, 16, 1.0, 1.0, 1.0, 0, 0, None) == -1
    assert b"grid lengths must be among" in L.ghom_last_error(None)
    assert L.ghom_create(ctypes.byref(out), 16, 16, 16, 1.0, 1.0, 1.0, 7, 0, None) == -1
    assert L.ghom_create(ctypes.byref(out), 16, 16, 16, -1.0, 1.0, 1.0, 0, 0, None) == -1
    assert L.ghom_create(None, 16, 16, 16, 1.0, 1.0, 1.0, 0, 0, None) == -1
    assert L.ghom_set_control(None, None) == -1


@pytest.mark.skipif(not os.path.exists(ghom.LIB_PATH), reason="libghom.so not built")
def test_new_entry_points_reject_null_contexts():
    L = ghom.lib()
    assert L.ghom_set_time_step(None, 1.0) == -1
    assert L.ghom_set_material_visco(None, None, 1, None, None, None) == -1
    assert L.ghom_step_adaptive(None, 4, 2, None, None, None) == -1
    assert L.ghom_set_option(None, 4, 1) == -1
    assert L.ghom_get_control(None, None, None) == -1


def test_binding_checks_device_buffers_before_the_abi():
    """The C ABI takes no lengths: the binding refuses host tensors, wrong dtypes, wrong
    sizes and other devices before passing a pointer."""
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError, match="device tensor"):
        ghom._field_ptr(torch.zeros(9 * 8), 9 * 8, torch.float64, 0, "x")


def test_missing_library_fails_loudly(monkeypatch):
    """No CPU fallback: without the built library every call raises."""
    monkeypatch.setattr(ghom, "LIB_PATH", "/nonexistent/libghom.so")
    monkeypatch.setattr(ghom, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        ghom.lib()
    with pytest.raises(RuntimeError, match="not built"):
        ghom.Solver((16, 16, 16))
