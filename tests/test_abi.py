"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/sg.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sg.h")).read()
    return sorted(set(re.findall(r"\b(sg_[a-z_]+)\s*\(", text)) - {"sg_plan"})


def _lib():
    import paper_1904_07400_amd as sg
    if not os.path.exists(sg.LIB_PATH):
        pytest.skip("libsg.so not built")
    return sg, sg.lib()


def test_every_declared_symbol_is_exported():
    sg, L = _lib()
    names = _declared()
    assert "sg_forces" in names and "sg_plan_create" in names and "sg_weights" in names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_arg_errors():
    sg, L = _lib()
    assert sg.sg_status_string(0) == "SG_OK"
    assert "ARG" in sg.sg_status_string(1)
    h = ctypes.c_void_p()
    # no grids
    assert L.sg_plan_create(ctypes.byref(h), None, 0, 0, None, 0) == 1
    assert "grid" in sg.sg_last_error_message()
    # bad order / sizes / domain / precision / flags: rejected before any device call
    bad = [
        (sg.sg_grid(64, 64, -1, 1, -1, 1, 6), 0, 0, 2),
        (sg.sg_grid(64, 64, -1, 1, -1, 1, 0), 0, 0, 2),
        (sg.sg_grid(1, 64, -1, 1, -1, 1, 3), 0, 0, 1),
        (sg.sg_grid(64, 64, 1, -1, -1, 1, 3), 0, 0, 1),
        (sg.sg_grid(64, 64, -1, 1, -1, float("nan"), 3), 0, 0, 1),
        (sg.sg_grid(100, 64, -1, 1, -1, 1, 3), 0, 0, 2),
        (sg.sg_grid(96, 6, -1, 1, -1, 1, 3), 0, 0, 2),
        (sg.sg_grid(3072, 64, -1, 1, -1, 1, 3), 0, 0, 2),
        (sg.sg_grid(16384, 64, -1, 1, -1, 1, 3), 0, 0, 2),
        (sg.sg_grid(64, 16384, -1, 1, -1, 1, 3), 1, 0, 2),
        (sg.sg_grid(64, 64, -1, 1, -1, 1, 3), 7, 0, 1),
        (sg.sg_grid(64, 64, -1, 1, -1, 1, 3), 0, 0x80, 1),
        (sg.sg_grid(3072, 64, -1, 1, -1, 1, 3), 1, 0, 2),
    ]
    for g, prec, flags, want in bad:
        arr = (sg.sg_grid * 1)(g)
        assert L.sg_plan_create(ctypes.byref(h), arr, 1, prec, None, flags) == want
        assert sg.sg_last_error_message() != ""
    assert L.sg_plan_create(None, None, 1, 0, None, 0) == 1
    # NULL plan handling
    assert L.sg_plan_destroy(None) == 0
    assert L.sg_forces(None, None, None, None) == 1
    assert L.sg_weights(None, 0, None, None) == 1
    assert L.sg_bspline_coeffs(None, None, None) == 1
    assert L.sg_forces_adjoint(None, None, None, None) == 1
    assert L.sg_plan_layout(None, None) == 1
    assert L.sg_plan_tuning(None, 0, None) == 1
