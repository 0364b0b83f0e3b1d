"""CPU checks of the Python binding's argument validation: a tensor of the
wrong dtype, length, device or layout is rejected with SG_ERR_ARG before any
call reaches the library (a short or mistyped buffer would otherwise be read
or written out of bounds by the kernels)."""
import pytest
import torch

import paper_1904_07400_amd as sg


def _fake_plan(prec=sg.SG_FP64, total=64):
    # a Plan object without a device-side plan: only the host-side checks run
    p = object.__new__(sg.Plan)
    p.grids = [(8, 8, -1.0, 1.0, -1.0, 1.0, 3)]
    p.prec = prec
    p.dtype = torch.float64 if prec == sg.SG_FP64 else torch.float32
    p.device = torch.device("cuda", 0)
    p.offsets = [0, total]
    p.handle = None
    return p


def _expect_arg(fn, what):
    with pytest.raises(sg.SGError) as e:
        fn()
    assert e.value.status == 1 and what in str(e.value)


def test_wrong_dtype_length_device_layout_rejected():
    p = _fake_plan()
    good_cpu = torch.zeros(64, dtype=torch.float64)
    # the plan lives on cuda:0, so a CPU tensor is on the wrong device
    _expect_arg(lambda: p._check_tensor("sigma", good_cpu), "on cpu")
    p.device = torch.device("cpu")  # from here on, check the other properties on the host
    p._check_tensor("sigma", good_cpu)
    _expect_arg(lambda: p._check_tensor("sigma", good_cpu.float()), "dtype")
    _expect_arg(lambda: p._check_tensor("fx", torch.zeros(63, dtype=torch.float64)), "63 elements")
    _expect_arg(lambda: p._check_tensor("fy", torch.zeros(128, dtype=torch.float64)[::2]), "contiguous")
    _expect_arg(lambda: p._check_tensor("gfx", [0.0] * 64), "torch.Tensor")


def test_forces_and_adjoint_check_before_the_call():
    p = _fake_plan(sg.SG_FP32_SPLIT)
    p.device = torch.device("cpu")
    s = torch.zeros(64, dtype=torch.float32)
    bad = torch.zeros(64, dtype=torch.float64)
    # every entry point validates each tensor before the library is called
    # (the handle is None, so reaching the library would fail differently)
    _expect_arg(lambda: p.forces(bad, s.clone(), s.clone()), "sigma")
    _expect_arg(lambda: p.forces(s, bad, s.clone()), "fx")
    _expect_arg(lambda: p.forces(s, s.clone(), torch.zeros(32, dtype=torch.float32)), "fy")
    _expect_arg(lambda: p.adjoint(s, bad, s.clone()), "gfy")
    _expect_arg(lambda: p.adjoint(s, s.clone(), bad), "out")
    _expect_arg(lambda: p.coeffs(bad, s.clone()), "sigma")
