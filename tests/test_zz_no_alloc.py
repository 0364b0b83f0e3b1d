"""sg_forces_noalloc (the entry point for callers that cannot allocate)
against sg_forces through the C ABI: the same kernels on a workspace in the
library's fixed device array instead of the plan's, so the forces must be
bit-identical.  Two calls in a row on two plans, the second smaller (the
array keeps the first call's contents), in both precisions; a plan of
several grids; and a plan whose workspace exceeds the array is refused with
SG_ERR_ARG before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sg():
    import paper_1904_07400_amd as sg
    return sg


def _noalloc(sg, plan, sigma):
    import torch
    fx, fy = plan.empty(), plan.empty()
    st = sg.lib().sg_forces_noalloc(ctypes.c_void_p(plan.handle), ctypes.c_void_p(sigma.data_ptr()),
                                    ctypes.c_void_p(fx.data_ptr()), ctypes.c_void_p(fy.data_ptr()))
    assert st == 0, sg.sg_last_error_message()
    torch.cuda.synchronize()
    return fx, fy


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32split"])
def test_noalloc_matches_forces_two_calls(prec):
    sg = _sg()
    import torch
    cases = [[(1024, 512, -1.0, 1.0, -0.5, 0.5, 3)],
             [(96, 48, -1.0, 1.0, -1.0, 1.0, 2), (64, 64, -1.0, 1.0, -1.0, 1.0, 5)]]
    rng = np.random.default_rng(7 + prec)
    for grids in cases:  # the second call smaller than the first
        plan = sg.Plan(grids, prec)
        try:
            sigma = torch.as_tensor(rng.standard_normal(plan.total), dtype=plan.dtype, device="cuda")
            rx, ry = plan.forces(sigma)
            torch.cuda.synchronize()
            gx, gy = _noalloc(sg, plan, sigma)
            assert torch.equal(gx, rx) and torch.equal(gy, ry), grids
            assert float(rx.abs().max()) > 0
        finally:
            plan.close()


def test_noalloc_refuses_a_workspace_beyond_the_array():
    sg = _sg()
    import torch
    plan = sg.Plan([(2048, 2048, -1.0, 1.0, -1.0, 1.0, 3)], sg.SG_FP64)  # 48 B x 4M cells > 64 MiB
    try:
        s = torch.zeros(plan.total, dtype=plan.dtype, device="cuda")
        fx, fy = plan.empty(), plan.empty()
        st = sg.lib().sg_forces_noalloc(ctypes.c_void_p(plan.handle), ctypes.c_void_p(s.data_ptr()),
                                        ctypes.c_void_p(fx.data_ptr()), ctypes.c_void_p(fy.data_ptr()))
        assert st == 1
        assert "no-allocation scratch" in sg.sg_last_error_message()
    finally:
        plan.close()
