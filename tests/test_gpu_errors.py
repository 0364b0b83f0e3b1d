"""Error paths of the C ABI on the GPU, forced from the host (no kernel is
made to fault):

* SG_FAULT_INJECT=alloc:N refuses the N-th device allocation of
  sg_plan_create.  Every N up to the plan's allocation count must give
  SG_ERR_NOMEM and release everything allocated before it (device memory
  returns to its level before the call).
* SG_FAULT_INJECT=device makes the next per-step call fail as a HIP error
  would: SG_ERR_DEVICE, after which the plan is sticky (SG_ERR_STATE for
  every per-step call) until it is destroyed, and a fresh plan works.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sg():
    import paper_1904_07400_amd as sg
    return sg


GRID = (1024, 512, -1.0, 1.0, -1.0, 1.0, 3)


def _free_bytes(torch):
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_every_allocation_failure_releases_the_plan(monkeypatch):
    sg = _sg()
    import torch
    base = _free_bytes(torch)
    failures = 0
    for n in range(1, 65):
        monkeypatch.setenv("SG_FAULT_INJECT", f"alloc:{n}")
        try:
            plan = sg.Plan([GRID], sg.SG_FP64)
        except sg.SGError as e:
            assert e.status == 3, str(e)
            assert "SG_FAULT_INJECT" in str(e)
            failures += 1
            continue
        # n is past the plan's last allocation: creation succeeds
        monkeypatch.delenv("SG_FAULT_INJECT")
        plan.close()
        break
    else:
        pytest.fail("plan creation never succeeded within 64 allocations")
    assert failures >= 5, failures
    # the plans that failed left nothing behind (4 MB of allocator slack)
    assert _free_bytes(torch) >= base - (4 << 20), (base, _free_bytes(torch))
    monkeypatch.setenv("SG_FAULT_INJECT", "alloc")
    with pytest.raises(sg.SGError) as e:
        sg.Plan([GRID], sg.SG_FP32_SPLIT)
    assert e.value.status == 3


def test_device_error_makes_the_plan_sticky(monkeypatch):
    sg = _sg()
    import torch
    plan = sg.Plan([GRID], sg.SG_FP32_SPLIT)
    try:
        s = torch.zeros(plan.total, dtype=plan.dtype, device="cuda")
        fx, fy = plan.forces(s)  # a working plan
        monkeypatch.setenv("SG_FAULT_INJECT", "device")
        with pytest.raises(sg.SGError) as e:
            plan.forces(s, fx, fy)
        assert e.value.status == 4, str(e.value)
        monkeypatch.delenv("SG_FAULT_INJECT")
        for call in (lambda: plan.forces(s, fx, fy), lambda: plan.adjoint(fx, fy),
                     lambda: plan.coeffs(s), lambda: plan.weights(0)):
            with pytest.raises(sg.SGError) as e:
                call()
            assert e.value.status == 5, str(e.value)
    finally:
        plan.close()  # destroying a sticky plan succeeds
    fresh = sg.Plan([GRID], sg.SG_FP32_SPLIT)
    try:
        s = torch.ones(fresh.total, dtype=fresh.dtype, device="cuda")
        fx, fy = fresh.forces(s)
        torch.cuda.synchronize()
        assert np.isfinite(fx.cpu().numpy()).all() and float(fx.abs().max()) > 0
    finally:
        fresh.close()
