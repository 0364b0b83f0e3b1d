"""Helpers for the GPU tests: plan construction, host<->device copies, error metrics."""
import numpy as np


def torch_cuda():
    import torch
    return torch


def to_dev(a, dtype):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run_forces(grid, prec, sigma):
    """One grid: returns (Fx, Fy) as float64 numpy arrays of shape (ny, nx)."""
    import paper_1904_07400_amd as sg
    torch = torch_cuda()
    plan = sg.Plan([grid], prec)
    try:
        s = to_dev(np.asarray(sigma).ravel(), plan.dtype)
        fx, fy = plan.forces(s)
        torch.cuda.synchronize()
        ny, nx = grid[1], grid[0]
        return (fx.double().cpu().numpy().reshape(ny, nx), fy.double().cpu().numpy().reshape(ny, nx))
    finally:
        plan.close()


def rel_max_err(got_x, got_y, ref_x, ref_y):
    """max_{cells, d} |F_d - F_d^ref| / max |F^ref| (the accuracy metric of the FP32-split path)."""
    scale = max(np.max(np.abs(ref_x)), np.max(np.abs(ref_y)))
    err = max(np.max(np.abs(got_x - ref_x)), np.max(np.abs(got_y - ref_y)))
    return err / scale
