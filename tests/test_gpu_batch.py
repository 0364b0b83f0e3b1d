"""GPU tests of batched plans: many grids of mixed sizes (2^a and 3*2^a),
orders and domains in one plan, run as one launch per pass and size class,
optionally autotuned and replayed from a captured HIP graph.

Every line of every grid is transformed independently, so the batched
results must equal, bit for bit, those of one plan per grid; small grids
are also checked against the oracle (FP64 1e-12, FP32-split 1e-6).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

GRIDS = [
    (96, 96, -1.0, 1.0, -1.0, 1.0, 3),
    (128, 64, -1.0, 1.0, -1.0, 1.0, 1),
    (96, 96, -1.0, 1.0, -1.0, 1.0, 3),      # same class, same spectra
    (48, 192, -1.0, 1.0, -2.0, 2.0, 2),
    (96, 96, -2.0, 1.0, -1.0, 1.0, 3),      # same class, other cell shape
    (256, 256, -1.0, 1.0, -1.0, 1.0, 2),
    (12, 24, -1.0, 1.0, -1.0, 1.0, 1),
    (384, 96, -1.0, 1.0, -0.5, 0.5, 3),
    (128, 64, -1.0, 1.0, -1.0, 1.0, 1),
    (96, 96, -1.0, 1.0, -1.0, 1.0, 5),
    (64, 128, -1.0, 1.0, -1.0, 1.0, 4),
    (96, 96, -1.0, 1.0, -1.0, 1.0, 4),      # same size as the k = 3, 5 grids, own class
]


def _sg():
    import paper_1904_07400_amd as sg
    return sg


def _sigma(grids):
    parts = []
    for gi, g in enumerate(grids):
        xs, ys = oracle.sample_lattice(g[6], g[0], g[1], g[2:6])
        parts.append(workloads.clump_sigma(workloads.clump_params(40 + gi, 4 + 4 * gi), xs, ys).ravel())
    return np.concatenate(parts)


def _single(grids, prec, sigma):
    """Forces of each grid from a plan of its own."""
    sg = _sg()
    import torch
    outx, outy, off = [], [], 0
    for g in grids:
        n = g[0] * g[1]
        plan = sg.Plan([g], prec)
        try:
            fx, fy = plan.forces(to_dev(sigma[off:off + n], plan.dtype))
            torch.cuda.synchronize()
            outx.append(fx.cpu().numpy())
            outy.append(fy.cpu().numpy())
        finally:
            plan.close()
        off += n
    return np.concatenate(outx), np.concatenate(outy)


@pytest.mark.parametrize("flags", [0, 4], ids=["default-tiles", "autotuned"])
def test_batched_equals_single_plans_and_oracle(flags):
    sg = _sg()
    import torch
    sigma = _sigma(GRIDS)
    for prec, tol in ((sg.SG_FP64, 1e-12), (sg.SG_FP32_SPLIT, 1e-6)):
        plan = sg.Plan(GRIDS, prec, flags=flags)
        try:
            classes = sg.sg_plan_classes(plan.handle)
            fx, fy = plan.forces(to_dev(sigma, plan.dtype))
            torch.cuda.synchronize()
            bx, by = fx.cpu().numpy(), fy.cpu().numpy()
            offs = plan.offsets
        finally:
            plan.close()
        # classes of equal (nx, ny, order), in order of first appearance
        assert [c[:4] for c in classes] == [(96, 96, 3, 3), (128, 64, 1, 2), (48, 192, 2, 1), (256, 256, 2, 1),
                                            (12, 24, 1, 1), (384, 96, 3, 1), (96, 96, 5, 1), (64, 128, 4, 1),
                                            (96, 96, 4, 1)]
        assert all(c[4] >= 1 and c[5] >= 1 and c[6] >= 1 for c in classes)
        sx, sy = _single(GRIDS, prec, sigma)
        assert np.array_equal(bx, sx) and np.array_equal(by, sy)
        for gi in (0, 3, 4, 6, 9, 10):
            g = GRIDS[gi]
            a, b = offs[gi], offs[gi + 1]
            rx, ry = oracle.forces(sigma[a:b].reshape(g[1], g[0]), g[6], g[2:6])
            sc = max(np.abs(rx).max(), np.abs(ry).max())
            err = max(np.abs(bx[a:b].reshape(g[1], g[0]) - rx).max(), np.abs(by[a:b].reshape(g[1], g[0]) - ry).max())
            assert err <= tol * sc, (prec, gi, err / sc)


def test_graph_replays_match_eager():
    """SG_FLAG_GRAPH: captured step replayed several times, with eager work
    and synchronisations between replays, and with two buffer sets."""
    sg = _sg()
    import torch
    sigma = _sigma(GRIDS)
    for prec in (sg.SG_FP32_SPLIT, sg.SG_FP64):
        eager = sg.Plan(GRIDS, prec)
        graph = sg.Plan(GRIDS, prec, flags=sg.SG_FLAG_GRAPH)
        try:
            s0 = to_dev(sigma, eager.dtype)
            s = torch.empty_like(s0)  # one input buffer: replays see new contents
            bufs = [(graph.empty(), graph.empty()), (graph.empty(), graph.empty())]
            for rep in range(6):
                s.copy_(s0 * (1.0 + 0.25 * rep) - 0.1 * rep)   # eager work between replays
                ex, ey = eager.forces(s)
                gx, gy = bufs[rep % 2]
                gx.fill_(float("nan"))
                gy.fill_(float("nan"))
                sg.sg_forces(graph.handle, s, gx, gy)
                torch.cuda.synchronize()
                assert torch.equal(gx, ex) and torch.equal(gy, ey), (prec, rep)
        finally:
            eager.close()
            graph.close()


def test_graph_plan_reuses_captures_for_same_buffers():
    sg = _sg()
    import torch
    grids = GRIDS[:3]
    sigma = to_dev(_sigma(grids), torch.float32)
    plan = sg.Plan(grids, sg.SG_FP32_SPLIT, flags=sg.SG_FLAG_GRAPH | sg.SG_FLAG_AUTOTUNE)
    try:
        fx, fy = plan.empty(), plan.empty()
        outs = []
        for _ in range(3):
            sg.sg_forces(plan.handle, sigma, fx, fy)
            torch.cuda.synchronize()
            outs.append((fx.clone(), fy.clone()))
    finally:
        plan.close()
    for ox, oy in outs[1:]:
        assert torch.equal(ox, outs[0][0]) and torch.equal(oy, outs[0][1])
