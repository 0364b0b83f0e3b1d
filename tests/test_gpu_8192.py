"""GPU parity at the largest size, 8192 (columns of 8192 take the four-step
column pass in both precisions; rows of 8192 the row passes):

* square 8192^2 grids with seeded impulses C (sigma = S C, Eq. (sigmaW)),
  every order, against the oracle's exact superposition at sampled cells and
  around every impulse (FP64 1e-12, FP32-split 1e-6 relative to max|F|);
* long-thin grids with 8192-long rows or columns (8192 x 4, 4 x 8192,
  64 x 8192, 8192 x 64) with impulses in the four corners, where the zero
  padding and the packed spectral bins matter most;
* the adjoint: the identity <F(s), g> = <s, F^T g> in FP64, and the
  FP32-split adjoint of the same random gradients against the FP64 one.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import run_forces

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-6


def _sg():
    import paper_1904_07400_amd as sg
    return sg


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_forces_8192_sparse_impulses(k):
    sg = _sg()
    M = N = 8192
    dom = (-1.0, 1.0, -1.0, 1.0)
    si, sj, sc = workloads.sparse_coeffs(500 + k, M, N, 12)
    C = np.zeros((N, M))
    np.add.at(C, (sj, si), sc)
    sigma = oracle.bspline_apply(C, k)
    del C
    near = [int(min(max(b + db, 0), N - 1)) * M + int(min(max(a + da, 0), M - 1))
            for a, b in zip(si, sj) for da in (-1, 0, 1) for db in (-1, 0, 1)]
    cells = workloads.sample_cells(600 + k, M, N, 200, extra=near)
    rx, ry = oracle.forces_sparse(k, 2.0 / M, 2.0 / N, M, si, sj, sc, cells)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    for prec, tol in ((sg.SG_FP64, FP64_TOL), (sg.SG_FP32_SPLIT, FP32_TOL)):
        gx, gy = run_forces((M, N, *dom, k), prec, sigma)
        err = max(np.abs(gx.ravel()[cells] - rx).max(), np.abs(gy.ravel()[cells] - ry).max()) / scale
        assert err <= tol, (prec, err)


THIN = [(k, M, N) for k in (3, 2, 5) for (M, N) in ((8192, 4), (4, 8192), (64, 8192), (8192, 64))]


@pytest.mark.parametrize("k,M,N", THIN, ids=[f"k{c[0]}-{c[1]}x{c[2]}" for c in THIN])
def test_long_thin_corner_impulses(k, M, N):
    sg = _sg()
    dom = (-1.0, 1.0, -0.5, 0.5)
    si = np.array([0, M - 1, 0, M - 1], np.int32)
    sj = np.array([0, 0, N - 1, N - 1], np.int32)
    sc = np.array([1.0, -0.75, 0.5, 0.25])
    C = np.zeros((N, M))
    C[sj, si] = sc
    sigma = oracle.bspline_apply(C, k)
    rows = [0, 1, N - 2, N - 1]
    cols = [0, 1, M - 2, M - 1]
    edge = {j * M + i for j in rows for i in range(M)} | {j * M + i for j in range(N) for i in cols}
    rng = np.random.default_rng(17)
    cells = np.array(sorted(edge | set(rng.integers(0, M * N, 300).tolist())), np.int64)
    rx, ry = oracle.forces_sparse(k, (dom[1] - dom[0]) / M, (dom[3] - dom[2]) / N, M, si, sj, sc, cells)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    for prec, tol in ((sg.SG_FP64, FP64_TOL), (sg.SG_FP32_SPLIT, FP32_TOL)):
        gx, gy = run_forces((M, N, *dom, k), prec, sigma)
        ex = np.abs(gx.ravel()[cells] - rx).max() / scale
        ey = np.abs(gy.ravel()[cells] - ry).max() / scale
        assert max(ex, ey) <= tol, (prec, ex, ey)


@pytest.mark.parametrize("k", [3, 2])
def test_adjoint_8192(k):
    sg = _sg()
    import torch
    n = 8192
    grid = (n, n, -1.0, 1.0, -1.0, 1.0, k)
    g = torch.Generator(device="cuda").manual_seed(8192 + k)
    s = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
    gx = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
    gy = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
    plan = sg.Plan([grid], sg.SG_FP64)
    try:
        fx, fy = plan.forces(s)
        gs64 = plan.adjoint(gx, gy)
        lhs = (fx * gx).sum() + (fy * gy).sum()
        rhs = (s * gs64).sum()
        scale = (fx.abs() * gx.abs()).sum() + (fy.abs() * gy.abs()).sum()
        ident = ((lhs - rhs).abs() / scale).item()
        del fx, fy
    finally:
        plan.close()
    assert ident <= 1e-13, ident
    p32 = sg.Plan([grid], sg.SG_FP32_SPLIT)
    try:
        gs32 = p32.adjoint(gx.float(), gy.float())
        torch.cuda.synchronize()
        err = ((gs32.double() - gs64).abs().max() / gs64.abs().max()).item()
    finally:
        p32.close()
    # random gradients: the FP32 transforms' rounding (~ eps32 log2 N) and
    # the rounding of the inputs to float, relative to max|g_sigma|
    assert err <= 2e-6, err
