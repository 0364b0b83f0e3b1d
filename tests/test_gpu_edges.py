"""GPU edge cases of the forward path.

* sigma = 0 gives F = 0 exactly (both precisions, smallest and ragged sizes).
* Impulses in the four corner cells, where the zero padding and the packed
  spectral bins (p = 0 and p = M, q = 0 and q = N) matter most, against the
  oracle's exact superposition (FP64 1e-12, FP32-split 1e-6 relative to
  max|F|), for each order and for 2^a, 3 * 2^a and long-thin grids.
* SG_FLAG_CHECK_FINITE: a NaN or an Inf in sigma is rejected with
  SG_ERR_STATE before any transform runs; the plan stays usable.
"""
import numpy as np
import pytest

import oracle
from gpu_util import run_forces, to_dev

pytestmark = pytest.mark.gpu


def _sg():
    import paper_1904_07400_amd as sg
    return sg


@pytest.mark.parametrize("grid", [(4, 4, -1.0, 1.0, -1.0, 1.0, 3), (96, 48, -1.0, 1.0, -2.0, 2.0, 2),
                                  (64, 4, -1.0, 1.0, -1.0, 1.0, 5), (12, 96, -1.0, 1.0, -1.0, 1.0, 4),
                                  (1024, 12, -1.0, 1.0, -1.0, 1.0, 1), (4096, 4, -1.0, 1.0, -1.0, 1.0, 3)])
def test_zero_density_gives_zero_forces(grid):
    sg = _sg()
    sigma = np.zeros(grid[0] * grid[1])
    for prec in (sg.SG_FP64, sg.SG_FP32_SPLIT):
        fx, fy = run_forces(grid, prec, sigma)
        assert not np.any(fx) and not np.any(fy), prec


CORNER_CASES = [(k, M, N) for k in (1, 2, 3, 4, 5) for (M, N) in ((64, 32), (1536, 24), (8, 4096))]


@pytest.mark.parametrize("k,M,N", CORNER_CASES, ids=[f"k{c[0]}-{c[1]}x{c[2]}" for c in CORNER_CASES])
def test_corner_impulses_against_oracle(k, M, N):
    sg = _sg()
    dom = (-1.0, 1.0, -0.5, 0.5)
    si = np.array([0, M - 1, 0, M - 1], np.int32)
    sj = np.array([0, 0, N - 1, N - 1], np.int32)
    sc = np.array([1.0, -0.75, 0.5, 0.25])
    C = np.zeros((N, M))
    C[sj, si] = sc
    sigma = oracle.bspline_apply(C, k)
    # every cell of the first and last two rows and columns, and seeded interior cells
    rows = [0, 1, N - 2, N - 1]
    cols = [0, 1, M - 2, M - 1]
    edge = {j * M + i for j in rows for i in range(M)} | {j * M + i for j in range(N) for i in cols}
    rng = np.random.default_rng(13)
    cells = np.array(sorted(edge | set(rng.integers(0, M * N, 200).tolist())), np.int64)
    rx, ry = oracle.forces_sparse(k, (dom[1] - dom[0]) / M, (dom[3] - dom[2]) / N, M, si, sj, sc, cells)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    for prec, tol in ((sg.SG_FP64, 1e-12), (sg.SG_FP32_SPLIT, 1e-6)):
        gx, gy = run_forces((M, N, *dom, k), prec, sigma)
        err = max(np.abs(gx.ravel()[cells] - rx).max(), np.abs(gy.ravel()[cells] - ry).max()) / scale
        assert err <= tol, (prec, err)


def test_check_finite_flag_rejects_nan_and_inf():
    sg = _sg()
    import torch
    grid = (64, 32, -1.0, 1.0, -1.0, 1.0, 3)
    rng = np.random.default_rng(3)
    good = rng.standard_normal(64 * 32)
    for prec in (sg.SG_FP64, sg.SG_FP32_SPLIT):
        plan = sg.Plan([grid], prec, flags=sg.SG_FLAG_CHECK_FINITE)
        try:
            ref = sg.Plan([grid], prec)
            try:
                rx, ry = (t.clone() for t in ref.forces(to_dev(good, ref.dtype)))
            finally:
                ref.close()
            for bad in (float("nan"), float("inf"), -float("inf")):
                s = good.copy()
                s[777] = bad
                with pytest.raises(sg.SGError) as e:
                    plan.forces(to_dev(s, plan.dtype))
                assert e.value.status == 5, (prec, bad)
            # the plan still works, and a finite input gives the plain plan's forces
            fx, fy = plan.forces(to_dev(good, plan.dtype))
            torch.cuda.synchronize()
            assert torch.equal(fx, rx) and torch.equal(fy, ry), prec
        finally:
            plan.close()
