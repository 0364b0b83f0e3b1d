"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars: FP64 path <= 1e-12 relative
(max-norm over cells and components, scaled by max|F|); FP32-split path
<= 1e-6 relative; weights <= 1e-14 of max|w|; coefficients <= 1e-13 (FP64)
relative to max|C|.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import rel_max_err, run_forces, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-6


def _sg():
    import paper_1904_07400_amd as sg
    return sg


def _clumps(k, M, N, domain, seed=2, n=32):
    xs, ys = oracle.sample_lattice(k, M, N, domain)
    return workloads.clump_sigma(workloads.clump_params(seed, n), xs, ys)


@pytest.mark.parametrize("k,M,N,dom", [
    (1, 8, 8, (-1, 1, -1, 1)), (2, 16, 8, (-1, 1, -1, 1)), (3, 16, 16, (-1, 1, -1, 1)),
    (3, 32, 64, (-1, 1, -0.5, 1.0)), (2, 64, 64, (-1, 1, -1, 1)), (1, 128, 32, (0, 3, 0, 1)),
    (3, 256, 256, (-1, 1, -1, 1)), (4, 16, 8, (-1, 1, -1, 1)), (5, 32, 64, (-1, 1, -0.5, 1.0)),
    (4, 64, 64, (-1, 1, -1, 1)), (5, 96, 48, (-1, 1, -2, 2)), (4, 48, 96, (0, 3, 0, 1))])
def test_weights_match_oracle(k, M, N, dom):
    sg = _sg()
    import torch
    grid = (M, N, *dom, k)
    plan = sg.Plan([grid], sg.SG_FP64)
    try:
        wx, wy = plan.weights(0)
        torch.cuda.synchronize()
        gx, gy = wx.cpu().numpy(), wy.cpu().numpy()
    finally:
        plan.close()
    hx, hy = (dom[1] - dom[0]) / M, (dom[3] - dom[2]) / N
    ox, oy = oracle.weights(k, M, N, hx, hy)
    s = max(np.abs(ox).max(), np.abs(oy).max())
    assert np.abs(gx - ox).max() <= 1e-14 * s
    assert np.abs(gy - oy).max() <= 1e-14 * s


def test_sample_points_match_oracle():
    sg = _sg()
    for k in (1, 2, 3, 4, 5):
        grid = (16, 8, -1.0, 1.0, -0.5, 0.5, k)
        plan = sg.Plan([grid], sg.SG_FP64)
        try:
            xs, ys = plan.sample_points(0)
        finally:
            plan.close()
        oxs, oys = oracle.sample_lattice(k, 16, 8, (-1.0, 1.0, -0.5, 0.5))
        assert np.allclose(xs, oxs, rtol=0, atol=1e-15) and np.allclose(ys, oys, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", [3, 4, 5])
@pytest.mark.parametrize("M,N", [(4, 4), (16, 16), (64, 32), (8, 256), (256, 256), (96, 12)])
def test_coeffs_match_oracle(M, N, k):
    sg = _sg()
    import torch
    rng = np.random.default_rng(M * 1000 + N)
    sigma = rng.standard_normal((N, M))
    ref = oracle.bspline_coeffs(sigma, k)
    for prec, tol in ((sg.SG_FP64, 1e-13), (sg.SG_FP32_SPLIT, 1e-6)):
        plan = sg.Plan([(M, N, -1.0, 1.0, -1.0, 1.0, k)], prec)
        try:
            c = plan.coeffs(to_dev(sigma.ravel(), plan.dtype))
            torch.cuda.synchronize()
            got = c.double().cpu().numpy().reshape(N, M)
        finally:
            plan.close()
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (prec, np.abs(got - ref).max())


CASES = [
    # (k, M, N, domain, input)
    (1, 64, 64, (-1, 1, -1, 1), "disk3"),     # 64^2, first order, D3 disk of radius 0.8
    (2, 64, 64, (-1, 1, -1, 1), "clumps"),
    (3, 64, 64, (-1, 1, -1, 1), "clumps"),
    (3, 128, 64, (-1, 1, -0.5, 0.5), "clumps"),
    (2, 32, 128, (-1, 1, -2, 2), "random"),
    (1, 16, 16, (-1, 1, -1, 1), "random"),
    (3, 4, 4, (-1, 1, -1, 1), "random"),
    (3, 8, 512, (-1, 1, -1, 1), "random"),
    (3, 256, 256, (-1, 1, -1, 1), "clumps"),
    # sizes 3 * 2^a (a radix-3 stage in every transform)
    (3, 96, 96, (-1, 1, -1, 1), "clumps"),
    (2, 48, 192, (-1, 1, -1, 1), "random"),
    (1, 12, 24, (-1, 1, -1, 1), "random"),
    (3, 384, 96, (-1, 1, -0.5, 0.5), "clumps"),
    (3, 12, 12, (-1, 1, -1, 1), "random"),
    # cubic and quartic splines (k = 4, 5)
    (4, 64, 64, (-1, 1, -1, 1), "clumps"),
    (5, 64, 64, (-1, 1, -1, 1), "clumps"),
    (4, 128, 64, (-1, 1, -0.5, 0.5), "clumps"),
    (5, 32, 128, (-1, 1, -2, 2), "random"),
    (4, 4, 4, (-1, 1, -1, 1), "random"),
    (5, 4, 4, (-1, 1, -1, 1), "random"),
    (5, 8, 512, (-1, 1, -1, 1), "random"),
    (4, 256, 256, (-1, 1, -1, 1), "clumps"),
    (5, 96, 96, (-1, 1, -1, 1), "clumps"),
    (4, 48, 192, (-1, 1, -1, 1), "random"),
    (5, 384, 96, (-1, 1, -0.5, 0.5), "clumps"),
    (4, 12, 12, (-1, 1, -1, 1), "random"),
    # columns of 1536 (FP32: the radix-3 column pass of three waves), every order
    (1, 8, 1536, (-0.5, 0.5, -96, 96), "random"),
    (2, 8, 1536, (-0.5, 0.5, -96, 96), "random"),
    (3, 16, 1536, (-1, 1, -96, 96), "random"),
    (4, 8, 1536, (-0.5, 0.5, -96, 96), "random"),
    (5, 8, 1536, (-0.5, 0.5, -96, 96), "random"),
    # columns of 768 (FP32: the radix-3 column pass with 256-point waves)
    (1, 8, 768, (-0.5, 0.5, -48, 48), "random"),
    (2, 16, 768, (-1, 1, -48, 48), "random"),
    (3, 8, 768, (-0.5, 0.5, -48, 48), "random"),
    (4, 8, 768, (-0.5, 0.5, -48, 48), "random"),
    (5, 16, 768, (-1, 1, -48, 48), "random"),
    # rows of 1536 and 768, every order but one
    (1, 1536, 8, (-96, 96, -0.5, 0.5), "random"),
    (3, 1536, 16, (-96, 96, -1, 1), "random"),
    (4, 1536, 8, (-96, 96, -0.5, 0.5), "random"),
    (2, 768, 8, (-48, 48, -0.5, 0.5), "random"),
    (5, 768, 16, (-48, 48, -1, 1), "random"),
]


def _input(kind, k, M, N, dom):
    if kind == "disk3":
        xs, ys = oracle.sample_lattice(k, M, N, dom)
        return workloads.disk_sigma(3, 0.8, xs, ys)
    if kind == "clumps":
        return _clumps(k, M, N, dom)
    return np.random.default_rng(M + 7 * N + k).standard_normal((N, M))


@pytest.mark.parametrize("k,M,N,dom,kind", CASES, ids=[f"k{c[0]}-{c[1]}x{c[2]}-{c[4]}" for c in CASES])
def test_forces_fp64_and_fp32_match_oracle(k, M, N, dom, kind):
    sg = _sg()
    sigma = _input(kind, k, M, N, dom)
    ref_x, ref_y = oracle.forces(sigma, k, dom)
    grid = (M, N, *dom, k)
    gx, gy = run_forces(grid, sg.SG_FP64, sigma)
    e64 = rel_max_err(gx, gy, ref_x, ref_y)
    assert e64 <= FP64_TOL, e64
    fx, fy = run_forces(grid, sg.SG_FP32_SPLIT, sigma)
    e32 = rel_max_err(fx, fy, ref_x, ref_y)
    assert e32 <= FP32_TOL, e32


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n", [1024, 4096, 1536])
def test_forces_full_size_sparse_impulses(k, n):
    """Full-size grids: C = a few seeded impulses (sigma = S C, Eq. (sigmaW)),
    so the oracle's exact superposition gives F at sampled cells."""
    sg = _sg()
    M = N = n
    dom = (-1.0, 1.0, -1.0, 1.0)
    si, sj, sc = workloads.sparse_coeffs(100 + k, M, N, 12)
    C = np.zeros((N, M))
    np.add.at(C, (sj, si), sc)
    sigma = oracle.bspline_apply(C, k)
    # sampled cells plus every impulse's neighbourhood, where max|F| lies, so
    # that the scale of the relative error is the field's max|F|
    near = [int(min(max(b + db, 0), N - 1)) * M + int(min(max(a + da, 0), M - 1))
            for a, b in zip(si, sj) for da in (-1, 0, 1) for db in (-1, 0, 1)]
    cells = workloads.sample_cells(200 + k, M, N, 200, extra=near)
    rx, ry = oracle.forces_sparse(k, 2.0 / M, 2.0 / N, M, si, sj, sc, cells)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    for prec, tol in ((sg.SG_FP64, FP64_TOL), (sg.SG_FP32_SPLIT, FP32_TOL)):
        gx, gy = run_forces((M, N, *dom, k), prec, sigma)
        err = max(np.abs(gx.ravel()[cells] - rx).max(), np.abs(gy.ravel()[cells] - ry).max()) / scale
        assert err <= tol, (prec, err)


ANISO = [(k, M, N, dom) for k in (1, 2, 3)
         for (M, N, dom) in ((2048, 2048, (-2.0, 2.0, -1.0, 1.0)), (4096, 1024, (-1.0, 1.0, -1.0, 1.0)),
                             (1536, 768, (-1.0, 1.0, -0.25, 0.25)))] + [
    (4, 2048, 2048, (-2.0, 2.0, -1.0, 1.0)), (5, 1536, 768, (-1.0, 1.0, -0.25, 0.25)),
    (5, 4096, 1024, (-1.0, 1.0, -1.0, 1.0))]


@pytest.mark.parametrize("k,M,N,dom", ANISO, ids=[f"k{c[0]}-{c[1]}x{c[2]}-dx{(c[3][1]-c[3][0])/c[1]/((c[3][3]-c[3][2])/c[2]):g}dy"
                                                 for c in ANISO])
def test_forces_anisotropic_full_size(k, M, N, dom):
    """Non-square cells at full size on rectangular domains (dx = 2 dy and
    dx = dy / 4, for 2^a and 3 * 2^a sizes): seeded impulses, the oracle's
    exact superposition at sampled cells and around every impulse."""
    sg = _sg()
    hx, hy = (dom[1] - dom[0]) / M, (dom[3] - dom[2]) / N
    si, sj, sc = workloads.sparse_coeffs(300 + k, M, N, 12)
    C = np.zeros((N, M))
    np.add.at(C, (sj, si), sc)
    sigma = oracle.bspline_apply(C, k)
    near = [int(min(max(b + db, 0), N - 1)) * M + int(min(max(a + da, 0), M - 1))
            for a, b in zip(si, sj) for da in (-1, 0, 1) for db in (-1, 0, 1)]
    cells = workloads.sample_cells(400 + k, M, N, 200, extra=near)
    rx, ry = oracle.forces_sparse(k, hx, hy, M, si, sj, sc, cells)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    for prec, tol in ((sg.SG_FP64, FP64_TOL), (sg.SG_FP32_SPLIT, FP32_TOL)):
        gx, gy = run_forces((M, N, *dom, k), prec, sigma)
        err = max(np.abs(gx.ravel()[cells] - rx).max(), np.abs(gy.ravel()[cells] - ry).max()) / scale
        assert err <= tol, (prec, err)


def test_forces_deterministic_and_linear():
    sg = _sg()
    import torch
    M = N = 128
    grid = (M, N, -1.0, 1.0, -1.0, 1.0, 3)
    rng = np.random.default_rng(9)
    a = rng.standard_normal(M * N)
    b = rng.standard_normal(M * N)
    plan = sg.Plan([grid], sg.SG_FP64)
    try:
        ta, tb = to_dev(a, torch.float64), to_dev(b, torch.float64)
        f1 = [t.clone() for t in plan.forces(ta)]
        f2 = [t.clone() for t in plan.forces(ta)]
        fb = [t.clone() for t in plan.forces(tb)]
        fab = [t.clone() for t in plan.forces(2.0 * ta - 3.0 * tb)]
        torch.cuda.synchronize()
    finally:
        plan.close()
    assert torch.equal(f1[0], f2[0]) and torch.equal(f1[1], f2[1])
    for d in range(2):
        lin = 2.0 * f1[d] - 3.0 * fb[d]
        assert (fab[d] - lin).abs().max().item() <= 1e-12 * lin.abs().max().item()
