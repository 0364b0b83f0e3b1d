"""GPU parity of the hand-written adjoint (sg_forces_adjoint) and its
torch.autograd wrapper.

Gradient bar for the FP32-split path: the loss gradient is the adjoint of
the residual F - F_target, so the forces bar (1e-6 max|F|) becomes
1e-6 max|F| / max|F - F_target| relative to the gradient (plus 1e-6 for the
adjoint's own rounding).

* against the oracle's direct transposed sum on small grids (FP64 <= 1e-12,
  FP32-split <= 1e-6 relative to max|g_sigma|);
* the adjoint identity <F(s), g> = <s, F^T g> at full size (FP64, 1e-12);
* autograd gradient of L = sum |F - F_target|^2 against the oracle at 256^2;
* central finite differences of L on the FP64 path at 256 x 128 (L is
  quadratic in sigma, so the differences are exact up to rounding);
* 8192^2 (and 4096^2) plus four 2048^2 grids in one plan: FP32-split
  gradient against the FP64 gradient, and finite differences at 64 seeded
  cells of the large grid;
* the FP32-split adjoint of the cubic and quartic splines (k = 4, 5) at
  1024^2 and 4096^2 against the FP64 adjoint of the same gradients.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _sg():
    import paper_1904_07400_amd as sg
    return sg


ADJ_CASES = [(1, 16, 16, (-1, 1, -1, 1)), (2, 32, 16, (-1, 1, -1, 1)), (3, 64, 64, (-1, 1, -1, 1)),
             (3, 8, 128, (-1, 1, -0.5, 1.5)), (2, 4, 4, (-1, 1, -1, 1)), (3, 256, 128, (-1, 1, -1, 1)),
             (3, 96, 48, (-1, 1, -1, 1)), (2, 24, 12, (-1, 1, -1, 1)), (1, 192, 96, (-1, 1, -1, 1)),
             (4, 32, 64, (-1, 1, -1, 1)), (5, 64, 32, (-1, 1, -0.5, 0.5)), (5, 96, 48, (-1, 1, -1, 1)),
             (4, 4, 4, (-1, 1, -1, 1)), (5, 256, 128, (-1, 1, -1, 1))]


@pytest.mark.parametrize("k,M,N,dom", ADJ_CASES, ids=[f"k{c[0]}-{c[1]}x{c[2]}" for c in ADJ_CASES])
def test_adjoint_matches_oracle(k, M, N, dom):
    sg = _sg()
    import torch
    rng = np.random.default_rng(M * 3 + N + k)
    gx = rng.standard_normal((N, M))
    gy = rng.standard_normal((N, M))
    ref = oracle.forces_adjoint(gx, gy, k, dom)
    for prec, tol in ((sg.SG_FP64, 1e-12), (sg.SG_FP32_SPLIT, 1e-6)):
        plan = sg.Plan([(M, N, *dom, k)], prec)
        try:
            out = plan.adjoint(to_dev(gx.ravel(), plan.dtype), to_dev(gy.ravel(), plan.dtype))
            torch.cuda.synchronize()
            got = out.double().cpu().numpy().reshape(N, M)
        finally:
            plan.close()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= tol, (prec, err)


@pytest.mark.parametrize("n,k", [(1024, 3), (4096, 3), (4096, 4), (4096, 5)])
def test_adjoint_identity_full_size(n, k):
    sg = _sg()
    import torch
    plan = sg.Plan([(n, n, -1.0, 1.0, -1.0, 1.0, k)], sg.SG_FP64)
    try:
        g = torch.Generator(device="cuda").manual_seed(n)
        s = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
        gx = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
        gy = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
        fx, fy = plan.forces(s)
        gs = plan.adjoint(gx, gy)
        lhs = (fx * gx).sum() + (fy * gy).sum()
        rhs = (s * gs).sum()
        scale = (fx.abs() * gx.abs()).sum() + (fy.abs() * gy.abs()).sum()
        err = ((lhs - rhs).abs() / scale).item()
    finally:
        plan.close()
    assert err <= 1e-13, err


def _loss_setup(n, k, seed=5, n_clumps=64):
    xs, ys = oracle.sample_lattice(k, n, n)
    params = workloads.clump_params(seed, n_clumps)
    sigma = workloads.clump_sigma(params, xs, ys)
    target = workloads.clump_sigma(workloads.perturb_clumps(params, 55), xs, ys)
    return sigma, target


def test_autograd_gradient_against_oracle_256():
    sg = _sg()
    import torch
    n, k = 256, 3
    sigma, target_sigma = _loss_setup(n, k)
    tx, ty = oracle.forces(target_sigma, k)
    fx0, fy0 = oracle.forces(sigma, k)
    ref = oracle.forces_adjoint(2 * (fx0 - tx), 2 * (fy0 - ty), k)
    # the gradient is the adjoint of the residual F - F_target; an error of
    # 1e-6 max|F| in F (the FP32-split bar) becomes 1e-6 max|F| / max|residual|
    # relative to the gradient
    amp = max(np.abs(fx0).max(), np.abs(fy0).max()) / max(np.abs(fx0 - tx).max(), np.abs(fy0 - ty).max())
    for prec, tol in ((sg.SG_FP64, 1e-12), (sg.SG_FP32_SPLIT, 1e-6 * amp + 1e-6)):
        plan = sg.Plan([(n, n, -1.0, 1.0, -1.0, 1.0, k)], prec)
        try:
            s = to_dev(sigma.ravel(), plan.dtype).requires_grad_(True)
            fx, fy = sg.ThinDiskForces.apply(s, plan)
            loss = ((fx - to_dev(tx.ravel(), plan.dtype)) ** 2).sum() + ((fy - to_dev(ty.ravel(), plan.dtype)) ** 2).sum()
            loss.backward()
            torch.cuda.synchronize()
            got = s.grad.double().cpu().numpy().reshape(n, n)
        finally:
            plan.close()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= tol, (prec, err)


def _fd_check(plan, sigma_t, target, grad, cells, delta):
    """Central differences of L(sigma) = sum |F - target|^2 at the given cells."""
    import torch
    tx, ty = target
    out = []
    for c in cells:
        vals = []
        for sgn in (1.0, -1.0):
            s = sigma_t.clone()
            s[c] += sgn * delta
            fx, fy = plan.forces(s)
            vals.append(((fx - tx) ** 2).sum() + ((fy - ty) ** 2).sum())
        out.append(((vals[0] - vals[1]) / (2 * delta)).item())
    torch.cuda.synchronize()
    fd = np.array(out)
    g = grad[cells]
    return np.abs(fd - g).max() / np.abs(g).max()


def test_gradient_central_differences_fp64():
    """256 x 128 cells (every kernel instantiation it uses has run cleanly in
    the other GPU tests)."""
    sg = _sg()
    import torch
    M, N, k = 256, 128, 3
    xs, ys = oracle.sample_lattice(k, M, N)
    params = workloads.clump_params(5, 64)
    sigma = workloads.clump_sigma(params, xs, ys)
    target_sigma = workloads.clump_sigma(workloads.perturb_clumps(params, 55), xs, ys)
    plan = sg.Plan([(M, N, -1.0, 1.0, -1.0, 1.0, k)], sg.SG_FP64)
    try:
        s = to_dev(sigma.ravel(), torch.float64)
        tgt = plan.forces(to_dev(target_sigma.ravel(), torch.float64))
        fx, fy = plan.forces(s)
        grad = plan.adjoint(2 * (fx - tgt[0]), 2 * (fy - tgt[1])).cpu().numpy()
        cells = workloads.sample_cells(555, M, N, 64)
        # L is exactly quadratic: any step gives the exact derivative, and a
        # step of order sigma keeps the rounding of L small beside it
        err = _fd_check(plan, s, tgt, grad, cells, 0.5)
    finally:
        plan.close()
    assert err <= 1e-8, err


def _at_scale(grids):
    """Config-5 style check on one plan of several grids (the first one
    large): FP64 gradient of L = sum |F - F_target|^2 against central
    differences at 64 seeded cells of the first grid (exact for a quadratic
    L), and the FP32-split autograd gradient against the FP64 one per grid
    (bar R10)."""
    sg = _sg()
    import torch
    k = grids[0][6]
    sig_parts, tgt_parts = [], []
    for gi, g in enumerate(grids):
        xs, ys = oracle.sample_lattice(k, g[0], g[1])
        params = workloads.clump_params(5 + gi, 64)
        sig_parts.append(workloads.clump_sigma_torch(params, xs, ys).reshape(-1))
        tgt_parts.append(workloads.clump_sigma_torch(workloads.perturb_clumps(params, 55), xs, ys).reshape(-1))
    s64 = torch.cat(sig_parts)
    tsig = torch.cat(tgt_parts)
    del sig_parts, tgt_parts
    p64 = sg.Plan(grids, sg.SG_FP64)
    try:
        tgt = [t.clone() for t in p64.forces(tsig)]
        fx, fy = p64.forces(s64)
        g64 = p64.adjoint(2 * (fx - tgt[0]), 2 * (fy - tgt[1]))
        amps = []
        for gi in range(len(grids)):
            a, b = p64.offsets[gi], p64.offsets[gi + 1]
            fmax = max(fx[a:b].abs().max().item(), fy[a:b].abs().max().item())
            rmax = max((fx[a:b] - tgt[0][a:b]).abs().max().item(), (fy[a:b] - tgt[1][a:b]).abs().max().item())
            amps.append(fmax / rmax)
        # finite differences on the first grid (offset 0), exact for a quadratic loss
        cells = workloads.sample_cells(555, grids[0][0], grids[0][1], 64)
        fd_err = _fd_check(p64, s64, tgt, g64.cpu().numpy(), cells, 1e-2)
        tgt32 = (tgt[0].float(), tgt[1].float())
        g64h = g64.cpu().numpy()
    finally:
        p64.close()
    assert fd_err <= 1e-6, fd_err
    p32 = sg.Plan(grids, sg.SG_FP32_SPLIT)
    try:
        s32 = s64.float().requires_grad_(True)
        fx, fy = sg.ThinDiskForces.apply(s32, p32)
        loss = ((fx - tgt32[0]) ** 2).sum() + ((fy - tgt32[1]) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        g32 = s32.grad.double().cpu().numpy()
        offs = p32.offsets
    finally:
        p32.close()
    for gi in range(len(grids)):
        a, b = offs[gi], offs[gi + 1]
        err = np.abs(g32[a:b] - g64h[a:b]).max() / np.abs(g64h[a:b]).max()
        assert err <= 1e-6 * amps[gi] + 1e-6, (gi, err, amps[gi])


def test_differentiation_at_scale_multigrid_4096():
    """4096^2 with four 2048^2 grids alongside, in one plan (packed buffers)."""
    _at_scale([(4096, 4096, -1.0, 1.0, -1.0, 1.0, 3)] + [(2048, 2048, -1.0, 1.0, -1.0, 1.0, 3)] * 4)


def test_differentiation_at_scale_multigrid():
    """8192^2 with four 2048^2 grids alongside, in one plan (packed buffers)."""
    _at_scale([(8192, 8192, -1.0, 1.0, -1.0, 1.0, 3)] + [(2048, 2048, -1.0, 1.0, -1.0, 1.0, 3)] * 4)


def test_autograd_multigrid_plan_equals_single_plans():
    """A plan of several grids (mixed sizes and orders): its autograd
    gradient equals, bit for bit, that of one plan per grid."""
    sg = _sg()
    import torch
    grids = [(96, 48, -1.0, 1.0, -1.0, 1.0, 3), (64, 64, -1.0, 1.0, -1.0, 1.0, 2), (96, 48, -1.0, 1.0, -1.0, 1.0, 3),
             (32, 128, -1.0, 1.0, -2.0, 2.0, 1)]
    rng = np.random.default_rng(77)
    sig = [rng.standard_normal(g[0] * g[1]) for g in grids]
    tgt = [rng.standard_normal(2 * g[0] * g[1]) for g in grids]
    for prec in (sg.SG_FP64, sg.SG_FP32_SPLIT):
        plan = sg.Plan(grids, prec)
        try:
            s = to_dev(np.concatenate(sig), plan.dtype).requires_grad_(True)
            fx, fy = sg.ThinDiskForces.apply(s, plan)
            tx = to_dev(np.concatenate([t[: t.size // 2] for t in tgt]), plan.dtype)
            ty = to_dev(np.concatenate([t[t.size // 2:] for t in tgt]), plan.dtype)
            (((fx - tx) ** 2).sum() + ((fy - ty) ** 2).sum()).backward()
            torch.cuda.synchronize()
            batched = s.grad.clone()
            offs = plan.offsets
        finally:
            plan.close()
        for gi, g in enumerate(grids):
            p1 = sg.Plan([g], prec)
            try:
                s1 = to_dev(sig[gi], p1.dtype).requires_grad_(True)
                fx, fy = sg.ThinDiskForces.apply(s1, p1)
                n = g[0] * g[1]
                tx = to_dev(tgt[gi][:n], p1.dtype)
                ty = to_dev(tgt[gi][n:], p1.dtype)
                (((fx - tx) ** 2).sum() + ((fy - ty) ** 2).sum()).backward()
                torch.cuda.synchronize()
                assert torch.equal(s1.grad, batched[offs[gi]:offs[gi + 1]]), (prec, gi)
            finally:
                p1.close()


@pytest.mark.parametrize("n,k", [(1024, 4), (1024, 5), (4096, 4), (4096, 5)])
def test_adjoint_fp32_higher_orders_full_size(n, k):
    """The FP32-split adjoint of k = 4, 5 at full size (its row pass carries
    the banded x-solve of those orders) against the FP64 adjoint."""
    sg = _sg()
    import torch
    grid = (n, n, -1.0, 1.0, -1.0, 1.0, k)
    g = torch.Generator(device="cuda").manual_seed(n + k)
    gx = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
    gy = torch.randn(n * n, dtype=torch.float64, device="cuda", generator=g)
    plan = sg.Plan([grid], sg.SG_FP64)
    try:
        ref = plan.adjoint(gx, gy)
    finally:
        plan.close()
    p32 = sg.Plan([grid], sg.SG_FP32_SPLIT)
    try:
        got = p32.adjoint(gx.float(), gy.float())
        torch.cuda.synchronize()
        err = ((got.double() - ref).abs().max() / ref.abs().max()).item()
    finally:
        p32.close()
    # random gradients: FP32 transform rounding and input rounding, relative to max|g_sigma|
    assert err <= 2e-6, err
