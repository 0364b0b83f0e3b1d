"""Plain FP64 CPU implementation of the method (test infrastructure only).

Arrays are row-major ``[N][M]`` (index ``[j, i]``, x fastest), cell (i, j)
of the paper (1-based) at ``[j-1, i-1]``.
"""
from __future__ import annotations

import math

import numpy as np

from . import _lib

build = _lib.build


# ----------------------------------------------------------------- grid ---
def cell_centres(n: int, lo: float, hi: float) -> np.ndarray:
    """Cell centres x_i = (x_{i-1/2} + x_{i+1/2}) / 2 with x_{i+1/2} = L + i dx
    (Sec. 2.2, definition of the grid points before Sec. 2.1)."""
    h = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * h


def sample_lattice(k: int, M: int, N: int, domain=(-1.0, 1.0, -1.0, 1.0)):
    """Points where sigma must be sampled so that C can be obtained from it.

    Odd k: the cell centres (Sec. 2.3, interpolation condition Eq. (eqnSigmaB)).
    Even k: the spline attached to C_i' is centred on the vertex
    x_{i'+1/2} = L + i' dx, i' = 1..M (k = 2 spans x_{i'-1/2} .. x_{i'+3/2},
    Case 2, and C = sigma there by the "C = sigma for k = 1, 2" remark of
    Sec. 2.3; k = 4 spans x_{i'-3/2} .. x_{i'+5/2}).
    """
    x0, x1, y0, y1 = domain
    hx, hy = (x1 - x0) / M, (y1 - y0) / N
    if k % 2 == 1:
        return cell_centres(M, x0, x1), cell_centres(N, y0, y1)
    return x0 + hx * np.arange(1, M + 1, dtype=np.float64), y0 + hy * np.arange(1, N + 1, dtype=np.float64)


# ----------------------------------------------------------- B-splines ---
def bspline_value(k: int, knots, x: float) -> float:
    """Order-k B-spline with knots t_0..t_k at x, Cox-de Boor (Eq. (eqnBk))."""
    t = np.ascontiguousarray(knots, dtype=np.float64)
    assert t.shape == (k + 1,)
    return float(_lib.lib().oracle_bspline(k, _lib.dptr(t), float(x)))


# ---------------------------------------------------- coefficient solve ---
def thomas(a: float, b: float, c: float, d: np.ndarray, axis: int) -> np.ndarray:
    """Solve the constant tridiagonal system (a x_{i-1} + b x_i + c x_{i+1} = d_i,
    x = 0 outside) along ``axis`` of ``d`` by Gaussian elimination without
    pivoting (the Thomas algorithm), independently for every line."""
    d = np.moveaxis(np.array(d, dtype=np.float64, copy=True), axis, 0)
    n = d.shape[0]
    cp = np.empty(n)
    dp = np.empty_like(d)
    cp[0] = c / b
    dp[0] = d[0] / b
    for i in range(1, n):
        den = b - a * cp[i - 1]
        cp[i] = c / den
        dp[i] = (d[i] - a * dp[i - 1]) / den
    x = np.empty_like(d)
    x[n - 1] = dp[n - 1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return np.moveaxis(x, 0, axis)


# Orders above 3 (the extension the end of Sec. 2.3 and Case 3 of Sec. 2.2
# state): the interpolation condition of Eq. (sigmaW) with the order-k
# spline in place of the quadratic one.  Per axis, sigma at a sample point is
# the sum of the coefficients of the splines that cover it, each times that
# spline's value there: the uniform cubic at its centre and one cell away
# (4/6, 1/6), the uniform quartic at its centre, one and two cells away
# (230/384, 76/384, 1/384).  With C = 0 outside the grid, as after
# Eq. (C_system), each axis is a symmetric banded Toeplitz system.
STENCIL = {4: (1.0 / 6, 4.0 / 6, 1.0 / 6),
           5: (1.0 / 384, 76.0 / 384, 230.0 / 384, 76.0 / 384, 1.0 / 384)}


def banded_solve(stencil, d: np.ndarray, axis: int) -> np.ndarray:
    """Solve the Toeplitz system with the symmetric ``stencil`` (x = 0 outside
    the line) along ``axis`` of ``d`` for every line, by LAPACK's banded LU
    (scipy.linalg.solve_banded)."""
    from scipy.linalg import solve_banded
    h = len(stencil) // 2
    d = np.moveaxis(np.array(d, dtype=np.float64, copy=True), axis, 0)
    n = d.shape[0]
    ab = np.zeros((2 * h + 1, n))
    for r in range(2 * h + 1):
        ab[r, :] = stencil[r]
    x = solve_banded((h, h), ab, d.reshape(n, -1)).reshape(d.shape)
    return np.moveaxis(x, 0, axis)


def bspline_coeffs(sigma: np.ndarray, k: int) -> np.ndarray:
    """sigma -> C (Sec. 2.3).

    k = 1, 2: C = sigma (normalised splines, sampled on ``sample_lattice``).
    k = 3: first the z-system of Eq. (z_system), tridiag(1,6,1) z_{i,.} = sigma_{i,.}
    along j for every i, then the C-system of Eq. (C_system),
    (1/64) tridiag(1,6,1) C_{.,j} = z_{.,j} along i for every j; C = 0 outside
    the grid (isolated boundary condition stated after Eq. (C_system)).
    """
    s = np.asarray(sigma, dtype=np.float64)
    if k in (1, 2):
        return s.copy()
    if k in STENCIL:  # k = 4, 5: along j, then along i
        return banded_solve(STENCIL[k], banded_solve(STENCIL[k], s, axis=0), axis=1)
    if k != 3:
        raise ValueError("oracle implements k = 1..5")
    z = thomas(1.0, 6.0, 1.0, s, axis=0)              # along j (rows of the [N][M] array)
    return thomas(1.0 / 64, 6.0 / 64, 1.0 / 64, z, axis=1)   # along i


def bspline_apply(C: np.ndarray, k: int) -> np.ndarray:
    """The interpolation operator itself, C -> sigma at the sample lattice,
    Eq. (sigmaW) with W of Eq. (weight_matrix) (identity for k = 1, 2)."""
    C = np.asarray(C, dtype=np.float64)
    if k in (1, 2):
        return C.copy()
    if k in STENCIL:
        st = STENCIL[k]
        h = len(st) // 2
        P = np.zeros((C.shape[0] + 2 * h, C.shape[1] + 2 * h))
        P[h:-h, h:-h] = C
        out = np.zeros_like(C)
        for dj in range(2 * h + 1):
            for di in range(2 * h + 1):
                out += st[dj] * st[di] * P[dj:dj + C.shape[0], di:di + C.shape[1]]
        return out
    P = np.zeros((C.shape[0] + 2, C.shape[1] + 2))
    P[1:-1, 1:-1] = C
    Wm = np.array([[1, 6, 1], [6, 36, 6], [1, 6, 1]], dtype=np.float64) / 64.0
    out = np.zeros_like(C)
    for dj in range(3):
        for di in range(3):
            out += Wm[dj, di] * P[dj:dj + C.shape[0], di:di + C.shape[1]]
    return out


def coeffs_transpose_solve(g: np.ndarray, k: int) -> np.ndarray:
    """Transpose of sigma -> C.  The two matrices of Eqs. (z_system) and
    (C_system) are symmetric (so are the banded ones of k = 4, 5), so the
    transpose is the same two solves."""
    return bspline_coeffs(g, k)


# -------------------------------------------------------------- weights ---
def weights_at(k: int, hx: float, hy: float, ms, ns):
    """w^x_{m,n}, w^y_{m,n} of Eq. (eqnwB) at the given offsets (m = i - i',
    n = j - j'), by quadrature of the defining integral."""
    ms = np.ascontiguousarray(ms, dtype=np.int32).ravel()
    ns = np.ascontiguousarray(ns, dtype=np.int32).ravel()
    wx = np.empty(ms.size)
    wy = np.empty(ms.size)
    rc = _lib.lib().oracle_weights_at(k, float(hx), float(hy), ms.size, _lib.i32ptr(ms),
                                      _lib.i32ptr(ns), _lib.dptr(wx), _lib.dptr(wy))
    if rc:
        raise ValueError("oracle_weights_at failed")
    return wx, wy


def weights(k: int, M: int, N: int, hx: float, hy: float):
    """Full weight tables, shape (2N-1, 2M-1); entry (m, n) at [n+N-1, m+M-1]."""
    wx = np.empty((2 * N - 1, 2 * M - 1))
    wy = np.empty((2 * N - 1, 2 * M - 1))
    rc = _lib.lib().oracle_weights_full(k, M, N, float(hx), float(hy), _lib.dptr(wx), _lib.dptr(wy))
    if rc:
        raise ValueError("oracle_weights_full failed")
    return wx, wy


# --------------------------------------------------------------- forces ---
def forces_from_coeffs(C: np.ndarray, wx: np.ndarray, wy: np.ndarray, cells=None):
    """Eq. (eqnF) by direct summation.  ``cells``: flat indices j*M+i, or None
    for every cell (then the result has the grid's shape)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    N, M = C.shape
    assert wx.shape == (2 * N - 1, 2 * M - 1) and wy.shape == wx.shape
    wx = np.ascontiguousarray(wx)
    wy = np.ascontiguousarray(wy)
    L = _lib.lib()
    if cells is None:
        fx = np.empty((N, M))
        fy = np.empty((N, M))
        L.oracle_forces(M, N, _lib.dptr(C), _lib.dptr(wx), _lib.dptr(wy), 0, None,
                        _lib.dptr(fx), _lib.dptr(fy))
        return fx, fy
    cells = np.ascontiguousarray(cells, dtype=np.int64).ravel()
    fx = np.empty(cells.size)
    fy = np.empty(cells.size)
    L.oracle_forces(M, N, _lib.dptr(C), _lib.dptr(wx), _lib.dptr(wy), cells.size,
                    _lib.i64ptr(cells), _lib.dptr(fx), _lib.dptr(fy))
    return fx, fy


def forces(sigma: np.ndarray, k: int, domain=(-1.0, 1.0, -1.0, 1.0), cells=None):
    """sigma (on ``sample_lattice``) -> (Fx, Fy) at the cell centres, G = 1."""
    sigma = np.asarray(sigma, dtype=np.float64)
    N, M = sigma.shape
    x0, x1, y0, y1 = domain
    C = bspline_coeffs(sigma, k)
    wx, wy = weights(k, M, N, (x1 - x0) / M, (y1 - y0) / N)
    return forces_from_coeffs(C, wx, wy, cells)


def forces_sparse(k: int, hx: float, hy: float, M: int, src_i, src_j, src_c, cells):
    """Forces at ``cells`` from a sparse set of coefficients C (impulse
    superposition of Eq. (eqnF); weights evaluated per pair)."""
    ip = np.ascontiguousarray(src_i, dtype=np.int32)
    jp = np.ascontiguousarray(src_j, dtype=np.int32)
    cv = np.ascontiguousarray(src_c, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64).ravel()
    fx = np.empty(cells.size)
    fy = np.empty(cells.size)
    rc = _lib.lib().oracle_forces_sparse(k, float(hx), float(hy), M, ip.size, _lib.i32ptr(ip),
                                         _lib.i32ptr(jp), _lib.dptr(cv), cells.size,
                                         _lib.i64ptr(cells), _lib.dptr(fx), _lib.dptr(fy))
    if rc:
        raise ValueError("oracle_forces_sparse failed")
    return fx, fy


def forces_adjoint(gx: np.ndarray, gy: np.ndarray, k: int, domain=(-1.0, 1.0, -1.0, 1.0)):
    """Transpose of sigma -> (Fx, Fy): g_sigma = S^-T (W_x^T gx + W_y^T gy)."""
    gx = np.ascontiguousarray(gx, dtype=np.float64)
    gy = np.ascontiguousarray(gy, dtype=np.float64)
    N, M = gx.shape
    x0, x1, y0, y1 = domain
    wx, wy = weights(k, M, N, (x1 - x0) / M, (y1 - y0) / N)
    gc = np.empty((N, M))
    _lib.lib().oracle_forces_transpose(M, N, _lib.dptr(gx), _lib.dptr(gy), _lib.dptr(wx),
                                       _lib.dptr(wy), _lib.dptr(gc))
    return coeffs_transpose_solve(gc, k)


# ------------------------------------------------------- analytic disks ---
def disk_force_radial(n: int, R, alpha: float, sigma0: float = 1.0, G: float = 1.0):
    """Radial force in the plane of the generalised Maclaurin disk D_n,
    n = 3 or 4, as printed in Sec. 3 (eta = alpha / R).  F_R = 0 at R = 0."""
    R = np.asarray(R, dtype=np.float64)
    out = np.zeros_like(R)
    pos = R > 0
    eta = np.where(pos, alpha / np.where(pos, R, 1.0), 1.0)
    inside = pos & (eta >= 1.0)
    outside = pos & (eta < 1.0)
    e = eta
    if n == 3:
        p = -15.0 / 8 * e**4 + 45.0 / 16 * e**2 - 75.0 / 64
        q = 5.0 / 8 * e**5 - 65.0 / 32 * e**3 + 75.0 / 64 * e
        npow = 5
    elif n == 4:
        p = -35.0 / 16 * e**6 + 315.0 / 64 * e**4 - 525.0 / 128 * e**2 + 1225.0 / 1024
        q = 35.0 / 64 * e**7 - 1085.0 / 384 * e**5 + 5075.0 / 1536 * e**3 - 1225.0 / 1024 * e
        npow = 7
    else:
        raise ValueError("analytic forces are given for D3 and D4 only")
    ein = e**(-npow)
    out[inside] = (math.pi**2 * sigma0 * G / 2.0) * (ein * p)[inside]
    eo = np.minimum(e, 1.0)
    val = math.pi * sigma0 * G * ein * (p * np.arcsin(eo) + q * np.sqrt(np.maximum(0.0, 1.0 - eo**2)))
    out[outside] = val[outside]
    return out


# ---------------------------------------------------------------- norms ---
def error_norms(num: np.ndarray, ana: np.ndarray, dx: float, dy: float):
    """(L1, L2, Linf) of Eqs. (oneNormErr)-(inftyNormErr) as the tables use
    them: the sums are weighted by the cell area dx*dy (the printed 1/N^2
    read as the cell area of the [-1,1]^2 domain up to its constant factor:
    only this weighting reproduces the tabulated L1 and L2 values)."""
    e = np.abs(np.asarray(num) - np.asarray(ana))
    return float(e.sum() * dx * dy), float(math.sqrt((e * e).sum() * dx * dy)), float(e.max())


def accuracy_order(err_coarse: float, err_fine: float) -> float:
    """Order of accuracy between N and 2N: log2(L_N / L_2N) (Sec. 3.1)."""
    return math.log2(err_coarse / err_fine)


# ----------------------------------------------- closed forms (mpmath) ---
def antiderivative(x, y, alpha: int, beta: int):
    """F(x, y, alpha, beta) of Appendix A (alpha + beta <= 4), an
    antiderivative with d^2F/dxdy = x^alpha y^beta / r^3.  mpmath numbers."""
    import mpmath as mp
    x = mp.mpf(x)
    y = mp.mpf(y)
    r = mp.sqrt(x * x + y * y)
    a, b = alpha, beta
    if (a, b) == (0, 0):
        return -r / (x * y)
    if (a, b) == (1, 0):
        return -mp.log(y + r)
    if (a, b) == (2, 0):
        return y * mp.log(x + r)
    if (a, b) == (1, 1):
        return -r
    if (a, b) == (3, 0):
        return y * r
    if (a, b) == (2, 1):
        return -x * r / 2 + y * y * mp.log(x + r) / 2
    if (a, b) == (4, 0):
        return x * y * r / 2 - y**3 * mp.log(x + r) / 2
    if (a, b) == (3, 1):
        return -r * (x * x - 2 * y * y) / 3
    if (a, b) == (2, 2):
        return -x * y * r / 3 + y**3 * mp.log(x + r) / 3 + x**3 * mp.log(y + r) / 3
    if a < b:
        return antiderivative(y, x, b, a)
    raise ValueError("Appendix A lists alpha + beta <= 4 only")


def _G(x, a, alpha: int):
    """G(x, a, alpha) = int x^alpha / (x^2 + a^2)^{3/2} dx: the bases of
    Eqs. (B11)-(B13) and the recursion of Eq. (intMoment)."""
    import mpmath as mp
    r = mp.sqrt(x * x + a * a)
    if alpha == 0:
        return x / (a * a * r)
    if alpha == 1:
        return -1 / r
    if alpha == 2:
        return -x / r + mp.log(abs(x + r))
    return x**(alpha - 1) / ((alpha - 2) * r) - mp.mpf(alpha - 1) / (alpha - 2) * a * a * _G(x, a, alpha - 2)


def antiderivative_intF(x, y, alpha: int, beta: int):
    """F(x, y, alpha, beta) by Eq. (intF) with G from Eq. (intMoment);
    valid for alpha + beta != 1."""
    import mpmath as mp
    x = mp.mpf(x)
    y = mp.mpf(y)
    s = alpha + beta - 1
    return (y**(beta + 1) * _G(x, y, alpha) + x**(alpha + 1) * _G(y, x, beta)) / s
