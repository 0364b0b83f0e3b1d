"""Reference of the column pass (pass B) in numpy, written from its
definition, for the CPU emulation tests of the column kernels: for each
column c of the row spectra X (column 0 packing the real bins 0 and M):
[the y-solve of order k], the 2N-point transform of the zero-padded column,
the products with i A^x, i A^y (A from the quarter tables by the reflection
q -> 2N - q, and for even k the half-cell phase), the unnormalised inverse
cropped to N, and V(c) = Yx + i Yy, V(2M - c) = conj(Yx) + i conj(Yy)."""
import numpy as np
import scipy.linalg

STENCIL = {3: [1.0, 6.0, 1.0], 4: [1.0, 4.0, 1.0], 5: [1.0, 76.0, 230.0, 76.0, 1.0]}


def band_solve(k, a):
    """Solve (stencil / sum(stencil)) y = a along axis 0 (C = 0 outside)."""
    st = np.array(STENCIL[k])
    st = st / st.sum()
    h = len(st) // 2
    n = a.shape[0]
    ab = np.zeros((2 * h + 1, n))
    for d in range(-h, h + 1):
        ab[h - d, max(d, 0):n + min(d, 0)] = st[h + d]
    return scipy.linalg.solve_banded((h, h), ab, a)


def full_table(tab_row, N, eps):
    """A(q) for q in [0, 2N) from a stored row of N + 1 entries: half 0
    (q = 2q') at [0, N/2], half 1 (q = 2q' + 1) at N/2 + 1 + [0, N/2)."""
    A = np.zeros(2 * N)
    for qq in range(N):
        A[2 * qq] = tab_row[qq] if qq <= N // 2 else eps * tab_row[N - qq]
        A[2 * qq + 1] = tab_row[N // 2 + 1 + qq] if qq < N // 2 else eps * tab_row[N // 2 + 1 + N - 1 - qq]
    return A


def column_pass(X, tx, ty, k, M, N):
    """X: (M, N) complex columns; tx, ty: (M + 1, N + 1) real tables.
    Returns V as (2M, N) complex (row p = bin p)."""
    kind = 1 if k % 2 == 0 else 0
    ex = -1.0 if kind else 1.0
    V = np.zeros((2 * M, N), complex)
    q = np.arange(2 * N)
    for c in range(M):
        a = X[c].astype(complex)
        if k >= 3:
            a = band_solve(k, a.real) + 1j * band_solve(k, a.imag)
        Z = np.fft.fft(np.concatenate([a, np.zeros(N)]))
        if c == 0:
            Zm = np.conj(Z[(-q) % (2 * N)])
            parts = [(0, 0.5 * (Z + Zm)), (M, (Z - Zm) / 2j)]
        else:
            parts = [(c, Z)]
        Y = []
        for p, Zp in parts:
            Ax = full_table(tx[p], N, ex)
            Ay = full_table(ty[p], N, -ex)
            ph = np.exp(-1j * np.pi * (p / (2 * M) + q / (2 * N))) if kind else 1.0
            gx = Zp * ph * 1j * Ax
            gy = Zp * ph * 1j * Ay
            yx = np.fft.ifft(gx)[:N] * 2 * N
            yy = np.fft.ifft(gy)[:N] * 2 * N
            Y.append((yx, yy))
        if c == 0:
            (y0x, y0y), (ymx, ymy) = Y
            yx = y0x + 1j * ymx
            yy = y0y + 1j * ymy
            V[0] = yx.real + 1j * yy.real
            V[M] = yx.imag + 1j * yy.imag
        else:
            yx, yy = Y[0]
            V[c] = yx + 1j * yy
            V[2 * M - c] = np.conj(yx) + 1j * np.conj(yy)
    return V


def untile(Vt, M, N, tj):
    """The tiled V layout of the kernels -> (2M, N): element (p, j) at
    ((j // tj * 2 + p % 2) * M + p // 2) * tj + j % tj."""
    out = np.zeros((2 * M, N), Vt.dtype)
    p = np.arange(2 * M)[:, None]
    j = np.arange(N)[None, :]
    out[:] = Vt[((j // tj * 2 + p % 2) * M + p // 2) * tj + j % tj]
    return out


def adjoint_column_pass(Xx, Xy, tx, ty, k, M, N):
    """The adjoint column pass: per column the zero-padded transforms of the
    gradient spectra, products with the conjugate spectra summed over x and y,
    the unnormalised inverse cropped to N, then the y-solve.  Returns (M, N)."""
    kind = 1 if k % 2 == 0 else 0
    ex = -1.0 if kind else 1.0
    Y = np.zeros((M, N), complex)
    q = np.arange(2 * N)
    for c in range(M):
        Zx = np.fft.fft(np.concatenate([Xx[c], np.zeros(N)]))
        Zy = np.fft.fft(np.concatenate([Xy[c], np.zeros(N)]))

        def conj_prod(Zxp, Zyp, p):
            Ax = full_table(tx[p], N, ex)
            Ay = full_table(ty[p], N, -ex)
            ph = np.exp(-1j * np.pi * (p / (2 * M) + q / (2 * N))) if kind else 1.0
            return Zxp * np.conj(1j * Ax * ph) + Zyp * np.conj(1j * Ay * ph)

        if c == 0:
            def split(Z):
                Zm = np.conj(Z[(-q) % (2 * N)])
                return 0.5 * (Z + Zm), (Z - Zm) / 2j
            x0, xm = split(Zx)
            y0, ym = split(Zy)
            H = conj_prod(x0, y0, 0) + 1j * conj_prod(xm, ym, M)
        else:
            H = conj_prod(Zx, Zy, c)
        h = np.fft.ifft(H)[:N] * 2 * N
        if k >= 3:
            h = band_solve(k, h.real) + 1j * band_solve(k, h.imag)
        Y[c] = h
    return Y


def untile_half(Yt, M, N, tj):
    """The packed gC spectra layout -> (M, N): bin p of row j at
    ((j // tj * 2 + p % 2) * (M // 2) + p // 2) * tj + j % tj."""
    p = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    return Yt[((j // tj * 2 + p % 2) * (M // 2) + p // 2) * tj + j % tj]


def spectrum_columns(Sg, k, M, N, scale):
    """Stored spectrum tables from the row spectra S (M columns of 2N): the
    2N-point transform of each column scaled, column 0 split into bins 0 and
    M, A = Im W (odd k) or Im(W conj(ph)) (even k), on the quarter."""
    kind = 1 if k % 2 == 0 else 0
    tab = np.zeros((M + 1, N + 1))
    q = np.arange(2 * N)
    for c in range(M):
        Z = np.fft.fft(Sg[c]) * scale
        if c == 0:
            Zm = np.conj(Z[(-q) % (2 * N)])
            parts = [(0, 0.5 * (Z + Zm)), (M, (Z - Zm) / 2j)]
        else:
            parts = [(c, Z)]
        for p, W in parts:
            if kind:
                ph = np.exp(-1j * np.pi * (p / (2 * M) + q / (2 * N)))
                A = (W * np.conj(ph)).imag
            else:
                A = W.imag
            tab[p, :N // 2 + 1] = A[0:N + 1:2]
            tab[p, N // 2 + 1:] = A[1:N:2]
    return tab
