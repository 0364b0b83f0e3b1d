"""Oracle pin: reproduce the paper's Tables 4-9 (Sec. 3.1).

The whole oracle chain (sample lattice, coefficient solve, weights, direct
sum, norms) and the analytic D3/D4 forces it is compared with must give the
printed error norms.  The setup is that of Sec. 3: [-1,1]^2, sigma0 = G = 1,
disk size 0.5.  N <= 256 must match every printed digit (a difference of one
unit in the last printed digit is accepted: two N = 256, k = 3, D4 values sit
on a rounding boundary); N = 512 (all six order/disk cases) must match to 0.5 % (the paper's own
weight round-off shows in the third digit of its k = 3 L1 values there).
"""
import csv
import math
import os

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows():
    out = []
    with open(os.path.join(HERE, "golden", "paper_tables_4_9.csv")) as f:
        for row in csv.reader(line for line in f if not line.startswith("#")):
            k, n, N = int(row[0]), int(row[1]), int(row[2])
            out.append((k, n, N, [float(v) for v in row[3:]], row[3:]))
    return out


def _norms(k, n, N, alpha=0.5):
    xs, ys = oracle.sample_lattice(k, N, N)
    sigma = workloads.disk_sigma(n, alpha, xs, ys)
    fx, fy = oracle.forces(sigma, k)
    xc = oracle.cell_centres(N, -1.0, 1.0)
    X, Y = np.meshgrid(xc, xc)
    R = np.hypot(X, Y)
    FR = oracle.disk_force_radial(n, R, alpha)
    h = 2.0 / N
    ex = oracle.error_norms(fx, FR * X / R, h, h)
    eR = oracle.error_norms((X * fx + Y * fy) / R, FR, h, h)
    return list(ex) + list(eR)


def _last_digit_unit(text):
    mant, exp = text.lower().split("e")
    decimals = len(mant.split(".")[1]) if "." in mant else 0
    return 10.0 ** (int(exp) - decimals)


ROWS = _rows()
FAST = [r for r in ROWS if r[2] <= 256]
SLOW = [r for r in ROWS if r[2] == 512]


@pytest.mark.parametrize("k,n,N,printed,texts", FAST, ids=[f"k{r[0]}-D{r[1]}-N{r[2]}" for r in FAST])
def test_tables_all_digits(k, n, N, printed, texts):
    got = _norms(k, n, N)
    for g, p, t in zip(got, printed, texts):
        assert abs(g - p) <= 1.0001 * _last_digit_unit(t), (g, t)


@pytest.mark.slow
@pytest.mark.parametrize("k,n,N,printed,texts", SLOW, ids=[f"k{r[0]}-D{r[1]}-N{r[2]}" for r in SLOW])
def test_tables_n512(k, n, N, printed, texts):
    got = _norms(k, n, N)
    for g, p in zip(got, printed):
        assert abs(g / p - 1.0) < 5e-3, (g, p)


def test_observed_orders():
    """Orders of accuracy approach k for the D4 disk (Sec. 3.1, Tables 7-9)."""
    for k in (1, 2, 3):
        e = [_norms(k, 4, N)[2] for N in (64, 128, 256)]
        orders = [oracle.accuracy_order(e[i], e[i + 1]) for i in range(2)]
        assert abs(orders[-1] - k) < 0.25, (k, orders)
    # D3 is not smooth enough for k = 3 in the max norm (Sec. 3.1): order ~2.5
    e = [_norms(3, 3, N)[2] for N in (64, 128, 256)]
    o = oracle.accuracy_order(e[1], e[2])
    assert 2.2 < o < 2.7 and math.isfinite(o)
