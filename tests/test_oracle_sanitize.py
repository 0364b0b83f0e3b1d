"""The oracle's C part (oracle/csrc/sg_oracle.c) under AddressSanitizer and
UndefinedBehaviorSanitizer: a small C driver exercises every entry point
(weights at listed offsets and in full for every order, the direct force
sum, its sparse and transposed forms) on a 6 x 5 grid with anisotropic
cells; the sanitized build must report nothing and print the same numbers as
the library the tests load (same compiler flags apart from the sanitizers)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "csrc", "sg_oracle.c")
GCC = shutil.which("gcc")

M, N, HX, HY = 6, 5, 0.3, 0.2

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int oracle_weights_at(int, double, double, int64_t, const int32_t*, const int32_t*, double*, double*);
int oracle_weights_full(int, int, int, double, double, double*, double*);
int oracle_forces(int, int, const double*, const double*, const double*, int64_t, const int64_t*, double*, double*);
int oracle_forces_sparse(int, double, double, int, int64_t, const int32_t*, const int32_t*, const double*, int64_t,
                         const int64_t*, double*, double*);
int oracle_forces_transpose(int, int, const double*, const double*, const double*, const double*, double*);
int main(void) {
  enum { M = %(M)d, N = %(N)d, W = (2 * M - 1) * (2 * N - 1) };
  const double hx = %(HX).17g, hy = %(HY).17g;
  double* wx = malloc(sizeof(double) * W);
  double* wy = malloc(sizeof(double) * W);
  double C[M * N], fx[M * N], fy[M * N], gs[M * N];
  for (int i = 0; i < M * N; ++i) C[i] = (double)((i * 37) %% 11) / 11.0 - 0.4;
  for (int k = 1; k <= 5; ++k) {
    if (oracle_weights_full(k, M, N, hx, hy, wx, wy)) return 2;
    double s = 0;
    for (int i = 0; i < W; ++i) s += wx[i] * (i + 1) + wy[i] * (i + 2);
    printf("weights %%d %%.17g\n", k, s);
    if (oracle_forces(M, N, C, wx, wy, 0, NULL, fx, fy)) return 3;
    s = 0;
    for (int i = 0; i < M * N; ++i) s += fx[i] * (i + 1) - fy[i] * (i + 3);
    printf("forces %%d %%.17g\n", k, s);
    if (oracle_forces_transpose(M, N, fx, fy, wx, wy, gs)) return 4;
    s = 0;
    for (int i = 0; i < M * N; ++i) s += gs[i] * (i + 1);
    printf("transpose %%d %%.17g\n", k, s);
    int32_t ip[3] = {0, 3, 5}, jp[3] = {0, 2, 4};
    double cv[3] = {1.0, -0.5, 0.25};
    int64_t cells[4] = {0, 7, 13, 29};
    double sx[4], sy[4];
    if (oracle_forces_sparse(k, hx, hy, M, 3, ip, jp, cv, 4, cells, sx, sy)) return 5;
    printf("sparse %%d %%.17g %%.17g\n", k, sx[1] + 2 * sx[2] + 3 * sx[3], sy[0] - sy[1] + sy[3]);
    int32_t ms[3] = {-5, 0, 4}, ns[3] = {3, 0, -4};
    double ax[3], ay[3];
    if (oracle_weights_at(k, hx, hy, 3, ms, ns, ax, ay)) return 6;
    printf("at %%d %%.17g %%.17g\n", k, ax[0] + ax[1] + ax[2], ay[0] - ay[2]);
  }
  free(wx);
  free(wy);
  return 0;
}
"""


def _reference_lines():
    """The same computation through the oracle library the tests load."""
    L = _lib.lib()
    W = (2 * M - 1) * (2 * N - 1)
    C = np.array([((i * 37) % 11) / 11.0 - 0.4 for i in range(M * N)])
    out = []
    for k in range(1, 6):
        wx, wy = np.zeros(W), np.zeros(W)
        assert L.oracle_weights_full(k, M, N, HX, HY, _lib.dptr(wx), _lib.dptr(wy)) == 0
        idx = np.arange(W, dtype=np.float64)
        s = 0.0
        for i in range(W):  # the driver's summation order
            s += wx[i] * (idx[i] + 1) + wy[i] * (idx[i] + 2)
        out.append(("weights", k, s))
        fx, fy = np.zeros(M * N), np.zeros(M * N)
        assert L.oracle_forces(M, N, _lib.dptr(C), _lib.dptr(wx), _lib.dptr(wy), 0, None, _lib.dptr(fx),
                               _lib.dptr(fy)) == 0
        s = 0.0
        for i in range(M * N):
            s += fx[i] * (i + 1) - fy[i] * (i + 3)
        out.append(("forces", k, s))
    return out


@pytest.mark.skipif(GCC is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER % {"M": M, "N": N, "HX": HX, "HY": HY})
    exe = tmp_path / "oracle_san"
    cmd = [GCC, "-O2", "-g", "-fopenmp", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           SRC, str(drv), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    # verify_asan_link_order=0: the environment may preload other libraries ahead of the runtime
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    got = {}
    for line in r.stdout.splitlines():
        parts = line.split()
        got[(parts[0], int(parts[1]))] = [float(x) for x in parts[2:]]
    assert len(got) == 25
    for name, k, s in _reference_lines():
        assert got[(name, k)][0] == pytest.approx(s, rel=1e-13, abs=1e-15), (name, k)
