"""CPU emulation of the four-step column kernels (paper_1904_07400_amd/csrc/
colfs.hpp, colfs3.hpp), built with g++ and ThreadSanitizer: one host thread per GPU
thread, workgroup barriers and wave-local barriers as real barriers.  Each
case checks the kernel's output against the column pass written from its
definition in numpy (tests/emu/colpass_ref.py), and that ThreadSanitizer
reports no data race on the LDS (an access that no barrier orders against
another thread's access to the same element).  Covers the shapes the GPU
runs (N = 2048, 4096 and 8192 in FP32 and FP64, 1024 in FP64, every LDS plan
and the component split; the radix-3 form for N = 1536 and 768), and 1024 in FP32,
which the library leaves to the Stockham kernel, on a few columns each."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, os.path.join(HERE, "emu"))
import colpass_ref as cr  # noqa: E402

pytestmark = pytest.mark.slow

GXX = shutil.which("g++")


def _build(tmp, kernel, prec, N, E, slots, k, to, split, pf=0):
    R = "float" if prec == 32 else "double"
    exe = os.path.join(tmp, f"emu_{kernel}_{prec}_{N}_{E}_{slots}_{k}_{to}_{split}_{pf}")
    cmd = [GXX, "-std=c++20", "-O1", "-g", "-fsanitize=thread", "-I" + os.path.join(HERE, "emu"),
           "-I" + os.path.join(ROOT, "paper_1904_07400_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
           f"-DEMU_KERNEL={kernel}", f"-DEMU_R={R}", f"-DEMU_TO={to}", f"-DEMU_N={N}", f"-DEMU_E={E}",
           f"-DEMU_SLOTS={slots}", f"-DEMU_MODE={k - 1}", f"-DEMU_SPLIT={split}", f"-DEMU_PF={pf}",
           os.path.join(HERE, "emu", "colfs_driver.cpp"), "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _tables(rng, M, N, to):
    tx = rng.standard_normal((M + 1, N + 1))
    ty = rng.standard_normal((M + 1, N + 1))
    out = []
    for t in (tx, ty):
        if to == "float2":
            hi = t.astype(np.float32)
            out.append(np.stack([hi, (t - hi.astype(np.float64)).astype(np.float32)], -1))
        elif to == "float":
            out.append(t.astype(np.float32))
        else:
            out.append(t)
    if to == "float":
        tx, ty = (t.astype(np.float32).astype(np.float64) for t in (tx, ty))
    return tx, ty, out


def _run(exe, M, path_in, path_out):
    r = subprocess.run([exe, str(M), path_in, path_out], capture_output=True, text=True, timeout=600)
    races = r.stderr.count("WARNING: ThreadSanitizer")
    assert r.returncode == 0 or races, r.stderr[-3000:]
    return races


FWD = [(32, 4096, 8, 4, 3, "float2", 0, 0), (32, 4096, 8, 4, 2, "float", 0, 0), (32, 4096, 8, 4, 5, "float2", 0, 0),
       (32, 8192, 16, 2, 4, "float", 1, 0), (64, 4096, 8, 2, 3, "double", 1, 0), (64, 8192, 16, 1, 2, "double", 1, 0),
       (32, 4096, 8, 4, 3, "float", 0, 1), (32, 4096, 8, 4, 1, "float", 0, 1),
       (32, 2048, 8, 4, 3, "float", 0, 0), (32, 2048, 8, 4, 2, "float2", 0, 0), (64, 2048, 8, 2, 5, "double", 0, 0),
       (32, 2048, 8, 2, 3, "float", 0, 0), (32, 2048, 8, 2, 2, "float", 0, 0), (32, 2048, 8, 2, 1, "float2", 0, 0),
       (32, 1024, 8, 4, 3, "float", 0, 0), (32, 1024, 8, 4, 2, "float2", 0, 0), (64, 1024, 8, 2, 5, "double", 0, 0),
       (64, 1024, 8, 2, 1, "double", 0, 0),
       (32, 8192, 16, 2, 3, "float", 2, 0), (32, 8192, 16, 2, 2, "float2", 2, 0)]


@pytest.mark.skipif(GXX is None, reason="g++ not found")
@pytest.mark.parametrize("prec,N,E,slots,k,to,split,pf", FWD,
                         ids=[f"fp{c[0]}-{c[1]}-s{c[3]}-k{c[4]}-{c[5]}-split{c[6]}-pf{c[7]}" for c in FWD])
def test_column_pass(tmp_path, prec, N, E, slots, k, to, split, pf):
    _column_case(tmp_path, 0, prec, N, E, slots, k, to, split, pf)


# the radix-3 column pass of 1536 and 768 (k_colfs3, FP32): every order, both table forms
FWD3 = [(1536, 3, "float2"), (1536, 1, "float2"), (1536, 2, "float2"), (1536, 4, "float"), (1536, 5, "float2"),
        (768, 3, "float2"), (768, 1, "float"), (768, 2, "float2"), (768, 4, "float2"), (768, 5, "float")]


@pytest.mark.skipif(GXX is None, reason="g++ not found")
@pytest.mark.parametrize("N,k,to", FWD3, ids=[f"{c[0]}-k{c[1]}-{c[2]}" for c in FWD3])
def test_column_pass_radix3(tmp_path, N, k, to):
    _column_case(tmp_path, 3, 32, N, N // 192, 4, k, to, 0, 0)


def _column_case(tmp_path, kernel, prec, N, E, slots, k, to, split, pf):
    M = 5 if pf else 4  # the prefetching loop: two workgroups over five columns
    exe = _build(str(tmp_path), kernel, prec, N, E, slots, k, to, split, pf)
    rng = np.random.default_rng(k * 11 + N)
    X = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    tx, ty, stored = _tables(rng, M, N, to)
    cdt = np.complex64 if prec == 32 else np.complex128
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as f:
        X.astype(cdt).tofile(f)
        for t in stored:
            t.tofile(f)
        np.exp(-1j * np.pi * np.arange(2 * N) / N).astype(cdt).tofile(f)
    races = _run(exe, M, fin, fout)
    tj = int(np.fromfile(fout, dtype=np.int32, count=1)[0])
    V = cr.untile(np.fromfile(fout, dtype=cdt, offset=4), M, N, tj)
    ref = cr.column_pass(X.astype(cdt).astype(complex), tx, ty, k, M, N)
    err = np.abs(V - ref).max() / np.abs(ref).max()
    assert races == 0
    assert err <= (1e-6 if prec == 32 else 1e-13), err


ADJ = [(32, 4096, 8, 2, 3, "float2"), (32, 4096, 8, 2, 2, "float"), (32, 8192, 16, 2, 5, "float2"),
       (64, 8192, 16, 1, 3, "double"), (64, 4096, 8, 2, 4, "double"), (32, 2048, 8, 2, 3, "float"),
       (64, 2048, 8, 2, 2, "double"), (32, 1024, 8, 2, 3, "float"), (64, 1024, 8, 2, 4, "double")]


@pytest.mark.skipif(GXX is None, reason="g++ not found")
@pytest.mark.parametrize("prec,N,E,slots,k,to", ADJ, ids=[f"fp{c[0]}-{c[1]}-s{c[3]}-k{c[4]}-{c[5]}" for c in ADJ])
def test_adjoint_column_pass(tmp_path, prec, N, E, slots, k, to):
    M = 4
    exe = _build(str(tmp_path), 1, prec, N, E, slots, k, to, 0)
    rng = np.random.default_rng(k * 13 + N + 1)
    Xx = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    Xy = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    tx, ty, stored = _tables(rng, M, N, to)
    cdt = np.complex64 if prec == 32 else np.complex128
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as f:
        Xx.astype(cdt).tofile(f)
        Xy.astype(cdt).tofile(f)
        for t in stored:
            t.tofile(f)
        np.exp(-1j * np.pi * np.arange(2 * N) / N).astype(cdt).tofile(f)
    races = _run(exe, M, fin, fout)
    tj = int(np.fromfile(fout, dtype=np.int32, count=1)[0])
    Y = cr.untile_half(np.fromfile(fout, dtype=cdt, offset=4), M, N, tj)
    ref = cr.adjoint_column_pass(Xx.astype(cdt).astype(complex), Xy.astype(cdt).astype(complex), tx, ty, k, M, N)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert races == 0
    assert err <= (1e-6 if prec == 32 else 1e-13), err


SPEC = [(3, "double"), (2, "float2"), (4, "float")]


@pytest.mark.skipif(GXX is None, reason="g++ not found")
@pytest.mark.parametrize("k,to", SPEC, ids=[f"k{c[0]}-{c[1]}" for c in SPEC])
def test_spectrum_columns(tmp_path, k, to):
    M, N = 4, 8192
    exe = _build(str(tmp_path), 2, 64, N, 16, 1, k, to, 0)
    rng = np.random.default_rng(k + 3)
    Sg = rng.standard_normal((M, 2 * N)) + 1j * rng.standard_normal((M, 2 * N))
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as f:
        Sg.tofile(f)
        np.exp(-1j * np.pi * np.arange(2 * N) / N).tofile(f)
    races = _run(exe, M, fin, fout)
    raw = np.fromfile(fout, dtype={"double": np.float64, "float": np.float32, "float2": np.float32}[to], offset=4)
    got = raw.reshape(M + 1, N + 1, 2).astype(np.float64).sum(-1) if to == "float2" else \
        raw.reshape(M + 1, N + 1).astype(np.float64)
    ref = cr.spectrum_columns(Sg, k, M, N, 0.25)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert races == 0
    assert err <= (1e-7 if to == "float" else 1e-13), err
