"""GPU tests of the launch tuning: per class, the variant of each pass
(kernels of the same transform with other buffering or elements per thread)
and its tile, chosen by timing under SG_FLAG_AUTOTUNE, kept in the
process-wide store and in the SG_TUNE_CACHE file.

Checked: a first autotuned plan times its classes (source 1) and writes the
cache; a second plan, with or without the flag, takes the stored choices
(source 2) and gives bit-identical forces, as do one-grid plans; a fresh
process reads the file and times nothing; SG_TUNE=off keeps the defaults;
malformed cache lines are skipped; the tuned plan meets the FP32-split bar
against the FP64 path.  Also the diagnostics from the environment: SG_LOG
(launch choices and errors on stderr) and SG_ROCTX (roctx ranges).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads
from gpu_util import rel_max_err, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# sizes with two variants of a pass (the Stockham column pass up to 1536,
# the inverse row pass from 512) that no other test tunes
GRIDS = [
    (512, 512, -1.0, 1.0, -1.0, 1.0, 3),
    (768, 768, -1.0, 1.0, -1.0, 1.0, 1),
    (512, 512, -1.0, 1.0, -1.0, 1.0, 3),
    (1024, 256, -2.0, 2.0, -0.5, 0.5, 2),
]


def _sg():
    import paper_1904_07400_amd as sg
    return sg


def _sigma(grids):
    import oracle
    parts = []
    for gi, g in enumerate(grids):
        xs, ys = oracle.sample_lattice(g[6], g[0], g[1], g[2:6])
        parts.append(workloads.clump_sigma(workloads.clump_params(70 + gi, 8), xs, ys).ravel())
    return np.concatenate(parts)


def _tuning(sg, plan):
    return [sg.sg_plan_tuning(plan.handle, c) for c in range(len(sg.sg_plan_classes(plan.handle)))]


def _forces(plan, sigma):
    import torch
    fx, fy = plan.forces(to_dev(sigma, plan.dtype))
    torch.cuda.synchronize()
    return fx.cpu().numpy(), fy.cpu().numpy()


def test_store_cache_and_identical_results(tmp_path, monkeypatch):
    sg = _sg()
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SG_TUNE_CACHE", str(cache))
    monkeypatch.delenv("SG_TUNE", raising=False)
    sigma = _sigma(GRIDS)
    p1 = sg.Plan(GRIDS, sg.SG_FP32_SPLIT, flags=sg.SG_FLAG_AUTOTUNE)
    try:
        t1 = _tuning(sg, p1)
        f1 = _forces(p1, sigma)
        offs = p1.offsets
    finally:
        p1.close()
    assert len(t1) == 3 and all(src == 1 for _, _, src in t1), t1
    assert all(t >= 1 for _, tiles, _ in t1 for t in tiles)
    # the cache file: valid JSON with a variant and a tile entry per class
    doc = json.loads(cache.read_text())
    assert doc["sg_tune_cache"] == 1
    for (nx, ny, k), (var, tiles, _) in zip([(512, 512, 3), (768, 768, 1), (1024, 256, 2)], t1):
        vk = [key for key in doc["variants"] if key.endswith(f"/fp32/{nx}x{ny}/k{k}")]
        tk = [key for key in doc["tiles"] if f"/fp32/{nx}x{ny}/k{k}/g" in key]
        assert len(vk) == 1 and tuple(doc["variants"][vk[0]]) == var
        assert len(tk) == 1 and tuple(doc["tiles"][tk[0]]) == tiles
    # second plans: stored choices, identical results
    for flags in (sg.SG_FLAG_AUTOTUNE, 0, sg.SG_FLAG_GRAPH):
        p2 = sg.Plan(GRIDS, sg.SG_FP32_SPLIT, flags=flags)
        try:
            t2 = _tuning(sg, p2)
            f2 = _forces(p2, sigma)
        finally:
            p2.close()
        assert all(src == 2 for _, _, src in t2), (flags, t2)
        assert [t[:2] for t in t2] == [t[:2] for t in t1]
        assert np.array_equal(f2[0], f1[0]) and np.array_equal(f2[1], f1[1]), flags
    # one-grid plans take the stored variants: the same forces bit for bit
    for gi, g in enumerate(GRIDS):
        ps = sg.Plan([g], sg.SG_FP32_SPLIT)
        try:
            fs = _forces(ps, sigma[offs[gi]:offs[gi + 1]])
        finally:
            ps.close()
        assert np.array_equal(fs[0], f1[0][offs[gi]:offs[gi + 1]]), gi
        assert np.array_equal(fs[1], f1[1][offs[gi]:offs[gi + 1]]), gi
    # accuracy of the tuned plan against the FP64 path
    p64 = sg.Plan(GRIDS, sg.SG_FP64)
    try:
        g64 = _forces(p64, sigma)
    finally:
        p64.close()
    for gi in range(len(GRIDS)):
        a, b = offs[gi], offs[gi + 1]
        err = rel_max_err(f1[0][a:b], f1[1][a:b], g64[0][a:b], g64[1][a:b])
        assert err <= 1e-6, (gi, err)


def test_fresh_process_reads_the_cache(tmp_path):
    """A new process with the same SG_TUNE_CACHE times nothing."""
    cache = tmp_path / "tune.json"
    script = (
        "import sys, json\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import paper_1904_07400_amd as sg\n"
        f"grids = {GRIDS!r}\n"
        "p = sg.Plan(grids, sg.SG_FP32_SPLIT, flags=sg.SG_FLAG_AUTOTUNE)\n"
        "n = len(sg.sg_plan_classes(p.handle))\n"
        "print(json.dumps([sg.sg_plan_tuning(p.handle, c) for c in range(n)]))\n"
        "p.close()\n")
    env = dict(os.environ, SG_TUNE_CACHE=str(cache))
    env.pop("SG_TUNE", None)
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert all(t[2] == 1 for t in outs[0]) or all(t[2] == 2 for t in outs[0])
    assert all(t[2] == 2 for t in outs[1]), outs[1]
    assert [t[:2] for t in outs[1]] == [t[:2] for t in outs[0]]


def test_tune_off_and_malformed_cache(tmp_path, monkeypatch):
    sg = _sg()
    cache = tmp_path / "bad.json"
    cache.write_text('{"sg_tune_cache": 1,\n "variants": {\n  "no slash": [1, 1, 1],\n  garbage line\n'
                     '  "x/y": [1, 2\n },\n "tiles": {\n  "a/b/c": [9999, 1, 1]\n }\n}\n')
    monkeypatch.setenv("SG_TUNE_CACHE", str(cache))
    grids = [(256, 128, -1.0, 1.0, -0.5, 0.5, 3)]
    sigma = _sigma(grids)
    monkeypatch.setenv("SG_TUNE", "off")
    p = sg.Plan(grids, sg.SG_FP32_SPLIT, flags=sg.SG_FLAG_AUTOTUNE)
    try:
        (var, tiles, src), = _tuning(sg, p)
        f0 = _forces(p, sigma)
    finally:
        p.close()
    assert src == 0 and tiles == (0, 0, 0) and var == (0, 0, 0)
    monkeypatch.setenv("SG_TUNE", "quick")
    p = sg.Plan(grids, sg.SG_FP32_SPLIT)
    try:
        (var_q, tiles_q, src_q), = _tuning(sg, p)
        fq = _forces(p, sigma)
    finally:
        p.close()
    # quick: tiles timed, variants left at their defaults; the same results
    assert src_q == 1 and var_q == (0, 0, 0) and all(t >= 1 for t in tiles_q)
    assert np.array_equal(fq[0], f0[0]) and np.array_equal(fq[1], f0[1])


def test_log_and_roctx_ranges():
    """SG_LOG prints each plan's launch choices and each error to stderr;
    SG_ROCTX marks the entry points with roctx ranges (run here without a
    profiler attached: the calls must succeed and change nothing)."""
    script = (
        "import sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import torch\n"
        "import paper_1904_07400_amd as sg\n"
        "p = sg.Plan([(256, 128, -1.0, 1.0, -0.5, 0.5, 3), (2048, 2048, -1.0, 1.0, -1.0, 1.0, 1)], sg.SG_FP32_SPLIT)\n"
        "s = torch.zeros(p.total, device='cuda')\n"
        "fx, fy = p.forces(s)\n"
        "g = torch.empty_like(s)\n"
        "p.adjoint(fx, fy, g)\n"
        "torch.cuda.synchronize()\n"
        "print('zero forces', float(fx.abs().max()), float(g.abs().max()))\n"
        "try:\n"
        "    sg.Plan([(100, 64, -1.0, 1.0, -1.0, 1.0, 3)], sg.SG_FP32_SPLIT)\n"
        "except sg.SGError as e:\n"
        "    print('refused', e.status)\n"
        "p.close()\n")
    env = dict(os.environ, SG_LOG="1", SG_ROCTX="1")
    env.pop("SG_TUNE", None)
    env.pop("SG_TUNE_CACHE", None)
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "zero forces 0.0 0.0" in r.stdout and "refused 2" in r.stdout, r.stdout
    assert "sg: plan" in r.stderr and "2 grids, FP32-split" in r.stderr, r.stderr[-2000:]
    assert "256x128 k=3 grids=1: columns Stockham" in r.stderr, r.stderr[-2000:]
    assert "2048x2048 k=1 grids=1: columns four-step" in r.stderr and "spectra 4 B per bin" in r.stderr
    assert "sg: error 2:" in r.stderr, r.stderr[-2000:]
