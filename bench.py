#!/usr/bin/env python3
"""Benchmark: thin-disk self-gravity forces (Fx + Fy), order k = 3, on one MI355X.

One step = the whole per-step path of the method for one surface density
sigma already resident in HBM: coefficient solve (Sec. 2.3), one forward and
two inverse zero-padded FFT convolutions with the kernel-weight spectra
(Sec. 4.2), Fx and Fy written at every cell centre.  Plan time (weights and
their spectra, done once per the end of Sec. 2.2) is outside the timed region
and reported separately.

Workload (default): 4096 x 4096 cells on [-1,1]^2, k = 3, sigma = 32 seeded
Gaussian clumps times a taper (``workloads``).  ``value`` is the FP32-split
path's cells/s; the FP64 path is timed on the same input and the FP32-split
error against it (max over cells and components, scaled by max|F|) is
reported.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# bytes per spectrum bin and component in FP32-split plans of the headline
# size (single floats; SG_FLAG_SPECTRA_SPLIT keeps float hi + lo pairs)
TABLE_BYTES_FP32 = 4


def bytes_per_cell(prec_fp64: bool, table_bytes=None):
    """Algorithmic HBM bytes per output cell, per pass (A, B, C).

    A: read sigma, write the row spectra X (one complex per cell).
    B: read X, read the weight spectra, write V (two complex per cell).
    C: read V, write Fx and Fy.
    The spectra: one real per (p, q) bin for each of the two components,
    ``table_bytes`` each (a double; a float; or a float hi + lo pair).  The
    model of the path's byte budget takes 8 bytes per bin for both components
    together (FP32: one float each; FP64: the budget of one double table)."""
    r = 8 if prec_fp64 else 4          # real
    c = 2 * r                          # complex
    sw = 8 if table_bytes is None else 2 * table_bytes
    return {"A": r + c, "B": c + sw + 2 * c, "C": 2 * c + 2 * r}


def time_plan(sg, torch, grid, prec, sigma_np, steps, warmup, flags=0):
    plan_t0 = time.perf_counter()
    plan = sg.Plan([grid], prec, flags=flags)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - plan_t0
    sigma = torch.as_tensor(sigma_np.ravel(), dtype=plan.dtype, device="cuda")
    fx, fy = plan.empty(), plan.empty()
    for _ in range(warmup):
        plan.forces(sigma, fx, fy)
    torch.cuda.synchronize()
    sg.sg_plan_set_timing(plan.handle, True)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        plan.forces(sigma, fx, fy)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    pass_ms, calls = sg.sg_plan_pass_times(plan.handle)
    sg.sg_plan_set_timing(plan.handle, False)
    out = (fx.double().cpu().numpy(), fy.double().cpu().numpy())
    plan.close()
    return ms, [p / calls for p in pass_ms], plan_s, out


KERNEL_SOURCES = ["paper_1904_07400_amd/csrc/sg_kernels.hip", "paper_1904_07400_amd/csrc/sg_colfs.hip",
                  "paper_1904_07400_amd/csrc/fft.hpp", "paper_1904_07400_amd/csrc/fft4.hpp",
                  "paper_1904_07400_amd/csrc/colfs.hpp", "paper_1904_07400_amd/csrc/colfs3.hpp",
                  "paper_1904_07400_amd/csrc/kcommon.hpp",
                  "paper_1904_07400_amd/csrc/tridiag.hpp", "paper_1904_07400_amd/csrc/sg_internal.h",
                  "paper_1904_07400_amd/build.py"]
# per-step kernels of the three passes (pass B: the four-step column kernel
# for columns of 2048, 4096 and 8192, its radix-3 form for 1536, the
# Stockham kernel otherwise)
PASS_KERNELS = r"k_(row_fwd|colfs3|colfs|col|row_inv)<"
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "forces_4096_k3_fp32_traffic.md")


def kernel_source_hash():
    """SHA-256 of the kernel sources and build flags (ties a counter profile to a build)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def calibration_copy(torch, mib):
    """A plain device copy of known size (torch.neg: reads and writes mib MiB),
    the reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b


def pmc_summary(fetch_csv, write_csv, mib, cells):
    """Per-kernel HBM bytes from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch), each scaled so that the calibration copy
    (the torch.neg kernel of ``mib`` MiB) reads and writes exactly its size."""
    import csv
    import re
    known = mib * (1 << 20)

    def load(path, counter):
        per = {}
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] != counter:
                continue
            name = row["Kernel_Name"]
            per.setdefault(name, []).append(float(row["Counter_Value"]) * 1024.0)
        return per

    fetch, write = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    cal = [k for k in fetch if "neg" in k.lower()]
    if not cal:
        raise SystemExit("calibration copy (torch.neg) not found in " + fetch_csv)
    f_scale = known / max(fetch[cal[0]])
    w_scale = known / max(write[cal[0]])
    rows = []
    for name in fetch:
        if not re.search(PASS_KERNELS, name) or name not in write:
            continue
        f = sum(fetch[name]) / len(fetch[name]) * f_scale
        w = sum(write[name]) / len(write[name]) * w_scale
        short = re.sub(r"\(.*", "", name).replace("sg::", "").replace("void ", "")
        rows.append((short, len(fetch[name]), f, w, (f + w) / cells))
    return f_scale, w_scale, rows


def sq_summary(csvs):
    """Per-kernel averages (per dispatch) of the instruction counters of one
    or more rocprofv3 --pmc runs, for the per-step kernels."""
    import csv
    import re
    per = {}
    for path in csvs:
        for row in csv.DictReader(open(path)):
            name = row["Kernel_Name"]
            if not re.search(PASS_KERNELS, name):
                continue
            per.setdefault(name, {}).setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    names = sorted({c for d in per.values() for c in d})
    out = ["| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    for name, d in per.items():
        short = re.sub(r"HIP_vector_type<(\w+), (\d)u>", r"\1\2", name).replace("sg::", "").replace("void ", "")
        short = re.sub(r"\(.*", "", short)
        vals = [f"{sum(d[c]) / len(d[c]):.4g}" if c in d else "" for c in names]
        out.append(f"| `{short}` | " + " | ".join(vals) + " |")
    return "\n".join(out)


def trace_summary(stats_csv, trace_csv):
    """Markdown table of a rocprofv3 kernel-trace run: durations from the
    stats file, launch shape and LDS from the trace file."""
    import csv
    import re
    shape = {r["Kernel_Name"]: r for r in csv.DictReader(open(trace_csv))}
    out = ["| kernel | calls | avg us | min us | max us | % of GPU time | workgroup | grid (threads) | LDS B |",
           "|---|---|---|---|---|---|---|---|---|"]
    for r in csv.DictReader(open(stats_csv)):
        if float(r["Percentage"]) < 0.05:
            continue
        m = shape.get(r["Name"], {})
        nm = re.sub(r"HIP_vector_type<(\w+), (\d)u>", r"\1\2", r["Name"]).replace("sg::", "").replace("void ", "")
        nm = re.sub(r"\(.*", "", nm)
        if nm.startswith("at::native"):
            nm = "at::native (PyTorch)"
        out.append(f"| `{nm}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} | {m.get('Workgroup_Size_X', '')} | "
                   f"{m.get('Grid_Size_X', '')} | {m.get('LDS_Block_Size', '')} |")
    return "\n".join(out)


def batch_trace_summary(trace_csv, per_step):
    """Per-step spans and per-length kernel time of a rocprofv3 kernel trace of
    `bench.py --batch-only`: of the FP32 per-step kernels, the graph replays
    are the launches on streams other than the plan's, the eager steps the
    first as many launches on the plan's stream after them; per_step =
    launches per step (three per class)."""
    import csv
    import re
    step_kernel = re.compile(r"sg::k_(row_fwd|row_inv|col|colfs|colfs3)<float")
    rows = sorted((r for r in csv.DictReader(open(trace_csv)) if step_kernel.search(r["Kernel_Name"])),
                  key=lambda r: int(r["Start_Timestamp"]))
    home = rows[0]["Stream_Id"]
    graph = [r for r in rows if r["Stream_Id"] != home]
    last = max(int(r["Start_Timestamp"]) for r in graph)
    eager = [r for r in rows if r["Stream_Id"] == home and int(r["Start_Timestamp"]) > last][:len(graph)]

    def steps(rs):
        return [rs[i:i + per_step] for i in range(0, len(rs) - per_step + 1, per_step)]

    def span(st):
        return (max(int(r["End_Timestamp"]) for r in st) - min(int(r["Start_Timestamp"]) for r in st)) / 1e6

    def kind(name):
        nm = re.sub(r"HIP_vector_type<(\w+), (\d)u>", r"\1\2", name)
        m = re.search(r"sg::(k_\w+)<([^>]*)>", nm)
        k, args = m.group(1), [a.strip() for a in m.group(2).split(",")]
        if k == "k_row_fwd":
            return "A", int(args[2]), k
        if k == "k_row_inv":
            return "C", int(args[2]), k
        if k == "k_colfs3":
            return "B", 3 * int(args[-1]), k
        return "B", int(args[2]), k

    gs, es = steps(graph), steps(eager)
    out = ["- graph: " + str([round(span(s), 3) for s in gs]),
           "- eager: " + str([round(span(s), 3) for s in es]), ""]
    timed = es[2:] if len(es) > 2 else es
    tab, bk = {}, {}
    for st in timed:
        for r in st:
            ps, n, k = kind(r["Kernel_Name"])
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 / len(timed)
            tab.setdefault(n, {"A": 0.0, "B": 0.0, "C": 0.0})[ps] += us
            if ps == "B":
                bk[n] = k
    out += ["| length | pass A | pass B | pass C | sum | pass B kernel |", "|---|---|---|---|---|---|"]
    tot = {"A": 0.0, "B": 0.0, "C": 0.0}
    for n in sorted(tab):
        t = tab[n]
        for ps in tot:
            tot[ps] += t[ps]
        out.append(f"| {n} | {t['A']:.0f} | {t['B']:.0f} | {t['C']:.0f} | {sum(t.values()):.0f} | `{bk.get(n, '')}` |")
    out.append(f"| all | {tot['A']:.0f} | {tot['B']:.0f} | {tot['C']:.0f} | {sum(tot.values()):.0f} | |")
    return "\n".join(out)


def measured_traffic(kname, n):
    """HBM bytes per launch of the FP32 kernel from the committed counter
    profile, or None if there is none for this size or the kernels changed
    since it was taken."""
    import re
    if n != 4096 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    m = re.search(r"source hash: (\w+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    for line in text.splitlines():
        if line.startswith("| `" + kname + "<float"):
            cols = [c.strip() for c in line.strip("|").split("|")]
            return round((float(cols[2]) + float(cols[3])) * 1e6)
    return None


def batch_bench(sg, torch, steps, warmup, count=256):
    """Batched disks: ``count`` seeded square grids of mixed sizes (2^a and
    3*2^a, 96..2048) and orders on [-1,1]^2, FP32-split.  Times one step of
    (a) one plan with SG_FLAG_GRAPH | SG_FLAG_AUTOTUNE, (b) the same plan
    without graph or tuning, (c) a host loop of single-grid plans, and checks
    that all three give bit-identical forces."""
    import workloads
    disks = workloads.batch_disks(4, count)
    grids = [(n, n, -1.0, 1.0, -1.0, 1.0, k) for n, k, _ in disks]
    prec = sg.SG_FP32_SPLIT
    t0 = time.perf_counter()
    pg = sg.Plan(grids, prec, flags=sg.SG_FLAG_GRAPH | sg.SG_FLAG_AUTOTUNE)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    sigma = torch.empty(pg.total, dtype=torch.float32, device="cuda")
    for gi, (n, k, params) in enumerate(disks):
        xs, ys = pg.sample_points(gi)
        sigma[pg.offsets[gi]:pg.offsets[gi + 1]] = workloads.clump_sigma_torch(params, xs, ys).ravel().float()
    cells = pg.total

    def timed(step):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    gx, gy = pg.empty(), pg.empty()
    ms_graph = timed(lambda: sg.sg_forces(pg.handle, sigma, gx, gy))
    classes = sg.sg_plan_classes(pg.handle)
    pb = sg.Plan(grids, prec)
    bx, by = pb.empty(), pb.empty()
    ms_batch = timed(lambda: sg.sg_forces(pb.handle, sigma, bx, by))
    singles = [sg.Plan([g], prec) for g in grids]
    lx, ly = pg.empty(), pg.empty()
    views = [(sigma[pg.offsets[i]:pg.offsets[i + 1]], lx[pg.offsets[i]:pg.offsets[i + 1]],
              ly[pg.offsets[i]:pg.offsets[i + 1]]) for i in range(len(grids))]

    def loop():
        for p, (s_, x_, y_) in zip(singles, views):
            sg.sg_forces(p.handle, s_, x_, y_)

    ms_loop = timed(loop)
    same = bool(torch.equal(gx, bx) and torch.equal(gy, by) and torch.equal(gx, lx) and torch.equal(gy, ly))
    # FP32-split error against the FP64 path, per grid (max|dF| / max|F|), worst grid
    p64 = sg.Plan(grids, sg.SG_FP64)
    hx, hy = p64.forces(sigma.double())
    torch.cuda.synchronize()
    err = 0.0
    for i in range(len(grids)):
        a, b = pg.offsets[i], pg.offsets[i + 1]
        scale = max(hx[a:b].abs().max().item(), hy[a:b].abs().max().item())
        dev = max((gx[a:b].double() - hx[a:b]).abs().max().item(), (gy[a:b].double() - hy[a:b]).abs().max().item())
        err = max(err, dev / scale)
    p64.close()
    for p in singles:
        p.close()
    pb.close()
    pg.close()
    return {"workload": f"{count} disks on [-1,1]^2, n ~ U{{96,128,192,256,384,512,768,1024,1536,2048}}, "
                        "k ~ U{1,2,3}, 4-64 seeded clumps each (seed 4), FP32-split",
            "cells": cells, "classes": len(classes), "steps": steps,
            "value": cells / (ms_graph * 1e-3), "unit": "cells/s", "ms_per_step": round(ms_graph, 4),
            "batched_no_graph": {"value": cells / (ms_batch * 1e-3), "ms_per_step": round(ms_batch, 4)},
            "loop_of_single_plans": {"value": cells / (ms_loop * 1e-3), "ms_per_step": round(ms_loop, 4)},
            "speedup_vs_loop": round(ms_loop / ms_graph, 3), "plan_s": round(plan_s, 3),
            "bit_identical": same, "rel_err_vs_fp64_worst_grid": err}


def aniso_bench(sg, torch, k, steps, warmup):
    """Non-square cells on a rectangular domain: 4096 x 2048 cells on
    [-2,2] x [-0.5,0.5] (dx = 2 dy), the same clump recipe, FP32-split timed
    and checked against FP64."""
    import numpy as np
    import workloads
    M, N = 4096, 2048
    grid = (M, N, -2.0, 2.0, -0.5, 0.5, k)
    hx, hy = 4.0 / M, 1.0 / N
    off = 0.5 if k % 2 == 1 else 1.0  # cell centres (odd k) or vertices x0 + (i+1) dx (k = 2)
    xs = -2.0 + hx * (off + np.arange(M))
    ys = -0.5 + hy * (off + np.arange(N))
    sigma = workloads.clump_sigma(workloads.clump_params(2, 32), xs, ys)
    ms64, _, _, (gx, gy) = time_plan(sg, torch, grid, sg.SG_FP64, sigma, steps, warmup)
    ms32, pass32, _, (fx, fy) = time_plan(sg, torch, grid, sg.SG_FP32_SPLIT, sigma, steps, warmup)
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    err = max(np.abs(fx - gx).max(), np.abs(fy - gy).max()) / scale
    return {"workload": f"{M}x{N} cells on [-2,2]x[-0.5,0.5] (dx = 2 dy), k={k}, 32 seeded clumps x taper",
            "value": M * N / (ms32 * 1e-3), "unit": "cells/s", "ms_per_step": round(ms32, 4),
            "pass_ms": [round(x, 4) for x in pass32], "fp64_ms_per_step": round(ms64, 4),
            "rel_err_vs_fp64": err, "meets_1e-6": bool(err <= 1e-6)}


def grad_bench(sg, torch, steps, warmup, big=8192):
    """Differentiation at scale: one plan of a big^2 grid with four 2048^2
    grids alongside, k = 3, 64 seeded clumps per grid.  A step is the forward
    forces, the loss residual 2 (F - F_t) and the adjoint (dL/dsigma for
    L = sum |F - F_t|^2, F_t from perturbed clumps).  FP32-split timed; its
    gradient checked against the FP64 plan's per grid."""
    import workloads
    grids = [(big, big, -1.0, 1.0, -1.0, 1.0, 3)] + [(2048, 2048, -1.0, 1.0, -1.0, 1.0, 3)] * 4
    out = {"workload": f"{big}^2 + 4 x 2048^2 in one plan, k=3, 64 seeded clumps each; forward + adjoint of "
                       "L = sum |F - F_t|^2 (F_t from perturbed clumps)"}
    grads = {}
    for prec in (sg.SG_FP64, sg.SG_FP32_SPLIT):
        plan = sg.Plan(grids, prec)
        try:
            sig = torch.empty(plan.total, dtype=plan.dtype, device="cuda")
            tsig = torch.empty_like(sig)
            for gi in range(len(grids)):
                xs, ys = plan.sample_points(gi)
                params = workloads.clump_params(5 + gi, 64)
                a, b = plan.offsets[gi], plan.offsets[gi + 1]
                sig[a:b] = workloads.clump_sigma_torch(params, xs, ys).ravel().to(plan.dtype)
                tsig[a:b] = workloads.clump_sigma_torch(workloads.perturb_clumps(params, 55), xs, ys).ravel().to(
                    plan.dtype)
            tx, ty = (t.clone() for t in plan.forces(tsig))
            fx, fy, g = plan.empty(), plan.empty(), plan.empty()

            def step():
                plan.forces(sig, fx, fy)
                plan.adjoint(2 * (fx - tx), 2 * (fy - ty), g)

            def timed(fn):
                for _ in range(warmup):
                    fn()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(steps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / steps

            ms = timed(step)
            grads[prec] = g.double().cpu().numpy()
            # the two halves alone: the forward pass, and the adjoint of fixed residuals
            rx, ry = 2 * (fx - tx), 2 * (fy - ty)
            ms_fwd = timed(lambda: plan.forces(sig, fx, fy))
            ms_adj = timed(lambda: plan.adjoint(rx, ry, g))
            pre = "fp64_" if prec == sg.SG_FP64 else ""
            out[pre + "ms_per_step"] = round(ms, 4)
            out[pre + "forward_ms"] = round(ms_fwd, 4)
            out[pre + "adjoint_ms"] = round(ms_adj, 4)
            if prec == sg.SG_FP32_SPLIT:
                out["value"] = plan.total / (ms * 1e-3)
                out["unit"] = "cells/s (forward + adjoint)"
                offs = plan.offsets
        finally:
            plan.close()
    g64, g32 = grads[sg.SG_FP64], grads[sg.SG_FP32_SPLIT]
    out["rel_err_vs_fp64_per_grid"] = [
        float(abs(g32[offs[i]:offs[i + 1]] - g64[offs[i]:offs[i + 1]]).max() / abs(g64[offs[i]:offs[i + 1]]).max())
        for i in range(len(grids))]
    return out


def orders_bench(sg, torch, n, steps, warmup):
    """The cubic and quartic splines (k = 4, 5) on the headline grid: n x n
    cells on [-1,1]^2, the same clump recipe, FP32-split timed and checked
    against FP64."""
    import numpy as np
    import workloads
    out = {}
    h = 2.0 / n
    for k in (4, 5):
        grid = (n, n, -1.0, 1.0, -1.0, 1.0, k)
        off = 0.5 if k % 2 == 1 else 1.0  # cell centres (odd k) or vertices x0 + (i+1) dx (even k)
        xs = -1.0 + h * (off + np.arange(n))
        sigma = workloads.clump_sigma(workloads.clump_params(2, 32), xs, xs)
        ms64, pass64, _, (gx, gy) = time_plan(sg, torch, grid, sg.SG_FP64, sigma, steps, warmup)
        ms32, pass32, plan32, (fx, fy) = time_plan(sg, torch, grid, sg.SG_FP32_SPLIT, sigma, steps, warmup)
        scale = max(np.abs(gx).max(), np.abs(gy).max())
        err = max(np.abs(fx - gx).max(), np.abs(fy - gy).max()) / scale
        out[f"k{k}"] = {"value": n * n / (ms32 * 1e-3), "unit": "cells/s", "ms_per_step": round(ms32, 4),
                        "pass_ms": [round(x, 4) for x in pass32], "plan_s": round(plan32, 3),
                        "fp64_ms_per_step": round(ms64, 4), "fp64_pass_ms": [round(x, 4) for x in pass64],
                        "rel_err_vs_fp64": err, "meets_1e-6": bool(err <= 1e-6)}
    return out


def cpu_baseline(n, k, sigma_np, sample):
    """The oracle (direct O(N^4) FP64 sum, OpenMP) on a bounded sample of cells."""
    import numpy as np
    import oracle
    import workloads
    h = 2.0 / n
    t0 = time.perf_counter()
    C = oracle.bspline_coeffs(sigma_np, k)
    t_solve = time.perf_counter() - t0
    t0 = time.perf_counter()
    wx, wy = oracle.weights(k, n, n, h, h)
    t_tab = time.perf_counter() - t0
    cells = workloads.sample_cells(7, n, n, sample)
    t0 = time.perf_counter()
    oracle.forces_from_coeffs(C, wx, wy, cells)
    t_sum = time.perf_counter() - t0
    # per-cell cost of a step: the full coefficient solve spread over all cells
    per_cell = t_sum / cells.size + t_solve / (n * n)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / per_cell, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": (f"{cells.size} of {n}x{n} cells (seeded), direct FP64 sum with the full weight table; "
                       f"coefficient solve on the full grid {t_solve:.2f} s (apportioned per cell); "
                       f"weight-table build {t_tab:.1f} s excluded, like GPU plan time"),
            "host_cpu": _cpu_model()}


def cpu_fft_reference(sg, torch, n, k, sigma_np, ref_fx, ref_fy):
    """CPU FFT reference (not the oracle): the same forces by FP64
    zero-padded FFT convolution with scipy.fft on all host cores.  The
    weights come from the library (sg_weights, FP64) and are transformed once
    (excluded, like plan time); the timed part is the coefficient solve (banded
    solves along both axes), one forward real 2-D FFT, the two spectral
    products and the two inverse real 2-D FFTs, cropped.  k = 1, 2, 3."""
    import numpy as np
    import scipy.fft
    import scipy.linalg
    if k not in (1, 2, 3):
        return None
    workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    plan = sg.Plan([(n, n, -1.0, 1.0, -1.0, 1.0, k)], sg.SG_FP64)
    try:
        wx, wy = (w.cpu().numpy() for w in plan.weights(0))
    finally:
        plan.close()
    P = 2 * n

    def padded(w):
        # w(m, n') at (m mod 2n, n' mod 2n); the slots m = n, n' = n stay 0 (odd k)
        out = np.zeros((P, P))
        idx = np.arange(-(n - 1), n) % P
        out[np.ix_(idx, idx)] = w
        return out

    Wx = scipy.fft.rfft2(padded(wx), workers=workers)
    Wy = scipy.fft.rfft2(padded(wy), workers=workers)
    ab = np.array([[1.0], [6.0], [1.0]]) * np.ones((3, n)) / 8.0  # tridiag(1,6,1)/8, Eqs. (z_system), (C_system)
    sig = np.asarray(sigma_np, dtype=np.float64)
    t0 = time.perf_counter()
    C = sig
    if k == 3:
        C = scipy.linalg.solve_banded((1, 1), ab, C.T).T       # along x (rows)
        C = scipy.linalg.solve_banded((1, 1), ab, C)           # along y (columns)
    Ch = scipy.fft.rfft2(C, s=(P, P), workers=workers)
    fx = scipy.fft.irfft2(Ch * Wx, s=(P, P), workers=workers)[:n, :n]
    fy = scipy.fft.irfft2(Ch * Wy, s=(P, P), workers=workers)[:n, :n]
    dt = time.perf_counter() - t0
    scale = max(np.abs(ref_fx).max(), np.abs(ref_fy).max())
    diff = max(np.abs(fx - ref_fx).max(), np.abs(fy - ref_fy).max()) / scale
    return {"value": n * n / dt, "unit": "cells/s", "cores": workers, "kind": "CPU FFT reference (not the oracle)",
            "seconds": round(dt, 3), "library": f"scipy.fft {scipy.__version__} (pocketfft), FP64",
            "rel_diff_vs_gpu_fp64": float(diff)}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-disks measurement")
    ap.add_argument("--batch-only", action="store_true", help="only the batched-disks measurement")
    ap.add_argument("--no-aniso", action="store_true", help="skip the anisotropic-cell measurement")
    ap.add_argument("--no-orders", action="store_true", help="skip the k = 4, 5 measurement")
    ap.add_argument("--no-grad", action="store_true", help="skip the forward + adjoint measurement")
    ap.add_argument("--prec", choices=["both", "fp32", "fp64"], default="both",
                    help="both (default, the metric) or one path only (profiling)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print per-kernel HBM traffic from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--trace-summary", nargs=2, metavar=("STATS_CSV", "TRACE_CSV"),
                    help="print a table of a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--batch-trace-summary", nargs=2, metavar=("TRACE_CSV", "LAUNCHES_PER_STEP"),
                    help="per-step spans and per-length kernel time of a --batch-only kernel trace")
    ap.add_argument("--sq-summary", nargs="+", metavar="PMC_CSV",
                    help="print per-kernel instruction counters of rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.trace_summary:
        print(trace_summary(*args.trace_summary))
        return
    if args.batch_trace_summary:
        print(batch_trace_summary(args.batch_trace_summary[0], int(args.batch_trace_summary[1])))
        return
    if args.sq_summary:
        print(f"source hash: {kernel_source_hash()}")
        print(sq_summary(args.sq_summary))
        return
    if args.pmc_summary:
        mib = args.copy_calibration_mib or 256
        fs, ws, rows = pmc_summary(*args.pmc_summary, mib, args.n * args.n)
        print(f"source hash: {kernel_source_hash()}")
        print(f"calibration: torch.neg copy of {mib} MiB; FETCH scale {fs:.4f}, WRITE scale {ws:.4f}")
        print("| kernel | dispatches | read MB/launch | written MB/launch | bytes/cell |")
        print("|---|---|---|---|---|")
        for name, nd, f, w, bpc in rows:
            print(f"| `{name}` | {nd} | {f / 1e6:.1f} | {w / 1e6:.1f} | {bpc:.1f} |")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the multi-GPU "
              "decomposition of this method is designed but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1904_07400_amd as sg
    import workloads

    n, k = args.n, args.k
    grid = (n, n, -1.0, 1.0, -1.0, 1.0, k)
    # sample lattice of the plan (cell centres for odd k)
    probe = sg.Plan([(8, 8, -1.0, 1.0, -1.0, 1.0, k)], sg.SG_FP64)
    xs0, ys0, _, _ = sg.sg_sample_points(probe.handle, 0)
    probe.close()
    h = 2.0 / n
    off = (xs0 + 1.0) / (2.0 / 8)  # 0.5 (centres) or 1.0 (vertices) in cell units
    xs = -1.0 + h * (off + np.arange(n))
    sigma = workloads.clump_sigma(workloads.clump_params(2, 32), xs, xs)

    if args.copy_calibration_mib:
        calibration_copy(torch, args.copy_calibration_mib)
    if args.batch_only:
        print(json.dumps(batch_bench(sg, torch, max(args.steps // 2, 3), 2)), flush=True)
        return
    if args.prec != "both":
        prec = sg.SG_FP32_SPLIT if args.prec == "fp32" else sg.SG_FP64
        ms, passes, plan_s, _ = time_plan(sg, torch, grid, prec, sigma, args.steps, args.warmup)
        print(json.dumps({"prec": args.prec, "ms_per_step": ms, "pass_ms": passes, "plan_s": plan_s}), flush=True)
        return
    ms64, pass64, plan64, (gx, gy) = time_plan(sg, torch, grid, sg.SG_FP64, sigma, args.steps, args.warmup)
    ms32, pass32, plan32, (fx, fy) = time_plan(sg, torch, grid, sg.SG_FP32_SPLIT, sigma, args.steps, args.warmup)
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    err32 = max(np.abs(fx - gx).max(), np.abs(fy - gy).max()) / scale
    # the same path with the spectra kept as hi + lo float pairs
    mss, passs, _, (sx, sy) = time_plan(sg, torch, grid, sg.SG_FP32_SPLIT, sigma, args.steps, args.warmup,
                                        flags=sg.SG_FLAG_SPECTRA_SPLIT)
    errs = max(np.abs(sx - gx).max(), np.abs(sy - gy).max()) / scale

    cells = n * n
    bpc = bytes_per_cell(False)                                 # the byte budget of the path
    bpc_impl = bytes_per_cell(False, TABLE_BYTES_FP32)          # what this build's tables hold
    dom = max(range(3), key=lambda i: pass32[i])
    name = "ABC"[dom]
    achieved = bpc[name] * cells / (pass32[dom] * 1e-3) / 1e9
    kname = {"A": "k_row_fwd", "B": "k_colfs" if n in (4096, 8192) else "k_col", "C": "k_row_inv"}[name]
    step_gbs = sum(bpc.values()) * cells / (ms32 * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": kname,
                "byte_model": "algorithmic (read X 8, weight spectra 4 + 4, write V 16 B/cell for pass B; "
                              "step 12 + 32 + 24 B/cell); traffic: FETCH_SIZE + WRITE_SIZE of the committed profile",
                "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(kname, n),
                "bytes_per_cell": bpc[name], "kernel_ms": round(pass32[dom], 4),
                "bytes_per_cell_impl": bpc_impl[name],
                "frac_impl": round(bpc_impl[name] * cells / (pass32[dom] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "step": {"bytes_per_cell": sum(bpc.values()), "achieved": round(step_gbs, 1),
                         "frac": round(step_gbs / PEAK_HBM_GBS, 4), "ms": round(ms32, 4)}}
    total_bytes = sum(bpc.values()) * cells
    line = {
        "metric": "force cells/s (Fx+Fy, 3rd order, 4096²): FP32-split vs FP64 at ≤1e-6 rel",
        "value": cells / (ms32 * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "precision_form": "FP32-split: f32 FFTs and products, f64 coefficient solve, f32 spectra "
                          "(the hi+lo spectra form is timed beside it: spectra_split)",
        "data": "synthetic",
        "config": {"workload": f"{n}x{n} cells on [-1,1]^2, k={k}, sigma = 32 seeded Gaussian clumps x taper "
                               f"(clump recipe of the 1024^2 precision case, at {n}^2)",
                   "grid": n, "order": k, "parallelism": "single GPU"},
        "fp64": {"value": cells / (ms64 * 1e-3), "ms_per_step": round(ms64, 4),
                 "pass_ms": [round(x, 4) for x in pass64], "plan_s": round(plan64, 3)},
        "fp32_split": {"pass_ms": [round(x, 4) for x in pass32], "plan_s": round(plan32, 3),
                       "rel_err_vs_fp64": err32, "meets_1e-6": bool(err32 <= 1e-6),
                       "step_gbs_algorithmic": round(total_bytes / (ms32 * 1e-3) / 1e9, 1)},
        "spectra_split": {"value": cells / (mss * 1e-3), "ms_per_step": round(mss, 4),
                          "pass_ms": [round(x, 4) for x in passs], "rel_err_vs_fp64": errs,
                          "meets_1e-6": bool(errs <= 1e-6)},
        "speedup_fp32split_vs_fp64": round(ms64 / ms32, 3),
        "roofline": roofline,
    }
    if not args.no_batch:
        line["batch"] = batch_bench(sg, torch, max(args.steps // 2, 3), 2)
    if not args.no_aniso:
        line["anisotropic"] = aniso_bench(sg, torch, k, max(args.steps // 2, 3), 2)
    if not args.no_orders:
        line["higher_orders"] = orders_bench(sg, torch, n, max(args.steps // 2, 3), 2)
    if not args.no_grad:
        line["differentiation"] = grad_bench(sg, torch, max(args.steps // 2, 3), 2)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n, k, sigma, args.cpu_sample)
        ref = cpu_fft_reference(sg, torch, n, k, sigma, gx.reshape(n, n), gy.reshape(n, n))
        if ref is not None:
            line["cpu_fft_reference"] = ref
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
