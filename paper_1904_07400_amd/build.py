"""Compile the HIP library (libsg.so) for gfx950, in-tree.

Sources: csrc/sg_kernels.hip (device kernels + launch dispatch, compiled as
four objects in parallel), csrc/sg_colfs.hip (the four-step column pass of
the long columns) and csrc/sg_api.cpp (the C ABI of include/sg.h).
Every call recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC, "--offload-arch=gfx950",
          # no packed FP32 instructions in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]
# (source, extra flags, object name): the kernel file is compiled in four
# parts (SG_PART, a bit mask of the parts) in parallel
UNITS = [("sg_kernels.hip", ["-DSG_PART=%d" % (1 << i)], "sg_kernels_p%d.o" % i) for i in range(4)] + \
        [("sg_colfs.hip", [], "sg_colfs.o"), ("sg_api.cpp", [], "sg_api.o")]


def _compile(unit, obj_dir: str) -> str:
    src, extra, name = unit
    obj = os.path.join(obj_dir, name)
    cmd = [HIPCC, *COMMON, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + src)
    return obj


# Largest per-lane private (scratch) segment a kernel may have.  Every
# dispatch on MI355X gets a 1024 B/lane scratch allocation up front; the two
# builds whose kernels needed more (register spills of 1.6 and 2.2 KB/lane)
# faulted the device, while every kernel at or below 656 B/lane has run
# cleanly, so the build refuses anything above that.
SCRATCH_LIMIT = 656


def kernel_resources(obj: str):
    """(name, scratch B/lane, LDS B, max workgroup size, VGPRs, AGPRs) of every
    gfx950 kernel in a compiled object, read from its code-object metadata."""
    llvm = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin")
    if not os.path.isdir(llvm):
        llvm = "/opt/rocm/llvm/bin"
    tmp = obj + ".meta"
    fat, elf = tmp + ".fatbin", tmp + ".elf"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", obj, fat], check=True)
    subprocess.run([os.path.join(llvm, "clang-offload-bundler"), "--type=o",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + fat, "--output=" + elf,
                    "--unbundle"], check=True)
    notes = subprocess.run([os.path.join(llvm, "llvm-readelf"), "--notes", elf], check=True,
                           capture_output=True, text=True).stdout
    for f in (fat, elf):
        os.remove(f)
    out, cur = [], {}
    keys = ("agpr_count", "group_segment_fixed_size", "max_flat_workgroup_size", "name",
            "private_segment_fixed_size", "vgpr_count")
    for line in notes.splitlines():
        t = line.strip()
        if not t.startswith(".") or ":" not in t:
            continue
        k, v = t[1:].split(":", 1)
        if k in keys:
            cur[k] = v.strip()
            if k == "vgpr_count":  # last key of each kernel record
                out.append((cur.get("name", "?"), int(cur.get("private_segment_fixed_size", 0)),
                            int(cur.get("group_segment_fixed_size", 0)),
                            int(cur.get("max_flat_workgroup_size", 0)), int(cur["vgpr_count"]),
                            int(cur.get("agpr_count", 0))))
                cur = {}
    return out


def check_resources(obj: str) -> None:
    res = kernel_resources(obj)
    if not res:
        raise RuntimeError("no kernel metadata found in " + obj)
    bad = [r for r in res if r[1] > SCRATCH_LIMIT]
    if bad:
        lines = "\n".join(f"  {r[0]}: {r[1]} B/lane" for r in bad)
        raise RuntimeError(f"kernels above the {SCRATCH_LIMIT} B/lane scratch limit:\n{lines}")


def build_id() -> str:
    """Hash of the library sources and compile flags: the build tag of the
    tuning store's entries (a rebuilt library with other kernels ignores
    entries of the old one)."""
    import hashlib
    h = hashlib.sha256(" ".join(COMMON).encode())
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp", ".h", ".cpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + f.read())
    with open(os.path.join(INCLUDE, "sg.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:12]


def build(verbose: bool = False) -> str:
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    bid = build_id()
    units = [(src, extra + (['-DSG_BUILD_ID="%s"' % bid] if src == "sg_api.cpp" else []), name)
             for src, extra, name in UNITS]
    with ThreadPoolExecutor(max_workers=len(units)) as ex:
        objs = list(ex.map(lambda u: _compile(u, obj_dir), units))
    for o, u in zip(objs, units):
        if u[0].endswith(".hip"):
            check_resources(o)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libsg.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
