"""Build and load the oracle's C part (``csrc/sg_oracle.c``) with gcc/OpenMP.

Test infrastructure only: see ``oracle/__init__.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "sg_oracle.c")
_LIB = os.path.join(_HERE, "csrc", "libsg_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C code into ``oracle/csrc/libsg_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            ip32 = ctypes.POINTER(ctypes.c_int32)
            ip64 = ctypes.POINTER(ctypes.c_int64)
            L.oracle_weights_at.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int64, ip32, ip32, dp, dp]
            L.oracle_weights_full.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, dp, dp]
            L.oracle_forces.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, ctypes.c_int64,
                                        ip64, dp, dp]
            L.oracle_forces_sparse.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int, ctypes.c_int64, ip32, ip32, dp,
                                               ctypes.c_int64, ip64, dp, dp]
            L.oracle_forces_transpose.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp]
            L.oracle_bspline.argtypes = [ctypes.c_int, dp, ctypes.c_double]
            L.oracle_bspline.restype = ctypes.c_double
            for f in ("oracle_weights_at", "oracle_weights_full", "oracle_forces",
                      "oracle_forces_sparse", "oracle_forces_transpose"):
                getattr(L, f).restype = ctypes.c_int
            _lib = L
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def i32ptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def i64ptr(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
