"""MI355X (gfx950) library for thin-disk self-gravity with order-k B-splines.

Thin ctypes binding over ``libsg.so`` (C ABI in ``include/sg.h``): the same
names as the C functions, argument marshalling only.  Every step of the
computation runs in the library's HIP kernels; PyTorch provides device
memory (tensors) and the HIP stream.  If the library is missing, every call
raises: there is no CPU fallback.

Method: Wang, Shiue, Wu & Yen, arXiv 1904.07400 — surface density sigma on a
uniform grid, order-k tensor B-spline interpolation (Sec. 2.3), forces at the
cell centres as discrete convolutions of the coefficients with the kernel
weights (Eqs. (eqnF), (eqnwB)), evaluated by zero-padded FFTs.
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = [
    "SG_FP64", "SG_FP32_SPLIT", "SG_FLAG_CHECK_FINITE", "SG_FLAG_GRAPH", "SG_FLAG_AUTOTUNE", "SG_FLAG_SPECTRA_SPLIT", "SGError",
    "sg_grid", "lib", "sg_plan_classes", "sg_plan_tuning",
    "sg_plan_create", "sg_plan_destroy", "sg_plan_layout", "sg_plan_info", "sg_sample_points",
    "sg_weights", "sg_bspline_coeffs", "sg_forces", "sg_forces_noalloc", "sg_forces_adjoint", "sg_status_string",
    "sg_last_error_message", "sg_plan_set_timing", "sg_plan_pass_times", "Plan", "ThinDiskForces",
]

SG_FP64 = 0
SG_FP32_SPLIT = 1
SG_FLAG_CHECK_FINITE = 0x1
SG_FLAG_GRAPH = 0x2
SG_FLAG_AUTOTUNE = 0x4
SG_FLAG_SPECTRA_SPLIT = 0x8
STATUS = {0: "SG_OK", 1: "SG_ERR_ARG", 2: "SG_ERR_UNSUPPORTED", 3: "SG_ERR_NOMEM",
          4: "SG_ERR_DEVICE", 5: "SG_ERR_STATE"}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsg.so")
_lock = threading.Lock()
_lib = None


class SGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class sg_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("order", ctypes.c_int32)]


def lib() -> ctypes.CDLL:
    """Load libsg.so (built by ``paper_1904_07400_amd.build``); raise if absent."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_1904_07400_amd.build` (no CPU fallback exists)")
            L = ctypes.CDLL(LIB_PATH)
            vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
            dp = ctypes.POINTER(ctypes.c_double)
            L.sg_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(sg_grid), i32, ctypes.c_int,
                                         vp, ctypes.c_uint32]
            L.sg_plan_destroy.argtypes = [vp]
            L.sg_plan_layout.argtypes = [vp, ctypes.POINTER(i64)]
            L.sg_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
            L.sg_sample_points.argtypes = [vp, i32, dp, dp, dp, dp]
            L.sg_weights.argtypes = [vp, i32, vp, vp]
            L.sg_bspline_coeffs.argtypes = [vp, vp, vp]
            L.sg_forces.argtypes = [vp, vp, vp, vp]
            L.sg_forces_adjoint.argtypes = [vp, vp, vp, vp]
            L.sg_forces_noalloc.argtypes = [vp, vp, vp, vp]
            L.sg_plan_set_timing.argtypes = [vp, i32]
            L.sg_plan_classes.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), i32]
            L.sg_plan_tuning.argtypes = [vp, i32, ctypes.POINTER(i32)]
            L.sg_plan_pass_times.argtypes = [vp, dp, ctypes.POINTER(i64)]
            L.sg_status_string.argtypes = [ctypes.c_int]
            L.sg_status_string.restype = ctypes.c_char_p
            L.sg_last_error_message.argtypes = []
            L.sg_last_error_message.restype = ctypes.c_char_p
            for f in ("sg_plan_create", "sg_plan_destroy", "sg_plan_layout", "sg_plan_info",
                      "sg_sample_points", "sg_weights", "sg_bspline_coeffs", "sg_forces", "sg_forces_noalloc",
                      "sg_forces_adjoint", "sg_plan_set_timing", "sg_plan_pass_times", "sg_plan_classes",
                      "sg_plan_tuning"):
                getattr(L, f).restype = ctypes.c_int
            _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise SGError(status, lib().sg_last_error_message().decode())


def _ptr(x):
    """Device address of a tensor (or an int address, or None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------ C-named wrappers --
def sg_status_string(status: int) -> str:
    return lib().sg_status_string(status).decode()


def sg_last_error_message() -> str:
    return lib().sg_last_error_message().decode()


def sg_plan_create(grids, prec: int = SG_FP64, stream=None, flags: int = 0) -> int:
    """grids: sequence of (nx, ny, x0, x1, y0, y1, order) or sg_grid."""
    arr = (sg_grid * len(grids))()
    for i, g in enumerate(grids):
        arr[i] = g if isinstance(g, sg_grid) else sg_grid(*g)
    h = ctypes.c_void_p()
    _check(lib().sg_plan_create(ctypes.byref(h), arr, len(grids), prec, _stream_handle(stream), flags))
    return h.value


def sg_plan_destroy(plan: int) -> None:
    _check(lib().sg_plan_destroy(plan))


def sg_plan_layout(plan: int, ngrids: int):
    offs = (ctypes.c_int64 * (ngrids + 1))()
    _check(lib().sg_plan_layout(plan, offs))
    return list(offs)


def sg_plan_info(plan: int):
    n, p, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().sg_plan_info(plan, ctypes.byref(n), ctypes.byref(p), ctypes.byref(b)))
    return n.value, p.value, b.value


def sg_plan_set_timing(plan: int, enable: bool) -> None:
    _check(lib().sg_plan_set_timing(plan, 1 if enable else 0))


def sg_plan_pass_times(plan: int):
    """(ms per pass summed since enabled [A, B, C], number of sg_forces calls)."""
    ms = (ctypes.c_double * 3)()
    calls = ctypes.c_int64()
    _check(lib().sg_plan_pass_times(plan, ms, ctypes.byref(calls)))
    return list(ms), calls.value


def sg_plan_classes(plan: int):
    """[(nx, ny, order, ngrids, tile_A, tile_B, tile_C), ...] of the plan's grid classes."""
    n = ctypes.c_int32()
    _check(lib().sg_plan_classes(plan, ctypes.byref(n), None, 0))
    info = (ctypes.c_int32 * (8 * max(n.value, 1)))()
    _check(lib().sg_plan_classes(plan, ctypes.byref(n), info, n.value))
    return [tuple(info[8 * i:8 * i + 7]) for i in range(n.value)]


def sg_plan_tuning(plan: int, cls: int):
    """(variants (A, B, C), tiles (A, B, C), source) of class cls: source 0 =
    defaults, 1 = timed at the plan's creation, 2 = from the tuning store."""
    out = (ctypes.c_int32 * 8)()
    _check(lib().sg_plan_tuning(plan, cls, out))
    return tuple(out[0:3]), tuple(out[3:6]), out[6]


def sg_sample_points(plan: int, g: int):
    v = [ctypes.c_double() for _ in range(4)]
    _check(lib().sg_sample_points(plan, g, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def sg_weights(plan: int, g: int, wx, wy) -> None:
    _check(lib().sg_weights(plan, g, _ptr(wx), _ptr(wy)))


def sg_bspline_coeffs(plan: int, sigma, coeffs) -> None:
    _check(lib().sg_bspline_coeffs(plan, _ptr(sigma), _ptr(coeffs)))


def sg_forces(plan: int, sigma, fx, fy) -> None:
    _check(lib().sg_forces(plan, _ptr(sigma), _ptr(fx), _ptr(fy)))


def sg_forces_noalloc(plan: int, sigma, fx, fy) -> None:
    _check(lib().sg_forces_noalloc(plan, _ptr(sigma), _ptr(fx), _ptr(fy)))


def sg_forces_adjoint(plan: int, gfx, gfy, gsigma) -> None:
    _check(lib().sg_forces_adjoint(plan, _ptr(gfx), _ptr(gfy), _ptr(gsigma)))


# ------------------------------------------------------------ Plan class --
class Plan:
    """A plan over one or more grids: ``Plan([(nx, ny, x0, x1, y0, y1, k), ...], prec)``.

    Arrays are torch tensors on the GPU, packed over the plan's grids
    (``offsets``); each grid row-major [ny][nx].  dtype float64 for SG_FP64,
    float32 for SG_FP32_SPLIT.
    """

    def __init__(self, grids, prec: int = SG_FP64, stream=None, flags: int = 0):
        import torch
        self.grids = [tuple(g) for g in grids]
        self.prec = prec
        self.dtype = torch.float64 if prec == SG_FP64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if isinstance(self.stream, int):
            self.stream = torch.cuda.ExternalStream(self.stream)
        self.handle = sg_plan_create(self.grids, prec, self.stream, flags)
        self.offsets = sg_plan_layout(self.handle, len(self.grids))

    def close(self):
        if getattr(self, "handle", None):
            sg_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def total(self) -> int:
        return self.offsets[-1]

    def empty(self):
        import torch
        return torch.empty(self.total, dtype=self.dtype, device=self.device)

    def view(self, buf, g: int):
        nx, ny = self.grids[g][0], self.grids[g][1]
        return buf[self.offsets[g]:self.offsets[g + 1]].view(ny, nx)

    def sample_points(self, g: int = 0):
        """(xs, ys) numpy arrays of the lattice where sigma of grid g is sampled."""
        import numpy as np
        xs0, ys0, dx, dy = sg_sample_points(self.handle, g)
        nx, ny = self.grids[g][0], self.grids[g][1]
        return xs0 + dx * np.arange(nx), ys0 + dy * np.arange(ny)

    # -- argument checks: every tensor handed to the kernels must be a
    # contiguous tensor of the plan's dtype on the plan's device holding
    # exactly the packed length (a short or mistyped buffer would be read or
    # written out of bounds by the kernels)
    def _check_tensor(self, name, t, numel=None, dtype=None):
        import torch
        dtype = self.dtype if dtype is None else dtype
        numel = self.total if numel is None else numel
        if not isinstance(t, torch.Tensor):
            raise SGError(1, f"{name}: expected a torch.Tensor, got {type(t).__name__}")
        if t.dtype != dtype:
            raise SGError(1, f"{name}: dtype {t.dtype}, the plan needs {dtype}")
        if t.device != self.device:
            raise SGError(1, f"{name}: on {t.device}, the plan is on {self.device}")
        if not t.is_contiguous():
            raise SGError(1, f"{name}: not contiguous")
        if t.numel() != numel:
            raise SGError(1, f"{name}: {t.numel()} elements, the plan needs {numel}")

    def _call(self, fn, ins, outs):
        """Run one library call on the plan's stream.  When the caller's
        current stream is another one, the plan's stream first waits for it
        (the inputs may still be being written there) and the caller's stream
        then waits for the plan's (the outputs are used there); every tensor
        is recorded on the plan's stream so that the caching allocator does
        not reuse its memory while the plan's kernels may still touch it."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        other = cur.cuda_stream != self.stream.cuda_stream
        if other:
            self.stream.wait_stream(cur)
        fn()
        if other:
            for t in (*ins, *outs):
                t.record_stream(self.stream)
            cur.wait_stream(self.stream)

    def weights(self, g: int = 0):
        import torch
        if not 0 <= g < len(self.grids):
            raise SGError(1, f"grid index {g} out of range")
        nx, ny = self.grids[g][0], self.grids[g][1]
        wx = torch.empty((2 * ny - 1, 2 * nx - 1), dtype=torch.float64, device=self.device)
        wy = torch.empty_like(wx)
        self._call(lambda: sg_weights(self.handle, g, wx, wy), (), (wx, wy))
        return wx, wy

    def coeffs(self, sigma, out=None):
        out = self.empty() if out is None else out
        self._check_tensor("sigma", sigma)
        self._check_tensor("out", out)
        self._call(lambda: sg_bspline_coeffs(self.handle, sigma, out), (sigma,), (out,))
        return out

    def forces(self, sigma, fx=None, fy=None):
        fx = self.empty() if fx is None else fx
        fy = self.empty() if fy is None else fy
        self._check_tensor("sigma", sigma)
        self._check_tensor("fx", fx)
        self._check_tensor("fy", fy)
        self._call(lambda: sg_forces(self.handle, sigma, fx, fy), (sigma,), (fx, fy))
        return fx, fy

    def adjoint(self, gfx, gfy, out=None):
        out = self.empty() if out is None else out
        self._check_tensor("gfx", gfx)
        self._check_tensor("gfy", gfy)
        self._check_tensor("out", out)
        self._call(lambda: sg_forces_adjoint(self.handle, gfx, gfy, out), (gfx, gfy), (out,))
        return out


def _autograd():
    import torch

    class ThinDiskForces(torch.autograd.Function):
        """(Fx, Fy) = forces(sigma) with the hand-written adjoint as backward."""

        @staticmethod
        def forward(ctx, sigma, plan):
            ctx.plan = plan
            s = sigma.contiguous()
            if s.dtype != plan.dtype:
                raise SGError(1, f"sigma: dtype {s.dtype}, the plan needs {plan.dtype}")
            return plan.forces(s)

        @staticmethod
        def backward(ctx, gfx, gfy):
            plan = ctx.plan
            gx = gfx.contiguous() if gfx is not None else torch.zeros(plan.total, dtype=plan.dtype, device=plan.device)
            gy = gfy.contiguous() if gfy is not None else torch.zeros(plan.total, dtype=plan.dtype, device=plan.device)
            return plan.adjoint(gx, gy), None

    return ThinDiskForces


class _Lazy:
    _fn = None

    def apply(self, sigma, plan):
        if _Lazy._fn is None:
            _Lazy._fn = _autograd()
        return _Lazy._fn.apply(sigma, plan)


ThinDiskForces = _Lazy()
