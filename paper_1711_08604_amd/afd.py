"""Python binding of libafd (argument marshalling only).

Every step of the decomposition runs in the HIP kernels of libafd.so; this
module only converts arrays to pointers and back.  Inputs may be numpy arrays
(host memory) or torch tensors on the GPU (device memory, used in place on
torch's current stream).  If the library is missing the import fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafd.so")

AFD_OK = 0
STATUS = {0: "AFD_OK", 1: "AFD_E_INVALID", 2: "AFD_E_NONFINITE", 3: "AFD_E_NOMEM", 4: "AFD_E_HIP",
          5: "AFD_E_UNSUPPORTED"}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_recheck": 1}


class AfdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("m", ctypes.c_int32),
        ("radii", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int),
        ("recheck_k", ctypes.c_int32),
        ("first_a_zero", ctypes.c_int32),
        ("recheck_band", ctypes.c_double),
        ("batch", ctypes.c_int32),
    ]


class ResultDesc(ctypes.Structure):
    _fields_ = [
        ("index", ctypes.c_void_p),
        ("a", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
        ("energy", ctypes.c_void_p),
        ("margin", ctypes.c_void_p),
        ("remainder", ctypes.c_void_p),
        ("recheck_count", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
        ("fp32_error", ctypes.c_void_p),
    ]


EXPORTS = [
    "afd_plan_create", "afd_decompose", "afd_replay", "afd_workspace_bytes", "afd_plan_destroy",
    "afd_status_string", "afd_last_error", "afd_plan_set_timing", "afd_plan_kernel_time",
    "afd_plan_radius_launch",
]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libafd.so (built by paper_1711_08604_amd.build); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libafd.so not found at {path}; build it with "
                          "`python -m paper_1711_08604_amd.build` (needs ROCm hipcc)")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.afd_plan_create.argtypes = [ctypes.POINTER(PlanDesc), vp, ctypes.POINTER(vp)]
    lib.afd_plan_create.restype = ctypes.c_int
    lib.afd_decompose.argtypes = [vp, vp, i32, ctypes.POINTER(ResultDesc)]
    lib.afd_decompose.restype = ctypes.c_int
    lib.afd_replay.argtypes = [vp, vp, i32, vp, ctypes.POINTER(ResultDesc)]
    lib.afd_replay.restype = ctypes.c_int
    lib.afd_workspace_bytes.argtypes = [ctypes.POINTER(PlanDesc)]
    lib.afd_workspace_bytes.restype = ctypes.c_size_t
    lib.afd_plan_destroy.argtypes = [vp]
    lib.afd_plan_destroy.restype = None
    lib.afd_status_string.argtypes = [ctypes.c_int]
    lib.afd_status_string.restype = ctypes.c_char_p
    lib.afd_last_error.argtypes = []
    lib.afd_last_error.restype = ctypes.c_char_p
    lib.afd_plan_set_timing.argtypes = [vp, ctypes.c_char_p, i32]
    lib.afd_plan_set_timing.restype = ctypes.c_int
    lib.afd_plan_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.afd_plan_kernel_time.restype = ctypes.c_int
    lib.afd_plan_radius_launch.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.afd_plan_radius_launch.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != AFD_OK:
        msg = _lib.afd_last_error().decode(errors="replace") if _lib else ""
        raise AfdError(status, msg)


def _make_desc(n, radii, precision, recheck_k, first_a_zero, recheck_band, batch=1):
    radii = np.ascontiguousarray(np.asarray(radii, dtype=np.float64))
    d = PlanDesc()
    d.n = int(n)
    d.m = int(radii.shape[0])
    d.radii = radii.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.precision = PRECISIONS[precision]
    d.recheck_k = int(recheck_k)
    d.first_a_zero = 1 if first_a_zero else 0
    d.recheck_band = float(recheck_band)
    d.batch = int(batch)
    return d, radii


def workspace_bytes(n, radii, precision="fp64", recheck_k=8, first_a_zero=False, recheck_band=0.0,
                    batch=1) -> int:
    lib = load_library()
    d, keep = _make_desc(n, radii, precision, recheck_k, first_a_zero, recheck_band, batch)
    return int(lib.afd_workspace_bytes(ctypes.byref(d)))


@dataclass
class Result:
    # shapes for one signal; a batched plan adds a leading batch dimension
    index: object      # (steps, 2) int32: (m_k, j_k)
    a: object          # (steps,) complex128
    coef: object       # (steps,) complex128
    energy: object     # (steps+1,) float64
    margin: object     # (steps,) float64
    remainder: object  # (N,) complex128
    recheck_count: object
    flags: object
    fp32_error: object  # (steps,) float64: FP32-vs-FP64 error of |.|^2 on the re-checked points

    @property
    def delta(self):
        return self.energy[1:] / self.energy[0]


def _is_torch_cuda(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


class Plan:
    """A decomposition plan: N samples, the radius grid, the precision mode;
    batch > 1 decomposes that many signals of length N together."""

    def __init__(self, n, radii, precision="fp64", recheck_k=8, first_a_zero=False, recheck_band=0.0,
                 stream=None, batch=1):
        self._lib = load_library()
        self.n = int(n)
        self.precision = precision
        self.batch = int(batch)
        d, self._radii = _make_desc(n, radii, precision, recheck_k, first_a_zero, recheck_band, self.batch)
        self.m = int(self._radii.shape[0])
        self._stream = stream
        h = ctypes.c_void_p()
        _check(self._lib.afd_plan_create(ctypes.byref(d), ctypes.c_void_p(stream), ctypes.byref(h)))
        self._h = h

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.afd_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- running
    def _outputs(self, signal, steps):
        lead = (self.batch,) if self.batch > 1 else ()
        shapes = {"index": ((steps, 2), "i32"), "a": ((steps,), "c128"), "coef": ((steps,), "c128"),
                  "energy": ((steps + 1,), "f64"), "margin": ((steps,), "f64"), "remainder": ((self.n,), "c128"),
                  "recheck_count": ((steps,), "i32"), "flags": ((steps,), "i32"), "fp32_error": ((steps,), "f64")}
        if _is_torch_cuda(signal):
            import torch
            dev = signal.device
            dt = {"i32": torch.int32, "f64": torch.float64, "c128": torch.complex128}
            out = Result(**{k: torch.empty(lead + shp, dtype=dt[t], device=dev) for k, (shp, t) in shapes.items()})
            ptr = lambda t: t.data_ptr()  # noqa: E731
        else:
            dt = {"i32": np.int32, "f64": np.float64, "c128": np.complex128}
            out = Result(**{k: np.empty(lead + shp, dtype=dt[t]) for k, (shp, t) in shapes.items()})
            ptr = lambda a: a.ctypes.data  # noqa: E731
        rd = ResultDesc()
        for name in ("index", "a", "coef", "energy", "margin", "remainder", "recheck_count", "flags", "fp32_error"):
            setattr(rd, name, ptr(getattr(out, name)))
        return out, rd

    def _signal_ptr(self, signal):
        total = self.n * self.batch
        if _is_torch_cuda(signal):
            import torch
            if signal.dtype == torch.float64:
                ok = signal.numel() == 2 * total
            else:
                ok = signal.dtype == torch.complex128 and signal.numel() == total
            if not (ok and signal.is_contiguous()):
                raise ValueError(f"signal must be {self.batch} x {self.n} contiguous complex128")
            return signal.data_ptr(), signal
        arr = np.ascontiguousarray(np.asarray(signal, dtype=np.complex128))
        want = (self.batch, self.n) if self.batch > 1 else (self.n,)
        if arr.shape != want:
            raise ValueError(f"signal must have shape {want}")
        return arr.ctypes.data, arr

    def decompose(self, signal, steps: int) -> Result:
        sp, keep = self._signal_ptr(signal)
        out, rd = self._outputs(signal, int(steps))
        _check(self._lib.afd_decompose(self._h, ctypes.c_void_p(sp), int(steps), ctypes.byref(rd)))
        return out

    def replay(self, signal, steps: int, forced) -> Result:
        sp, keep = self._signal_ptr(signal)
        out, rd = self._outputs(signal, int(steps))
        if _is_torch_cuda(forced):
            fptr, fkeep = forced.data_ptr(), forced
        else:
            fkeep = np.ascontiguousarray(np.asarray(forced, dtype=np.int32))
            if fkeep.size != 2 * int(steps) * self.batch:
                raise ValueError("forced must hold (m, j) for every step of every signal")
            fptr = fkeep.ctypes.data
        _check(self._lib.afd_replay(self._h, ctypes.c_void_p(sp), int(steps), ctypes.c_void_p(fptr),
                                    ctypes.byref(rd)))
        return out

    # -- measurement
    def set_timing(self, kernel: str = "radius", enable: bool = True):
        _check(self._lib.afd_plan_set_timing(self._h, kernel.encode(), 1 if enable else 0))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self._lib.afd_plan_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def radius_launch(self):
        b = ctypes.c_int64()
        t = ctypes.c_int32()
        l = ctypes.c_int32()
        _check(self._lib.afd_plan_radius_launch(self._h, ctypes.byref(b), ctypes.byref(t), ctypes.byref(l)))
        return b.value, t.value, l.value


def status_string(status: int) -> str:
    return load_library().afd_status_string(int(status)).decode()
