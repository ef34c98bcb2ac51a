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
        ("concurrent", ctypes.c_int32),
        ("sample_turns", ctypes.POINTER(ctypes.c_double)),
        ("sample_weights", ctypes.POINTER(ctypes.c_double)),
        ("samples", ctypes.c_int64),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("split_tail", ctypes.c_int32),
        ("no_queue", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("ms", ctypes.c_double),
        ("ms_default", ctypes.c_double),
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
        ("pick_index", ctypes.c_void_p),
        ("pick_p", ctypes.c_void_p),
        ("pick_margin", ctypes.c_void_p),
        ("pick_flags", ctypes.c_void_p),
    ]


EXPORTS = [
    "afd_plan_create", "afd_decompose", "afd_decompose_noalloc", "afd_replay", "afd_workspace_bytes", "afd_plan_destroy",
    "afd_status_string", "afd_last_error", "afd_plan_set_timing", "afd_plan_kernel_time",
    "afd_plan_radius_launch", "afd_reconstruct", "afd_analytic",
    "afd_graph_create", "afd_graph_launch", "afd_graph_status", "afd_graph_destroy",
    "afd_group_create", "afd_group_launch", "afd_group_status", "afd_group_destroy", "afd_plan_tune",
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
    lib.afd_decompose_noalloc.argtypes = [vp, vp, i32, ctypes.POINTER(ResultDesc)]
    lib.afd_decompose_noalloc.restype = ctypes.c_int
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
    lib.afd_reconstruct.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.afd_reconstruct.restype = ctypes.c_int
    lib.afd_analytic.argtypes = [vp, vp, vp]
    lib.afd_analytic.restype = ctypes.c_int
    lib.afd_graph_create.argtypes = [vp, vp, i32, ctypes.POINTER(ResultDesc), ctypes.POINTER(vp)]
    lib.afd_graph_create.restype = ctypes.c_int
    lib.afd_graph_launch.argtypes = [vp]
    lib.afd_graph_launch.restype = ctypes.c_int
    lib.afd_graph_status.argtypes = [vp]
    lib.afd_graph_status.restype = ctypes.c_int
    lib.afd_graph_destroy.argtypes = [vp]
    lib.afd_graph_destroy.restype = None
    lib.afd_group_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(i32),
                                     ctypes.POINTER(ResultDesc), ctypes.POINTER(vp)]
    lib.afd_group_create.restype = ctypes.c_int
    lib.afd_group_launch.argtypes = [vp]
    lib.afd_group_launch.restype = ctypes.c_int
    lib.afd_group_status.argtypes = [vp]
    lib.afd_group_status.restype = ctypes.c_int
    lib.afd_group_destroy.argtypes = [vp]
    lib.afd_group_destroy.restype = None
    lib.afd_plan_tune.argtypes = [vp, vp, i32, ctypes.POINTER(Tuning)]
    lib.afd_plan_tune.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != AFD_OK:
        msg = _lib.afd_last_error().decode(errors="replace") if _lib else ""
        raise AfdError(status, msg)


def _make_desc(n, radii, precision, recheck_k, first_a_zero, recheck_band, batch=1, concurrent=False,
               sample_turns=None, sample_weights=None):
    """The plan descriptor and the host arrays it points to (kept alive by the caller)."""
    radii = np.ascontiguousarray(np.asarray(radii, dtype=np.float64))
    d = PlanDesc()
    keep = [radii]
    if sample_turns is not None:
        t = np.ascontiguousarray(np.asarray(sample_turns, dtype=np.float64).reshape(-1))
        d.sample_turns = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.samples = int(t.shape[0])
        keep.append(t)
        if sample_weights is not None:
            w = np.ascontiguousarray(np.asarray(sample_weights, dtype=np.float64).reshape(-1))
            if w.shape != t.shape:
                raise ValueError("sample_weights must have one weight per sample")
            d.sample_weights = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            keep.append(w)
    d.n = int(n)
    d.m = int(radii.shape[0])
    d.radii = radii.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.precision = PRECISIONS[precision]
    d.recheck_k = int(recheck_k)
    d.first_a_zero = 1 if first_a_zero else 0
    d.recheck_band = float(recheck_band)
    d.batch = int(batch)
    d.concurrent = 1 if concurrent else 0
    return d, keep


def workspace_bytes(n, radii, precision="fp64", recheck_k=8, first_a_zero=False, recheck_band=0.0,
                    batch=1, sample_turns=None, sample_weights=None) -> int:
    lib = load_library()
    d, keep = _make_desc(n, radii, precision, recheck_k, first_a_zero, recheck_band, batch,
                         sample_turns=sample_turns, sample_weights=sample_weights)
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
    # replay only: the selection's own choice at each replayed step (None after decompose)
    pick_index: object = None   # (steps, 2) int32
    pick_p: object = None       # (steps,) float64: its |<G_k, e_a>~|^2
    pick_margin: object = None  # (steps,) float64
    pick_flags: object = None   # (steps,) int32: bit 4 = the forced point was on the FP32 short-list

    @property
    def delta(self):
        return self.energy[1:] / self.energy[0]


def _is_torch_cuda(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


class Plan:
    """A decomposition plan: N samples, the radius grid, the precision mode;
    batch > 1 decomposes that many signals of length N together."""

    def __init__(self, n, radii, precision="fp64", recheck_k=8, first_a_zero=False, recheck_band=0.0,
                 stream=None, batch=1, concurrent=False, sample_turns=None, sample_weights=None):
        """`concurrent`: the stream runs beside other streams' work on the device
        (no step-tail grid barriers, see afd_plan_desc.concurrent).
        `sample_turns` (and optionally `sample_weights`): non-uniform samples at
        z = e^{2 pi i t}; the signal then holds one value per position and `n`
        is the number of grid angles (afd_plan_desc.sample_turns)."""
        self._lib = load_library()
        self.n = int(n)
        self.precision = precision
        self.batch = int(batch)
        d, keep = _make_desc(n, radii, precision, recheck_k, first_a_zero, recheck_band, self.batch,
                             concurrent, sample_turns, sample_weights)
        self._radii = keep[0]
        self.samples = int(d.samples) if sample_turns is not None else self.n
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
    def _outputs(self, signal, steps, picks=False):
        lead = (self.batch,) if self.batch > 1 else ()
        shapes = {"index": ((steps, 2), "i32"), "a": ((steps,), "c128"), "coef": ((steps,), "c128"),
                  "energy": ((steps + 1,), "f64"), "margin": ((steps,), "f64"),
                  "remainder": ((self.samples,), "c128"),
                  "recheck_count": ((steps,), "i32"), "flags": ((steps,), "i32"), "fp32_error": ((steps,), "f64")}
        if picks:
            shapes.update({"pick_index": ((steps, 2), "i32"), "pick_p": ((steps,), "f64"),
                           "pick_margin": ((steps,), "f64"), "pick_flags": ((steps,), "i32")})
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
        for name in shapes:
            setattr(rd, name, ptr(getattr(out, name)))
        return out, rd

    def _signal_ptr(self, signal):
        total = self.samples * self.batch
        if _is_torch_cuda(signal):
            import torch
            if signal.dtype == torch.float64:
                ok = signal.numel() == 2 * total
            else:
                ok = signal.dtype == torch.complex128 and signal.numel() == total
            if not (ok and signal.is_contiguous()):
                raise ValueError(f"signal must be {self.batch} x {self.samples} contiguous complex128")
            return signal.data_ptr(), signal
        arr = np.ascontiguousarray(np.asarray(signal, dtype=np.complex128))
        want = (self.batch, self.samples) if self.batch > 1 else (self.samples,)
        if arr.shape != want:
            raise ValueError(f"signal must have shape {want}")
        return arr.ctypes.data, arr

    def decompose(self, signal, steps: int) -> Result:
        sp, keep = self._signal_ptr(signal)
        out, rd = self._outputs(signal, int(steps))
        _check(self._lib.afd_decompose(self._h, ctypes.c_void_p(sp), int(steps), ctypes.byref(rd)))
        return out

    def decompose_noalloc(self, signal, steps: int) -> Result:
        """decompose() through afd_decompose_noalloc: the library allocates
        nothing in the call (results staged in its static device scratch)."""
        sp, keep = self._signal_ptr(signal)
        out, rd = self._outputs(signal, int(steps))
        _check(self._lib.afd_decompose_noalloc(self._h, ctypes.c_void_p(sp), int(steps), ctypes.byref(rd)))
        return out

    def replay(self, signal, steps: int, forced) -> Result:
        """Decompose along the forced indices (steps x 2, or batch x steps x 2):
        every step still runs the whole path and reports its own choice in
        pick_index / pick_p / pick_margin / pick_flags (afd_replay)."""
        sp, keep = self._signal_ptr(signal)
        out, rd = self._outputs(signal, int(steps), picks=True)
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

    def tune(self, signal=None, steps: int = 0) -> dict:
        """afd_plan_tune: time the plan's result-invariant launch choices on
        `steps` steps of `signal` and keep the fastest (steps = 0: report the
        current choices)."""
        sp, keep = self._signal_ptr(signal) if signal is not None else (None, None)
        t = Tuning()
        _check(self._lib.afd_plan_tune(self._h, ctypes.c_void_p(sp), int(steps), ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def graph(self, signal, steps: int) -> "Graph":
        """A decomposition of `signal` (a torch tensor on the GPU) captured as a HIP
        graph (afd_graph_create); every launch() decomposes what the tensor then
        holds into the Graph's device outputs."""
        if not _is_torch_cuda(signal):
            raise ValueError("a captured decomposition needs the signal on the device")
        return Graph(self, signal, int(steps))

    # -- outputs around the loop
    def _complex_in(self, x, count, name):
        """Pointer to `count` complex128 values (numpy or torch on the GPU) and a keep-alive."""
        if _is_torch_cuda(x):
            import torch
            if not (x.is_contiguous() and ((x.dtype == torch.complex128 and x.numel() == count)
                                           or (x.dtype == torch.float64 and x.numel() == 2 * count))):
                raise ValueError(f"{name} must hold {count} contiguous complex128 values")
            return x.data_ptr(), x
        arr = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
        if arr.size != count:
            raise ValueError(f"{name} must hold {count} complex values")
        return arr.ctypes.data, arr

    def reconstruct(self, a, coef, signal=None, partial_sum: bool = True):
        """Partial sum S_n = sum_k c_k B_k on the N circle points and, with the
        signal, delta_k = ||G - S_k||^2/||G||^2 for k = 1..n (afd_reconstruct).
        `a`, `coef`: the decomposition's parameters and coefficients, shape
        (steps,) or (batch, steps).  Returns (S or None, delta or None) as numpy
        arrays, or torch tensors on the device when `a` is one."""
        steps = int(np.shape(a)[-1]) if not _is_torch_cuda(a) else int(a.shape[-1])
        count = steps * self.batch
        ap, akeep = self._complex_in(a, count, "a")
        cp, ckeep = self._complex_in(coef, count, "coef")
        sp, skeep = (self._signal_ptr(signal) if signal is not None else (None, None))
        lead = (self.batch,) if self.batch > 1 else ()
        on_dev = _is_torch_cuda(a)
        if on_dev:
            import torch
            S = torch.empty(lead + (self.samples,), dtype=torch.complex128, device=a.device) if partial_sum else None
            D = torch.empty(lead + (steps,), dtype=torch.float64, device=a.device) if signal is not None else None
            ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        else:
            S = np.empty(lead + (self.samples,), dtype=np.complex128) if partial_sum else None
            D = np.empty(lead + (steps,), dtype=np.float64) if signal is not None else None
            ptr = lambda t: t.ctypes.data if t is not None else None  # noqa: E731
        _check(self._lib.afd_reconstruct(self._h, ctypes.c_void_p(ap), ctypes.c_void_p(cp), steps,
                                         ctypes.c_void_p(sp), ctypes.c_void_p(ptr(S)), ctypes.c_void_p(ptr(D))))
        return S, D

    def analytic(self, x):
        """Analytic (H^2) part of the samples x: IDFT(h . DFT(x)) with the DC and
        Nyquist bins kept, positive bins doubled and negative bins removed
        (afd_analytic).  Same shape and location (host or device) as x."""
        xp, keep = self._complex_in(x, self.n * self.batch, "x")
        lead = (self.batch,) if self.batch > 1 else ()
        if _is_torch_cuda(x):
            import torch
            g = torch.empty(lead + (self.n,), dtype=torch.complex128, device=x.device)
            gp = g.data_ptr()
        else:
            g = np.empty(lead + (self.n,), dtype=np.complex128)
            gp = g.ctypes.data
        _check(self._lib.afd_analytic(self._h, ctypes.c_void_p(xp), ctypes.c_void_p(gp)))
        return g

    # -- measurement
    def set_timing(self, kernel: str = "radius", enable=True):
        """Time the kernel class; enable = n >= 1 samples every n-th launch (True: every one), 0/False stops."""
        _check(self._lib.afd_plan_set_timing(self._h, kernel.encode(), int(enable)))

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


class Graph:
    """One decomposition captured as a HIP graph; `result` holds its device outputs."""

    def __init__(self, plan: Plan, signal, steps: int):
        self._plan = plan
        self._lib = plan._lib
        sp, self._signal = plan._signal_ptr(signal)
        self.result, rd = plan._outputs(signal, steps)
        h = ctypes.c_void_p()
        _check(self._lib.afd_graph_create(plan._h, ctypes.c_void_p(sp), steps, ctypes.byref(rd), ctypes.byref(h)))
        self._h = h

    def launch(self):
        """Enqueue one replay on the plan's stream (asynchronous)."""
        _check(self._lib.afd_graph_launch(self._h))

    def status(self):
        """Wait for the plan's stream; raise AfdError if the last replay's signal was not finite."""
        _check(self._lib.afd_graph_status(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.afd_graph_destroy(self._h)
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


class Group:
    """Decompositions of several plans (uneven N) captured into one HIP graph
    (afd_group_create): members = [(plan, signal on the device, steps), ...];
    `results[i]` holds member i's device outputs after launch() + status()."""

    def __init__(self, members):
        if not members:
            raise ValueError("a group needs at least one member")
        self._lib = members[0][0]._lib
        self._plans = [m[0] for m in members]
        self._keep = []
        self.results = []
        count = len(members)
        hs = (ctypes.c_void_p * count)()
        sig = (ctypes.c_void_p * count)()
        st = (ctypes.c_int32 * count)()
        rds = (ResultDesc * count)()
        for i, (plan, signal, steps) in enumerate(members):
            if not _is_torch_cuda(signal):
                raise ValueError("a group member's signal must be on the device")
            sp, keep = plan._signal_ptr(signal)
            res, rd = plan._outputs(signal, int(steps))
            self._keep.append(keep)
            self.results.append(res)
            hs[i] = plan._h.value
            sig[i] = sp
            st[i] = int(steps)
            rds[i] = rd
        h = ctypes.c_void_p()
        _check(self._lib.afd_group_create(hs, count, sig, st, rds, ctypes.byref(h)))
        self._h = h

    def launch(self):
        """One graph launch runs every member's decomposition (asynchronous)."""
        _check(self._lib.afd_group_launch(self._h))

    def status(self):
        """Wait; raise AfdError for the first member whose signal was not finite."""
        _check(self._lib.afd_group_status(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.afd_group_destroy(self._h)
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


def status_string(status: int) -> str:
    return load_library().afd_status_string(int(status)).decode()
