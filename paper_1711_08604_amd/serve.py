"""Serving: a continuous-batching request loop for Core-AFD decompositions on one GPU.

Requests (samples, radii, steps, precision) of differing N and step counts
are queued in arrival order.  A request is admitted as soon as a slot is free
and the HBM its plan needs (``afd_workspace_bytes``) fits the budget; a
request that arrives while others run starts as soon as that holds.  Each
slot owns a HIP stream, a worker thread and the plans it has built: a plan
(its tables and device workspace, including the remainder) stays resident
for the next request of the same shape unless its memory is needed.
Admitted requests run concurrently on their slots' streams, so their kernels
overlap on the device.  Every step of every request runs in the library's HIP
kernels; this module only schedules.

The plan of a request is the same object a caller would build alone, and the
kernels are deterministic, so a request's result does not depend on what else
is in flight.
"""
from __future__ import annotations

import threading
import time
from collections import OrderedDict, deque
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from .afd import Plan, workspace_bytes


@dataclass
class Request:
    signal: np.ndarray          # (N,) complex128 boundary samples
    radii: np.ndarray           # (M,) radii in [0, 1)
    steps: int
    precision: str = "fp32"
    submitted: float = field(default_factory=time.perf_counter)


@dataclass
class Served:
    result: object              # afd.Result (numpy arrays)
    submitted: float            # times from time.perf_counter()
    started: float
    finished: float
    slot: int

    @property
    def latency(self) -> float:
        return self.finished - self.submitted


def _plan_key(req: Request):
    return (int(req.signal.shape[0]), req.precision, np.ascontiguousarray(req.radii, dtype=np.float64).tobytes())


class Server:
    """Admission by free slot and HBM budget; concurrent execution on per-slot streams."""

    def __init__(self, slots: int = 8, hbm_budget: int = 64 << 30, device: str = "cuda:0", streams=None):
        """`streams`: one HIP stream handle per slot (default: new torch streams on `device`)."""
        self.slots = int(slots)
        self.budget = int(hbm_budget)
        self._lock = threading.Condition()
        self._queue: deque = deque()
        self._free_slots = list(range(self.slots))
        self._used = 0                       # bytes of resident plans and running requests
        self._plans = [OrderedDict() for _ in range(self.slots)]  # per slot: key -> (plan, bytes)
        if streams is None:
            import torch
            dev = torch.device(device)
            self._torch_streams = [torch.cuda.Stream(device=dev) for _ in range(self.slots)]
            self._streams = [st.cuda_stream for st in self._torch_streams]
        else:
            self._streams = list(streams)
        self._closed = False
        self._busy = 0
        self.peak_used = 0                   # largest HBM accounted at once (bytes)
        self._dispatcher = threading.Thread(target=self._dispatch, name="afd-dispatch", daemon=True)
        self._dispatcher.start()

    # -- public
    def submit(self, signal, radii, steps: int, precision: str = "fp32") -> Future:
        req = Request(np.ascontiguousarray(np.asarray(signal, dtype=np.complex128)),
                      np.ascontiguousarray(np.asarray(radii, dtype=np.float64)), int(steps), precision)
        need = workspace_bytes(req.signal.shape[0], req.radii, req.precision)
        if need == 0:
            raise ValueError("request rejected by the plan validation (see afd_workspace_bytes)")
        if need > self.budget:
            raise ValueError(f"request needs {need} bytes of HBM, above the budget {self.budget}")
        fut: Future = Future()
        with self._lock:
            if self._closed:
                raise RuntimeError("server closed")
            self._queue.append((req, need, fut))
            self._lock.notify_all()
        return fut

    def drain(self):
        """Wait until every submitted request has finished."""
        with self._lock:
            while self._queue or self._busy:
                self._lock.wait()

    def close(self):
        self.drain()
        with self._lock:
            self._closed = True
            self._lock.notify_all()
        self._dispatcher.join()
        for cache in self._plans:
            for plan, _ in cache.values():
                plan.close()
            cache.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- scheduling
    def _reclaim(self, need: int, keep_slot: int, keep_key) -> bool:
        """Free cached plans of idle slots (least recently used first) until `need` fits."""
        for s in range(self.slots):
            if s not in self._free_slots and s != keep_slot:
                continue
            cache = self._plans[s]
            for key in list(cache.keys()):
                if self._used + need <= self.budget:
                    return True
                if s == keep_slot and key == keep_key:
                    continue
                plan, b = cache.pop(key)
                plan.close()
                self._used -= b
        return self._used + need <= self.budget

    def _dispatch(self):
        while True:
            with self._lock:
                while not self._closed and not self._queue:
                    self._lock.wait()
                if self._closed and not self._queue:
                    return
                req, need, fut = self._queue[0]
                key = _plan_key(req)
                # prefer a free slot that already holds this plan
                slot = next((s for s in self._free_slots if key in self._plans[s]), None)
                if slot is None and self._free_slots:
                    slot = self._free_slots[0]
                if slot is None:
                    self._lock.wait()
                    continue
                extra = 0 if key in self._plans[slot] else need
                if self._used + extra > self.budget and not self._reclaim(extra, slot, key):
                    self._lock.wait()  # wait for running requests to finish
                    continue
                self._queue.popleft()
                self._free_slots.remove(slot)
                self._used += extra
                self.peak_used = max(self.peak_used, self._used)
                self._busy += 1
            threading.Thread(target=self._run, args=(slot, req, need, key, fut), daemon=True).start()

    def _run(self, slot: int, req: Request, need: int, key, fut: Future):
        started = time.perf_counter()
        try:
            cache = self._plans[slot]
            if key in cache:
                plan, _ = cache.pop(key)
            else:
                plan = Plan(req.signal.shape[0], req.radii, precision=req.precision, stream=self._streams[slot])
            cache[key] = (plan, need)  # most recently used last
            res = plan.decompose(req.signal, req.steps)
            fut.set_result(Served(res, req.submitted, started, time.perf_counter(), slot))
        except Exception as e:  # the request fails, the server goes on
            with self._lock:
                if key in self._plans[slot]:
                    plan, b = self._plans[slot].pop(key)
                    plan.close()
                    self._used -= b
                elif need:
                    self._used -= need
            fut.set_exception(e)
        finally:
            with self._lock:
                self._free_slots.append(slot)
                self._busy -= 1
                self._lock.notify_all()
