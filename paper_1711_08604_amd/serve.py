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

Shared launches: requests of one shape (N <= 2^14, radii, precision) run as
the members of a group on one slot.  The group advances every member by a
segment of AFD steps per call of a batched plan (every kernel launch covers
all members), and between segments it admits the requests of that shape
that arrived meanwhile and retires the ones that are done.  A member's next
segment starts from the remainder its last one returned; each AFD step
depends on the remainder alone, so the segments concatenate to the
decomposition of the whole request.  Batches are padded with zero signals
to a power of two, so a group reuses a few plans.  With the server's own
device streams a member's remainder and its segments' outputs stay in device
memory between segments (gathered into the batch's input on the device);
only the finished request is copied to the host.

Plans are created with `concurrent=True`: their streams run beside other
slots' kernels, so no launch of theirs waits at a grid barrier for
workgroups that other streams keep from becoming resident.

The plan of a request (or of a group) is the same object a caller would
build, and the kernels are deterministic (a signal's result in a batch
equals its result alone), so a request's result does not depend on what
else is in flight.
"""
from __future__ import annotations

import threading
import time
from collections import OrderedDict, deque
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from .afd import Plan, Result, workspace_bytes


@dataclass
class Request:
    signal: np.ndarray          # (N,) complex128 boundary samples
    radii: np.ndarray           # (M,) radii in [0, 1)
    steps: int
    precision: str = "fp32"
    submitted: float = field(default_factory=time.perf_counter)


SHARE_MAX_N = 1 << 14  # batched plans cover N <= 2^14

RESULT_FIELDS = ("index", "a", "coef", "energy", "margin", "remainder", "recheck_count", "flags", "fp32_error")


@dataclass
class _Member:
    req: Request
    fut: Future
    started: float
    g: object                   # the remainder the next segment starts from (numpy, or a device tensor)
    left: int                   # AFD steps still to run
    parts: list = field(default_factory=list)


def _is_tensor(x) -> bool:
    return type(x).__module__.startswith("torch")


def _member_result(res, i: int, batched: bool):
    """Signal i of a (batched) Result: views of the batch's arrays (device
    tensors stay on the device; each call's outputs are fresh arrays)."""
    if _is_tensor(res.index):
        return Result(**{k: (getattr(res, k)[i] if batched else getattr(res, k)) for k in RESULT_FIELDS})
    return Result(**{k: np.array(getattr(res, k)[i] if batched else getattr(res, k)) for k in RESULT_FIELDS})


def _concat(parts) -> "Result":
    """The segments of one request as one decomposition (numpy): per-step
    arrays concatenated; energies E_0 of the first segment, then each
    segment's E_1.. (its own E_0 is the previous segment's last); the last
    remainder.  Device segments are joined on the device and copied once."""
    on_dev = _is_tensor(parts[0].index)
    if on_dev:
        import torch
        cat = torch.cat
    else:
        cat = np.concatenate
    out = {k: cat([getattr(p, k) for p in parts]) for k in RESULT_FIELDS if k not in ("energy", "remainder")}
    out["energy"] = cat([parts[0].energy] + [p.energy[1:] for p in parts[1:]])
    out["remainder"] = parts[-1].remainder
    if on_dev:
        out = {k: v.cpu().numpy() for k, v in out.items()}
    return Result(**out)


def _bucket(count: int) -> int:
    b = 1
    while b < count:
        b *= 2
    return b


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
    """Admission by free slot and HBM budget; concurrent execution on per-slot
    streams; requests of one shape share their launches."""

    def __init__(self, slots: int = 8, hbm_budget: int = 64 << 30, device: str = "cuda:0", streams=None,
                 share: bool = True, segment: int = 16, max_batch: int = 32):
        """`streams`: one HIP stream handle per slot (default: new torch streams on `device`).
        `share`: run requests of one shape (N <= 2^14) as a group with shared
        launches, `segment` AFD steps per call, at most `max_batch` at once."""
        self.slots = int(slots)
        self.budget = int(hbm_budget)
        self.share = bool(share)
        self.segment = max(1, int(segment))
        self.max_batch = _bucket(max(1, int(max_batch)))
        self._groups = {}                    # shape key -> pending members of the group running it
        self._group_threads = []
        self.shared_calls = 0                # batched calls made by groups
        self.shared_members = 0              # member-segments they covered
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
            self._device = dev
        else:
            self._streams = list(streams)
            self._torch_streams = None
            self._device = None  # caller's streams: groups keep their remainders on the host
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
        for th in list(self._group_threads):  # their plans are closed by their threads
            th.join()
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

    def _shareable(self, req: Request) -> bool:
        return self.share and req.signal.shape[0] <= SHARE_MAX_N and req.steps > 0

    def _group_size(self, req: Request):
        """(largest batch, HBM of every batched plan up to it) for a group of
        this shape: the largest power of two up to max_batch whose plans (one
        per power of two) fit the budget together; (0, 0) if none does."""
        best, total, b = (0, 0), 0, 1
        while b <= self.max_batch:
            total += workspace_bytes(req.signal.shape[0], req.radii, req.precision, batch=b)
            if total > self.budget:
                break
            best = (b, total)
            b *= 2
        return best

    def _dispatch(self):
        while True:
            with self._lock:
                while not self._closed and not self._queue:
                    self._lock.wait()
                if self._closed and not self._queue:
                    return
                req, need, fut = self._queue[0]
                key = _plan_key(req)
                if self._shareable(req):
                    if key in self._groups:  # a group of this shape is running: it takes the request
                        self._queue.popleft()
                        self._groups[key].append((req, fut))
                        self._busy += 1
                        continue
                    if not self._free_slots:
                        self._lock.wait()
                        continue
                    gmax, gneed = self._group_size(req)
                    if gmax == 0:
                        self._queue.popleft()
                        fut.set_exception(ValueError(f"a request of this shape needs more than the HBM budget "
                                                     f"{self.budget}"))
                        continue
                    slot = self._free_slots[0]
                    if self._used + gneed > self.budget and not self._reclaim(gneed, slot, None):
                        self._lock.wait()  # wait for running requests to finish
                        continue
                    self._queue.popleft()
                    self._free_slots.remove(slot)
                    self._used += gneed
                    self.peak_used = max(self.peak_used, self._used)
                    self._busy += 1
                    self._groups[key] = deque([(req, fut)])
                    target, args = self._run_group, (slot, key, gmax, gneed)
                    self._group_threads = [t for t in self._group_threads if t.is_alive()]
                else:
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
                    target, args = self._run, (slot, req, need, key, fut)
            th = threading.Thread(target=target, args=args, daemon=True)
            if target == self._run_group:
                with self._lock:
                    self._group_threads.append(th)
            th.start()

    def _run_group(self, slot: int, key, gmax: int, gneed: int):
        """Run the group of shape `key` on `slot` (at most gmax members at a
        time) until no member is left."""
        n, precision, _ = key
        pending = self._groups[key]
        radii = np.frombuffer(key[2], dtype=np.float64)
        plans = {}
        members = []
        try:
            while True:
                with self._lock:
                    while pending and len(members) < gmax:
                        req, fut = pending.popleft()
                        members.append(_Member(req, fut, time.perf_counter(), req.signal, req.steps))
                    if not members:
                        del self._groups[key]  # later requests of this shape start a new group
                        return
                nb = _bucket(len(members))
                if nb not in plans:
                    plans[nb] = Plan(n, radii, precision=precision, stream=self._streams[slot], batch=nb,
                                     concurrent=True)
                seg = min(self.segment, min(m.left for m in members))
                res = self._segment(slot, plans[nb], members, nb, n, seg)
                self.shared_calls += 1
                self.shared_members += len(members)
                for i, m in enumerate(members):
                    part = _member_result(res, i, nb > 1)
                    m.parts.append(part)
                    m.g = part.remainder
                    m.left -= seg
                done = [m for m in members if m.left == 0]
                for m in done:
                    out = Served(_concat(m.parts), m.req.submitted, m.started, time.perf_counter(), slot)
                    members = [x for x in members if x is not m]
                    m.fut.set_result(out)
                    with self._lock:
                        self._busy -= 1
                        self._lock.notify_all()
        except Exception as e:  # the group's requests fail, the server goes on
            with self._lock:
                failed = members + [_Member(r, f, 0.0, r.signal, 0) for r, f in pending]
                pending.clear()
                self._groups.pop(key, None)
                for m in failed:
                    m.fut.set_exception(e)
                    self._busy -= 1
        finally:
            for plan in plans.values():
                plan.close()
            with self._lock:
                self._used -= gneed
                self._free_slots.append(slot)
                self._lock.notify_all()

    def _segment(self, slot, plan, members, nb: int, n: int, seg: int):
        """One call of the batched plan over the members' remainders (zero
        padding to nb signals): on the device when the server owns its
        streams (torch work on the slot's stream, in order with the plan's
        kernels), else through host memory."""
        if self._device is None:
            sig = np.zeros((nb, n), dtype=np.complex128)
            for i, m in enumerate(members):
                sig[i] = m.g
            return plan.decompose(sig if nb > 1 else sig[0], seg)
        import torch
        with torch.cuda.stream(self._torch_streams[slot]):
            sig = torch.zeros((nb, n), dtype=torch.complex128, device=self._device)
            for i, m in enumerate(members):
                if not torch.is_tensor(m.g):
                    m.g = torch.from_numpy(m.g).to(self._device, non_blocking=False)
                sig[i].copy_(m.g)
            return plan.decompose(sig if nb > 1 else sig[0], seg)

    def _run(self, slot: int, req: Request, need: int, key, fut: Future):
        started = time.perf_counter()
        try:
            cache = self._plans[slot]
            if key in cache:
                plan, _ = cache.pop(key)
            else:
                plan = Plan(req.signal.shape[0], req.radii, precision=req.precision, stream=self._streams[slot],
                            concurrent=True)
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
