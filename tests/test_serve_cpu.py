"""The serving scheduler's admission logic on the CPU, with a stand-in plan
(no GPU): slots and the HBM budget are never exceeded, every request
finishes, a failing request does not stop the others, and cached plans are
reused and evicted when memory is needed.  Requests of one shape that share
launches (segments of a batched plan, members joining and leaving between
segments) get the decomposition they would get alone."""
import threading
import time

import numpy as np
import pytest

import paper_1711_08604_amd.serve as S


class FakePlan:
    live = 0
    peak = 0
    built = 0
    lock = threading.Lock()

    def __init__(self, n, radii, precision="fp32", stream=None, batch=1, concurrent=False):
        with FakePlan.lock:
            FakePlan.built += 1
        self.n = n

    def decompose(self, signal, steps):
        with FakePlan.lock:
            FakePlan.live += 1
            FakePlan.peak = max(FakePlan.peak, FakePlan.live)
        time.sleep(0.002 * steps)
        with FakePlan.lock:
            FakePlan.live -= 1
        if steps == 13:
            raise RuntimeError("planted failure")
        return (self.n, steps)

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(S, "Plan", FakePlan)
    monkeypatch.setattr(S, "workspace_bytes", lambda n, radii, precision="fp32", batch=1: 1000 * n * batch)
    FakePlan.live = FakePlan.peak = FakePlan.built = 0
    return FakePlan


def test_slots_budget_and_completion(fake):
    rng = np.random.default_rng(0)
    ns = [int(2 ** rng.integers(6, 10)) for _ in range(40)]
    budget = 3 * 1000 * 512
    srv = S.Server(slots=4, hbm_budget=budget, streams=[None] * 4, share=False)
    futs = [srv.submit(np.zeros(n, complex), [0.0, 0.5], 2 + i % 5) for i, n in enumerate(ns)]
    out = [f.result(timeout=30) for f in futs]
    srv.close()
    assert [o.result for o in out] == [(n, 2 + i % 5) for i, n in enumerate(ns)]
    assert fake.peak <= 4
    assert srv.peak_used <= budget
    assert all(o.finished >= o.started >= o.submitted for o in out)


def test_failure_is_isolated_and_plans_are_reused(fake):
    srv = S.Server(share=False, slots=2, hbm_budget=10 ** 9, streams=[None] * 2)
    futs = [srv.submit(np.zeros(64, complex), [0.0, 0.5], s) for s in (3, 13, 4, 5, 6)]
    res = []
    for f in futs:
        try:
            res.append(f.result(timeout=30).result)
        except RuntimeError:
            res.append("failed")
    srv.close()
    assert res == [(64, 3), "failed", (64, 4), (64, 5), (64, 6)]
    assert fake.built <= 3  # one plan per slot, rebuilt once after the failure


def test_rejects_oversized(fake):
    srv = S.Server(slots=1, hbm_budget=1000 * 64, streams=[None])
    with pytest.raises(ValueError):
        srv.submit(np.zeros(128, complex), [0.5], 2)
    srv.close()


class HalvingPlan:
    """A stand-in decomposition whose step k only depends on the remainder:
    index (m, j) and coefficient from the first sample, remainder halved
    (exact in binary), energies of the remainders.  Batched like the library."""
    calls = []
    lock = threading.Lock()
    gate = threading.Event()  # calls wait for it: requests join groups while a segment runs

    def __init__(self, n, radii, precision="fp32", stream=None, batch=1, concurrent=False):
        self.n, self.batch = n, batch

    def _one(self, x, steps):
        idx = np.zeros((steps, 2), np.int32)
        coef = np.zeros(steps, complex)
        energy = np.zeros(steps + 1)
        energy[0] = np.mean(np.abs(x) ** 2)
        for k in range(steps):
            idx[k] = (int(abs(x[0]) * 1e6) % 97, int(abs(x[1]) * 1e6) % 89)
            coef[k] = x[0]
            x = x * 0.5
            energy[k + 1] = np.mean(np.abs(x) ** 2)
        f = np.full(steps, 1.0)
        return dict(index=idx, a=coef * 0.1, coef=coef, energy=energy, margin=f, remainder=x,
                    recheck_count=np.ones(steps, np.int32), flags=np.zeros(steps, np.int32), fp32_error=f * 0)

    def decompose(self, signal, steps):
        assert HalvingPlan.gate.wait(30)
        with HalvingPlan.lock:
            HalvingPlan.calls.append((self.batch, steps))
        sig = np.asarray(signal).reshape(self.batch, self.n)
        outs = [self._one(sig[b].copy(), steps) for b in range(self.batch)]
        if self.batch == 1:
            return S.Result(**outs[0])
        return S.Result(**{k: np.stack([o[k] for o in outs]) for k in outs[0]})

    def close(self):
        pass


def test_shared_launches_equal_alone(monkeypatch):
    monkeypatch.setattr(S, "Plan", HalvingPlan)
    monkeypatch.setattr(S, "workspace_bytes", lambda n, radii, precision="fp32", batch=1: 1000 * batch)
    HalvingPlan.calls = []
    HalvingPlan.gate.clear()
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(30):
        n = 64 if i % 3 else 128
        g = rng.normal(size=n) + 1j * rng.normal(size=n)
        reqs.append((g, np.array([0.0, 0.5]), int(rng.integers(1, 40)), "fp32"))
    srv = S.Server(slots=2, streams=[None] * 2, segment=7, max_batch=8)
    futs = []
    for i, r in enumerate(reqs):
        futs.append(srv.submit(*r))
        if i == 5:
            time.sleep(0.01)  # the first groups have started and hold their first segment
    HalvingPlan.gate.set()  # later requests joined groups already running
    served = [f.result(timeout=30) for f in futs]
    srv.close()
    calls = list(HalvingPlan.calls)
    for (g, radii, steps, prec), s in zip(reqs, served):
        alone = HalvingPlan(g.shape[0], radii).decompose(g, steps)
        for k in S.RESULT_FIELDS:
            np.testing.assert_array_equal(getattr(s.result, k), getattr(alone, k), err_msg=k)
    # launches were shared: fewer batched calls than member-segments, every batch a power of two
    assert srv.shared_members > srv.shared_calls
    assert all(b & (b - 1) == 0 and b <= 8 for b, _ in calls)
    assert all(st <= 7 for _, st in calls)
    assert max(b for b, _ in calls) > 1
