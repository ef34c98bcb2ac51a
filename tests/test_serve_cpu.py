"""The serving scheduler's admission logic on the CPU, with a stand-in plan
(no GPU): slots and the HBM budget are never exceeded, every request
finishes, a failing request does not stop the others, and cached plans are
reused and evicted when memory is needed."""
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

    def __init__(self, n, radii, precision="fp32", stream=None):
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
    monkeypatch.setattr(S, "workspace_bytes", lambda n, radii, precision="fp32": 1000 * n)
    FakePlan.live = FakePlan.peak = FakePlan.built = 0
    return FakePlan


def test_slots_budget_and_completion(fake):
    rng = np.random.default_rng(0)
    ns = [int(2 ** rng.integers(6, 10)) for _ in range(40)]
    budget = 3 * 1000 * 512
    srv = S.Server(slots=4, hbm_budget=budget, streams=[None] * 4)
    futs = [srv.submit(np.zeros(n, complex), [0.0, 0.5], 2 + i % 5) for i, n in enumerate(ns)]
    out = [f.result(timeout=30) for f in futs]
    srv.close()
    assert [o.result for o in out] == [(n, 2 + i % 5) for i, n in enumerate(ns)]
    assert fake.peak <= 4
    assert srv.peak_used <= budget
    assert all(o.finished >= o.started >= o.submitted for o in out)


def test_failure_is_isolated_and_plans_are_reused(fake):
    srv = S.Server(slots=2, hbm_budget=10 ** 9, streams=[None] * 2)
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
