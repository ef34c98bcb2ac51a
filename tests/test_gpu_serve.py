"""Serving: requests of differing N and step counts admitted by free slot and
HBM budget and run concurrently, those of one shape in shared launches; each
result must equal the same request decomposed alone (bit for bit) and match
the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.parity_tools import TOL, compare

torch = pytest.importorskip("torch")
from paper_1711_08604_amd import Plan, workspace_bytes  # noqa: E402
from paper_1711_08604_amd.serve import Server  # noqa: E402

pytestmark = pytest.mark.gpu

FIELDS = ("index", "a", "coef", "energy", "margin", "recheck_count", "flags", "fp32_error", "remainder")


def _requests(count, seed=11):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(2 ** rng.integers(8, 13))          # 256 .. 4096
        m = max(n // 8, 4)
        steps = int(rng.integers(3, 13))
        prec = "fp32" if i % 3 else "fp64"
        g, radii, _ = W.shaped_like_config2(n, m, steps, item=1000 + i)
        reqs.append((g, radii, steps, prec))
    return reqs


def _alone(g, radii, steps, prec):
    with Plan(g.shape[0], radii, precision=prec) as p:
        return p.decompose(g, steps)


def _large_requests():
    """N = 2^15 and 2^16 (M = N/8): two-pass radius transforms on slots of their own."""
    out = []
    for i, (k, steps, prec) in enumerate(((15, 4, "fp32"), (16, 3, "fp64"), (15, 3, "fp64"), (16, 4, "fp32"))):
        g, radii, _ = W.shaped_like_config2(1 << k, (1 << k) // 8, steps, item=2000 + i)
        out.append((g, radii, steps, prec))
    return out


def test_mix_equals_alone_and_oracle():
    """Requests of one shape share launches: segments of 4 AFD steps of a
    batched plan, members joining (also while the group runs) and leaving
    between segments; requests of N = 2^15 and 2^16 run beside them on slots
    of their own."""
    reqs = _requests(24)
    reqs = reqs[:6] + _large_requests()[:2] + reqs[6:18] + _large_requests()[2:] + reqs[18:]
    with Server(slots=4, segment=4) as srv:
        futs = []
        for i, r in enumerate(reqs):
            futs.append(srv.submit(*r))
            if i == 15:
                futs[0].result(timeout=120)  # the rest arrive while groups run
        served = [f.result(timeout=120) for f in futs]
        shared = (srv.shared_calls, srv.shared_members)
    slots_used = {s.slot for s in served}
    assert len(slots_used) > 1
    assert shared[1] > shared[0], shared  # some calls covered several requests
    for i, ((g, radii, steps, prec), s) in enumerate(zip(reqs, served)):
        alone = _alone(g, radii, steps, prec)
        for k in FIELDS:
            np.testing.assert_array_equal(getattr(s.result, k), getattr(alone, k), err_msg=f"request {i} field {k}")
        if i % 4 == 0 and g.shape[0] <= 4096:
            compare(s.result, O.decompose(g, radii, steps), TOL[prec], signal=g, radii=radii)
    assert any(g.shape[0] >= 1 << 15 for g, _, _, _ in reqs)


def test_admission_respects_budget():
    reqs = _requests(12, seed=5)
    need = max(workspace_bytes(g.shape[0], radii, prec) for g, radii, _, prec in reqs)
    budget = 2 * need
    with Server(slots=4, hbm_budget=budget) as srv:
        served = [f.result(timeout=120) for f in [srv.submit(*r) for r in reqs]]
        assert srv.peak_used <= budget
    for (g, radii, steps, prec), s in zip(reqs, served):
        alone = _alone(g, radii, steps, prec)
        np.testing.assert_array_equal(s.result.index, alone.index)
        np.testing.assert_array_equal(s.result.coef, alone.coef)


def test_rejected_requests():
    with Server(slots=2, hbm_budget=1 << 20) as srv:
        with pytest.raises(ValueError):
            srv.submit(np.ones(64, complex), [0.5, 1.5], 2)        # radius outside [0, 1)
        with pytest.raises(ValueError):
            srv.submit(np.ones(1 << 14, complex), np.linspace(0, 0.9, 1000), 2)  # above the budget
        ok = srv.submit(np.ones(64, complex), [0.0, 0.5], 2).result(timeout=60)
        assert ok.result.index.shape == (2, 2)
