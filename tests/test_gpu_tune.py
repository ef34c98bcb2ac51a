"""The autotuner (afd_plan_tune): every launch choice it times gives the same
results bit for bit (the tuner checks each candidate against the first), the
tuned plan decomposes exactly as the untuned one, and a plan created later
with the same shape starts from the choices found."""
import numpy as np
import pytest

import workloads as W
from tests.parity_tools import to_numpy

torch = pytest.importorskip("torch")
from paper_1711_08604_amd import Plan  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FIELDS = ("index", "a", "coef", "energy", "margin", "remainder", "recheck_count", "flags", "fp32_error")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("n,m,prec,cands", [
    (16384, 1000, "fp64", 4),    # fused or three-launch tail x work queue on or off
    (4096, 300, "fp32", 2),      # the tail only
    (1 << 16, 300, "fp64", 3),   # radii per two-pass chunk: allocated, half, quarter
    (729, 60, "fp64", 1),        # nothing to choose
    (1000, 60, "fp32", 1),       # nor for a mixed radix
], ids=str)
def test_tune_keeps_results(n, m, prec, cands):
    g, radii, _ = W.shaped_like_config2(n, m, 6, item=600)
    stream = torch.cuda.current_stream().cuda_stream
    with Plan(n, radii, precision=prec, stream=stream) as plan:
        before = to_numpy(plan.decompose(_dev(g), 6))
        rep = plan.tune(_dev(g), 3)
        print(f"case tune N={n} M={m} {prec}: {rep}", flush=True)
        assert rep["candidates"] == cands
        if cands > 1:
            assert rep["ms"] > 0 and rep["ms"] <= rep["ms_default"]
        after = to_numpy(plan.decompose(_dev(g), 6))
        for k in FIELDS:
            assert np.array_equal(before[k], after[k], equal_nan=True), k
    with Plan(n, radii, precision=prec, stream=stream) as again:
        now = again.tune()
        for k in ("split_tail", "no_queue", "chunk"):
            assert now[k] == rep[k], (k, now, rep)
