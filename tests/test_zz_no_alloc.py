"""afd_decompose_noalloc (results staged in the library's static device
scratch, no allocation in the call) against afd_decompose through the C ABI:
bit for bit on two calls in a row, the second with a smaller input, and the
smaller one against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.parity_tools import TOL, compare, to_numpy

torch = pytest.importorskip("torch")
from paper_1711_08604_amd import AfdError, Plan  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FIELDS = ("index", "a", "coef", "energy", "margin", "remainder", "recheck_count", "flags", "fp32_error")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_decompose(prec):
    cases = [W.config2(), W.config1()]  # N = 16384, M = 1000, 50 steps; then N = 1024, M = 100, 10 steps
    last = None
    for g, radii, steps in cases:
        n = g.shape[0]
        print(f"case noalloc N={n} M={len(radii)} steps={steps} {prec}", flush=True)
        with Plan(n, radii, precision=prec) as plan:
            a = to_numpy(plan.decompose_noalloc(_dev(g), steps))  # first call on the plan: nothing allocated yet
            b = to_numpy(plan.decompose(_dev(g), steps))
            h = to_numpy(plan.decompose_noalloc(g, steps))  # host input and outputs
        for k in FIELDS:
            assert np.array_equal(a[k], b[k], equal_nan=True), (n, k)
            assert np.array_equal(h[k], b[k], equal_nan=True), (n, k)
        last = (g, radii, steps, a)
    g, radii, steps, a = last
    compare(_Res(a), O.decompose(g, radii, steps), TOL[prec], signal=g, radii=radii)


def test_noalloc_rejects_beyond_scratch():
    with Plan(64, W.uniform_radii(5), precision="fp64") as plan:
        g = np.ones(64, complex)
        with pytest.raises(AfdError) as ei:
            plan.decompose_noalloc(_dev(g), 6000)
        assert ei.value.status == 1
        r = to_numpy(plan.decompose_noalloc(_dev(g), 3))  # still usable
        assert r["energy"].shape == (4,)


class _Res:
    def __init__(self, d):
        self.__dict__.update(d)
