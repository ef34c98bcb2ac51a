"""A decomposition captured as a HIP graph (afd_graph_create) against the
same decomposition run eagerly: every replay equal bit for bit, with eager
work of the same plan and synchronisations between the replays, a new
signal written into the captured buffer, and a non-finite signal reported."""
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


def _case(name):
    if name == "n1024_m100":  # fused step tail
        g, radii, steps = W.config1()
        g2, _, _ = W.config1(item=1)
        return g, g2, radii, steps, 1
    if name == "n16384_m1000":  # fused step tail; the double-precision radius kernel's work queue
        g, radii, _ = W.config2()
        g2, _, _ = W.config2(item=1)
        return g, g2, radii, 12, 1
    if name == "n256_m41":  # the last radius workgroup merges; separate update
        g, radii, steps = W.config2(n=256, m=41, steps=6)
        g2, _, _ = W.config2(item=1, n=256, m=41, steps=6)
        return g, g2, radii, steps, 1
    if name == "n65536_m9":  # two-pass radius transforms and their merge launch
        g, radii, steps = W.config2(n=1 << 16, m=9, steps=3)
        g2, _, _ = W.config2(item=1, n=1 << 16, m=9, steps=3)
        return g, g2, radii, steps, 1
    if name == "batch4_n4096":  # batched plan
        g = np.stack([W.config3(i) for i in range(4)])
        g2 = np.stack([W.config3(i + 10) for i in range(4)])
        return g, g2, W.uniform_radii(64), 5, 4
    raise ValueError(name)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["n1024_m100", "n16384_m1000", "n256_m41", "n65536_m9", "batch4_n4096"])
def test_graph_replays_equal_eager(name, prec):
    g, g2, radii, steps, batch = _case(name)
    n = g.shape[-1]
    print(f"case graph {name} steps={steps} {prec}", flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    with Plan(n, radii, precision=prec, stream=stream, batch=batch) as plan:
        eager = to_numpy(plan.decompose(_dev(g), steps))
        eager2 = to_numpy(plan.decompose(_dev(g2), steps))
        sig = _dev(g)
        with plan.graph(sig, steps) as gr:
            for rep in range(3):
                gr.launch()
                gr.status()
                r = to_numpy(gr.result)
                for k in FIELDS:
                    assert np.array_equal(r[k], eager[k], equal_nan=True), (rep, k)
                # eager work of the same plan, and of torch, between the replays
                other = to_numpy(plan.decompose(_dev(g2), steps))
                assert np.array_equal(other["coef"], eager2["coef"])
                (sig * 2).sum().item()
                torch.cuda.synchronize()
            sig.copy_(_dev(g2))
            gr.launch()
            gr.status()
            r = to_numpy(gr.result)
            for k in FIELDS:
                assert np.array_equal(r[k], eager2[k], equal_nan=True), ("new signal", k)
            if batch == 1 and n <= 4096:
                compare(_Res(r), O.decompose(g2, radii, steps), TOL[prec], signal=g2, radii=radii)
            bad = g.copy()
            bad.reshape(-1)[7] = np.nan
            sig.copy_(_dev(bad))
            gr.launch()
            with pytest.raises(AfdError) as ei:
                gr.status()
            assert ei.value.status == 2
            sig.copy_(_dev(g))
            gr.launch()
            gr.status()
            r = to_numpy(gr.result)
            assert np.array_equal(r["coef"], eager["coef"])


def test_graph_needs_device_buffers():
    radii = W.uniform_radii(9)
    with Plan(64, radii) as plan:
        with pytest.raises(ValueError):
            plan.graph(np.ones(64, complex), 2)


class _Res:
    def __init__(self, d):
        self.__dict__.update(d)
