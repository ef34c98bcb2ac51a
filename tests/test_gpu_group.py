"""Batches of uneven N (afd_group_*): one decomposition each of plans of
different N, precision and sampling, captured into one HIP graph whose
branches run concurrently.  Every member equals its own afd_decompose bit for
bit on every launch (with other work of the plans and of torch between the
launches), a member is checked against the oracle, and a non-finite signal is
reported for its member only."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.parity_tools import TOL, compare, to_numpy

torch = pytest.importorskip("torch")
from paper_1711_08604_amd import AfdError, Group, Plan  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FIELDS = ("index", "a", "coef", "energy", "margin", "remainder", "recheck_count", "flags", "fp32_error")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _members(stream):
    """Plans of N = 256, 1024 (FP32), 4096, 729 (= 3^6), 16384 (FP32), 2^15,
    1000 and 12288 (mixed radix; FP32), 3125 (= 5^5, FP32), a batch of
    3 x 2048, and non-uniform samples on a 1024-angle grid."""
    out = []
    for k, (n, m, steps, prec) in enumerate(((256, 41, 6, "fp64"), (1024, 100, 8, "fp32"), (4096, 64, 5, "fp64"),
                                              (729, 60, 6, "fp32"), (16384, 200, 4, "fp32"),
                                              (1 << 15, 40, 3, "fp64"), (1000, 60, 5, "fp64"),
                                              (12288, 40, 3, "fp32"), (3125, 50, 4, "fp32"))):
        g, radii, _ = W.shaped_like_config2(n, m, steps, item=500 + k)
        out.append((Plan(n, radii, precision=prec, stream=stream), g, steps, radii))
    sigs = np.stack([W.shaped_like_config2(2048, 33, 4, item=520 + i)[0] for i in range(3)])
    out.append((Plan(2048, W.uniform_radii(33), precision="fp64", stream=stream, batch=3), sigs, 4, None))
    g, t = W.nonuniform_kernel_signal(1300, item=530)
    out.append((Plan(1024, W.uniform_radii(50, 0.95), precision="fp64", stream=stream, sample_turns=t), g, 5,
                None))
    return out


def test_group_equals_alone_and_oracle():
    stream = torch.cuda.current_stream().cuda_stream
    members = _members(stream)
    alone = [to_numpy(p.decompose(_dev(g), steps)) for p, g, steps, _ in members]
    sigs = [_dev(g) for _, g, _, _ in members]
    with Group([(p, s, steps) for (p, _, steps, _), s in zip(members, sigs)]) as grp:
        for rep in range(3):
            print(f"case group launch {rep}", flush=True)
            grp.launch()
            grp.status()
            for i, res in enumerate(grp.results):
                r = to_numpy(res)
                for k in FIELDS:
                    assert np.array_equal(r[k], alone[i][k], equal_nan=True), (rep, i, k)
            # other work of the same plans, and of torch, between the launches
            p, g, steps, _ = members[1]
            assert np.array_equal(to_numpy(p.decompose(_dev(g), steps))["coef"], alone[1]["coef"])
            (sigs[0] * 2).sum().item()
            torch.cuda.synchronize()
        p, g, steps, radii = members[0]
        compare(grp.results[0], O.decompose(g, radii, steps), TOL["fp64"], signal=g, radii=radii)
        # a non-finite signal fails its member only
        bad = members[2][1].copy()
        bad[5] = np.nan
        sigs[2].copy_(_dev(bad))
        grp.launch()
        with pytest.raises(AfdError) as ei:
            grp.status()
        assert ei.value.status == 2
        r = to_numpy(grp.results[3])
        assert np.array_equal(r["coef"], alone[3]["coef"])
    for p, _, _, _ in members:
        p.close()


def test_group_rejects():
    stream = torch.cuda.current_stream().cuda_stream
    g, radii, steps = W.shaped_like_config2(256, 9, 2, item=540)
    with Plan(256, radii, stream=stream) as p:
        s = _dev(g)
        with pytest.raises(AfdError):
            Group([(p, s, steps), (p, s, steps)])      # a plan twice
        with pytest.raises(ValueError):
            Group([(p, g, steps)])                      # host signal
