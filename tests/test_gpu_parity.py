"""GPU path (libafd through its C ABI) against the FP64 oracle.

Small and medium sizes, and the N = 16384, M = 1000 workload: every step
free-running (indices bit-exact while the oracle's lead exceeds 1e-6, then a
validity check of the near-tie choice) and every step replayed along the
oracle's trajectory, with the whole path (forward DFT, radius transforms,
selection, re-check) running on each replayed remainder and its own choice
checked against the oracle's grid maximum.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.parity_tools import TOL, compare, compare_replay, to_numpy

torch = pytest.importorskip("torch")
from paper_1711_08604_amd import AfdError, Plan  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def oracle_workers():
    """Threads for the oracle's streamed grids: the host cores this process may use, at most 16."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _signal(n, item, rmax=0.9, count=6):
    rng = W.rng_for(100 + n, item)
    g, _, _ = W.random_kernel_signal(rng, n, count, rmax)
    return W.add_noise(rng, g, 40.0)


SMALL = [  # (N, M, steps)  -- M chosen so the last radius block is ragged where blocks hold several radii
    (2, 3, 2), (4, 5, 3), (8, 7, 3), (16, 9, 4), (32, 17, 4), (64, 21, 5), (128, 33, 5), (256, 41, 6),
    (512, 51, 6), (1024, 100, 10), (2048, 65, 5), (4096, 64, 5), (8192, 48, 4), (16384, 40, 4),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,m,steps", SMALL, ids=lambda v: str(v))
def test_free_run_and_replay(n, m, steps, prec):
    print(f"case N={n} M={m} steps={steps} {prec}", flush=True)
    g = _signal(n, 0)
    radii = W.uniform_radii(m, 0.999) if n >= 64 else W.uniform_radii(m, 0.95)
    ref = O.decompose(g, radii, steps)
    with Plan(n, radii, precision=prec) as plan:
        res = plan.decompose(_dev(g), steps)
        torch.cuda.synchronize()
        compare(res, ref, TOL[prec], signal=g, radii=radii)
        rep = plan.replay(_dev(g), steps, ref.index.astype(np.int32))
        compare_replay(rep, ref, prec, radii=radii)
        r = to_numpy(res)
        if prec == "fp32":
            assert np.all(r["recheck_count"] >= 1)
            assert np.all((r["flags"] & 3) == 0), r["flags"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config1_full(prec):
    """N = 1024, 5 kernels, 100 radii m/100, 10 steps: every lead exceeds 1e-6."""
    g, radii, steps = W.config1()
    ref = O.decompose(g, radii, steps)
    assert np.all(ref.margin > 1e-6)
    with Plan(1024, radii, precision=prec) as plan:
        res = plan.decompose(_dev(g), steps)
        upto, rep = compare(res, ref, TOL[prec], signal=g, radii=radii)
        assert upto == steps
        # both precisions re-evaluate or carry FP64 coefficients: far inside the bar
        assert rep["worst_coef"] < 1e-11


_C2 = {}


def _config2_oracle():
    """The oracle's own 50-step trajectory on the N = 16384, M = 1000 workload
    (the grid streamed by radius chunks over threads; equal to decompose())."""
    if "ref" not in _C2:
        g, radii, steps = W.config2()
        ref = O.decompose_streamed(g, radii, steps, chunk=25, workers=oracle_workers())
        _C2["ref"] = (g, radii, steps, ref)
    return _C2["ref"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config2_every_step(prec):
    """N = 16384, M = 1000, 50 steps (the benchmark's launch configuration; in
    double precision the radius kernel takes its slots from the work queue).
    Every step is replayed along the oracle's trajectory with the whole path
    running: the path's own choice on each replayed remainder against the
    oracle's grid maximum, the coefficient at the forced point against the
    oracle's.  The free-running decomposition is compared until its first
    near-tie, and all 50 of its steps satisfy the aliasing-corrected energy
    identity."""
    g, radii, steps, ref = _config2_oracle()
    print(f"case config2 N=16384 M=1000 steps={steps} {prec}; oracle margins "
          f"min {np.min(ref.margin):.2e} median {np.median(ref.margin):.2e}", flush=True)
    with Plan(16384, radii, precision=prec) as plan:
        rep = plan.replay(_dev(g), steps, ref.index.astype(np.int32))
        report = compare_replay(rep, ref, prec, radii=radii)
        print("replay:", report, flush=True)
        assert report["picks_compared"] >= steps // 2
        res = plan.decompose(_dev(g), steps)
        upto, rr = compare(res, ref, TOL[prec], signal=g, radii=radii)
        print("free run:", rr, flush=True)
        r = to_numpy(res)
        # energy identity E_k = E_{k-1} - |c_k|^2 (1 - 3 rho)/(1 - rho), rho = |a_k|^N
        rho = np.abs(r["a"]) ** 16384
        pred = r["energy"][:-1] - np.abs(r["coef"]) ** 2 * (1 - 3 * rho) / (1 - rho)
        assert np.max(np.abs(pred - r["energy"][1:])) <= 1e-11 * r["energy"][0]
        assert np.all(r["energy"][1:] <= r["energy"][:-1] * (1 + 1e-12))
        if prec == "fp32":
            assert np.all((r["flags"] & 3) == 0), r["flags"]
            assert np.all(r["recheck_count"] >= 8)
            # the re-check band (4e-6 by default) must cover twice the measured FP32 error
            print("max FP32 error of |.|^2:", float(np.max(r["fp32_error"])), flush=True)
            assert np.max(r["fp32_error"]) * 2 < 4e-6
        else:
            # replayed with its own choices, the decomposition comes back bit for bit
            own = to_numpy(plan.replay(_dev(g), steps, r["index"].astype(np.int32)))
            for k in ("index", "a", "coef", "energy", "remainder"):
                assert np.array_equal(own[k], r[k]), k
            assert np.array_equal(own["pick_index"], r["index"])
            assert np.array_equal(own["pick_margin"], r["margin"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1 << 14, 1 << 15, 1 << 20], ids=lambda v: f"N={v}")
def test_zero_radius_ring_tie(n, prec):
    """radii = {0, 0.2, 0.4} and a dominant mean: the r = 0 ring (every one
    of its N values the same number) is the maximum of step 1, and the first
    maximum of the scan, flat index 0, must be chosen: on the LDS-resident
    radius kernel (2^14), the two-pass path (2^15) and the row pass (2^20)."""
    g = _signal(n, 1)
    g = 0.01 * (g - g.mean()) + 5.0
    radii = np.array([0.0, 0.2, 0.4])
    ref = O.decompose(g, radii, 2)
    assert tuple(ref.index[0]) == (0, 0) and ref.margin[0] == 0.0
    with Plan(n, radii, precision=prec) as plan:
        res = plan.decompose(_dev(g), 2)
        r = to_numpy(res)
        assert tuple(r["index"][0]) == (0, 0), r["index"][0]
        compare(res, ref, TOL[prec], signal=g, radii=radii)
        rep = to_numpy(plan.replay(_dev(g), 2, ref.index.astype(np.int32)))
        assert tuple(rep["pick_index"][0]) == (0, 0), rep["pick_index"][0]


def test_paper_case1_first_a_zero():
    """Table 4 of the paper on the GPU: f1, N = 1024, radii 0..0.8, a_1 = 0."""
    from tests.oracle_pins import load_golden
    radii = W.paper_radii()
    f1 = W.paper_f1(1024)
    ref = O.decompose(f1, radii, 10, first_a_zero=True)
    for prec in ("fp64", "fp32"):
        with Plan(1024, radii, precision=prec, first_a_zero=True) as plan:
            res = plan.decompose(_dev(f1), 10)
            compare(res, ref, TOL[prec], signal=f1, radii=radii, forced_first=True)
            d = to_numpy(res)
            delta = d["energy"][1:] / d["energy"][0]
            assert np.max(np.abs(delta - load_golden("paper_table4_f1_delta.txt"))) < 1.5e-3


def test_zero_radius_reduces_to_dft():
    n = 256
    g = _signal(n, 1)
    C = np.fft.fft(g)
    for prec in ("fp64", "fp32"):
        with Plan(n, [0.0], precision=prec) as plan:
            r = to_numpy(plan.decompose(_dev(g), 8))
        assert np.all(r["index"] == 0)
        assert np.max(np.abs(r["coef"] - C[:8] / n)) <= 1e-12 * np.sqrt(r["energy"][0])


def test_single_kernel_recovery():
    n = 1024
    radii = np.round(np.arange(100) / 100.0, 12)
    b = radii[50] * np.exp(2j * np.pi * 3 / n)
    w = 0.7 - 1.1j
    g = w * O.szego(b, O.circle_points(n))
    for prec in ("fp64", "fp32"):
        with Plan(n, radii, precision=prec) as plan:
            r = to_numpy(plan.decompose(_dev(g), 1))
        assert tuple(r["index"][0]) == (50, 3)
        rho = 0.5 ** n
        assert abs(r["coef"][0] - w * (1 + rho) / (1 - rho)) < 1e-13
        assert r["energy"][1] < 1e-25


def test_zero_signal_and_zero_steps():
    n = 512
    radii = W.uniform_radii(33)
    for prec in ("fp64", "fp32"):
        with Plan(n, radii, precision=prec) as plan:
            r = to_numpy(plan.decompose(_dev(np.zeros(n, complex)), 3))
            assert np.all(r["index"] == 0) and np.all(r["coef"] == 0) and np.all(r["energy"] == 0)
            r0 = to_numpy(plan.decompose(_dev(_signal(n, 2)), 0))
            assert r0["energy"].shape == (1,) and r0["energy"][0] > 0


def test_deterministic_and_host_device_equal():
    n, m, steps = 4096, 128, 6
    g = _signal(n, 3)
    radii = W.uniform_radii(m)
    for prec in ("fp64", "fp32"):
        with Plan(n, radii, precision=prec) as plan:
            a = to_numpy(plan.decompose(_dev(g), steps))
            b = to_numpy(plan.decompose(_dev(g), steps))
            c = to_numpy(plan.decompose(g, steps))  # host input and outputs
        for k in ("index", "a", "coef", "energy", "margin", "remainder"):
            assert np.array_equal(a[k], b[k], equal_nan=True), k
            assert np.array_equal(a[k], c[k], equal_nan=True), k


def test_errors_on_device():
    n = 64
    with Plan(n, W.uniform_radii(5), precision="fp64") as plan:
        bad = _signal(n, 4)
        bad[7] = np.nan
        with pytest.raises(AfdError) as ei:
            plan.decompose(_dev(bad), 2)
        assert ei.value.status == 2
        with pytest.raises(AfdError) as ei:
            plan.decompose(bad, 2)
        assert ei.value.status == 2
        with pytest.raises(AfdError) as ei:
            plan.replay(_dev(_signal(n, 4)), 1, np.array([[5, 0]], np.int32))
        assert ei.value.status == 1
        # the plan still works after the errors
        g = _signal(n, 5)
        ref = O.decompose(g, W.uniform_radii(5), 2)
        compare(plan.decompose(_dev(g), 2), ref, TOL["fp64"], signal=g, radii=W.uniform_radii(5))
