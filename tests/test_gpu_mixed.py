"""Mixed-radix N (several of the primes 2, 3, 5, 7; N <= 16384): the run-time
pass kernels against the FP64 oracle, through the C ABI.  The paper's fast
algorithm does not depend on N being a power of two (its closing remark);
the oracle's FFT and direct forms take any N.

One size for every value-per-thread count E (6, 10, ..., 30) and the
largest sizes of several, free-running and replayed along the oracle's
trajectory, the r = 0 ring tie, a_1 = 0, the DFT reduction of radii = {0},
batches equal to lone signals bit for bit, captured graphs equal to eager
calls, reconstruction, and the errors of unsupported sizes."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.parity_tools import TOL, compare, compare_replay, to_numpy

torch = pytest.importorskip("torch")
from paper_1711_08604_amd import AfdError, Plan  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _signal(n, item, rmax=0.9, count=6):
    rng = W.rng_for(500 + n % 1000, item)
    g, _, _ = W.random_kernel_signal(rng, n, count, rmax)
    return W.add_noise(rng, g, 40.0)


SIZES = [  # (N, M, steps): E = 6, 10, 12, 14, 15, 18, 20, 21, 24, 28, 30 and large sizes of several
    (6, 3, 2), (10, 4, 3), (12, 5, 3), (14, 5, 3), (15, 6, 3), (36, 7, 3), (100, 11, 4), (147, 9, 4),
    (288, 13, 4), (392, 17, 4), (1000, 37, 5), (1536, 41, 5), (3087, 29, 4), (5625, 23, 4), (6000, 31, 4),
    (9604, 19, 4), (10125, 27, 4), (12288, 33, 4), (14336, 21, 4), (15360, 25, 4),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,m,steps", SIZES, ids=lambda v: str(v))
def test_free_run_and_replay(n, m, steps, prec):
    print(f"case mixed N={n} M={m} steps={steps} {prec}", flush=True)
    g = _signal(n, 0)
    if n > 6561:
        g = g - g.mean()  # keep step 1's maximum off a nearly flat small-radius ring
    radii = W.uniform_radii(m, 0.999) if n >= 81 else W.uniform_radii(m, 0.95)
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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [1000, 12288], ids=lambda v: f"N={v}")
def test_shaped_like_n16384_workload(n, prec):
    """M = 1000 radii uniform in [0, 0.999], 40 normalised Szego kernels +
    noise (the single-signal workload's recipe), 10 steps, every step
    replayed."""
    g, radii, _ = W.shaped_like_config2(n, 1000, 10, item=9)
    ref = O.decompose(g, radii, 10)
    with Plan(n, radii, precision=prec) as plan:
        res = plan.decompose(_dev(g), 10)
        compare(res, ref, TOL[prec], signal=g, radii=radii)
        rep = plan.replay(_dev(g), 10, ref.index.astype(np.int32))
        compare_replay(rep, ref, prec, radii=radii)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [12, 1000, 14336], ids=lambda v: f"N={v}")
def test_zero_radius_ring_tie(n, prec):
    """The r = 0 ring (all N values the same number) is the maximum of step
    1; the first maximum of the scan, flat index 0, must be chosen."""
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


@pytest.mark.parametrize("n", [360, 6000], ids=lambda v: f"N={v}")
def test_zero_radius_reduces_to_dft(n):
    """radii = {0}: index 0 every step and c_k = DFT(G)[k-1] / N."""
    g = _signal(n, 2)
    C = np.fft.fft(g)
    for prec in ("fp64", "fp32"):
        with Plan(n, [0.0], precision=prec) as plan:
            r = to_numpy(plan.decompose(_dev(g), 8))
        assert np.all(r["index"] == 0)
        assert np.max(np.abs(r["coef"] - C[:8] / n)) < 1e-12 * np.max(np.abs(C[:8] / n))


def test_first_a_zero():
    n = 1536
    g = _signal(n, 3)
    g = g - g.mean()
    radii = np.concatenate([[0.0], W.uniform_radii(30, 0.99)[1:]])
    ref = O.decompose(g, radii, 6, first_a_zero=True)
    for prec in ("fp64", "fp32"):
        with Plan(n, radii, precision=prec, first_a_zero=True) as plan:
            res = plan.decompose(_dev(g), 6)
            compare(res, ref, TOL[prec], signal=g, radii=radii, forced_first=True)
            assert tuple(to_numpy(res)["index"][0]) == (0, 0)


@pytest.mark.parametrize("n,jb", [(1000, 777), (15360, 12345)], ids=lambda v: str(v))
def test_single_kernel_recovery(n, jb):
    """G = w e_b with b on the grid: step 1 finds b and w (1 + rho)/(1 - rho)."""
    radii = np.round(np.arange(0, 100) / 100.0, 12)
    mb, w = 50, 0.7 - 1.1j
    b = radii[mb] * np.exp(2j * np.pi * jb / n)
    g = w * O.szego(b, O.circle_points(n))
    rho = abs(b) ** n
    for prec in ("fp64", "fp32"):
        with Plan(n, radii, precision=prec) as plan:
            r = to_numpy(plan.decompose(_dev(g), 1))
        assert tuple(r["index"][0]) == (mb, jb)
        assert abs(r["coef"][0] - w * (1 + rho) / (1 - rho)) < 1e-12 * abs(w)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_alone(prec):
    n, m, batch, steps = 1000, 33, 3, 4
    sigs = np.stack([_signal(n, 10 + i) for i in range(batch)])
    radii = W.uniform_radii(m, 0.999)
    with Plan(n, radii, precision=prec, batch=batch) as plan:
        rb = to_numpy(plan.decompose(_dev(sigs), steps))
    for i in range(batch):
        with Plan(n, radii, precision=prec) as plan:
            ra = to_numpy(plan.decompose(_dev(sigs[i]), steps))
        for k in ("index", "coef", "energy", "margin"):
            np.testing.assert_array_equal(rb[k][i], ra[k], err_msg=f"signal {i} field {k}")
    ref = O.decompose(sigs[1], radii, steps)
    assert np.array_equal(rb["index"][1], ref.index)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replays_equal_eager(prec):
    n, m, steps = 6000, 60, 5
    g = _signal(n, 4)
    radii = W.uniform_radii(m, 0.999)
    stream = torch.cuda.current_stream().cuda_stream
    with Plan(n, radii, precision=prec, stream=stream) as plan:
        eager = to_numpy(plan.decompose(_dev(g), steps))
        with plan.graph(_dev(g), steps) as gr:
            for rep in range(3):
                gr.launch()
                gr.status()
                got = to_numpy(gr.result)
                for k in ("index", "coef", "energy", "margin", "remainder"):
                    assert np.array_equal(got[k], eager[k], equal_nan=True), (rep, k)
                plan.decompose(_dev(g), 1)  # eager work of the same plan between the replays
                torch.cuda.synchronize()


def test_reconstruct_matches_oracle():
    n, steps = 1000, 8
    g = _signal(n, 5)
    radii = W.uniform_radii(40, 0.999)
    with Plan(n, radii, precision="fp64") as plan:
        d = plan.decompose(_dev(g), steps)
        r = to_numpy(d)
        S, delta = plan.reconstruct(r["a"], r["coef"], signal=g)
    z = O.circle_points(n)
    ref = O.partial_sum(r["coef"], r["a"], z)
    assert np.max(np.abs(np.asarray(S) - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(np.asarray(delta) - O.relative_errors(g, r["coef"], r["a"]))) < 1e-12


def test_unsupported_sizes():
    for n in (22, 1001, 121):            # a prime beyond 7
        with pytest.raises(AfdError):
            Plan(n, [0.5])
    for n in (35, 42, 3 << 14, 2 * 3 ** 8):  # primes whose product exceeds 30, too many threads, beyond 16384
        with pytest.raises(AfdError):
            Plan(n, [0.5])
    with Plan(1000, [0.0, 0.5]) as plan:
        with pytest.raises(AfdError):
            plan.analytic(np.ones(1000))  # the analytic part needs N = 2^K
