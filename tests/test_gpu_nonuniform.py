"""Non-uniform samples (Sec. 3.2, the remark after Step 2) on the GPU against
the FP64 oracle's quadrature form.

Jittered and clustered positions with trapezoidal weights (or given
weights), every step free-running and replayed along the oracle's
trajectory, the r = 0 ring tie, a_1 = 0, uniform positions against the
uniform oracle, captured graphs against eager calls, and the errors of what
a non-uniform plan does not support; reconstruction at the sample points.  The largest radius of each grid is
one whose kernel series is negligible from l = N on (the plan rejects
others)."""
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


CASES = [  # (N grid angles, samples, M, steps, largest radius, positions)
    (64, 80, 9, 4, 0.5, "jitter"),
    (256, 300, 21, 5, 0.8, "cluster"),
    (1024, 1500, 60, 6, 0.95, "jitter"),
    (4096, 5000, 50, 5, 0.985, "cluster"),
    (8192, 9000, 30, 3, 0.993, "jitter"),
]


_REF = {}


def _oracle(g, t, w, radii, n, steps, key):
    # the quadrature rule itself where it is affordable, else the pinned series
    # form; one oracle run serves both precisions
    if key not in _REF:
        form = "direct" if n * len(t) * len(radii) <= 2e8 else "series"
        _REF[key] = O.decompose_nu(g, t, w, radii, n, steps, form=form)
    return _REF[key]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ns,m,steps,rmax,kind", CASES, ids=lambda v: str(v))
def test_free_run_and_replay(n, ns, m, steps, rmax, kind, prec):
    print(f"case nonuniform N={n} samples={ns} M={m} steps={steps} {kind} {prec}", flush=True)
    g, t = W.nonuniform_kernel_signal(ns, item=n, kind=kind)
    w = O.trapezoid_weights(t)
    radii = W.uniform_radii(m, rmax)
    ref = _oracle(g, t, w, radii, n, steps, key=(n, ns, m, steps, rmax, kind))
    with Plan(n, radii, precision=prec, sample_turns=t) as plan:
        res = plan.decompose(_dev(g), steps)
        compare(res, ref, TOL[prec], signal=g, radii=radii, nonuniform=(t, w, n))
        assert to_numpy(res)["remainder"].shape == (ns,)
        rep = plan.replay(_dev(g), steps, ref.index.astype(np.int32))
        compare_replay(rep, ref, prec, radii=radii)


def test_given_weights():
    """Explicit quadrature weights (not the trapezoid's) reach the grid values,
    the update's energy and the re-check."""
    n, ns, m, steps = 512, 700, 24, 5
    g, t = W.nonuniform_kernel_signal(ns, item=5, kind="cluster")
    rng = W.rng_for(60, 0)
    w = O.trapezoid_weights(t) * (1.0 + 0.5 * rng.random(ns))
    radii = W.uniform_radii(m, 0.9)
    ref = O.decompose_nu(g, t, w, radii, n, steps)
    for prec in ("fp64", "fp32"):
        with Plan(n, radii, precision=prec, sample_turns=t, sample_weights=w) as plan:
            res = plan.decompose(_dev(g), steps)
            compare(res, ref, TOL[prec], signal=g, radii=radii, nonuniform=(t, w, n))


def test_uniform_positions_match_uniform_oracle():
    """t_n = n/N with w_n = 1/N: the non-uniform path computes the uniform
    decomposition (through the non-uniform DFT instead of the FFT)."""
    n, m, steps = 1024, 40, 6
    rng = W.rng_for(61, 0)
    g, _, _ = W.random_kernel_signal(rng, n, 6, 0.9)
    radii = W.uniform_radii(m, 0.95)
    t = np.arange(n) / n
    ref = O.decompose(g, radii, steps)
    with Plan(n, radii, sample_turns=t, sample_weights=np.full(n, 1.0 / n)) as plan:
        res = plan.decompose(_dev(g), steps)
        compare(res, ref, TOL["fp64"], signal=g, radii=radii)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_radius_ring_tie(prec):
    n, ns = 256, 333
    g, t = W.nonuniform_kernel_signal(ns, item=7)
    g = 0.01 * (g - g.mean()) + 5.0
    w = O.trapezoid_weights(t)
    radii = np.array([0.0, 0.2, 0.4])
    ref = O.decompose_nu(g, t, w, radii, n, 2)
    assert tuple(ref.index[0]) == (0, 0) and ref.margin[0] == 0.0
    with Plan(n, radii, precision=prec, sample_turns=t) as plan:
        r = to_numpy(plan.decompose(_dev(g), 2))
        assert tuple(r["index"][0]) == (0, 0), r["index"][0]
        rep = to_numpy(plan.replay(_dev(g), 2, ref.index.astype(np.int32)))
        assert tuple(rep["pick_index"][0]) == (0, 0), rep["pick_index"][0]


def test_first_a_zero():
    n, ns = 512, 640
    g, t = W.nonuniform_kernel_signal(ns, item=8, kind="cluster")
    w = O.trapezoid_weights(t)
    radii = W.uniform_radii(30, 0.9)
    ref = O.decompose_nu(g, t, w, radii, n, 5, first_a_zero=True)
    for prec in ("fp64", "fp32"):
        with Plan(n, radii, precision=prec, first_a_zero=True, sample_turns=t) as plan:
            res = plan.decompose(_dev(g), 5)
            compare(res, ref, TOL[prec], signal=g, radii=radii, forced_first=True, nonuniform=(t, w, n))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replays_equal_eager(prec):
    n, ns, steps = 1024, 1200, 5
    g, t = W.nonuniform_kernel_signal(ns, item=9)
    radii = W.uniform_radii(40, 0.95)
    stream = torch.cuda.current_stream().cuda_stream
    with Plan(n, radii, precision=prec, stream=stream, sample_turns=t) as plan:
        eager = to_numpy(plan.decompose(_dev(g), steps))
        with plan.graph(_dev(g), steps) as gr:
            for rep in range(3):
                gr.launch()
                gr.status()
                got = to_numpy(gr.result)
                for k in ("index", "coef", "energy", "margin", "remainder"):
                    assert np.array_equal(got[k], eager[k], equal_nan=True), (rep, k)
                plan.decompose(_dev(g), 1)
                torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ns,m,steps,rmax", [(1024, 1200, 40, 5, 0.999), (256, 300, 25, 4, 0.995)],
                         ids=lambda v: str(v))
def test_radii_near_one(n, ns, m, steps, rmax, prec):
    """Radii whose kernel series outlasts N terms (up to 0.999 on a 1024-angle
    grid: about 41600 terms): the non-uniform DFT computes K N modes and those
    radii read folded spectra; against the quadrature rule itself, every step
    free-running and replayed."""
    print(f"case nonuniform near one N={n} samples={ns} M={m} rmax={rmax} {prec}", flush=True)
    g, t = W.nonuniform_kernel_signal(ns, item=70, kind="cluster", rmax=0.95)
    w = O.trapezoid_weights(t)
    radii = W.uniform_radii(m, rmax)
    assert n * ns * m <= 2e8  # the oracle's quadrature rule itself (not the series cut at N)
    ref = _oracle(g, t, w, radii, n, steps, key=("near", n, ns, m, steps, rmax))
    with Plan(n, radii, precision=prec, sample_turns=t) as plan:
        res = plan.decompose(_dev(g), steps)
        compare(res, ref, TOL[prec], signal=g, radii=radii, nonuniform=(t, w, n))
        rep = plan.replay(_dev(g), steps, ref.index.astype(np.int32))
        compare_replay(rep, ref, prec, radii=radii)
        alone = to_numpy(res)
    # a batch of two on the same (clustered) positions: the first equals its lone decomposition
    g1, t1 = W.nonuniform_kernel_signal(ns, item=71, kind="cluster", rmax=0.95)
    assert np.array_equal(t1, t)
    with Plan(n, radii, precision=prec, sample_turns=t, batch=2) as plan:
        rb = to_numpy(plan.decompose(_dev(np.stack([g, g1])), steps))
    for k in ("index", "coef", "energy", "remainder"):
        assert np.array_equal(rb[k][0], alone[k], equal_nan=True), k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_alone(prec):
    """A batch of three signals on one set of positions: each equals its own
    decomposition bit for bit, and one is checked against the oracle."""
    n, ns, m, steps, batch = 1024, 1300, 40, 5, 3
    made = [W.nonuniform_kernel_signal(ns, item=40 + i, kind="cluster") for i in range(batch)]
    t = made[0][1]
    assert all(np.array_equal(ti, t) for _, ti in made)  # clustered positions do not depend on the item
    sigs = np.stack([g for g, _ in made])
    radii = W.uniform_radii(m, 0.95)
    with Plan(n, radii, precision=prec, sample_turns=t, batch=batch) as plan:
        rb = to_numpy(plan.decompose(_dev(sigs), steps))
        S, delta = plan.reconstruct(rb["a"], rb["coef"], signal=sigs)
    w = O.trapezoid_weights(t)
    for i in range(batch):
        # partial sums at the sample points and relative errors, per signal
        S_ref = O.partial_sum(rb["coef"][i], rb["a"][i], O.sample_points(t))
        assert np.max(np.abs(S[i] - S_ref)) < 1e-12 * np.max(np.abs(S_ref))
        assert np.max(np.abs(delta[i] - O.relative_errors_nu(sigs[i], t, w, rb["coef"][i], rb["a"][i]))) < 1e-12
    for i in range(batch):
        with Plan(n, radii, precision=prec, sample_turns=t) as plan:
            ra = to_numpy(plan.decompose(_dev(sigs[i]), steps))
        for k in ("index", "coef", "energy", "margin", "remainder"):
            np.testing.assert_array_equal(rb[k][i], ra[k], err_msg=f"signal {i} field {k}")
    ref = O.decompose_nu(sigs[1], t, w, radii, n, steps)
    assert np.array_equal(rb["index"][1], ref.index)


def test_unsupported():
    t = np.arange(100) / 100 + 0.001
    with pytest.raises(AfdError):
        Plan(256, [0.0, 0.99999], sample_turns=t)    # r = 0.99999 needs more than 2^18 terms
    with pytest.raises(AfdError):
        Plan(243, [0.0, 0.5], sample_turns=t)        # the grid must be 2^K
    with Plan(256, [0.0, 0.5], sample_turns=t) as plan:
        with pytest.raises(AfdError):
            plan.analytic(np.ones(256))
        bad = np.ones(100, complex)
        bad[3] = np.nan
        with pytest.raises(AfdError):
            plan.decompose(bad, 2)


def test_reconstruct_at_sample_points():
    """Partial sums at the sample points and the relative errors in the
    quadrature norm against the oracle; they equal E_n/E_0 of the GPU's own
    decomposition."""
    n, ns, steps = 1024, 1400, 8
    g, t = W.nonuniform_kernel_signal(ns, item=11, kind="cluster")
    w = O.trapezoid_weights(t)
    radii = W.uniform_radii(40, 0.95)
    with Plan(n, radii, sample_turns=t) as plan:
        r = to_numpy(plan.decompose(_dev(g), steps))
        S, delta = plan.reconstruct(r["a"], r["coef"], signal=g)
    S_ref = O.partial_sum(r["coef"], r["a"], O.sample_points(t))
    assert np.max(np.abs(S - S_ref)) < 1e-12 * np.max(np.abs(S_ref))
    assert np.max(np.abs(delta - O.relative_errors_nu(g, t, w, r["coef"], r["a"]))) < 1e-12
    assert np.max(np.abs(delta - r["energy"][1:] / r["energy"][0])) < 1e-11
