"""The FP64 oracle against closed forms, brute force, invariants and the paper's tables.

Also: every planted mistake (a dropped term, a wrong sign, a swapped index, a
conjugate lost) must make at least one pin fail, so the battery is shown to be
able to catch the kinds of slips that could hide in the oracle.
"""
import types

import numpy as np
import pytest

import oracle as O
from oracle import afd_oracle as OA
from tests import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(O)


def test_first_a_zero_requires_zero_radius():
    with pytest.raises(ValueError):
        O.decompose(np.ones(8, complex), np.array([0.1, 0.2]), 1, first_a_zero=True)


# ---------------------------------------------------------------- planted mistakes
def _mutant(**overrides):
    ns = types.SimpleNamespace(**{name: getattr(OA, name) for name in OA.__all__})
    for k, v in overrides.items():
        setattr(ns, k, v)

    # decompose must route through the mutated helpers
    def decompose(G, radii, steps, first_a_zero=False, forced=None, form="fft"):
        G = np.asarray(G, dtype=np.complex128).copy()
        radii = np.asarray(radii, dtype=np.float64)
        N = G.shape[0]
        grid = ns.grid_fft if form == "fft" else ns.grid_direct
        idx, a_l, c_l, e_l, mg = [], [], [], [ns.energy(G)], []
        zero = int(np.nonzero(radii == 0.0)[0][0]) if first_a_zero else None
        for k in range(steps):
            V = grid(G, radii)
            f = tuple(forced[k]) if forced is not None else ((zero, 0) if first_a_zero and k == 0 else None)
            (m, j), margin = ns.select(V, f)
            a = radii[m] * np.exp(2j * np.pi * j / N)
            G = ns.update(G, a, V[m, j])
            idx.append((m, j)); a_l.append(a); c_l.append(V[m, j]); e_l.append(ns.energy(G)); mg.append(margin)
        return OA.Decomposition(idx, a_l, c_l, e_l, mg, G)

    def decompose_nu(G, turns, weights, radii, n, steps, first_a_zero=False, forced=None, form="direct"):
        G = np.asarray(G, dtype=np.complex128).copy()
        radii = np.asarray(radii, dtype=np.float64)
        z = ns.sample_points(turns)
        grid = ns.grid_direct_nu if form == "direct" else ns.grid_series_nu
        idx, a_l, c_l, e_l, mg = [], [], [], [ns.energy_nu(G, weights)], []
        zero = int(np.nonzero(radii == 0.0)[0][0]) if first_a_zero else None
        for k in range(steps):
            V = grid(G, turns, weights, radii, n)
            f = tuple(forced[k]) if forced is not None else ((zero, 0) if first_a_zero and k == 0 else None)
            (m, j), margin = ns.select(V, f)
            a = radii[m] * np.exp(2j * np.pi * j / n)
            G = ns.update_nu(G, z, a, V[m, j])
            idx.append((m, j)); a_l.append(a); c_l.append(V[m, j]); e_l.append(ns.energy_nu(G, weights))
            mg.append(margin)
        return OA.Decomposition(idx, a_l, c_l, e_l, mg, G)

    if "decompose" not in overrides:
        ns.decompose = decompose
    if "decompose_nu" not in overrides:
        ns.decompose_nu = decompose_nu
    return ns


def _grid_fft_forward_sign(G, radii):
    N = len(G)
    c = np.fft.fft(G)
    return np.array([np.sqrt(1 - r * r) / (1 - r ** N) * np.fft.fft(c * OA._radius_power(r, N)) / N
                     for r in radii])


def _grid_fft_no_alias(G, radii):
    c = np.fft.fft(G)
    return np.array([np.sqrt(1 - r * r) * np.fft.ifft(c * OA._radius_power(r, len(G))) for r in radii])


def _grid_fft_no_sqrt(G, radii):
    N = len(G)
    c = np.fft.fft(G)
    return np.array([1 / (1 - r ** N) * np.fft.ifft(c * OA._radius_power(r, N)) for r in radii])


def _grid_fft_shifted_weight(G, radii):
    N = len(G)
    c = np.fft.fft(G)
    return np.array([np.sqrt(1 - r * r) / (1 - r ** N) * np.fft.ifft(c * r ** np.arange(1, N + 1)) for r in radii])


def _szego_no_conj(a, z):
    return np.sqrt(1 - abs(a) ** 2) / (1 - a * z)


def _update_wrong_factor(G, a, coef):
    z = OA.circle_points(len(G))
    return (G - coef * OA.szego(a, z)) * (1 - a * z) / (z - a)


def _update_no_subtract(G, a, coef):
    z = OA.circle_points(len(G))
    return G * (1 - np.conj(a) * z) / (z - a)


def _select_last_max(V, forced=None):
    if forced is not None:
        return tuple(forced), float("nan")
    M, N = V.shape
    P = np.abs(V.ravel()) ** 2
    f = len(P) - 1 - int(np.argmax(P[::-1]))
    return (f // N, f % N), 0.0


def _select_transposed(V, forced=None):
    if forced is not None:
        return tuple(forced), float("nan")
    M, N = V.shape
    P = np.abs(V.ravel()) ** 2
    f = int(np.argmax(P))
    return (f % M, f // M), 0.0


def _analytic_szego_projection(x):
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    h = np.zeros(n)
    h[: n // 2] = 1.0
    return np.fft.ifft(np.fft.fft(x) * h)


def _analytic_negative_bins(x):
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    h = np.zeros(n)
    h[0] = 1.0
    h[n // 2 + 1:] = 2.0
    h[n // 2] = 1.0
    return np.fft.ifft(np.fft.fft(x) * h)


def _analytic_no_nyquist(x):
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    h = np.zeros(n)
    h[0] = 1.0
    h[1:n // 2] = 2.0
    return np.fft.ifft(np.fft.fft(x) * h)


def _relative_errors_off_by_one(G, coefs, a_list):
    return np.concatenate([[1.0], OA.relative_errors(G, coefs, a_list)[:-1]])


def _energy_sum(G):
    return float(np.sum(np.abs(G) ** 2))


def _grid_direct_nu_unweighted(G, turns, weights, radii, n):
    return OA.grid_direct_nu(G, turns, np.full(len(G), 1.0 / len(G)), radii, n)


def _nudft_plus_sign(u, turns, count):
    return np.conj(OA.nudft(np.conj(u), turns, count))


def _update_nu_uniform_points(G, z, a, coef):
    return OA.update_nu(G, OA.circle_points(len(G)), a, coef)


def _energy_nu_unweighted(G, weights):
    return OA.energy(G)


def _relative_errors_nu_uniform_norm(G, turns, weights, coefs, a_list):
    return OA.relative_errors_nu(G, turns, np.full(len(G), 1.0 / len(G)), coefs, a_list)


MUTANTS = {
    "forward-sign inverse DFT": dict(grid_fft=_grid_fft_forward_sign),
    "aliasing factor 1/(1-r^N) dropped": dict(grid_fft=_grid_fft_no_alias),
    "sqrt(1-r^2) dropped": dict(grid_fft=_grid_fft_no_sqrt),
    "weights r^(l+1)": dict(grid_fft=_grid_fft_shifted_weight),
    "szego kernel without conjugate": dict(szego=_szego_no_conj),
    "Moebius factor without conjugate": dict(update=_update_wrong_factor),
    "projection not subtracted": dict(update=_update_no_subtract),
    "ties to the last maximum": dict(select=_select_last_max),
    "flat index transposed": dict(select=_select_transposed),
    "energy without 1/N": dict(energy=_energy_sum),
    "analytic part as the Szego projection": dict(analytic_part=_analytic_szego_projection),
    "analytic part keeps the negative bins": dict(analytic_part=_analytic_negative_bins),
    "analytic part drops the Nyquist bin": dict(analytic_part=_analytic_no_nyquist),
    "relative errors shifted by one step": dict(relative_errors=_relative_errors_off_by_one),
    "quadrature weights dropped": dict(grid_direct_nu=_grid_direct_nu_unweighted),
    "non-uniform DFT with the inverse sign": dict(nudft=_nudft_plus_sign),
    "non-uniform update at the uniform points": dict(update_nu=_update_nu_uniform_points),
    "quadrature energy without weights": dict(energy_nu=_energy_nu_unweighted),
    "non-uniform relative errors in the unweighted norm": dict(relative_errors_nu=_relative_errors_nu_uniform_norm),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    ns = _mutant(**MUTANTS[name])
    failures = 0
    for pin in P.ALL_PINS:
        try:
            pin(ns)
        except (AssertionError, ValueError, IndexError, FloatingPointError):
            failures += 1
    assert failures > 0, f"no pin caught the planted mistake: {name}"
