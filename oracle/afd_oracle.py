"""FP64 CPU oracle for the FFT-based Core-AFD maximal-selection loop.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously-correct
reference that the GPU path is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and the two
share no code.

Paper: Gao, Ku, Qian, "Fast algorithm of adaptive Fourier series"
(arXiv 1711.08604).  Equations are cited by section and by the label the
paper's source gives them (the compiled number in brackets):

* Sec. 2, eq. (1) [1]      inner product on the circle
* Sec. 2, eq. (2) [2]      Takenaka-Malmquist system B_k
* Sec. 2, eqs. (3)-(4)     one-step Core-AFD decomposition, e_a
* Sec. 2, eq. ak [8]       maximal selection principle
* Sec. 2, eq. (7) [7]      remainder recursion (Blaschke / Moebius division)
* Sec. 2, eq. (9) [9]      energy identity
* Sec. 3.1, eq. term81 [14] rectangle-rule grid value <G, e_{a_j}>~
* Sec. 3.1, eqs. ku12 [15], term4 [16], rcl [17]  aliased geometric series,
  forward DFT of the samples, per-radius inverse DFT
* Sec. 3.2, Steps 1 and 2  all grid values, then the maximum
* Sec. 4, eq. er [24]      relative error delta
* Sec. 4 (case 2)          analytic (H^2) part of real boundary samples
* Sec. 3.2, remark after Step 2  non-uniform samples through a non-uniform DFT

Readings adopted where the paper is silent or inconsistent (each is also
listed with its reason in the design notes):

* The circle measure is dt/2pi (so e_a has unit continuous norm and the
  discrete inner product is (1/N) * sum); the stray 1/sqrt(2pi) of eq. (2)
  and the 2pi constants of eqs. ku12/rcl are replaced by this normalisation
  and by N respectively.  Every function takes any N: the aliased series of
  Sec. 3.1 does not use N = 2^K, which the paper's closing remark extends to
  N = p^K (pinned at N = 3^K as well).
* Grid order is radius-major: flat index f = m*N + j, a_{m,j} = r_m e^{2 pi i j/N}.
  Ties in the maximal selection go to the lowest flat index (the first
  maximum of a linear scan, Sec. 3.2 Step 2).
* 0^0 = 1 for the radius r = 0.
* Optional first_a_zero forces a_1 = 0 (the convention the paper's Sec. 4
  tables follow: their first row is exactly 1.0000 on zero-mean signals).

Parity status: every function here is pinned by tests against closed forms,
brute force or the paper's printed tables (see tests/test_oracle_pins.py);
none is "parity unpinned".
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "circle_points",
    "szego",
    "grid_direct",
    "grid_fft",
    "select",
    "update",
    "energy",
    "decompose",
    "select_streamed",
    "decompose_streamed",
    "tm_basis",
    "partial_sum",
    "relative_errors",
    "analytic_part",
    "sample_points",
    "trapezoid_weights",
    "grid_direct_nu",
    "nudft",
    "grid_series_nu",
    "update_nu",
    "energy_nu",
    "decompose_nu",
    "relative_errors_nu",
    "Decomposition",
]


def circle_points(n: int) -> np.ndarray:
    """Uniform samples z_n = e^{2 pi i n / N}, n = 0..N-1 (Sec. 3.1, t_m = 2 pi m / 2^K)."""
    t = 2.0 * np.pi * np.arange(n) / n
    return np.exp(1j * t)


def szego(a: complex, z: np.ndarray) -> np.ndarray:
    """Normalised Szego kernel e_a(z) = sqrt(1-|a|^2) / (1 - conj(a) z) (Sec. 2, after eq. (3))."""
    a = complex(a)
    return np.sqrt(1.0 - abs(a) ** 2) / (1.0 - np.conj(a) * z)


def _radius_power(r: float, n: int) -> np.ndarray:
    """r^l for l = 0..n-1 with 0^0 = 1."""
    w = np.empty(n, dtype=np.float64)
    w[0] = 1.0
    if n > 1:
        w[1:] = float(r) ** np.arange(1, n, dtype=np.float64)
    return w


def grid_direct(G: np.ndarray, radii: np.ndarray) -> np.ndarray:
    """Grid values by the rectangle rule, Sec. 3.1 eq. term81.

    V[m, j] = (sqrt(1 - r_m^2) / N) * sum_n G[n] / (1 - a_{m,j} e^{-2 pi i n/N}),
    with a_{m,j} = r_m e^{2 pi i j/N}.  Cost O(M N^2): the direct form the paper
    compares against (Sec. 3.3 remark), used here as the brute-force reference.
    """
    G = np.asarray(G, dtype=np.complex128)
    N = G.shape[0]
    z = circle_points(N)
    V = np.empty((len(radii), N), dtype=np.complex128)
    for m, r in enumerate(radii):
        a = r * z  # a_{m,j}, j = 0..N-1
        # denominator[j, n] = 1 - a_j * conj(z_n)
        den = 1.0 - np.outer(a, np.conj(z))
        V[m] = np.sqrt(1.0 - r * r) / N * (den ** -1 @ G)
    return V


def grid_fft(G: np.ndarray, radii: np.ndarray) -> np.ndarray:
    """Grid values by the FFT form, Sec. 3.1 eqs. term4 and rcl.

    c = DFT(G) (eq. term4, unnormalised, e^{-2 pi i l m/N}); for each radius the
    inverse DFT of f(l) = r^l c_l, scaled by sqrt(1-r^2) / (N (1 - r^N))
    (eq. rcl with the constant N, see the module notes).  numpy's ifft carries
    the 1/N.
    """
    G = np.asarray(G, dtype=np.complex128)
    N = G.shape[0]
    c = np.fft.fft(G)
    V = np.empty((len(radii), N), dtype=np.complex128)
    for m, r in enumerate(radii):
        w = _radius_power(r, N)
        V[m] = np.sqrt(1.0 - r * r) / (1.0 - float(r) ** N) * np.fft.ifft(c * w)
    return V


def select(V: np.ndarray, forced: tuple[int, int] | None = None):
    """Maximal selection on the grid, Sec. 2 eq. ak and Sec. 3.2 Step 2.

    Returns ((m, j), margin) where (m, j) is the first maximiser of |V|^2 in
    radius-major order (lowest flat index) and margin = (P1 - P2) / P1 with
    P1 >= P2 the two largest values of |V|^2 over the grid (0 when P1 = 0).
    With `forced`, that index is taken instead and the margin is NaN.
    """
    M, N = V.shape
    if forced is not None:
        return (int(forced[0]), int(forced[1])), float("nan")
    P = (V.real ** 2 + V.imag ** 2).ravel()
    f = int(np.argmax(P))
    p1 = P[f]
    if P.size > 1:
        p2 = np.partition(P, P.size - 2)[P.size - 2]
    else:
        p2 = 0.0
    margin = float((p1 - p2) / p1) if p1 > 0 else 0.0
    return (f // N, f % N), margin


def update(G: np.ndarray, a: complex, coef: complex) -> np.ndarray:
    """Remainder recursion, Sec. 2 eq. (7).

    G_{k+1}(z) = (G_k(z) - coef * e_a(z)) * (1 - conj(a) z) / (z - a) on the samples.
    """
    z = circle_points(G.shape[0])
    return (G - coef * szego(a, z)) * (1.0 - np.conj(a) * z) / (z - a)


def energy(G: np.ndarray) -> float:
    """Discrete squared norm (1/N) sum |G[n]|^2 (the dt/2pi measure of eq. (1), rectangle rule)."""
    G = np.asarray(G)
    return float(np.mean(G.real ** 2 + G.imag ** 2))


class Decomposition:
    """Per-step record: indices (m_k, j_k), parameters a_k, coefficients
    <G_k, e_{a_k}>~, energies E_0..E_S (E_k = ||G_{k+1}||^2_N), margins and the
    final remainder G_{S+1}."""

    def __init__(self, index, a, coef, energy, margin, remainder):
        self.index = np.asarray(index, dtype=np.int64).reshape(-1, 2)
        self.a = np.asarray(a, dtype=np.complex128)
        self.coef = np.asarray(coef, dtype=np.complex128)
        self.energy = np.asarray(energy, dtype=np.float64)
        self.margin = np.asarray(margin, dtype=np.float64)
        self.remainder = np.asarray(remainder, dtype=np.complex128)

    @property
    def delta(self) -> np.ndarray:
        """Relative error after n = 1..S steps, Sec. 4 eq. er: ||G - S_n||^2 / ||G||^2.

        Equal to E_n / E_0 because the Blaschke factor is unimodular on the
        circle, so ||G - S_n||_N = ||G_{n+1}||_N at every sample (expansion (Sn)).
        """
        return self.energy[1:] / self.energy[0]


def decompose(G, radii, steps: int, first_a_zero: bool = False, forced=None,
              form: str = "fft") -> Decomposition:
    """Run `steps` steps of Core-AFD on the samples G (Sec. 2 and Sec. 3.2).

    Per step k: grid values (Step 1; `form` = "fft" for eqs. term4/rcl, "direct"
    for eq. term81), maximal selection (Step 2, eq. ak), coefficient
    c_k = <G_k, e_{a_k}>~ (eq. (3)), remainder update (eq. (7)) and energy.
    `forced` (steps x 2 indices) replaces the selection at every step (replay);
    `first_a_zero` replaces it at step 1 by the r = 0 grid point.
    """
    G = np.asarray(G, dtype=np.complex128).copy()
    radii = np.asarray(radii, dtype=np.float64)
    N = G.shape[0]
    grid = grid_fft if form == "fft" else grid_direct
    zero_idx = None
    if first_a_zero:
        hits = np.nonzero(radii == 0.0)[0]
        if hits.size == 0:
            raise ValueError("first_a_zero needs a radius equal to 0")
        zero_idx = int(hits[0])
    idx, a_list, c_list, e_list, mg = [], [], [], [energy(G)], []
    for k in range(steps):
        V = grid(G, radii)
        f = None
        if forced is not None:
            f = tuple(forced[k])
        elif first_a_zero and k == 0:
            f = (zero_idx, 0)
        (m, j), margin = select(V, f)
        a = radii[m] * np.exp(2j * np.pi * j / N)
        coef = V[m, j]
        G = update(G, a, coef)
        idx.append((m, j))
        a_list.append(a)
        c_list.append(coef)
        e_list.append(energy(G))
        mg.append(margin)
    return Decomposition(idx, a_list, c_list, e_list, mg, G)


def select_streamed(G: np.ndarray, radii: np.ndarray, chunk: int = 16, workers: int = 1):
    """Sec. 3.2 Steps 1 and 2 without holding the whole M x N grid.

    The grid values of eqs. term4/rcl are formed `chunk` radii at a time by
    grid_fft (each radius' row is computed exactly as there), and every chunk
    is reduced to its largest |V|^2 (first maximiser in radius-major order),
    its second largest |V|^2 and the grid value at the maximiser.  Chunks are
    combined in index order, so the result is select(grid_fft(G, radii))
    bit for bit: ((m, j), margin) plus V[m, j] and P1 = |V[m, j]|^2.
    `workers` > 1 evaluates chunks on that many threads (the FFTs release
    the interpreter lock); the combination order does not change.
    """
    G = np.asarray(G, dtype=np.complex128)
    radii = np.asarray(radii, dtype=np.float64)
    N = G.shape[0]
    starts = list(range(0, len(radii), chunk))

    def part(m0):
        V = grid_fft(G, radii[m0:m0 + chunk])
        P = (V.real ** 2 + V.imag ** 2).ravel()
        f = int(np.argmax(P))
        p2 = np.partition(P, P.size - 2)[P.size - 2] if P.size > 1 else -1.0
        return P[f], p2, m0 * N + f, V.ravel()[f]

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            parts = list(ex.map(part, starts))
    else:
        parts = [part(m0) for m0 in starts]
    p1, p2, f, v = parts[0]
    for q1, q2, g, w in parts[1:]:
        if q1 > p1:  # strictly larger: equal values keep the lower flat index
            p2 = max(p1, q2)
            p1, f, v = q1, g, w
        else:
            p2 = max(p2, q1)
    if len(radii) * N < 2:
        p2 = 0.0
    margin = float((p1 - p2) / p1) if p1 > 0 else 0.0
    return (f // N, f % N), margin, complex(v), float(p1)


def decompose_streamed(G, radii, steps: int, forced=None, chunk: int = 16, workers: int = 1) -> Decomposition:
    """decompose() with the grid streamed by select_streamed: the same loop
    (FFT form, maximal selection, coefficient, eq. (7) update, energy) for
    grids too large to hold; results equal decompose()'s bit for bit.
    `forced` (steps x 2) replaces the selection as in decompose()."""
    G = np.asarray(G, dtype=np.complex128).copy()
    radii = np.asarray(radii, dtype=np.float64)
    N = G.shape[0]
    idx, a_list, c_list, e_list, mg = [], [], [], [energy(G)], []
    for k in range(steps):
        if forced is not None:
            m, j = int(forced[k][0]), int(forced[k][1])
            coef = grid_fft(G, radii[m:m + 1])[0, j]
            margin = float("nan")
        else:
            (m, j), margin, coef, _ = select_streamed(G, radii, chunk, workers)
        a = radii[m] * np.exp(2j * np.pi * j / N)
        G = update(G, a, coef)
        idx.append((m, j))
        a_list.append(a)
        c_list.append(coef)
        e_list.append(energy(G))
        mg.append(margin)
    return Decomposition(idx, a_list, c_list, e_list, mg, G)


def tm_basis(a_list, z: np.ndarray) -> np.ndarray:
    """Takenaka-Malmquist system on the samples, Sec. 2 eq. (2) with the dt/2pi
    normalisation: B_k(z) = e_{a_k}(z) * prod_{l<k} (z - a_l) / (1 - conj(a_l) z).
    Returns an array of shape (len(a_list), len(z))."""
    out = np.empty((len(a_list), len(z)), dtype=np.complex128)
    blaschke = np.ones_like(z, dtype=np.complex128)
    for k, a in enumerate(a_list):
        out[k] = szego(a, z) * blaschke
        blaschke = blaschke * (z - a) / (1.0 - np.conj(a) * z)
    return out


def partial_sum(coefs, a_list, z: np.ndarray) -> np.ndarray:
    """S_n = sum_k <G_k, e_{a_k}> B_k on the samples (Sec. 2 expansion (Sn))."""
    B = tm_basis(a_list, z)
    return np.asarray(coefs) @ B


def relative_errors(G, coefs, a_list) -> np.ndarray:
    """delta_n = ||G - S_n||_N^2 / ||G||_N^2 for n = 1..len(a_list) (Sec. 4, eq. er),
    with S_n the partial sum of expansion (Sn) on the N samples."""
    G = np.asarray(G, dtype=np.complex128)
    z = circle_points(G.shape[0])
    B = tm_basis(a_list, z)
    S = np.zeros_like(G)
    out = []
    for k in range(len(a_list)):
        S = S + coefs[k] * B[k]
        out.append(energy(G - S) / energy(G))
    return np.asarray(out, dtype=np.float64)


def analytic_part(x) -> np.ndarray:
    """Boundary samples of the H^2 (analytic) function whose real part matches
    real samples x, by the DFT: bin 0 and (N even) bin N/2 kept, bins
    1..N/2-1 doubled, the negative-frequency bins N/2+1..N-1 removed.  This is
    how the non-analytic test function of Sec. 4 (case 2) is brought into the
    Hardy space before the decomposition."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    h = np.zeros(n)
    h[0] = 1.0
    if n % 2 == 0:
        h[1:n // 2] = 2.0
        h[n // 2] = 1.0
    else:
        h[1:(n + 1) // 2] = 2.0
    return np.fft.ifft(np.fft.fft(x) * h)


# ---------------------------------------------------------------- non-uniform samples
# Sec. 3.2, remark after Step 2: with samples at non-uniform positions the
# algorithm carries over once the DFT of the samples is replaced by a
# non-uniform DFT.  Readings (listed with the others in the design notes):
# * sample positions are given in turns t_n in [0, 1): z_n = e^{2 pi i t_n};
# * the discrete inner product is the quadrature sum_n w_n G(z_n) conj(F(z_n))
#   with weights w_n standing for dt/2pi (sum 1 for a consistent rule); the
#   uniform case is w_n = 1/N at t_n = n/N;
# * the selection grid stays the uniform polar grid a_{m,j} = r_m e^{2 pi i j/N}.


def sample_points(turns) -> np.ndarray:
    """z_n = e^{2 pi i t_n}, with the angle formed and the cosine and sine taken
    in extended precision, then rounded once to double."""
    t = np.asarray(turns, dtype=np.longdouble)
    two_pi = np.longdouble("6.283185307179586476925286766559005768")
    ang = two_pi * t
    return (np.cos(ang).astype(np.float64) + 1j * np.sin(ang).astype(np.float64)).astype(np.complex128)


def trapezoid_weights(turns) -> np.ndarray:
    """Periodic trapezoidal weights w_n = (t_{n+1} - t_{n-1}) / 2 for strictly
    increasing positions in [0, 1) (t_N = t_0 + 1, t_{-1} = t_{N-1} - 1); they
    sum to 1 and equal 1/N on the uniform positions."""
    t = np.asarray(turns, dtype=np.float64)
    if t.size == 1:
        return np.ones(1)
    nxt = np.concatenate([t[1:], [t[0] + 1.0]])
    prv = np.concatenate([[t[-1] - 1.0], t[:-1]])
    return (nxt - prv) / 2.0


def grid_direct_nu(G, turns, weights, radii, n: int) -> np.ndarray:
    """Grid values by the quadrature rule on non-uniform samples:
    V[m, j] = sqrt(1 - r_m^2) * sum_n w_n G_n / (1 - a_{m,j} conj(z_n)),
    a_{m,j} = r_m e^{2 pi i j/n} (eq. term81 with the weights in place of
    1/N).  Cost O(M n N_s): the plain definition."""
    G = np.asarray(G, dtype=np.complex128)
    w = np.asarray(weights, dtype=np.float64)
    z = sample_points(turns)
    grid = circle_points(n)
    V = np.empty((len(radii), n), dtype=np.complex128)
    for m, r in enumerate(radii):
        den = 1.0 - np.outer(r * grid, np.conj(z))
        V[m] = np.sqrt(1.0 - r * r) * ((den ** -1) @ (w * G))
    return V


def _turns_times(l, t):
    """frac(l * t) in [-1/2, 1/2] for integers l < 2^22 and doubles t: t splits
    into a 30-bit head (l * head is exact in double, so is its fractional
    part) and a tail (l * tail is below 2^-8 and rounds far below 1e-16)."""
    t = np.asarray(t, dtype=np.float64)
    head = np.round(t * 2.0 ** 30) / 2.0 ** 30
    tail = t - head
    ld = np.asarray(l, dtype=np.float64)
    prod = np.outer(ld, head)
    f = (prod - np.floor(prod)) + np.outer(ld, tail)
    return f - np.round(f)


def nudft(u, turns, count: int) -> np.ndarray:
    """Non-uniform DFT c_l = sum_n u_n e^{-2 pi i l t_n}, l = 0..count-1 (the
    series coefficients of the remark's non-uniform form of eq. term4); each
    phase from the fractional turn of l t_n, so its error does not grow with l."""
    u = np.asarray(u, dtype=np.complex128)
    out = np.empty(count, dtype=np.complex128)
    for l0 in range(0, count, 512):
        ls = np.arange(l0, min(count, l0 + 512))
        ph = 2.0 * np.pi * _turns_times(ls, turns)
        out[l0:l0 + len(ls)] = (np.cos(ph) - 1j * np.sin(ph)) @ u
    return out


def grid_series_nu(G, turns, weights, radii, n: int, terms: int = None) -> np.ndarray:
    """Grid values from the non-uniform DFT: with c_l = sum_n w_n G_n e^{-2 pi i l t_n},
    V[m, j] = sqrt(1 - r^2) sum_{l >= 0} r^l c_l e^{2 pi i l j/n} (the geometric
    expansion of the kernel, eq. ku12 without the periodicity that uniform
    samples give c_l).  The sum is cut at l < `terms` (default n), so this
    equals grid_direct_nu only where r^terms is negligible.  Since
    e^{2 pi i l j/n} depends on l mod n only, the terms l = l' + k n are
    summed into x[l'] = sum_k r^(l' + k n) c_(l' + k n), and the inverse DFT
    over j is numpy's (times n)."""
    terms = n if terms is None else int(terms)
    G = np.asarray(G, dtype=np.complex128)
    c = nudft(np.asarray(weights, dtype=np.float64) * G, turns, terms)
    V = np.empty((len(radii), n), dtype=np.complex128)
    for m, r in enumerate(radii):
        y = c * _radius_power(r, terms)
        x = np.zeros(n, dtype=np.complex128)
        for k0 in range(0, terms, n):
            part = y[k0:k0 + n]
            x[:len(part)] += part
        V[m] = np.sqrt(1.0 - r * r) * n * np.fft.ifft(x)
    return V


def update_nu(G, z, a: complex, coef: complex) -> np.ndarray:
    """Eq. (7) at the sample points z: (G - coef e_a(z)) (1 - conj(a) z) / (z - a)."""
    return (G - coef * szego(a, z)) * (1.0 - np.conj(a) * z) / (z - a)


def energy_nu(G, weights) -> float:
    """Quadrature squared norm sum_n w_n |G_n|^2."""
    G = np.asarray(G)
    return float(np.sum(np.asarray(weights, dtype=np.float64) * (G.real ** 2 + G.imag ** 2)))


def decompose_nu(G, turns, weights, radii, n: int, steps: int, first_a_zero: bool = False, forced=None,
                 form: str = "direct", terms: int = None) -> Decomposition:
    """Core-AFD on non-uniform samples: the loop of decompose() with the grid
    values of grid_direct_nu (`form` = "direct") or grid_series_nu ("series",
    cut at `terms`, default n), the update at the sample points and the
    quadrature energy.  Indices are (m, j) on the n-angle grid."""
    G = np.asarray(G, dtype=np.complex128).copy()
    radii = np.asarray(radii, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    z = sample_points(turns)
    if form == "direct":
        grid = grid_direct_nu
    else:
        def grid(G_, t_, w_, r_, n_):
            return grid_series_nu(G_, t_, w_, r_, n_, terms)
    zero_idx = None
    if first_a_zero:
        hits = np.nonzero(radii == 0.0)[0]
        if hits.size == 0:
            raise ValueError("first_a_zero needs a radius equal to 0")
        zero_idx = int(hits[0])
    idx, a_list, c_list, e_list, mg = [], [], [], [energy_nu(G, w)], []
    for k in range(steps):
        V = grid(G, turns, w, radii, n)
        f = None
        if forced is not None:
            f = tuple(forced[k])
        elif first_a_zero and k == 0:
            f = (zero_idx, 0)
        (m, j), margin = select(V, f)
        a = radii[m] * np.exp(2j * np.pi * j / n)
        coef = V[m, j]
        G = update_nu(G, z, a, coef)
        idx.append((m, j))
        a_list.append(a)
        c_list.append(coef)
        e_list.append(energy_nu(G, w))
        mg.append(margin)
    return Decomposition(idx, a_list, c_list, e_list, mg, G)


def relative_errors_nu(G, turns, weights, coefs, a_list) -> np.ndarray:
    """delta_n = ||G - S_n||^2 / ||G||^2 in the quadrature norm (Sec. 4, eq. er),
    with S_n the partial sum of expansion (Sn) at the sample points."""
    G = np.asarray(G, dtype=np.complex128)
    z = sample_points(turns)
    B = tm_basis(a_list, z)
    S = np.zeros_like(G)
    out = []
    for k in range(len(a_list)):
        S = S + coefs[k] * B[k]
        out.append(energy_nu(G - S, weights) / energy_nu(G, weights))
    return np.asarray(out, dtype=np.float64)
