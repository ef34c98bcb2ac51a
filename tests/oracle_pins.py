"""Pins for the FP64 oracle: each check compares the oracle with something other
than itself (a closed form, brute force, an invariant, or a value the paper
prints).  Every pin takes the oracle namespace as an argument so that the
planted-mistake test can run the same battery on a deliberately broken copy.
"""
from __future__ import annotations

import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def load_golden(name):
    vals = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(float(line))
    return np.array(vals)


# ------------------------------------------------------------------ P0 brute force
def _term81_loops(G, radii):
    """Sec. 3.1 eq. term81 written out with plain Python loops (tiny inputs only)."""
    import cmath
    import math
    N = len(G)
    out = []
    for r in radii:
        row = []
        for j in range(N):
            a = r * cmath.exp(2j * math.pi * j / N)
            s = 0j
            for n in range(N):
                s += complex(G[n]) / (1 - a * cmath.exp(-2j * math.pi * n / N))
            row.append(math.sqrt(1 - r * r) / N * s)
        out.append(row)
    return np.array(out)


def pin_bruteforce_loops(O):
    """Oracle grid values (both forms) and one full decomposition step against
    pure-Python loops of eq. term81 and an exhaustive scan."""
    rng = _rng(1)
    N = 8
    G = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    radii = np.array([0.0, 0.3, 0.75, 0.95])
    ref = _term81_loops(G, radii)
    assert _rel(O.grid_direct(G, radii), ref) < 1e-13
    assert _rel(O.grid_fft(G, radii), ref) < 1e-13
    # exhaustive scan for the maximum, first occurrence in radius-major order
    best, bi = -1.0, None
    for m in range(len(radii)):
        for j in range(N):
            p = abs(ref[m, j]) ** 2
            if p > best:
                best, bi = p, (m, j)
    d = O.decompose(G, radii, 1)
    assert tuple(d.index[0]) == bi
    assert abs(d.coef[0] - ref[bi]) < 1e-13 * abs(ref[bi])
    assert abs(d.a[0] - radii[bi[0]] * np.exp(2j * np.pi * bi[1] / N)) < 1e-15


# ------------------------------------------------------------------ P1
def pin_fft_equals_direct(O):
    """The aliased geometric series (eqs. ku12/term1) is exact: FFT form = direct form."""
    rng = _rng(2)
    for N in (16, 64, 256):
        G = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        radii = np.array([0.0, 0.1, 0.5, 0.9, 0.99, 0.999])
        assert _rel(O.grid_fft(G, radii), O.grid_direct(G, radii)) < 1e-12


# ------------------------------------------------------------------ P2
def pin_kernel_spectrum(O):
    """DFT of the sampled normalised Szego kernel has the closed form
    N sqrt(1-|b|^2) conj(b)^l / (1 - conj(b)^N) (geometric series)."""
    for N in (8, 64, 1024):
        z = O.circle_points(N)
        for b in (0.0, 0.37, 0.9 * np.exp(0.7j), 0.999 * np.exp(-2.1j)):
            l = np.arange(N)
            closed = N * np.sqrt(1 - abs(b) ** 2) * np.conj(b) ** l / (1 - np.conj(b) ** N)
            if b == 0.0:
                closed = np.zeros(N, complex)
                closed[0] = N
            assert _rel(np.fft.fft(O.szego(b, z)), closed) < 1e-12
    # sample points: angles 2 pi n / N, starting at 1
    z = O.circle_points(12)
    assert abs(z[0] - 1) < 1e-15 and abs(z[3] - 1j) < 1e-15 and abs(z[6] + 1) < 1e-15


# ------------------------------------------------------------------ P3
def pin_reproducing(O):
    """For a polynomial G of degree < N the grid value is
    sqrt(1-r^2) G(a) / (1 - r^N) (reproducing property; G(a) by Horner)."""
    rng = _rng(3)
    N = 32
    coeffs = rng.standard_normal(N - 3) + 1j * rng.standard_normal(N - 3)  # degree N-4
    z = O.circle_points(N)
    G = np.polyval(coeffs[::-1], z)
    radii = np.array([0.0, 0.2, 0.6, 0.97])
    V = O.grid_fft(G, radii)
    Vd = O.grid_direct(G, radii)
    for m, r in enumerate(radii):
        a = r * z
        ref = np.sqrt(1 - r * r) * np.polyval(coeffs[::-1], a) / (1 - r ** N)
        assert _rel(V[m], ref) < 1e-12
        assert _rel(Vd[m], ref) < 1e-12


# ------------------------------------------------------------------ P4
def pin_kernel_kernel(O):
    """<e_b, e_a>~ = sqrt((1-|a|^2)(1-|b|^2)) (1-(a conj b)^N) / ((1-a conj b)(1-a^N)(1-conj(b)^N))."""
    N = 64
    z = O.circle_points(N)
    b = 0.8 * np.exp(1.3j)
    G = O.szego(b, z)
    radii = np.array([0.0, 0.4, 0.8, 0.95])
    V = O.grid_fft(G, radii)
    for m, r in enumerate(radii):
        a = r * z
        ab = a * np.conj(b)
        ref = (np.sqrt((1 - abs(a) ** 2) * (1 - abs(b) ** 2)) * (1 - ab ** N)
               / ((1 - ab) * (1 - a ** N) * (1 - np.conj(b) ** N)))
        assert _rel(V[m], ref) < 1e-12


# ------------------------------------------------------------------ P5
def pin_single_kernel(O):
    """G = w e_b with b on the grid: one step selects b (when rho = |b|^N is
    negligible), with coefficient w (1+rho)/(1-rho) and remainder energy
    |w|^2 (2 rho/(1-rho))^2 (1+rho)/(1-rho); the two formulas are exact for
    any rho once a_1 = b (checked with the index forced at rho = 0.9^64)."""
    radii = np.round(np.arange(0, 100) / 100.0, 12)
    w = 0.7 - 1.1j
    for N, rb, jb, free in ((64, 0.9, 11, False), (64, 0.5, 40, True),
                            (256, 0.5, 200, True), (1024, 0.5, 3, True)):
        mb = int(round(rb * 100))
        b = radii[mb] * np.exp(2j * np.pi * jb / N)
        z = O.circle_points(N)
        G = w * O.szego(b, z)
        d = O.decompose(G, radii, 1, forced=None if free else [(mb, jb)])
        assert tuple(d.index[0]) == (mb, jb)
        rho = abs(b) ** N
        assert abs(d.coef[0] - w * (1 + rho) / (1 - rho)) < 1e-13 * abs(w)
        e1 = abs(w) ** 2 * (2 * rho / (1 - rho)) ** 2 * (1 + rho) / (1 - rho)
        assert abs(d.energy[1] - e1) < 1e-14 * abs(w) ** 2
        assert abs(d.energy[0] - abs(w) ** 2 * (1 + rho) / (1 - rho)) < 1e-13
        if free:
            # margin to the nearest grid neighbour: pseudo-hyperbolic distance squared
            cand = [radii[mb] * np.exp(2j * np.pi * (jb + 1) / N),
                    radii[mb + 1] * np.exp(2j * np.pi * jb / N),
                    radii[mb - 1] * np.exp(2j * np.pi * jb / N)]
            rho2 = min(abs(a - b) ** 2 / abs(1 - np.conj(b) * a) ** 2 for a in cand)
            assert abs(d.margin[0] - rho2) < 1e-6 * rho2


# ------------------------------------------------------------------ P6
def pin_zero_radius_is_dft(O):
    """With radii = {0} every grid value ties, index j = 0 is taken, and the
    decomposition peels off the DFT coefficients: c_k = DFT(G)[k-1]/N,
    E_k = sum_{l >= k} |DFT(G)_l|^2 / N^2 (Parseval)."""
    rng = _rng(6)
    N = 32
    G = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    C = np.fft.fft(G)
    d = O.decompose(G, np.array([0.0]), 6)
    assert np.all(d.index == 0)
    assert _rel(d.coef, C[:6] / N) < 1e-13
    ref_e = np.array([np.sum(np.abs(C[k:]) ** 2) / N ** 2 for k in range(7)])
    assert _rel(d.energy, ref_e) < 1e-13


# ------------------------------------------------------------------ P7
def pin_energy_with_aliasing(O):
    """Discrete energy bookkeeping: E_k = E_{k-1} - |c_k|^2 (1 - 3 rho)/(1 - rho),
    rho = |a_k|^N (the discrete norm of e_a is (1+rho)/(1-rho), not 1)."""
    rng = _rng(7)
    N = 64
    G = W.kernel_sum(N, 0.9 * np.exp(2j * np.pi * rng.random(4)), rng.standard_normal(4) + 0j)
    radii = np.array([0.0, 0.3, 0.6, 0.8, 0.9, 0.95])
    d = O.decompose(G, radii, 6)
    for k in range(6):
        rho = abs(d.a[k]) ** N
        pred = d.energy[k] - abs(d.coef[k]) ** 2 * (1 - 3 * rho) / (1 - rho)
        assert abs(pred - d.energy[k + 1]) < 1e-13 * d.energy[0]


# ------------------------------------------------------------------ P8
def pin_expansion(O):
    """Expansion (Sn): G = sum_k c_k B_k + G_{n+1} prod_k (z - a_k)/(1 - conj(a_k) z)
    at every sample, so ||G - S_n||_N = ||G_{n+1}||_N and delta = E_n/E_0."""
    g, radii, _ = W.config1()
    g = g[::8]  # N = 128
    N = g.shape[0]
    z = O.circle_points(N)
    d = O.decompose(g, radii[::5], 5)
    blaschke = np.ones(N, complex)
    for a in d.a:
        blaschke *= (z - a) / (1 - np.conj(a) * z)
    S = O.partial_sum(d.coef, d.a, z)
    assert _rel(S + d.remainder * blaschke, g) < 1e-12
    assert abs(np.mean(np.abs(g - S) ** 2) - d.energy[-1]) < 1e-12 * d.energy[0]
    # orthonormality of the TM system in the continuous sense, checked by a fine rule
    zf = O.circle_points(1 << 14)
    B = O.tm_basis(d.a, zf)
    gram = (B @ np.conj(B).T) / zf.shape[0]
    assert np.max(np.abs(gram - np.eye(len(d.a)))) < 1e-9


# ------------------------------------------------------------------ P9
def pin_invariances(O):
    """Cyclic shift of the samples by s shifts every selected angle index by s;
    scaling G by lambda scales every coefficient by lambda."""
    g, radii, _ = W.config1()
    g = g[::4]  # N = 256
    N = g.shape[0]
    radii = radii[::4]
    d0 = O.decompose(g, radii, 4)
    assert np.all(d0.margin > 1e-6)
    s = 37
    d1 = O.decompose(np.roll(g, s), radii, 4)
    assert np.all(d1.index[:, 0] == d0.index[:, 0])
    assert np.all(d1.index[:, 1] == (d0.index[:, 1] + s) % N)
    rot = np.exp(2j * np.pi * s / N)  # a_k rotates with the shift; coefficients keep their modulus
    assert _rel(d1.a, d0.a * rot) < 1e-12
    assert _rel(np.abs(d1.coef), np.abs(d0.coef)) < 1e-10
    assert _rel(d1.energy, d0.energy) < 1e-10
    lam = 2.5 - 0.5j
    d2 = O.decompose(lam * g, radii, 4)
    assert np.all(d2.index == d0.index)
    assert _rel(d2.coef, lam * d0.coef) < 1e-12


# ------------------------------------------------------------------ P10
def pin_paper_tables(O):
    """Tables 4 and 8 of the paper (delta after n steps, 4 decimals) with a_1 = 0,
    N = 1024, radii 0..0.8.  Weak pin: the printed digits agree to about 1e-3."""
    radii = W.paper_radii()
    d1 = O.decompose(W.paper_f1(1024), radii, 10, first_a_zero=True)
    assert np.max(np.abs(d1.delta - load_golden("paper_table4_f1_delta.txt"))) < 1.5e-3
    d2 = O.decompose(W.paper_f2(1024), radii, 10, first_a_zero=True)
    assert np.max(np.abs(d2.delta - load_golden("paper_table8_f2_delta.txt"))) < 1.5e-3


# ------------------------------------------------------------------ selection rules
def pin_selection_rules(O):
    """Ties go to the lowest flat index; margin = (P1 - P2)/P1; forced indices replay."""
    V = np.zeros((3, 4), complex)
    V[1, 2] = 2.0
    V[2, 1] = -2.0  # same |.|^2, later in radius-major order
    V[0, 3] = 1.0j
    (m, j), margin = O.select(V)
    assert (m, j) == (1, 2) and margin == 0.0
    V[2, 1] = 1.9
    (m, j), margin = O.select(V)
    assert (m, j) == (1, 2) and abs(margin - (4 - 1.9 ** 2) / 4) < 1e-15
    g, radii, _ = W.config1()
    g = g[::4]
    radii = radii[::4]
    d = O.decompose(g, radii, 3)
    r = O.decompose(g, radii, 3, forced=d.index)
    assert np.all(r.index == d.index)
    assert _rel(r.coef, d.coef) < 1e-15 and _rel(r.energy, d.energy) < 1e-15


def pin_streamed_selection(O):
    """The streamed grid (radius chunks, threads) selects exactly as the whole
    grid: the same first maximiser, margin and grid value bit for bit, for any
    chunk size, including exact ties split across chunks (a repeated radius
    repeats its row: the first copy must win with margin 0) and the r = 0
    ring tie; and decompose_streamed equals decompose."""
    rng = _rng(41)
    N = 128
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    for radii in (np.array([0.3, 0.5, 0.3, 0.5, 0.1]), np.array([0.0, 0.2, 0.0]), W.uniform_radii(13)):
        V = O.grid_fft(g, radii)
        (m, j), margin = O.select(V)
        for chunk, workers in ((1, 1), (2, 3), (3, 1), (64, 1)):
            (ms, js), mg, v, p1 = O.select_streamed(g, radii, chunk=chunk, workers=workers)
            assert (ms, js) == (m, j) and mg == margin and v == V[m, j], (radii, chunk)
            assert p1 == V[m, j].real ** 2 + V[m, j].imag ** 2
    # repeated rows: the first copy wins and the tie leaves no margin
    (m, j), margin, _, _ = O.select_streamed(g, np.array([0.3, 0.5, 0.3, 0.5]), chunk=1)
    P = np.abs(O.grid_fft(g, np.array([0.3, 0.5]))) ** 2
    assert m == int(np.argmax(P.max(axis=1))) and margin == 0.0
    # a dominant mean: the r = 0 ring ties exactly; flat index 0 wins
    (m, j), margin, _, _ = O.select_streamed(g * 0.01 + 5.0, np.array([0.0, 0.2, 0.0]), chunk=1)
    assert (m, j) == (0, 0) and margin == 0.0
    gc, radii, _ = W.config1()
    a = O.decompose(gc[::2], radii[::3], 5)
    b = O.decompose_streamed(gc[::2], radii[::3], 5, chunk=7, workers=2)
    for k in ("index", "a", "coef", "energy", "margin", "remainder"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    c = O.decompose_streamed(gc[::2], radii[::3], 5, forced=a.index)
    assert np.array_equal(c.coef, a.coef) and np.array_equal(c.energy, a.energy)


# ------------------------------------------------------------------ N = p^K
def pin_prime_power_sizes(O):
    """N = p^K for p = 3, 5, 7 (the paper's closing remark: the fast algorithm
    holds for N = p^K).  Nothing in the aliased series depends on N being a
    power of two: pure-Python loops of eq. term81 at N = 9, 27, 5, 25, 7 and
    49, the direct form at N = 81, 243, 125, 625 and 343, the reproducing
    closed form sqrt(1-r^2) G(a)/(1-r^N) at N = 243, 625 and 343, and one
    step on w e_b at N = 729, 3125 and 2401 (b on the grid) giving index b,
    coefficient w (1+rho)/(1-rho) and the closed-form remainder energy."""
    rng = _rng(43)
    for N in (9, 27, 5, 25, 7, 49):
        G = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        radii = np.array([0.0, 0.35, 0.8, 0.97])
        ref = _term81_loops(G, radii)
        assert _rel(O.grid_fft(G, radii), ref) < 1e-13
        assert _rel(O.grid_direct(G, radii), ref) < 1e-13
    for N in (81, 243, 125, 625, 343):
        G = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        radii = np.array([0.0, 0.1, 0.5, 0.9, 0.99, 0.999])
        assert _rel(O.grid_fft(G, radii), O.grid_direct(G, radii)) < 1e-12
    for N in (243, 625, 343):
        coeffs = rng.standard_normal(N - 5) + 1j * rng.standard_normal(N - 5)
        z = O.circle_points(N)
        G = np.polyval(coeffs[::-1], z)
        radii = np.array([0.0, 0.3, 0.9])
        V = O.grid_fft(G, radii)
        for m, r in enumerate(radii):
            ref = np.sqrt(1 - r * r) * np.polyval(coeffs[::-1], r * z) / (1 - r ** N)
            assert _rel(V[m], ref) < 1e-12
    w = 0.4 + 0.9j
    radii = np.round(np.arange(0, 100) / 100.0, 12)
    for N, mb, jb in ((729, 97, 500), (3125, 96, 2999), (2401, 95, 1717)):
        b = radii[mb] * np.exp(2j * np.pi * jb / N)
        d = O.decompose(w * O.szego(b, O.circle_points(N)), radii, 1)
        rho = abs(b) ** N
        assert tuple(d.index[0]) == (mb, jb)
        assert abs(d.coef[0] - w * (1 + rho) / (1 - rho)) < 1e-13 * abs(w)
        e1 = abs(w) ** 2 * (2 * rho / (1 - rho)) ** 2 * (1 + rho) / (1 - rho)
        assert abs(d.energy[1] - e1) < 1e-13 * abs(w) ** 2


# ------------------------------------------------------------------ mixed radix
def pin_mixed_radix_sizes(O):
    """N with several prime factors (2, 3, 5, 7): the aliased series holds
    for any N.  Pure-Python loops of eq. term81 at N = 6, 10, 12, 15 and 21,
    the direct form at N = 60, 100, 210 and 360, the reproducing closed form
    at N = 360 and 1000, and one step on w e_b at N = 1000 and 1536 (b on the
    grid) giving index b, coefficient w (1+rho)/(1-rho) and the closed-form
    remainder energy."""
    rng = _rng(44)
    for N in (6, 10, 12, 15, 21):
        G = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        radii = np.array([0.0, 0.35, 0.8, 0.97])
        ref = _term81_loops(G, radii)
        assert _rel(O.grid_fft(G, radii), ref) < 1e-13
        assert _rel(O.grid_direct(G, radii), ref) < 1e-13
    for N in (60, 100, 210, 360):
        G = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        radii = np.array([0.0, 0.1, 0.5, 0.9, 0.99, 0.999])
        assert _rel(O.grid_fft(G, radii), O.grid_direct(G, radii)) < 1e-12
    for N in (360, 1000):
        coeffs = rng.standard_normal(N - 7) + 1j * rng.standard_normal(N - 7)
        z = O.circle_points(N)
        G = np.polyval(coeffs[::-1], z)
        radii = np.array([0.0, 0.3, 0.9])
        V = O.grid_fft(G, radii)
        for m, r in enumerate(radii):
            ref = np.sqrt(1 - r * r) * np.polyval(coeffs[::-1], r * z) / (1 - r ** N)
            assert _rel(V[m], ref) < 1e-12
    w = -0.3 + 1.2j
    radii = np.round(np.arange(0, 100) / 100.0, 12)
    for N, mb, jb in ((1000, 93, 777), (1536, 97, 1111)):
        b = radii[mb] * np.exp(2j * np.pi * jb / N)
        d = O.decompose(w * O.szego(b, O.circle_points(N)), radii, 1)
        rho = abs(b) ** N
        assert tuple(d.index[0]) == (mb, jb)
        assert abs(d.coef[0] - w * (1 + rho) / (1 - rho)) < 1e-13 * abs(w)
        e1 = abs(w) ** 2 * (2 * rho / (1 - rho)) ** 2 * (1 + rho) / (1 - rho)
        assert abs(d.energy[1] - e1) < 1e-13 * abs(w) ** 2


# ------------------------------------------------------------------ non-uniform samples
def _nu_loops(G, turns, weights, radii, n):
    """The quadrature rule written out with plain Python loops (tiny inputs only)."""
    import cmath
    import math
    out = []
    for r in radii:
        row = []
        for j in range(n):
            a = r * cmath.exp(2j * math.pi * j / n)
            s = 0j
            for t, w, g in zip(turns, weights, G):
                s += w * complex(g) / (1 - a * cmath.exp(-2j * math.pi * t))
            row.append(math.sqrt(1 - r * r) * s)
        out.append(row)
    return np.array(out)


def _two_grids(n1, b1, n2, b2, alpha):
    """Union of two rotated uniform grids (positions in turns, sorted) with
    weights alpha/n1 and (1 - alpha)/n2: a quadrature exact for the
    trigonometric polynomials up to degree min(n1, n2) - 1."""
    t = np.concatenate([(b1 + np.arange(n1) / n1) % 1.0, (b2 + np.arange(n2) / n2) % 1.0])
    w = np.concatenate([np.full(n1, alpha / n1), np.full(n2, (1 - alpha) / n2)])
    order = np.argsort(t)
    return t[order], w[order]


def pin_nonuniform_rule(O):
    """Non-uniform samples (Sec. 3.2, remark after Step 2).  The quadrature
    grid values against pure-Python loops; the uniform positions t_n = n/N
    with w_n = 1/N give the uniform grid values and decomposition; trapezoid
    weights sum to 1 and are 1/N on uniform positions; on a union of two
    rotated grids (n1 at beta1, n2 at beta2, weights alpha/n1, (1-alpha)/n2)
    a polynomial of degree < min(n1, n2) has the closed form
    sqrt(1-r^2) G(a) [alpha/(1 - (a e^{-2 pi i beta1})^n1) + (1-alpha)/(1 - (a e^{-2 pi i beta2})^n2)]."""
    rng = _rng(51)
    t = np.sort(rng.random(7))
    w = rng.random(7) + 0.2
    G = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    radii = np.array([0.0, 0.3, 0.8])
    assert _rel(O.grid_direct_nu(G, t, w, radii, 8), _nu_loops(G, t, w, radii, 8)) < 1e-13
    wt = O.trapezoid_weights(t)
    assert abs(wt.sum() - 1.0) < 1e-15 and np.all(wt > 0)
    assert abs(wt[0] - (t[1] - (t[-1] - 1.0)) / 2) < 1e-16
    # clustered positions: the quadrature norm of e_b approaches its integral, 1
    sc = np.arange(2000) / 2000
    tc = sc + 0.3 * np.sin(2 * np.pi * sc) / (2 * np.pi)
    eb = O.szego(0.5 * np.exp(0.4j), O.sample_points(tc))
    assert abs(O.energy_nu(eb, O.trapezoid_weights(tc)) - 1.0) < 1e-4
    N = 64
    tu = np.arange(N) / N
    assert np.max(np.abs(O.trapezoid_weights(tu) - 1.0 / N)) < 1e-17
    Gu = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    radii = np.array([0.0, 0.2, 0.6, 0.9, 0.99])
    assert _rel(O.grid_direct_nu(Gu, tu, np.full(N, 1.0 / N), radii, N), O.grid_direct(Gu, radii)) < 1e-13
    du = O.decompose_nu(Gu, tu, np.full(N, 1.0 / N), radii, N, 4)
    d = O.decompose(Gu, radii, 4, form="direct")
    assert np.array_equal(du.index, d.index)
    assert _rel(du.coef, d.coef) < 1e-12 and _rel(du.energy, d.energy) < 1e-12
    assert _rel(du.remainder, d.remainder) < 1e-11
    n1, b1, n2, b2, alpha = 48, 0.0031, 80, 0.0117, 0.3
    t2, w2 = _two_grids(n1, b1, n2, b2, alpha)
    coeffs = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    z2 = O.sample_points(t2)
    Gp = np.polyval(coeffs[::-1], z2)
    radii = np.array([0.0, 0.35, 0.7, 0.93])
    V = O.grid_direct_nu(Gp, t2, w2, radii, 40)
    for m, r in enumerate(radii):
        a = r * O.circle_points(40)
        ref = np.sqrt(1 - r * r) * np.polyval(coeffs[::-1], a) * (
            alpha / (1 - (a * np.exp(-2j * np.pi * b1)) ** n1)
            + (1 - alpha) / (1 - (a * np.exp(-2j * np.pi * b2)) ** n2))
        assert _rel(V[m], ref) < 1e-12


def pin_nonuniform_series(O):
    """The non-uniform DFT and the series form: c_l of a single sample is
    u e^{-2 pi i l t}; the series form equals the quadrature rule once r^N is
    negligible (jittered positions, trapezoid weights), and for radii near 1
    once its cut (terms) makes r^terms negligible, while the cut at N misses
    their tail; the normalised Szego
    kernel e_b on the two-grid union has the closed form
    sqrt((1-|a|^2)(1-|b|^2)) sum_g alpha_g (1 - (xy)^n_g) / ((1 - xy)(1 - x^n_g)(1 - y^n_g)),
    x = conj(b) e^{2 pi i beta_g}, y = a e^{-2 pi i beta_g}; and one step on w e_b
    (b on the grid) selects b with that coefficient and the eq. (7) update."""
    c = O.nudft(np.array([2.0 - 1.0j]), np.array([0.1234567]), 9)
    ref = (2.0 - 1.0j) * np.exp(-2j * np.pi * np.arange(9) * 0.1234567)
    assert _rel(c, ref) < 1e-14
    rng = _rng(52)
    N = 256
    t = np.sort((np.arange(300) + 0.45 * rng.random(300)) / 300)
    w = O.trapezoid_weights(t)
    G = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    radii = np.array([0.0, 0.1, 0.5, 0.8, 0.85])
    assert _rel(O.grid_series_nu(G, t, w, radii, N), O.grid_direct_nu(G, t, w, radii, N)) < 1e-12
    # radii near 1: the series cut at N terms misses the tail that the
    # quadrature rule holds; cut at 32 N (0.99^8192 ~ 1e-36) it does not
    near = np.array([0.5, 0.95, 0.99])
    direct = O.grid_direct_nu(G, t, w, near, N)
    assert _rel(O.grid_series_nu(G, t, w, near, N), direct) > 1e-3
    assert _rel(O.grid_series_nu(G, t, w, near, N, terms=32 * N), direct) < 1e-12
    n1, b1, n2, b2, alpha = 48, 0.0031, 80, 0.0117, 0.3
    t2, w2 = _two_grids(n1, b1, n2, b2, alpha)
    z2 = O.sample_points(t2)
    n = 40
    b = 0.5 * np.exp(2j * np.pi * 13 / n)
    wk = 0.6 + 0.8j
    Gk = wk * O.szego(b, z2)
    radii = np.round(np.arange(0, 20) / 20.0, 12)

    def kernel_closed(a):
        tot = 0.0
        for ng, bg, ag in ((n1, b1, alpha), (n2, b2, 1 - alpha)):
            x = np.conj(b) * np.exp(2j * np.pi * bg)
            y = a * np.exp(-2j * np.pi * bg)
            tot = tot + ag * (1 - (x * y) ** ng) / ((1 - x * y) * (1 - x ** ng) * (1 - y ** ng))
        return np.sqrt((1 - abs(a) ** 2) * (1 - abs(b) ** 2)) * tot

    V = O.grid_direct_nu(Gk, t2, w2, radii, n)
    for m in (3, 10, 17):
        a = radii[m] * O.circle_points(n)
        assert _rel(V[m], wk * kernel_closed(a)) < 1e-12
    d = O.decompose_nu(Gk, t2, w2, radii, n, 1)
    assert tuple(d.index[0]) == (10, 13)
    assert abs(d.coef[0] - wk * kernel_closed(b)) < 1e-13
    e_a = np.sqrt(1 - abs(b) ** 2) / (1 - np.conj(b) * z2)
    rem = (Gk - d.coef[0] * e_a) * (1 - np.conj(b) * z2) / (z2 - b)
    assert _rel(d.remainder, rem) < 1e-13
    assert abs(d.energy[1] - np.sum(w2 * np.abs(rem) ** 2)) < 1e-14
    assert abs(d.energy[0] - np.sum(w2 * np.abs(Gk) ** 2)) < 1e-14 * d.energy[0]


def pin_nonuniform_relative_errors(O):
    """At non-uniform points the Blaschke factor is still unimodular, so the
    partial sums' errors equal the remainders' energies: delta_n = E_n / E_0
    of decompose_nu; uniform positions give the uniform relative errors."""
    g, t = W.nonuniform_kernel_signal(300, item=3, kind="cluster")
    w = O.trapezoid_weights(t)
    radii = W.uniform_radii(12, 0.8)
    d = O.decompose_nu(g, t, w, radii, 256, 5)
    dl = O.relative_errors_nu(g, t, w, d.coef, d.a)
    assert np.max(np.abs(dl - d.energy[1:] / d.energy[0])) < 1e-12
    gu, radii_u, _ = W.config1()
    gu = gu[::8]
    du = O.decompose(gu, radii_u[::5], 4)
    n = gu.shape[0]
    ref = O.relative_errors(gu, du.coef, du.a)
    assert np.max(np.abs(O.relative_errors_nu(gu, np.arange(n) / n, np.full(n, 1.0 / n), du.coef, du.a) - ref)) < 1e-13


# ------------------------------------------------------------------ relative error (Sec. 4, eq. er)
def pin_relative_errors(O):
    """delta_n from the partial sums equals E_n/E_0 from the remainders at every
    n (expansion (Sn) with a unimodular Blaschke factor); one kernel e_b picked
    at b reconstructs exactly (delta_1 = 0)."""
    g, radii, _ = W.config1()
    g = g[::8]
    d = O.decompose(g, radii[::5], 6)
    dl = O.relative_errors(g, d.coef, d.a)
    assert np.max(np.abs(dl - d.energy[1:] / d.energy[0])) < 1e-12
    N = 64
    z = O.circle_points(N)
    b = 0.4 * np.exp(2j * np.pi * 5 / N)
    gk = (1.5 - 0.5j) * O.szego(b, z)
    assert O.relative_errors(gk, [(1.5 - 0.5j)], [b])[0] < 1e-28


# ------------------------------------------------------------------ analytic part (Sec. 4, case 2)
def pin_analytic_part(O):
    """Closed forms: a positive tone cos(2 pi k n/N), 0 < k < N/2, becomes
    e^{2 pi i k n/N}; a negative-frequency exponential vanishes; the constant
    and the alternating (Nyquist) sequence are kept; for real samples the
    real part of the result is the input."""
    for N in (2, 8, 64, 1024):
        n = np.arange(N)
        for k in range(1, N // 2):
            x = np.cos(2 * np.pi * k * n / N)
            assert _rel(O.analytic_part(x), np.exp(2j * np.pi * k * n / N)) < 1e-13
            assert np.max(np.abs(O.analytic_part(np.exp(-2j * np.pi * k * n / N)))) < 1e-13
            if N > 64 and k > 3:
                break
        assert _rel(O.analytic_part(np.full(N, 2.0 + 1.0j)), np.full(N, 2.0 + 1.0j)) < 1e-14
        alt = (-1.0) ** n
        assert _rel(O.analytic_part(alt), alt) < 1e-13
        x = _rng(31).standard_normal(N)
        assert np.max(np.abs(O.analytic_part(x).real - x)) < 1e-13 * np.max(np.abs(x))


ALL_PINS = [
    pin_bruteforce_loops,
    pin_fft_equals_direct,
    pin_kernel_spectrum,
    pin_reproducing,
    pin_kernel_kernel,
    pin_single_kernel,
    pin_zero_radius_is_dft,
    pin_energy_with_aliasing,
    pin_prime_power_sizes,
    pin_mixed_radix_sizes,
    pin_nonuniform_rule,
    pin_nonuniform_series,
    pin_nonuniform_relative_errors,
    pin_expansion,
    pin_invariances,
    pin_paper_tables,
    pin_selection_rules,
    pin_streamed_selection,
    pin_relative_errors,
    pin_analytic_part,
]
