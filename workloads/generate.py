"""Synthetic signals and radius grids for the Core-AFD workloads.

Recipes (all complex128 samples on z_n = e^{2 pi i n/N}, n = 0..N-1):

* kernel sums: G(z) = sum_j w_j sqrt(1-|b_j|^2) / (1 - conj(b_j) z), a rational
  H^2 function with simple poles at 1/conj(b_j) outside the closed disc; poles
  b_j area-uniform in |b| <= R (|b| = R sqrt(U), arg b = 2 pi V); weights
  complex standard Gaussian CN(0,1) = (X + iY)/sqrt(2);
* optional complex white noise CN(0, s^2) at a stated SNR, s^2 = mean|G|^2 * 10^(-SNR/10);
* a real chirp + Gaussian-windowed tones + real white noise, reduced to its
  H^2 (analytic) part by zeroing the negative-frequency bins;
* the two closed-form signals of the paper's Sec. 4 experiments;
* non-uniform samples: positions t_n in turns, jittered (t_n = (n + j U_n)/N_s,
  j < 1) or clustered (t_n = s_n + c sin(2 pi s_n)/(2 pi), s_n = n/N_s, c < 1),
  with kernel sums evaluated at z_n = e^{2 pi i t_n}.

Seeds: numpy.random.SeedSequence([20171108, config, item]) with PCG64.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "SEED_ROOT",
    "rng_for",
    "circle",
    "kernel_sum",
    "random_kernel_signal",
    "add_noise",
    "analytic_part",
    "uniform_radii",
    "paper_f1",
    "paper_f2",
    "paper_radii",
    "config1",
    "config2",
    "config3",
    "config3_batch",
    "config5",
    "shaped_like_config2",
    "nonuniform_positions",
    "nonuniform_kernel_signal",
]

SEED_ROOT = 20171108


def rng_for(config: int, item: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence([SEED_ROOT, int(config), int(item)])
    return np.random.Generator(np.random.PCG64(ss))


def circle(n: int) -> np.ndarray:
    t = 2.0 * np.pi * np.arange(n) / n
    return np.exp(1j * t)


def kernel_sum(n: int, poles: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Samples of sum_j w_j sqrt(1-|b_j|^2)/(1 - conj(b_j) z) on the N-point circle."""
    z = circle(n)
    out = np.zeros(n, dtype=np.complex128)
    for b, w in zip(poles, weights):
        out += w * np.sqrt(1.0 - abs(b) ** 2) / (1.0 - np.conj(b) * z)
    return out


def _poles_area_uniform(rng, count: int, rmax: float) -> np.ndarray:
    rad = rmax * np.sqrt(rng.random(count))
    ang = 2.0 * np.pi * rng.random(count)
    return rad * np.exp(1j * ang)


def _cn01(rng, count: int) -> np.ndarray:
    return (rng.standard_normal(count) + 1j * rng.standard_normal(count)) / np.sqrt(2.0)


def random_kernel_signal(rng, n: int, count: int, rmax: float):
    poles = _poles_area_uniform(rng, count, rmax)
    weights = _cn01(rng, count)
    return kernel_sum(n, poles, weights), poles, weights


def add_noise(rng, g: np.ndarray, snr_db: float) -> np.ndarray:
    power = float(np.mean(np.abs(g) ** 2))
    sigma2 = power * 10.0 ** (-snr_db / 10.0)
    return g + np.sqrt(sigma2) * _cn01(rng, g.shape[0])


def analytic_part(x: np.ndarray) -> np.ndarray:
    """Analytic signal by FFT: keep DC and Nyquist, double positive bins, zero negative bins."""
    n = x.shape[0]
    X = np.fft.fft(x)
    h = np.zeros(n)
    h[0] = 1.0
    if n % 2 == 0:
        h[n // 2] = 1.0
        h[1:n // 2] = 2.0
    else:
        h[1:(n + 1) // 2] = 2.0
    return np.fft.ifft(X * h)


def uniform_radii(m: int, rmax: float = 0.999) -> np.ndarray:
    """r_k = rmax * k / (m - 1), k = 0..m-1 (both endpoints included)."""
    if m == 1:
        return np.zeros(1)
    return rmax * np.arange(m, dtype=np.float64) / (m - 1)


# ---------------------------------------------------------------- paper, Sec. 4
def paper_f1(n: int) -> np.ndarray:
    """Case 1 of Sec. 4: f1 = (0.0247 e^{3it} + 0.355 e^{2it}) / (1 - 0.3679 e^{it})."""
    z = circle(n)
    return (0.0247 * z ** 3 + 0.355 * z ** 2) / (1.0 - 0.3679 * z)


def paper_f2(n: int) -> np.ndarray:
    """Case 2 of Sec. 4: sgn(sin t), taken as its analytic (H^2) part."""
    t = 2.0 * np.pi * np.arange(n) / n
    return analytic_part(np.sign(np.sin(t)).astype(np.complex128))


def paper_radii() -> np.ndarray:
    """The radius grid r = 0, 0.1, ..., 0.8 of the Sec. 4 experiments."""
    return np.round(np.arange(9) * 0.1, 12)


# ---------------------------------------------------------------- workloads
def config1(item: int = 0):
    """N = 1024, 5 kernels |b| <= 0.9, radii m/100 (m = 0..99), 10 steps, FP64."""
    rng = rng_for(1, item)
    g, _, _ = random_kernel_signal(rng, 1024, 5, 0.9)
    radii = np.arange(100, dtype=np.float64) / 100.0
    return g, radii, 10


def config2(item: int = 0, n: int = 16384, m: int = 1000, steps: int = 50):
    """N = 16384, 40 kernels |b| <= 0.98 plus CN noise at 30 dB, M = 1000 radii
    uniform in [0, 0.999], 50 steps.  Smaller (n, m, steps) keep the recipe."""
    rng = rng_for(2, item)
    g, _, _ = random_kernel_signal(rng, n, 40, 0.98)
    g = add_noise(rng, g, 30.0)
    return g, uniform_radii(m), steps


def shaped_like_config2(n: int, m: int, steps: int, item: int = 0):
    return config2(item=item, n=n, m=m, steps=steps)


def config3(item: int, n: int = 4096):
    """One signal of the uniform batch: U{8..32} kernels, |b| <= 0.95, no noise."""
    rng = rng_for(3, item)
    count = int(rng.integers(8, 33))
    g, _, _ = random_kernel_signal(rng, n, count, 0.95)
    return g


def config3_batch(batch: int = 512, n: int = 4096, m: int = 512, steps: int = 30):
    """The uniform batch: `batch` signals of config3 (item = signal index), M radii
    uniform in [0, 0.999], 30 steps.  Returns (signals [batch][N], radii, steps)."""
    g = np.stack([config3(i, n) for i in range(batch)])
    return g, uniform_radii(m), steps


def config5(item: int = 0, n: int = 1 << 20, m: int = 2000, steps: int = 100):
    """Real chirp (0.01 -> 0.4 cycles/sample) + 3 Gaussian-windowed tones + real
    white noise at 20 dB, reduced to its analytic part; M radii uniform in [0, 0.999]."""
    rng = rng_for(5, item)
    k = np.arange(n, dtype=np.float64)
    x = np.cos(2.0 * np.pi * (0.01 * k + 0.39 * k * k / (2.0 * n)))
    for _ in range(3):
        mu = rng.uniform(0.1 * n, 0.9 * n)
        sig = n / 64.0
        f = rng.uniform(0.02, 0.45)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        x = x + np.exp(-(k - mu) ** 2 / (2.0 * sig * sig)) * np.cos(2.0 * np.pi * f * k + phi)
    power = float(np.mean(x * x))
    x = x + np.sqrt(power * 10.0 ** (-2.0)) * rng.standard_normal(n)
    return analytic_part(x.astype(np.complex128)), uniform_radii(m), steps


def nonuniform_positions(rng, ns: int, kind: str = "jitter", amount: float = 0.8) -> np.ndarray:
    """Strictly increasing sample positions in [0, 1) (turns): "jitter" moves
    each uniform position n/ns by amount * U[0, 1) of a spacing; "cluster"
    warps s = n/ns to s + amount sin(2 pi s)/(2 pi) (denser near s = 1/2)."""
    s = np.arange(ns, dtype=np.float64) / ns
    if kind == "jitter":
        return s + amount * rng.random(ns) / ns
    if kind == "cluster":
        return s + amount * np.sin(2.0 * np.pi * s) / (2.0 * np.pi)
    raise ValueError(kind)


def nonuniform_kernel_signal(ns: int, item: int = 0, kind: str = "jitter", count: int = 12, rmax: float = 0.9,
                             snr_db: float = 40.0):
    """Kernel sum (count poles area-uniform in |b| <= rmax, CN(0,1) weights) at
    non-uniform positions, plus CN noise at snr_db.  Returns (samples, turns)."""
    rng = rng_for(6, item)
    t = nonuniform_positions(rng, ns, kind)
    z = np.exp(2j * np.pi * t)
    poles = _poles_area_uniform(rng, count, rmax)
    weights = _cn01(rng, count)
    g = np.zeros(ns, dtype=np.complex128)
    for b, w in zip(poles, weights):
        g += w * np.sqrt(1.0 - abs(b) ** 2) / (1.0 - np.conj(b) * z)
    return add_noise(rng, g, snr_db), t
