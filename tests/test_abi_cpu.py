"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/afd.h declares, and rejects invalid arguments before
any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afd.h")


def _lib():
    from paper_1711_08604_amd import afd
    if not os.path.exists(afd.LIB_PATH):
        from paper_1711_08604_amd import build
        build.build()
    return afd, afd.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(afd_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    afd, lib = _lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(afd.EXPORTS)


def _desc(afd, n=1024, radii=(0.0, 0.5), precision=0, recheck_k=8, first_a_zero=0, band=0.0, batch=0):
    r = np.ascontiguousarray(np.asarray(radii, dtype=np.float64))
    d = afd.PlanDesc()
    d.n = n
    d.m = r.shape[0]
    d.radii = r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.precision = precision
    d.recheck_k = recheck_k
    d.first_a_zero = first_a_zero
    d.recheck_band = band
    d.batch = batch
    return d, r


@pytest.mark.parametrize("kw,status", [
    (dict(n=1001), 1), (dict(n=1), 1), (dict(n=0), 1), (dict(n=-4), 1),
    (dict(n=1 << 21), 5), (dict(radii=()), 1), (dict(radii=(0.2, 1.0)), 1), (dict(radii=(-0.1,)), 1),
    (dict(radii=(np.nan,)), 1), (dict(radii=(np.inf,)), 1), (dict(precision=7), 1),
    (dict(recheck_k=-1), 1), (dict(recheck_k=65), 1), (dict(band=-1e-3), 1), (dict(band=0.5), 1),
    (dict(first_a_zero=1, radii=(0.1, 0.2)), 1), (dict(n=1 << 16, radii=np.zeros(1 << 16)), 1),
    (dict(batch=-1), 1), (dict(n=1 << 15, batch=2), 5), (dict(n=1 << 14, batch=1 << 17), 1),
    (dict(n=3 ** 9), 5), (dict(n=22), 1), (dict(n=26), 1), (dict(n=3 ** 8 * 2), 5),
    (dict(n=5 ** 7), 5), (dict(n=7 ** 5), 5), (dict(n=11), 1), (dict(n=35), 5), (dict(n=42), 5),
    (dict(n=121), 1), (dict(n=3 << 14), 5), (dict(n=17 * 3), 1),
])
def test_plan_create_rejects(kw, status):
    afd, lib = _lib()
    d, keep = _desc(afd, **kw)
    h = ctypes.c_void_p(123)
    st = lib.afd_plan_create(ctypes.byref(d), None, ctypes.byref(h))
    assert st == status, (kw, st, lib.afd_last_error())
    assert h.value is None
    assert lib.afd_last_error().decode() != ""
    assert lib.afd_workspace_bytes(ctypes.byref(d)) == 0


def test_null_arguments():
    afd, lib = _lib()
    assert lib.afd_plan_create(None, None, None) == 1
    h = ctypes.c_void_p()
    assert lib.afd_plan_create(None, None, ctypes.byref(h)) == 1
    rd = afd.ResultDesc()
    assert lib.afd_decompose(None, None, 1, ctypes.byref(rd)) == 1
    assert lib.afd_replay(None, None, 1, None, ctypes.byref(rd)) == 1
    lib.afd_plan_destroy(None)
    assert lib.afd_plan_set_timing(None, b"radius", 1) == 1
    assert lib.afd_workspace_bytes(None) == 0
    assert lib.afd_reconstruct(None, None, None, 0, None, None, None) == 1
    assert lib.afd_analytic(None, None, None) == 1


def test_workspace_bytes_scales():
    afd, lib = _lib()
    d1, k1 = _desc(afd, n=1024, radii=np.linspace(0, 0.99, 100))
    d2, k2 = _desc(afd, n=16384, radii=np.linspace(0, 0.999, 1000), precision=1)
    b1 = lib.afd_workspace_bytes(ctypes.byref(d1))
    b2 = lib.afd_workspace_bytes(ctypes.byref(d2))
    assert 0 < b1 < b2
    # tables dominate: 16 B per sample of omega + the per-radius power tables
    assert b2 >= 16 * 16384 + 4 * 1000 * (512 + 32)


def test_workspace_bytes_two_pass():
    """N = 2^20: only the radii with long spectra (beyond 16 N2 = 16384 terms)
    run in two passes, over chunks whose intermediate is bounded (1 GiB; all
    4 such radii in double precision, all 3 in single precision; the 63 + 17
    / 45 + 11 of medium length run in the shifted splits' row passes), so the
    workspace does not grow with M * N; besides it, a step keeps the
    selection records of every radius (M x 256 lists of 528 bytes in single
    precision, M x 256 bests of 40 bytes in double precision: the largest
    record count of the row passes)."""
    afd, lib = _lib()
    r = np.linspace(0, 0.999, 2000)
    out = {}
    for prec in (0, 1):
        d, keep = _desc(afd, n=1 << 20, radii=r, precision=prec)
        out[prec] = lib.afd_workspace_bytes(ctypes.byref(d))
    base64 = 4 * (16 << 20) + 2000 * 256 * 40
    base32 = 3 * (8 << 20) + 2000 * 256 * 528
    assert base64 <= out[0] < base64 + (200 << 20), out
    assert base32 <= out[1] < base32 + (200 << 20), out
    d, keep = _desc(afd, n=1 << 15, radii=r[:7], precision=1)
    assert 0 < lib.afd_workspace_bytes(ctypes.byref(d)) < (16 << 20)


def test_workspace_bytes_batch():
    """A batch holds one copy of every per-signal buffer per signal and one copy of the tables."""
    afd, lib = _lib()
    r = np.linspace(0, 0.999, 512)
    sizes = []
    for batch in (1, 2, 512):
        d, keep = _desc(afd, n=4096, radii=r, precision=1, batch=batch)
        sizes.append(lib.afd_workspace_bytes(ctypes.byref(d)))
    per_signal = sizes[1] - sizes[0]
    assert per_signal > 16 * 4096  # at least the double remainder
    assert sizes[2] == pytest.approx(sizes[0] + 511 * per_signal, rel=1e-3)


def test_status_strings():
    afd, lib = _lib()
    for s in range(6):
        assert lib.afd_status_string(s).decode().startswith("AFD_")


@pytest.mark.parametrize("p,kmax", [(3, 8), (5, 6), (7, 4)])
def test_workspace_bytes_prime_powers(p, kmax):
    """N = p^K plans (p = 3, 5, 7): valid for K = 1..kmax (one radius per
    workgroup, records for M radii), growing with N and M."""
    afd, lib = _lib()
    sizes = []
    for k in range(1, kmax + 1):
        d, keep = _desc(afd, n=p ** k, radii=np.linspace(0, 0.99, 50))
        sizes.append(lib.afd_workspace_bytes(ctypes.byref(d)))
    assert all(b > 0 for b in sizes) and sizes == sorted(sizes), sizes
    d, keep = _desc(afd, n=p ** kmax, radii=np.linspace(0, 0.99, 50), precision=1, batch=4)
    assert lib.afd_workspace_bytes(ctypes.byref(d)) > sizes[-1]


@pytest.mark.parametrize("n", [6, 10, 12, 15, 18, 100, 1000, 1536, 6000, 10125, 12288, 14336, 15360])
def test_workspace_bytes_mixed_radix(n):
    """Mixed-radix N (several of the primes 2, 3, 5, 7): valid up to 16384,
    one radius per workgroup, growing with M and with the batch."""
    afd, lib = _lib()
    d, keep = _desc(afd, n=n, radii=np.linspace(0, 0.99, 50))
    a = lib.afd_workspace_bytes(ctypes.byref(d))
    d, keep = _desc(afd, n=n, radii=np.linspace(0, 0.99, 80))
    b = lib.afd_workspace_bytes(ctypes.byref(d))
    d, keep = _desc(afd, n=n, radii=np.linspace(0, 0.99, 50), precision=1, batch=3)
    c = lib.afd_workspace_bytes(ctypes.byref(d))
    assert 0 < a < b and a < c, (a, b, c)


def _nu_desc(afd, n=256, radii=(0.0, 0.5), turns=None, weights=None, batch=0, precision=0):
    d, keep = _desc(afd, n=n, radii=radii, batch=batch, precision=precision)
    t = np.ascontiguousarray(np.arange(100) / 100 + 0.001 if turns is None else np.asarray(turns, dtype=np.float64))
    d.sample_turns = t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.samples = t.shape[0]
    keep = [keep, t]
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        d.sample_weights = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        keep.append(w)
    return d, keep


@pytest.mark.parametrize("kw,status", [
    (dict(turns=[0.1, 0.1, 0.5]), 1),            # not strictly increasing
    (dict(turns=[0.2, 0.1]), 1),
    (dict(turns=[0.0, 1.0]), 1),                 # outside [0, 1)
    (dict(turns=[-0.1, 0.5]), 1),
    (dict(turns=[0.0, np.nan]), 1),
    (dict(weights=[np.inf] + [0.01] * 99), 1),
    (dict(radii=(0.0, 0.99999)), 5),             # kernel series longer than 2^18 terms
    (dict(n=243), 5),                            # the grid must be 2^K
    (dict(n=1 << 15), 5),
    (dict(turns=np.arange(1 << 17) / (1 << 17)), 5),
])
def test_nonuniform_rejects(kw, status):
    afd, lib = _lib()
    d, keep = _nu_desc(afd, **kw)
    h = ctypes.c_void_p(123)
    st = lib.afd_plan_create(ctypes.byref(d), None, ctypes.byref(h))
    assert st == status, (kw, st, lib.afd_last_error())
    assert h.value is None
    assert lib.afd_workspace_bytes(ctypes.byref(d)) == 0


def test_nonuniform_workspace():
    """A non-uniform plan sizes its per-sample buffers; samples without
    positions are rejected."""
    afd, lib = _lib()
    d1, k1 = _nu_desc(afd, n=1024, radii=np.linspace(0, 0.95, 20), turns=np.arange(1000) / 1000)
    d2, k2 = _nu_desc(afd, n=1024, radii=np.linspace(0, 0.95, 20), turns=np.arange(4000) / 4000)
    b1, b2 = lib.afd_workspace_bytes(ctypes.byref(d1)), lib.afd_workspace_bytes(ctypes.byref(d2))
    assert 0 < b1 < b2
    # 3000 more samples: position, weight, point, shifted weight and the remainder sample
    assert b2 - b1 >= 3000 * (8 + 8 + 16 + 16 + 16)
    # a batch of 3 holds three remainders and three gridding buffers (G = 4096 cells of
    # 16 bytes, three of them per signal)
    d3, k3 = _nu_desc(afd, n=1024, radii=np.linspace(0, 0.95, 20), turns=np.arange(1000) / 1000, batch=3)
    b3 = lib.afd_workspace_bytes(ctypes.byref(d3))
    assert b3 - b1 >= 2 * (1000 * 16 + 3 * 4096 * 16)
    d3, k3 = _desc(afd, n=1024)
    d3.samples = 1000
    assert lib.afd_workspace_bytes(ctypes.byref(d3)) == 0


def test_nonuniform_fold_workspace():
    """Radii whose kernel series outlasts N terms are accepted: the plan holds
    the K N modes the longest series needs (K a power of two) and one folded
    spectrum per such radius; series beyond 2^18 terms are rejected."""
    afd, lib = _lib()
    turns = np.arange(1000) / 1000
    # FP64: the series of r is cut where r^L / (1 - r) <= 2^-60
    need = lambda r: (60 * np.log(2) - np.log1p(-r)) / -np.log(r)
    d1, k1 = _nu_desc(afd, n=1024, radii=(0.0, 0.5, 0.6), turns=turns)     # every series within N
    d2, k2 = _nu_desc(afd, n=1024, radii=(0.0, 0.5, 0.99), turns=turns)    # 4596 terms: 8 N modes, one fold
    d3, k3 = _nu_desc(afd, n=1024, radii=(0.0, 0.99, 0.995), turns=turns)  # 9354 terms: 16 N modes, two folds
    assert 4096 < need(0.99) < 8192 < need(0.995) < 16384
    b1, b2, b3 = (lib.afd_workspace_bytes(ctypes.byref(d)) for d in (d1, d2, d3))
    assert 0 < b1 < b2 < b3
    assert b2 - b1 >= 16 * (8192 - 1024) + 16 * 1024
    assert b3 - b2 >= 16 * (16384 - 8192) + 16 * 1024
    # 2^18 modes at most: a series of about 250000 terms is accepted, 5.4e6 is not
    lo, hi = 0.99, 1.0 - 1e-9
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if need(mid) < 250000 else (lo, mid)
    r_ok = lo
    assert 249000 < need(r_ok) <= 250000 and need(0.99999) > 2 ** 18
    d4, k4 = _nu_desc(afd, n=1024, radii=(0.0, r_ok), turns=turns)
    assert lib.afd_workspace_bytes(ctypes.byref(d4)) > b3
    d5, k5 = _nu_desc(afd, n=1024, radii=(0.0, 0.99999), turns=turns)
    assert lib.afd_workspace_bytes(ctypes.byref(d5)) == 0


def test_flat_index_beyond_2p31():
    """M*N between 2^31 and 2^32 - 2 is accepted (unsigned flat indices)."""
    afd, lib = _lib()
    d, keep = _desc(afd, n=1 << 20, radii=np.linspace(0.0, 0.95, 2101))
    assert lib.afd_workspace_bytes(ctypes.byref(d)) > 0
    d, keep = _desc(afd, n=1 << 20, radii=np.linspace(0.0, 0.95, 4095))
    assert lib.afd_workspace_bytes(ctypes.byref(d)) > 0
    d, keep = _desc(afd, n=1 << 20, radii=np.linspace(0.0, 0.95, 4096))
    assert lib.afd_workspace_bytes(ctypes.byref(d)) == 0
