"""Comparison of a GPU decomposition with the FP64 oracle.

Bar (per step k, oracle values unhatted, GPU values hatted):
* selected grid indices bit-exact while the oracle's best leads its runner-up
  by more than 1e-6 relative (steps forced by first_a_zero or replay count
  as decided);
* at the first step whose lead is <= 1e-6 several answers are correct: the GPU's
  choice must be a point whose oracle |<G_k, e_a>~|^2 lies within 2e-6 of the
  oracle's maximum, and the comparison of the trajectories stops there;
* |c^_k - c_k| <= tol * max(|c_k|, sqrt(E_{k-1}))  (FFT errors are normwise);
* |E^_k - E_k| <= tol * max(E_0, E_k) (small N with radii near 1 can raise the
  discrete energy by orders of magnitude);  |a^_k - a_k| <= 1e-13.
tol = 1e-12 for the FP64 path and 1e-5 for the FP32 + FP64-recheck path.
"""
from __future__ import annotations

import numpy as np

import oracle as O

TOL = {"fp64": 1e-12, "fp32": 1e-5}
MARGIN_MIN = 1e-6


def to_numpy(res):
    out = {}
    for name in ("index", "a", "coef", "energy", "margin", "remainder", "recheck_count", "flags", "fp32_error"):
        v = getattr(res, name)
        if hasattr(v, "detach"):
            v = v.detach().cpu().numpy()
        out[name] = np.asarray(v)
    return out


def compare(gpu, ref: "O.Decomposition", tol: float, signal=None, radii=None, forced_first: bool = False,
            replay: bool = False):
    """Return (steps_compared, report dict); raise AssertionError on a violation."""
    g = to_numpy(gpu)
    S = ref.coef.shape[0]
    E0 = ref.energy[0]
    assert abs(g["energy"][0] - E0) <= tol * E0 + 1e-300, ("E0", g["energy"][0], E0)
    upto = S
    for k in range(S):
        decided = replay or (forced_first and k == 0) or (ref.margin[k] > MARGIN_MIN)
        if not decided:
            upto = k
            break
    worst_c = 0.0
    worst_e = 0.0
    for k in range(upto):
        assert tuple(g["index"][k]) == tuple(ref.index[k]), (k, g["index"][k], ref.index[k], ref.margin[k])
        assert abs(g["a"][k] - ref.a[k]) <= 1e-13, (k, g["a"][k], ref.a[k])
        den = max(abs(ref.coef[k]), np.sqrt(ref.energy[k]))
        ec = abs(g["coef"][k] - ref.coef[k]) / den
        ee = abs(g["energy"][k + 1] - ref.energy[k + 1]) / max(E0, ref.energy[k + 1])
        worst_c = max(worst_c, ec)
        worst_e = max(worst_e, ee)
        assert ec <= tol, (k, "coef", ec, g["coef"][k], ref.coef[k])
        assert ee <= tol, (k, "energy", ee, g["energy"][k + 1], ref.energy[k + 1])
    if upto < S and signal is not None and radii is not None:
        # near-tie: the GPU's choice must be one of the (nearly) equal maxima of the oracle grid
        Gk = O.decompose(signal, radii, upto, forced=ref.index[:upto]).remainder if upto > 0 else signal
        V = O.grid_fft(Gk, radii)
        P = np.abs(V) ** 2
        m, j = g["index"][upto]
        assert P[m, j] >= P.max() * (1 - 2e-6), ("near-tie choice not maximal", upto, P[m, j], P.max())
    return upto, {"worst_coef": worst_c, "worst_energy": worst_e, "steps_compared": upto, "steps": S}
