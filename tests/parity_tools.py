"""Comparison of a GPU decomposition with the FP64 oracle.

Bar (per step k, oracle values unhatted, GPU values hatted):
* selected grid indices bit-exact while the oracle's best leads its runner-up
  by more than 1e-6 relative (steps forced by first_a_zero count as decided),
  and on an exact tie of the r = 0 ring (every value of that ring is the same
  number, so the lowest flat index, j = 0, is the one answer);
* at the first step whose lead is <= 1e-6 several answers are correct: the
  GPU's choice must be a point whose oracle |<G_k, e_a>~|^2 lies within
  NEAR_TIE of the oracle's maximum (both modes decide in double: the FP64
  grid values, or the FP64 re-check of the FP32 short-list), and the
  comparison of the trajectories stops there;
* |c^_k - c_k| <= tol * max(|c_k|, sqrt(E_{k-1}))  (FFT errors are normwise),
  and |c^_k - c_k| <= tol * |c_k| wherever |c_k| >= REL_FLOOR * sqrt(E_{k-1});
* |E^_k - E_k| <= tol * max(E_0, E_k) (small N with radii near 1 can raise the
  discrete energy by orders of magnitude);  |a^_k - a_k| <= 1e-13;
* FP64 mode: the margin (P1 - P2)/P1 within 1e-10 of the oracle's.
tol = 1e-12 for the FP64 path and 1e-5 for the FP32 + FP64-recheck path.
Both paths update the remainder in double, with rounding errors of about
1e-16 of the signal's norm; once the oracle's remainder norm falls below
RESIDUAL_FLOOR / tol of the signal's (the decomposition has converged to
that accuracy, Sec. 2), its digits are below that rounding and the steps
from there on are not compared.

FP32 mode with flag bit 0 or 1 set at a step (the band, or a radius' list,
held more points than it could keep: a flat ring) re-checks the top of the
FP32 order only, so there its choice is a maximum within the FP32 accuracy:
the bars of that step use TOL["fp32"] in place of MARGIN_MIN, NEAR_TIE and
PICK_MARGIN, and the oracle's winner need not have been re-checked.

Replay (compare_replay) forces the oracle's own trajectory, so every step is
compared, and checks the path's own selection on each replayed remainder:
its choice equals the oracle's wherever the oracle's lead exceeds
PICK_MARGIN, its |.|^2 is within NEAR_TIE of the oracle's maximum at every
step, and (FP32 mode) the oracle's winner was on the re-checked short-list.
"""
from __future__ import annotations

import numpy as np

import oracle as O

TOL = {"fp64": 1e-12, "fp32": 1e-5}
MARGIN_MIN = 1e-6
NEAR_TIE = 1e-11
PICK_MARGIN = 1e-10
REL_FLOOR = 1e-2
RESIDUAL_FLOOR = 1e-16
FLAG_FORCED_LISTED = 16

FIELDS = ("index", "a", "coef", "energy", "margin", "remainder", "recheck_count", "flags", "fp32_error",
          "pick_index", "pick_p", "pick_margin", "pick_flags")


def to_numpy(res):
    out = {}
    for name in FIELDS:
        v = getattr(res, name, None)
        if v is None:
            continue
        if hasattr(v, "detach"):
            v = v.detach().cpu().numpy()
        out[name] = np.asarray(v)
    return out


def _ring_tie(ref, k, radii) -> bool:
    """Oracle step k picked (m, 0) on a zero radius with an exact tie: the r = 0 ring."""
    if radii is None or ref.margin[k] != 0.0:
        return False
    m, j = (int(v) for v in ref.index[k])
    return j == 0 and float(radii[m]) == 0.0


def _cut(flags, k, prec) -> bool:
    """FP32 mode: step k's band or a per-radius list was cut (flag bits 0, 1)."""
    return prec == "fp32" and bool(int(flags[k]) & 3)


def converged_step(ref, tol, steps=None) -> int:
    """The first step whose remainder (energy E_k entering it) is below the
    rounding level of the update: sqrt(E_k) <= RESIDUAL_FLOOR / tol * sqrt(E_0)."""
    S = ref.coef.shape[0] if steps is None else steps
    cut = (RESIDUAL_FLOOR / tol) ** 2 * ref.energy[0]
    for k in range(S):
        if ref.energy[k] <= cut:
            return k
    return S


def _check_step(g, ref, k, tol, prec, report):
    assert abs(g["a"][k] - ref.a[k]) <= 1e-13, (k, g["a"][k], ref.a[k])
    c = ref.coef[k]
    scale = np.sqrt(ref.energy[k])
    err = abs(g["coef"][k] - c)
    ec = err / max(abs(c), scale)
    assert ec <= tol, (k, "coef", ec, g["coef"][k], c)
    report["worst_coef"] = max(report["worst_coef"], ec)
    if abs(c) >= REL_FLOOR * scale and abs(c) > 0:
        er = err / abs(c)
        assert er <= tol, (k, "coef (relative)", er, g["coef"][k], c)
        report["worst_coef_rel"] = max(report["worst_coef_rel"], er)
    E0 = ref.energy[0]
    ee = abs(g["energy"][k + 1] - ref.energy[k + 1]) / max(E0, ref.energy[k + 1])
    assert ee <= tol, (k, "energy", ee, g["energy"][k + 1], ref.energy[k + 1])
    report["worst_energy"] = max(report["worst_energy"], ee)


def compare(gpu, ref: "O.Decomposition", tol: float, signal=None, radii=None, forced_first: bool = False,
            prec: str | None = None, nonuniform=None):
    """Free-running GPU decomposition against the oracle's.  Return
    (steps_compared, report dict); raise AssertionError on a violation.
    `nonuniform` = (turns, weights, n) for a decomposition of non-uniform
    samples (the near-tie check then evaluates the quadrature rule)."""
    g = to_numpy(gpu)
    prec = prec or ("fp64" if tol <= TOL["fp64"] else "fp32")
    S = ref.coef.shape[0]
    E0 = ref.energy[0]
    assert abs(g["energy"][0] - E0) <= tol * E0 + 1e-300, ("E0", g["energy"][0], E0)
    conv = converged_step(ref, tol)
    upto = conv
    for k in range(conv):
        lead = TOL["fp32"] if _cut(g["flags"], k, prec) else MARGIN_MIN
        decided = (forced_first and k == 0) or (ref.margin[k] > lead) or _ring_tie(ref, k, radii)
        if not decided:
            upto = k
            break
    report = {"worst_coef": 0.0, "worst_coef_rel": 0.0, "worst_energy": 0.0, "worst_margin": 0.0}
    if conv < S:
        report["converged_step"] = conv
    for k in range(upto):
        assert tuple(g["index"][k]) == tuple(ref.index[k]), (k, g["index"][k], ref.index[k], ref.margin[k])
        _check_step(g, ref, k, tol, prec, report)
        if prec == "fp64" and not (forced_first and k == 0):
            dm = abs(g["margin"][k] - ref.margin[k])
            assert dm <= 1e-10, (k, "margin", g["margin"][k], ref.margin[k])
            report["worst_margin"] = max(report["worst_margin"], dm)
    if upto < conv and signal is not None and radii is not None:
        # near-tie: the GPU's choice must be one of the (nearly) equal maxima of
        # the oracle grid, whose maximum is |c_k|^2 of the oracle's own step
        # (the trajectories agree up to here)
        m, j = (int(v) for v in g["index"][upto])
        if nonuniform is not None:
            t, w, n = nonuniform
            Gk = (O.decompose_nu(signal, t, w, radii, n, upto, forced=ref.index[:upto], form="series").remainder
                  if upto > 0 else signal)
            # the quadrature rule itself (the series cut at n terms misses radii near 1)
            p = abs(O.grid_direct_nu(Gk, t, w, np.asarray(radii)[m:m + 1], n)[0, j]) ** 2
        else:
            Gk = O.decompose_streamed(signal, radii, upto, forced=ref.index[:upto]).remainder if upto > 0 else signal
            p = abs(O.grid_fft(Gk, np.asarray(radii)[m:m + 1])[0, j]) ** 2
        pmax = abs(ref.coef[upto]) ** 2
        bar = TOL["fp32"] if _cut(g["flags"], upto, prec) else NEAR_TIE
        assert p >= pmax * (1 - bar), ("near-tie choice not maximal", upto, p, pmax, bar)
        report["near_tie_step"] = upto
        report["near_tie_gap"] = float((pmax - p) / pmax) if pmax > 0 else 0.0
    report["steps_compared"] = upto
    report["steps"] = S
    return upto, report


def compare_replay(gpu, ref: "O.Decomposition", prec: str, radii=None, steps=None):
    """A replay along the oracle's own trajectory (forced = ref.index) against
    the oracle, at every step.  Return a report dict; raise AssertionError on
    a violation."""
    g = to_numpy(gpu)
    tol = TOL[prec]
    S = ref.coef.shape[0] if steps is None else steps
    E0 = ref.energy[0]
    assert abs(g["energy"][0] - E0) <= tol * E0 + 1e-300, ("E0", g["energy"][0], E0)
    report = {"worst_coef": 0.0, "worst_coef_rel": 0.0, "worst_energy": 0.0, "worst_pick_p": 0.0,
              "picks_compared": 0, "steps": S}
    conv = converged_step(ref, tol, S)
    if conv < S:
        report["converged_step"] = conv
    for k in range(conv):
        assert tuple(g["index"][k]) == tuple(ref.index[k]), (k, g["index"][k], ref.index[k])
        _check_step(g, ref, k, tol, prec, report)
        # the path's own selection on the oracle's remainder G_k
        pmax = abs(ref.coef[k]) ** 2
        pp = g["pick_p"][k]
        dp = abs(pp - pmax) / pmax if pmax > 0 else abs(pp)
        cut = _cut(g["pick_flags"], k, prec)
        bar = TOL["fp32"] if cut else NEAR_TIE
        assert pp >= pmax * (1 - bar) and pp <= pmax * (1 + NEAR_TIE) + 1e-300, (k, "pick P", pp, pmax, bar)
        report["worst_pick_p"] = max(report["worst_pick_p"], dp)
        if ref.margin[k] > (TOL["fp32"] if cut else PICK_MARGIN) or _ring_tie(ref, k, radii):
            assert tuple(g["pick_index"][k]) == tuple(ref.index[k]), (k, "pick", g["pick_index"][k], ref.index[k],
                                                                      ref.margin[k])
            report["picks_compared"] += 1
        if prec == "fp64":
            assert abs(g["pick_margin"][k] - ref.margin[k]) <= 1e-10, (k, "pick margin", g["pick_margin"][k],
                                                                       ref.margin[k])
        elif not cut:
            # the oracle's winner was re-checked in double (it was within the band)
            assert g["pick_flags"][k] & FLAG_FORCED_LISTED, (k, "oracle winner not on the short-list",
                                                             g["pick_flags"][k])
            pm = g["pick_margin"][k]
            assert np.isnan(pm) or pm >= ref.margin[k] - 1e-10, (k, pm, ref.margin[k])
    return report
