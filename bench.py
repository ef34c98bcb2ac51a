#!/usr/bin/env python3
"""Benchmark of the FFT-based Core-AFD loop on one MI355X.

One benchmark step = one complete decomposition (afd_decompose) of the
workload: per AFD step the forward DFT of the remainder, the weighted
inverse DFT / |.|^2 / selection over the whole M x N polar grid, the
selection merge (FP32 mode: short-list + FP64 direct-rule recheck), the
Blaschke update and the energy.  Inputs are resident in HBM before the timed
region; outputs stay on the device.

Workload (default, `chirp1m`): the large single decomposition, N = 2^20,
M = 2000 radii uniform in [0, 0.999], 100 AFD steps of the analytic part of a
linear chirp + 3 Gaussian-windowed tones + white noise at 20 dB (seeded,
synthetic); its radius transforms run beyond the LDS (one row pass for short
spectra, two passes through HBM for the longest).  `value` is the FP64
path; the FP32 + double re-check path is under "fp32", and the N = 16384,
M = 1000, 50-step workload (40 Szego kernels + noise at 30 dB; LDS-resident
transforms) under "single16k", and the same recipe at N = 3^8 = 6561 (the
radix-3 transforms) under "tern6561" and at N = 5^6 = 15625 (the radix-5
transforms) under "pow5_15625".
`--workload single16k` (or `tern6561`, `pow5_15625`) times that workload alone;
`--workload mixed12288` the same recipe at N = 12288 = 3 * 2^12 (mixed-radix
transforms).
`--workload nonuni16k` times non-uniform samples (also the "nonuni16k" key
of the default line): 16384 jittered positions with trapezoidal weights, a
grid of N = 16384 angles, M = 1000 radii uniform in [0, 0.996], 50 steps.
`--workload batch512` times the uniform batch: 512 signals of N = 4096
(8..32 kernels, |b| <= 0.95), M = 512, 30 steps, decomposed together.
`--workload small1k` times the small latency-bound case: N = 1024, M = 100
radii m/100, 10 steps, FP64 only, 200 solves for p50/p99.
`--workload mixed` times a batch of uneven N (32 signals, N log-uniform over
2^10..2^14, M = N/8, 20 steps, FP64) one plan after another and as one group
graph (afd_group_launch).
`--workload serve` runs the served stream: 2000 requests with N log-uniform
over 2^10..2^16, M = N/8, 5..100 steps, signals as in the N = 16384
workload, one after another on one stream (the plain per-signal method), then
through the continuous-batching server all at once (throughput) and with
Poisson arrivals at 0.3, 0.5, 0.7 and 0.9 times that request rate (p50/p99
latency).

Prints ONE JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid evals/s (M·N·steps/s) FP32+recheck vs FP64; p50/p99 solve latency"
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}  # MI355X vector peaks (fp32 figure assumes packed math)
HBM_PEAK_BPS = 8.0e12  # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flops_per_eval(n: int) -> float:
    """Algorithmic work per grid value: one inverse-DFT share (5 log2 N, the
    standard nominal count of a complex FFT, used for every N) plus the weight
    multiply, |.|^2 and compare (6)."""
    return 5.0 * math.log2(n) + 6.0


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


# Measured HBM traffic of the radius kernels (rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by a copy of known size), valid only for the sources it was taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


# The translation unit each measured kernel is compiled from; its counters
# stay valid while that file and every header of csrc/ are unchanged.
KERNEL_SOURCES = {
    "k_big_": "afd_large.hip", "k_radius_pp": "afd_primepow.hip", "k_fwd_pp": "afd_primepow.hip",
    "k_radius_mixed": "afd_mixed.hip", "k_fwd_mixed": "afd_mixed.hip",
    "k_radius<": "afd_radius.hip", "k_advance": "afd_advance.hip", "k_fwd_": "afd_fwd.hip",
    "k_fft_fwd": "afd_fwd.hip", "k_nu_": "afd_nonuni.hip", "k_recon": "afd_recon.hip",
    "k_analytic": "afd_recon.hip",
}
STEP_KERNELS = ("k_update", "k_recheck", "k_prepare", "k_merge", "k_pick", "k_force", "k_zero")


def kernel_source(kernel: str) -> str:
    for prefix, f in KERNEL_SOURCES.items():
        if kernel.startswith(prefix):
            return f
    if kernel.startswith(STEP_KERNELS):
        return "afd_step.hip"
    return ""


def source_hashes() -> dict:
    """sha256 of each device source of csrc/ (every .hip and .h file except
    afd_api.hip, which holds the host side of the library only)."""
    csrc = os.path.join(ROOT, "paper_1711_08604_amd", "csrc")
    out = {}
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")) and f != "afd_api.hip":
            with open(os.path.join(csrc, f), "rb") as fh:
                out[f] = hashlib.sha256(fh.read()).hexdigest()
    return out


def measured_counters(kernel: str):
    """The counter record of `kernel` (bytes and VALU instructions per launch)
    if its translation unit and the headers are as they were measured, else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    then, now = t.get("sources", {}), source_hashes()
    unit = kernel_source(kernel)
    if not unit or then.get(unit) != now.get(unit):
        return None
    if any(then.get(f) != h for f, h in now.items() if f.endswith(".h")):
        return None
    return t.get("kernels", {}).get(kernel)


def measured_traffic(kernel: str):
    """Bytes per launch for `kernel` if measured on the current sources, else None."""
    k = measured_counters(kernel)
    return None if k is None else float(k["bytes_per_launch"])


# VALU issue capacity: each CU issues one wave64 vector instruction per clock
# (four SIMD16 units, four clocks per wave64 instruction)
CUS, CLOCK_HZ = 256, 2.4e9


def two_pass_radii(radii, n: int, prec: str) -> int:
    """Radii whose significant spectrum length exceeds 16 N2, N2 = 2^(K - K//2):
    only those go through the HBM intermediate (terms r^l below 2^-40 single /
    2^-60 double precision of the largest, summed, are dropped; lengths up to
    16 N2 run in row passes of the split shifted by a factor 4 or 16)."""
    bits = 60 if prec == "fp64" else 40
    k = int(math.log2(n))
    n2 = 16 << (k - k // 2)
    count = 0
    for r in radii:
        r = float(r)
        if r <= 0.0:
            continue
        need = (bits * math.log(2.0) - math.log1p(-r)) / -math.log(r)
        if math.ceil(need) > n2:
            count += 1
    return count


# The radius kernel's duration is measured on every TIMING_EVERY-th launch of
# the timed decompositions (7 is coprime with the step counts, so the sampled
# steps rotate): a stamped dispatch costs a few microseconds of stream time.
TIMING_EVERY = 7


def _kernel_name(prec, n):
    tname = "double" if prec == "fp64" else "float"
    if n & (n - 1):
        p = next(q for q in (3, 5, 7) if n % q == 0)
        k = round(math.log(n, p))
        if p ** k == n:  # N = p^K
            return f"k_radius_pp<{tname},{p},{k}>"
        return f"k_radius_mixed<{tname}>"  # mixed radix
    k = int(math.log2(n))
    return f"k_radius<{tname},{k}>" if n <= (1 << 14) else f"k_big_rows<{tname},{k}>"


def run_gpu(prec, sig, radii, afd_steps, steps, warmup, torch, kernel_timing=True, n_grid=None, plan_kw=None):
    """Time `steps` whole decompositions after `warmup` untimed ones; the
    dominant kernel (the radius kernel, or at N > 2^14 the row pass of the
    radius transforms, one launch per chunk of radii) is timed live on every
    TIMING_EVERY-th launch with events its dispatch stamps."""
    from paper_1711_08604_amd import Plan
    batch = int(sig.shape[0]) if sig.dim() == 2 else 1
    # (non-uniform samples: n_grid angles, the signal holds the samples)
    n = n_grid or int(sig.numel()) // batch
    m = len(radii)
    big = n > (1 << 14)
    kind = "rows" if big else "radius"
    stream = torch.cuda.current_stream().cuda_stream
    plan = Plan(n, radii, precision=prec, stream=stream, batch=batch, **(plan_kw or {}))
    per_solve = 0
    if kernel_timing:
        # launches of the timed kernel per decomposition (every one stamped, untimed)
        plan.set_timing(kind, 1)
        plan.decompose(sig, afd_steps)
        per_solve = plan.kernel_time()[1]
        plan.set_timing(kind, False)
    for _ in range(warmup):
        plan.decompose(sig, afd_steps)
    torch.cuda.synchronize()
    if kernel_timing:
        plan.set_timing(kind, TIMING_EVERY)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        res = plan.decompose(sig, afd_steps)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms, k_launches = plan.kernel_time()
    blocks, threads, lds = plan.radius_launch()
    plan.set_timing(kind, False)
    plan.close()
    evals = float(m) * n * afd_steps * steps * batch
    if not kernel_timing:  # (counter runs under a profiler: no stamped dispatches)
        return {"value": evals / wall, "ms_per_step": wall / steps * 1e3, "p50_ms": percentile(lat, 0.5) * 1e3,
                "p99_ms": percentile(lat, 0.99) * 1e3, "roofline": {"kernel": _kernel_name(prec, n), "frac": float("nan"),
                                                                     "avg_launch_us": float("nan")}}
    avg_kernel_s = (k_ms / 1e3) / max(k_launches, 1)
    # algorithmic work of one launch: the step's grid values share the launches
    # of the step (one radius-kernel launch, or one row pass per chunk of radii)
    launches_per_step = per_solve / afd_steps
    flop_launch = float(m) * n * flops_per_eval(n) * batch / launches_per_step
    achieved = flop_launch / avg_kernel_s / 1e12
    peak = PEAK_TFLOPS[prec]
    kname = _kernel_name(prec, n)
    traffic = measured_traffic(kname)
    cnt = measured_counters(kname)
    valu = None if cnt is None or "valu_insts_per_launch" not in cnt else float(cnt["valu_insts_per_launch"])
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic, "traffic_unit": "bytes/launch", "kernel": kname,
            "avg_launch_us": avg_kernel_s * 1e6, "launches_sampled": k_launches,
            "launches_per_afd_step": launches_per_step, "flop_per_launch": flop_launch,
            "hbm_gbs": None if traffic is None else traffic / avg_kernel_s / 1e9,
            "hbm_frac": None if traffic is None else traffic / avg_kernel_s / HBM_PEAK_BPS,
            "valu_insts_per_launch": valu,
            "valu_busy": None if valu is None else valu / (CUS * CLOCK_HZ * avg_kernel_s)}
    if big:
        roof["two_pass_radii"] = two_pass_radii(radii, n, prec)
        roof["row_grid"] = [blocks, threads, lds]
    else:
        roof["grid"] = [blocks, threads, lds]
    lat_sorted = sorted(lat)
    out = {
        "value": evals / wall,
        "ms_per_step": wall / steps * 1e3,
        "p50_ms": percentile(lat, 0.5) * 1e3,
        "p99_ms": percentile(lat, 0.99) * 1e3,
        "latency_ms": {"min": lat_sorted[0] * 1e3, "median": percentile(lat, 0.5) * 1e3,
                       "max": lat_sorted[-1] * 1e3},
        "roofline": roof,
    }
    if prec == "fp32":
        out["fp32_error_max"] = float(res.fp32_error.max().item())
        out["recheck_count_mean"] = float(res.recheck_count.double().mean().item())
    out["index_last"] = [int(x) for x in res.index.reshape(-1, 2)[-1].tolist()]
    return out


def run_graph(prec, sig, radii, afd_steps, steps, warmup, torch):
    """The same decompositions as run_gpu, each one replay of a HIP graph that
    captured the whole decomposition (afd_graph_create); per-solve latency is
    launch to completion."""
    from paper_1711_08604_amd import Plan
    batch = int(sig.shape[0]) if sig.dim() == 2 else 1
    n = int(sig.numel()) // batch
    stream = torch.cuda.current_stream().cuda_stream
    plan = Plan(n, radii, precision=prec, stream=stream, batch=batch)
    gr = plan.graph(sig, afd_steps)
    for _ in range(warmup):
        gr.launch()
    gr.status()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        gr.launch()
        torch.cuda.current_stream().synchronize()
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gr.status()
    gr.close()
    plan.close()
    evals = float(len(radii)) * n * afd_steps * steps * batch
    return {"value": evals / wall, "ms_per_step": wall / steps * 1e3, "p50_ms": percentile(lat, 0.5) * 1e3,
            "p99_ms": percentile(lat, 0.99) * 1e3}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, radii, steps_sample, total_steps):
    """The FP64 oracle as it stands, timed on this host on a bounded sample of
    the same workload: an all-cores leg (the oracle's grid streamed by radius
    chunks over one thread per usable core) and a one-worker leg."""
    import numpy as np

    import oracle as O
    cores = len(os.sched_getaffinity(0))
    batched = g.ndim == 2
    if batched:
        g = g[0]  # the oracle decomposes one signal at a time
    n = g.shape[0]
    base = {"unit": "grid evals/s", "kind": "oracle", "cpu_model": _cpu_model(), "affinity_cores": cores,
            "numpy": np.__version__}
    if n <= (1 << 14):
        t0 = time.perf_counter()
        O.decompose(g, radii, steps_sample)
        dt1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.decompose_streamed(g, radii, steps_sample, chunk=max(1, len(radii) // (4 * cores)), workers=cores)
        dta = time.perf_counter() - t0
        evals = float(len(radii)) * n * steps_sample
        what = f"first {steps_sample} of the {total_steps} AFD steps" + (" of signal 0 of the batch" if batched else "")
        one = {"value": evals / dt1, "seconds": dt1, "sample": f"decompose(), one thread, {what}"}
        return {**base, "value": evals / dta, "cores": cores, "seconds": dta,
                "sample": f"decompose_streamed(), {cores} threads, {what}", "one_worker": one}
    # N > 2^14: the whole grid of step 1 on every core, a twentieth of its radii on one
    t0 = time.perf_counter()
    O.decompose_streamed(g, radii, 1, chunk=4, workers=cores)
    dta = time.perf_counter() - t0
    sub = radii[::20]
    t0 = time.perf_counter()
    O.decompose_streamed(g, sub, 1, chunk=4, workers=1)
    dt1 = time.perf_counter() - t0
    one = {"value": float(len(sub)) * n / dt1, "seconds": dt1,
           "sample": f"grid, selection and update of AFD step 1 over {len(sub)} of the {len(radii)} radii, one thread"}
    return {**base, "value": float(len(radii)) * n / dta, "cores": cores, "seconds": dta,
            "sample": f"grid ({len(radii)} x {n}), selection and update of AFD step 1 of {total_steps}, "
                      f"{cores} threads", "one_worker": one}


def run_mixed(args, np, torch, W):
    """A batch of uneven N: 32 signals, N log-uniform over 2^10..2^14 (seeded),
    M = N/8 radii uniform in [0, 0.999], 20 AFD steps each, FP64, signals as
    in the N = 16384 workload.  Timed one plan after another on one stream
    (afd_decompose per signal), then as one group graph (afd_group_launch:
    a branch per plan, all concurrent)."""
    from paper_1711_08604_amd import Group, Plan
    rng = W.rng_for(7, 0)
    ks = rng.integers(10, 15, size=32)
    steps = 20
    stream = torch.cuda.current_stream().cuda_stream
    members, sigs = [], []
    for i, k in enumerate(ks):
        n = 1 << int(k)
        g, radii, _ = W.shaped_like_config2(n, n // 8, steps, item=700 + i)
        plan = Plan(n, radii, precision="fp64", stream=stream)
        sig = torch.from_numpy(g).to("cuda:0")
        members.append((plan, sig, steps))
        sigs.append(sig)
    evals = float(sum(p.m * p.n for p, _, _ in members)) * steps
    reps = max(args.steps or 5, 3)
    for p, s_, st in members:
        p.decompose(s_, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for p, s_, st in members:
            p.decompose(s_, st)
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) / reps
    with Group(members) as grp:
        grp.launch()
        grp.status()
        t0 = time.perf_counter()
        for _ in range(reps):
            grp.launch()
        grp.status()
        grouped = (time.perf_counter() - t0) / reps
    for p, _, _ in members:
        p.close()
    log(f"bench: mixed one after another {seq * 1e3:.2f} ms, group {grouped * 1e3:.2f} ms per batch")
    return {"metric": "grid evals/s of a batch of uneven N", "value": evals / grouped, "unit": "grid evals/s",
            "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": grouped * 1e3, "higher_is_better": True,
            "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "batch of 32 signals, N log-uniform over 2^10..2^14 (" +
                       ",".join(str(1 << int(k)) for k in ks) + "), M = N/8 radii uniform in [0,0.999], "
                       "20 AFD steps each, FP64; 40 normalised Szego kernels + CN noise at 30 dB"},
            "one_after_another": {"value": evals / seq, "ms_per_batch": seq * 1e3},
            "group_graph": {"value": evals / grouped, "ms_per_batch": grouped * 1e3}}


def run_serve(args, np, torch, W):
    """The served stream through paper_1711_08604_amd.serve.Server (FP32+recheck):
    the plain per-signal method (the requests one after another on one
    stream), then the server with every request present at once (saturated
    throughput), then Poisson arrivals at 0.3, 0.5, 0.7 and 0.9 times that
    request rate (p50/p99 latency from arrival to completion)."""
    from paper_1711_08604_amd.serve import Server
    rng = np.random.default_rng(20171108)
    reqs = []
    for i in range(args.requests):
        n = int(2 ** rng.integers(10, 17))
        steps = int(rng.integers(5, 101))
        g, radii, _ = W.shaped_like_config2(n, n // 8, steps, item=4000 + i)
        reqs.append((g, radii, steps))
    evals = float(sum(len(r) * g.shape[0] * s for g, r, s in reqs))
    log(f"bench: serve {len(reqs)} requests, {evals:.3e} grid evals")

    def stream(arrivals):
        with Server(slots=8) as srv:
            # warm the plans of every N (not timed)
            for n in sorted({g.shape[0] for g, _, _ in reqs}):
                g, r, s = next(q for q in reqs if q[0].shape[0] == n)
                srv.submit(g, r, 1).result()
            t0 = time.perf_counter()
            futs = []
            for (g, r, s), at in zip(reqs, arrivals):
                delay = t0 + at - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                futs.append(srv.submit(g, r, s))
            out = [f.result() for f in futs]
            wall = time.perf_counter() - t0
            shared = (srv.shared_calls, srv.shared_members)
        lat = [o.latency for o in out]
        return wall, lat, shared

    # the plain per-signal method: the same requests one after another on one stream
    from paper_1711_08604_amd import Plan
    plans = {}
    for g, r, s in reqs:
        if g.shape[0] not in plans:
            plans[g.shape[0]] = Plan(g.shape[0], r, precision="fp32")
            plans[g.shape[0]].decompose(g, 1)
    t0 = time.perf_counter()
    seq_lat = []
    for g, r, s in reqs:
        plans[g.shape[0]].decompose(g, s)
        seq_lat.append(time.perf_counter() - t0)  # all requests present at t0
    wall_seq = time.perf_counter() - t0
    for p in plans.values():
        p.close()
    log(f"bench: serve sequential (one stream) {evals / wall_seq:.3e} evals/s, {wall_seq:.1f} s")

    wall0, lat0, shared0 = stream([0.0] * len(reqs))
    rate = len(reqs) / wall0
    log(f"bench: serve saturated {evals / wall0:.3e} evals/s ({rate:.1f} req/s), p50 "
        f"{percentile(lat0, 0.5) * 1e3:.0f} ms, p99 {percentile(lat0, 0.99) * 1e3:.0f} ms")
    sweep = {}
    for frac in (0.3, 0.5, 0.7, 0.9):
        lam = frac * rate
        arrivals = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
        arrivals -= arrivals[0]
        wall, lat, shared = stream(list(arrivals))
        sweep[str(frac)] = {"rate_req_s": lam, "wall_s": wall, "evals_per_s": evals / wall,
                            "p50_ms": percentile(lat, 0.5) * 1e3, "p99_ms": percentile(lat, 0.99) * 1e3,
                            "shared_calls": shared[0], "shared_member_segments": shared[1]}
        log(f"bench: serve Poisson {frac}x = {lam:.1f} req/s: p50 {sweep[str(frac)]['p50_ms']:.1f} ms, "
            f"p99 {sweep[str(frac)]['p99_ms']:.1f} ms")
    at07 = sweep["0.7"]
    return {
        "metric": METRIC, "value": evals / wall0, "unit": "grid evals/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": wall0 * 1e3, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served stream: {len(reqs)} requests, N log-uniform over 2^10..2^16, M=N/8, steps "
                               "uniform in 5..100, signals as the N=16384 workload, 8 slots, FP32+recheck",
                   "requests": len(reqs), "grid_evals": evals},
        "p50_ms": at07["p50_ms"], "p99_ms": at07["p99_ms"],
        "serve": {"sequential_evals_per_s": evals / wall_seq, "sequential_wall_s": wall_seq,
                  "sequential_p50_ms": percentile(seq_lat, 0.5) * 1e3,
                  "sequential_p99_ms": percentile(seq_lat, 0.99) * 1e3,
                  "saturated_wall_s": wall0, "saturated_evals_per_s": evals / wall0,
                  "saturated_p50_ms": percentile(lat0, 0.5) * 1e3, "saturated_p99_ms": percentile(lat0, 0.99) * 1e3,
                  "saturated_shared_calls": shared0[0], "saturated_shared_member_segments": shared0[1],
                  "poisson": sweep},
    }


WORKLOADS = {
    "chirp1m": ("large single decomposition: N=2^20 samples, M=2000 radii uniform in [0,0.999], 100 AFD steps; "
                "analytic part of a linear chirp (0.01->0.4 cycles/sample) + 3 Gaussian-windowed tones + white "
                "noise at 20 dB", 5, 1),
    "single16k": ("single-signal Core-AFD: N=16384 samples, M=1000 radii uniform in [0,0.999], 50 AFD steps; 40 "
                  "normalised Szego kernels |b|<=0.98 + CN noise at 30 dB", 30, 3),
    "batch512": ("uniform batch: 512 signals of N=4096 samples (8..32 normalised Szego kernels, |b|<=0.95), M=512 "
                 "radii uniform in [0,0.999], 30 AFD steps each, decomposed together", 5, 1),
    "small1k": ("small single decomposition: N=1024 samples (5 normalised Szego kernels, |b|<=0.9), M=100 radii "
                "m/100, 10 AFD steps; launch-latency bound", 200, 10),
    "tern6561": ("single-signal Core-AFD at N=3^8=6561 samples (radix-3 transforms), M=1000 radii uniform in "
                 "[0,0.999], 50 AFD steps; 40 normalised Szego kernels |b|<=0.98 + CN noise at 30 dB", 30, 3),
    "pow5_15625": ("single-signal Core-AFD at N=5^6=15625 samples (radix-5 transforms), M=1000 radii uniform in "
                   "[0,0.999], 50 AFD steps; 40 normalised Szego kernels |b|<=0.98 + CN noise at 30 dB", 30, 3),
    "mixed12288": ("single-signal Core-AFD at N=12288=3*2^12 samples (mixed-radix transforms), M=1000 radii uniform "
                   "in [0,0.999], 50 AFD steps; 40 normalised Szego kernels |b|<=0.98 + CN noise at 30 dB", 30, 3),
    "nonuni16k": ("non-uniform samples: 16384 jittered positions (trapezoidal weights), a grid of N=16384 angles, "
                  "M=1000 radii uniform in [0,0.996], 50 AFD steps; 12 normalised Szego kernels |b|<=0.9 + CN noise "
                  "at 40 dB", 10, 2),
}

# grid angles of the non-uniform workload (its signal holds the samples)
NONUNI_GRID = 16384


def _workload(name, W):
    if name == "batch512":
        return W.config3_batch()
    if name == "small1k":
        return W.config1()
    if name == "chirp1m":
        return W.config5()
    if name == "tern6561":
        return W.shaped_like_config2(6561, 1000, 50)
    if name == "pow5_15625":
        return W.shaped_like_config2(15625, 1000, 50)
    if name == "mixed12288":
        return W.shaped_like_config2(12288, 1000, 50)
    if name == "nonuni16k":
        g, t = W.nonuniform_kernel_signal(16384, item=0, kind="jitter")
        return g, W.uniform_radii(1000, 0.996), 50, t
    return W.config2()


def _time_workload(name, W, torch, steps, warmup, only=None, kernel_timing=True):
    wl = _workload(name, W)
    g, radii, afd_steps = wl[:3]
    kw = {}
    if len(wl) > 3:  # non-uniform positions
        kw = {"n_grid": NONUNI_GRID, "plan_kw": {"sample_turns": wl[3]}}
    n, m = g.shape[-1], len(radii)
    log(f"bench: {name}: N={n} M={m} afd_steps={afd_steps} solves={steps} warmup={warmup}")
    sig = torch.from_numpy(g).to("cuda:0")
    torch.cuda.synchronize()
    res = {}
    for prec in ("fp64", "fp32"):
        if only and prec != only:
            continue
        res[prec] = run_gpu(prec, sig, radii, afd_steps, steps, warmup, torch, kernel_timing, **kw)
        log(f"bench: {name} {prec} {res[prec]['value']:.3e} evals/s, {res[prec]['ms_per_step']:.3f} ms/solve, "
            f"{res[prec]['roofline']['kernel']} {res[prec]['roofline']['avg_launch_us']:.1f} us per launch "
            f"({res[prec]['roofline']['frac']:.3f} of peak)")
    del sig
    return g, radii, afd_steps, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["chirp1m", "single16k", "batch512", "small1k", "tern6561", "pow5_15625",
                                           "mixed12288", "nonuni16k", "mixed", "serve"],
                    default="chirp1m")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests in the stream")
    ap.add_argument("--steps", type=int, default=None, help="timed decompositions (chirp1m: 5)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed decompositions (chirp1m: 1)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="chirp1m: skip the extra keys of the N=16384, 6561, 15625 and non-uniform workloads")
    ap.add_argument("--cpu-steps", type=int, default=5, help="AFD steps of the oracle sample (N <= 2^14)")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None)
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="no event-stamped dispatches (for hardware-counter runs); no roofline figures")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a known-size kernel for "
                         "scaling HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (the decomposition of one signal on one MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W

    if args.workload == "serve":
        print(json.dumps(run_serve(args, np, torch, W)), flush=True)
        return
    if args.workload == "mixed":
        print(json.dumps(run_mixed(args, np, torch, W)), flush=True)
        return

    wl_text, dsteps, dwarm = WORKLOADS[args.workload]
    if args.workload == "small1k":
        args.only = args.only or "fp64"
    args.steps = dsteps if args.steps is None else args.steps
    args.warmup = dwarm if args.warmup is None else args.warmup
    if args.copy_calibration_mib:
        n_el = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration {args.copy_calibration_mib} MiB read + {args.copy_calibration_mib} MiB written")
        del src, dst
    kt = not args.no_kernel_timing
    g, radii, afd_steps, res = _time_workload(args.workload, W, torch, args.steps, args.warmup, args.only, kt)
    n, m = g.shape[-1], len(radii)
    # the FP64 path is the primary figure (the paper computes in double); FP32 +
    # double re-check sits under its own key
    prim_key = "fp64" if "fp64" in res else "fp32"
    prim = res[prim_key]
    line = {
        "metric": METRIC,
        "value": prim["value"],
        "unit": "grid evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if prim_key == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": wl_text, "N": n, "M": m, "afd_steps": afd_steps,
                   "batch": int(g.shape[0]) if g.ndim == 2 else 1,
                   "mode": "FP64" if prim_key == "fp64" else "FP32 bulk + FP64 short-list recheck"},
        "p50_ms": prim["p50_ms"],
        "p99_ms": prim["p99_ms"],
        "latency_ms": prim.get("latency_ms"),
        "roofline": prim["roofline"],
    }
    if prim_key == "fp64" and "fp32" in res:
        f = res["fp32"]
        line["fp32"] = {k: f[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "latency_ms", "roofline",
                                          "fp32_error_max", "recheck_count_mean") if k in f}
        line["fp32"]["mode"] = "FP32 bulk + FP64 short-list recheck"
    if args.workload == "small1k":
        # the same solves replayed from a captured HIP graph
        sig = torch.from_numpy(g).to("cuda:0")
        gres = run_graph("fp64", sig, radii, afd_steps, args.steps, args.warmup, torch)
        log(f"bench: small1k graph {gres['value']:.3e} evals/s, p50 {gres['p50_ms']:.3f} ms, "
            f"p99 {gres['p99_ms']:.3f} ms")
        line["graph"] = gres
    if args.workload == "chirp1m" and not args.no_extra:
        # the N = 16384, M = 1000 workload: a second, VALU/LDS-bound regime
        _, _, _, r2 = _time_workload("single16k", W, torch, max(args.steps, 10), args.warmup, args.only, kt)
        line["single16k"] = {"workload": WORKLOADS["single16k"][0],
                             **{p: {k: v[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "roofline")}
                                for p, v in r2.items()}}
        # N = 3^8: the radix-3 transforms
        _, _, _, r3 = _time_workload("tern6561", W, torch, max(args.steps, 10), args.warmup, args.only, kt)
        line["tern6561"] = {"workload": WORKLOADS["tern6561"][0],
                            **{p: {k: v[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "roofline")}
                               for p, v in r3.items()}}
        # N = 5^6: the radix-5 transforms
        _, _, _, r5 = _time_workload("pow5_15625", W, torch, max(args.steps, 10), args.warmup, args.only, kt)
        line["pow5_15625"] = {"workload": WORKLOADS["pow5_15625"][0],
                              **{p: {k: v[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "roofline")}
                                 for p, v in r5.items()}}
        # non-uniform samples through the non-uniform DFT
        _, _, _, r4 = _time_workload("nonuni16k", W, torch, max(args.steps, 10), args.warmup, args.only, kt)
        line["nonuni16k"] = {"workload": WORKLOADS["nonuni16k"][0],
                             **{p: {k: v[k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "roofline")}
                                for p, v in r4.items()}}
    if args.workload == "nonuni16k" and not args.no_cpu:
        log("bench: no CPU oracle leg for the non-uniform workload (its oracle is the quadrature form)")
        args.no_cpu = True
    if not args.no_cpu:
        log("bench: CPU oracle baseline ...")
        line["cpu_baseline"] = cpu_baseline(g, radii, args.cpu_steps, afd_steps)
        log(f"bench: oracle {line['cpu_baseline']['value']:.3e} evals/s on {line['cpu_baseline']['cores']} cores, "
            f"{line['cpu_baseline']['one_worker']['value']:.3e} on one")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
