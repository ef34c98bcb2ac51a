#!/usr/bin/env python3
"""Benchmark of the FFT-based Core-AFD loop on one MI355X.

One benchmark step = one complete decomposition (afd_decompose) of the
workload below: 50 AFD steps, each a forward DFT of the remainder, the fused
weighted inverse DFT / |.|^2 / selection over the 1000 x 16384 polar grid, the
selection merge (FP32 mode: short-list + FP64 direct-rule recheck), the
Blaschke update and the energy.  Inputs are resident in HBM before the timed
region; outputs stay on the device.

Workload (default): single signal, N = 16384 samples, M = 1000 radii uniform
in [0, 0.999], 50 steps; G = 40 normalised Szego kernels with poles
|b| <= 0.98 and CN(0,1) weights plus CN noise at 30 dB SNR (seeded,
synthetic).  `--workload chirp1m` times the large decomposition instead:
N = 2^20, M = 2000, 100 steps of the analytic part of a chirp + 3 tones +
white noise at 20 dB, whose radius transforms run beyond the LDS (one row pass
for short spectra, two passes through HBM for the longest).
`--workload batch512` times the uniform batch: 512 signals of N = 4096
(8..32 kernels, |b| <= 0.95), M = 512, 30 steps, decomposed together.
`--workload small1k` times the small latency-bound case: N = 1024, M = 100
radii m/100, 10 steps, FP64 only, 200 solves for p50/p99.
`--workload serve` runs the served stream: requests with N log-uniform over
2^10..2^16, M = N/8, 5..100 steps, signals as in the default workload, through
the continuous-batching server, first all at once (throughput), then with
Poisson arrivals at 0.7x that request rate (p50/p99 latency).

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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flops_per_eval(n: int) -> float:
    """Algorithmic work per grid value: one inverse-DFT share (5 log2 N, the
    standard complex radix-2 count) plus the weight multiply, |.|^2 and compare (6)."""
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


def source_hash() -> str:
    """sha256 over the kernel sources and the C header (names and contents, sorted by name)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1711_08604_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    files.append(os.path.join(ROOT, "include", "afd.h"))
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """Bytes per launch for `kernel` if measured on the current sources, else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else float(k["bytes_per_launch"])


# bytes of the two-pass intermediate per grid value (written once, read once)
TWO_PASS_BYTES = {"fp32": 16, "fp64": 32}


def two_pass_radii(radii, n: int, prec: str) -> int:
    """Radii whose significant spectrum length exceeds N2 = 2^(K - K//2): only
    those go through the HBM intermediate (terms r^l below 2^-40 single /
    2^-60 double precision of the largest, summed, are dropped)."""
    bits = 60 if prec == "fp64" else 40
    k = int(math.log2(n))
    n2 = 1 << (k - k // 2)
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


def run_gpu(prec, sig, radii, afd_steps, steps, warmup, torch):
    from paper_1711_08604_amd import Plan
    batch = int(sig.shape[0]) if sig.dim() == 2 else 1
    n = int(sig.numel()) // batch
    m = len(radii)
    stream = torch.cuda.current_stream().cuda_stream
    plan = Plan(n, radii, precision=prec, stream=stream, batch=batch)
    for _ in range(warmup):
        plan.decompose(sig, afd_steps)
    torch.cuda.synchronize()
    plan.set_timing("radius", TIMING_EVERY)
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
    plan.set_timing("radius", False)
    plan.close()
    evals = float(m) * n * afd_steps * steps * batch
    avg_kernel_s = (k_ms / 1e3) / max(k_launches, 1)
    flop_launch = float(m) * n * flops_per_eval(n) * batch
    achieved = flop_launch / avg_kernel_s / 1e12
    peak = PEAK_TFLOPS[prec]
    tname = "double" if prec == "fp64" else "float"
    if n <= (1 << 14):
        kname = f"k_radius<{tname},{int(math.log2(n))}>"
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(kname), "traffic_unit": "bytes/launch",
                "kernel": kname,
                "avg_launch_us": avg_kernel_s * 1e6, "launches": k_launches,
                "flop_per_launch": flop_launch, "grid": [blocks, threads, lds]}
    else:
        # one timed unit = the column and row passes over all chunks of one AFD
        # step; only the radii with long spectra move through the intermediate,
        # the rest are formed in the row pass from the spectrum (ALU-bound)
        long_r = two_pass_radii(radii, n, prec)
        inter = float(long_r) * n * TWO_PASS_BYTES[prec]
        roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None,
                "kernel": f"k_big_rows<{tname},{int(math.log2(n))}> + k_big_cols (all radius chunks of a step)",
                "avg_launch_us": avg_kernel_s * 1e6, "launches": k_launches,
                "flop_per_launch": flop_launch, "two_pass_radii": long_r,
                "intermediate_bytes_per_launch": inter,
                "intermediate_gbs": inter / avg_kernel_s / 1e9,
                "row_grid": [blocks, threads, lds]}
    out = {
        "value": evals / wall,
        "ms_per_step": wall / steps * 1e3,
        "p50_ms": percentile(lat, 0.5) * 1e3,
        "p99_ms": percentile(lat, 0.99) * 1e3,
        "roofline": roof,
    }
    if prec == "fp32":
        out["fp32_error_max"] = float(res.fp32_error.max().item())
        out["recheck_count_mean"] = float(res.recheck_count.double().mean().item())
    out["index_last"] = [int(x) for x in res.index.reshape(-1, 2)[-1].tolist()]
    return out


def cpu_baseline(g, radii, steps_sample, total_steps):
    import numpy as np

    import oracle as O
    batched = g.ndim == 2
    if batched:
        g = g[0]  # the oracle decomposes one signal at a time
    n = g.shape[0]
    t0 = time.perf_counter()
    if batched:
        O.decompose(g, radii, steps_sample)
        evals = len(radii) * n * steps_sample
        what = f"first {steps_sample} of the {total_steps} AFD steps of signal 0 of the batch"
    elif n <= (1 << 14):
        O.decompose(g, radii, steps_sample)
        evals = len(radii) * n * steps_sample
        what = f"first {steps_sample} of the {total_steps} AFD steps of the same signal"
    else:
        # one step's grid over a subset of the radii (the full grid of one step
        # takes minutes and tens of GB on the host)
        sub = radii[:: max(1, len(radii) // 40)]
        O.select(O.grid_fft(g, sub))
        evals = len(sub) * n
        what = f"grid values and selection of step 1 over {len(sub)} of the {len(radii)} radii"
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "grid evals/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 FFT-form oracle (numpy pocketfft, single thread), {what}, {dt:.1f} s",
            "seconds": dt, "numpy": np.__version__}


def run_serve(args, np, torch, W):
    """The served stream through paper_1711_08604_amd.serve.Server (FP32+recheck)."""
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
        lat = [o.latency for o in out]
        return wall, lat

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
    log(f"bench: serve sequential (one stream) {evals / wall_seq:.3e} evals/s")

    wall0, lat0 = stream([0.0] * len(reqs))
    rate = len(reqs) / wall0
    lam = 0.7 * rate
    arrivals = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
    arrivals -= arrivals[0]
    wall1, lat1 = stream(list(arrivals))
    log(f"bench: serve saturated {evals / wall0:.3e} evals/s; Poisson at {lam:.1f} req/s: "
        f"p50 {percentile(lat1, 0.5) * 1e3:.1f} ms p99 {percentile(lat1, 0.99) * 1e3:.1f} ms")
    return {
        "metric": METRIC, "value": evals / wall0, "unit": "grid evals/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": wall0 * 1e3, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served stream: {len(reqs)} requests, N log-uniform over 2^10..2^16, M=N/8, steps "
                               "uniform in 5..100, signals as the default workload, 8 slots, FP32+recheck",
                   "requests": len(reqs), "grid_evals": evals},
        "p50_ms": percentile(lat1, 0.5) * 1e3, "p99_ms": percentile(lat1, 0.99) * 1e3,
        "serve": {"sequential_evals_per_s": evals / wall_seq, "sequential_wall_s": wall_seq,
                  "sequential_p50_ms": percentile(seq_lat, 0.5) * 1e3,
                  "sequential_p99_ms": percentile(seq_lat, 0.99) * 1e3,
                  "saturated_wall_s": wall0, "saturated_p50_ms": percentile(lat0, 0.5) * 1e3,
                  "saturated_p99_ms": percentile(lat0, 0.99) * 1e3, "poisson_rate_req_s": lam,
                  "poisson_wall_s": wall1, "poisson_evals_per_s": evals / wall1},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["single16k", "chirp1m", "batch512", "small1k", "serve"],
                    default="single16k")
    ap.add_argument("--requests", type=int, default=300, help="serve: requests in the stream")
    ap.add_argument("--steps", type=int, default=None, help="timed decompositions (30; chirp1m: 3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed decompositions (3; chirp1m: 1)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=5, help="AFD steps of the oracle sample")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None)
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

    if args.workload == "batch512":
        g, radii, afd_steps = W.config3_batch()
        wl_text = ("uniform batch: 512 signals of N=4096 samples (8..32 normalised Szego kernels, |b|<=0.95), "
                   "M=512 radii uniform in [0,0.999], 30 AFD steps each, decomposed together")
        dsteps, dwarm = 5, 1
    elif args.workload == "small1k":
        g, radii, afd_steps = W.config1()
        wl_text = ("small single decomposition: N=1024 samples (5 normalised Szego kernels, |b|<=0.9), "
                   "M=100 radii m/100, 10 AFD steps, FP64; launch-latency bound")
        dsteps, dwarm = 200, 10
        args.only = args.only or "fp64"
    elif args.workload == "chirp1m":
        g, radii, afd_steps = W.config5()
        wl_text = ("large single decomposition: N=2^20 samples, M=2000 radii uniform in [0,0.999], 100 AFD "
                   "steps; analytic part of a linear chirp + 3 Gaussian-windowed tones + white noise at 20 dB")
        dsteps, dwarm = 3, 1
    else:
        g, radii, afd_steps = W.config2()
        wl_text = ("single-signal Core-AFD: N=16384 samples, M=1000 radii uniform in [0,0.999], "
                   "50 AFD steps; 40 normalised Szego kernels |b|<=0.98 + CN noise at 30 dB")
        dsteps, dwarm = 30, 3
    args.steps = dsteps if args.steps is None else args.steps
    args.warmup = dwarm if args.warmup is None else args.warmup
    n, m = g.shape[-1], len(radii)
    log(f"bench: N={n} M={m} afd_steps={afd_steps} solves={args.steps} warmup={args.warmup}")
    sig = torch.from_numpy(g).to("cuda:0")
    torch.cuda.synchronize()
    if args.copy_calibration_mib:
        n_el = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration {args.copy_calibration_mib} MiB read + {args.copy_calibration_mib} MiB written")
        del src, dst
    res = {}
    for prec in ("fp32", "fp64"):
        if args.only and prec != args.only:
            continue
        res[prec] = run_gpu(prec, sig, radii, afd_steps, args.steps, args.warmup, torch)
        log(f"bench: {prec} {res[prec]['value']:.3e} evals/s, {res[prec]['ms_per_step']:.3f} ms/solve, "
            f"radius kernel(s) {res[prec]['roofline']['avg_launch_us']:.1f} us per AFD step")
    prim = res.get("fp32") or res.get("fp64")
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
        "dtype": "f32" if "fp32" in res else "f64",
        "data": "synthetic",
        "config": {"workload": wl_text, "N": n, "M": m, "afd_steps": afd_steps,
                   "batch": int(g.shape[0]) if g.ndim == 2 else 1,
                   "mode": "FP32 bulk + FP64 short-list recheck" if "fp32" in res else "FP64"},
        "p50_ms": prim["p50_ms"],
        "p99_ms": prim["p99_ms"],
        "roofline": prim["roofline"],
    }
    if "fp32_error_max" in prim:
        line["fp32_error_max"] = prim["fp32_error_max"]
        line["recheck_count_mean"] = prim["recheck_count_mean"]
    if "fp32" in res and "fp64" in res:
        line["fp64"] = {k: res["fp64"][k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms", "roofline")}
    if not args.no_cpu:
        log(f"bench: CPU oracle baseline, {args.cpu_steps} AFD steps ...")
        line["cpu_baseline"] = cpu_baseline(g, radii, args.cpu_steps, afd_steps)
        log(f"bench: oracle {line['cpu_baseline']['value']:.3e} evals/s")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
