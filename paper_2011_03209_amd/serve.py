"""Serving form: a Poisson stream of mapper requests over resident clouds.

Eight Gaussian-mixture clouds stay resident in one device arena; requests
(random lens, interval count, overlap, minPts; eps = 1.05 sqrt(2d)) are
submitted at their arrival times through mapper_submit and collected with
mapper_wait.  The library admits a request when a stream slot is free and its
workspace fits in the arena, so requests that arrive while others run overlap
on the device.  Latency = completion - arrival.

First the saturation throughput T is measured (all requests submitted at
once), then the stream is replayed at fractions of T; p50/p99 latency and
graphs/s are reported for each point, and the 0.7 T point is the headline.
"""
from __future__ import annotations

import json
import sys
import threading
import time

import numpy as np

from . import binding, synth


def _replay(ctx, clouds, reqs, t_origin):
    """Submit each request at its arrival time; return per-request latencies."""
    lat = [0.0] * len(reqs)
    lag = [0.0] * len(reqs)
    errs = []

    def one(k, t_arr, c, p):
        due = t_origin + t_arr
        delay = due - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        t_sub = time.perf_counter()
        try:
            tk = clouds[c].submit(p)
            binding.wait(ctx, tk)
        except Exception as e:    # reported, not hidden
            errs.append((k, repr(e)))
        # from the scheduled arrival: a client thread that wakes late still
        # counts its delay (reported on its own as the submission lag)
        lat[k] = time.perf_counter() - due
        lag[k] = max(0.0, t_sub - due)

    threads = [threading.Thread(target=one, args=(k, t, c, p)) for k, (t, c, p) in enumerate(reqs)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    if errs:
        raise RuntimeError(f"{len(errs)} requests failed, first: {errs[0]}")
    return np.array(lat), np.array(lag)


# Stream slots: measured on MI355X (one run each, 256 requests, at 70% of
# each setting's own saturation): 1 slot 289 graphs/s, p99 25 ms; 2 slots
# 437 graphs/s, p99 24 ms; 3 slots 536 graphs/s, p99 76 ms; 4 slots 573
# graphs/s, p99 36 ms.  More slots raise throughput, but large requests that
# share the chip with more others finish later, so two keep the lowest p99.
SLOTS = 2


def run(n_requests=256, slots=SLOTS, arena_gb=96.0, scale=1.0, fractions=(0.25, 0.5, 0.7, 0.9),
        precision=synth.PREC_BF16X3, log=sys.stderr):
    raw = synth.serving_clouds(scale=scale)
    ctx = binding.Context(arena_bytes=int(arena_gb * (1 << 30)), serving_streams=slots)
    clouds = [ctx.cloud(X) for X in raw]
    print(f"[serve] {len(clouds)} clouds resident", file=log, flush=True)
    base = synth.serving_requests(raw, n_requests, qps=1.0, precision=precision)
    # warm-up: the first request of each cloud
    seen = set()
    for _, c, p in base:
        if c not in seen:
            seen.add(c)
            clouds[c].run(p)
    # saturation: everything at t = 0
    sat = [(0.0, c, p) for (_, c, p) in base]
    t0 = time.perf_counter()
    _replay(ctx, clouds, sat, t0)
    t_sat = time.perf_counter() - t0
    T = n_requests / t_sat
    print(f"[serve] saturation {T:.2f} graphs/s", file=log, flush=True)
    points = []
    for fr in fractions:
        qps = fr * T
        reqs = synth.serving_requests(raw, n_requests, qps=qps, precision=precision)
        t0 = time.perf_counter()
        lat, lag = _replay(ctx, clouds, reqs, t0)
        wall = time.perf_counter() - t0
        points.append({"fraction_of_saturation": fr, "qps": qps, "graphs_per_s": n_requests / wall,
                       "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                       "p99_submit_lag_s": float(np.percentile(lag, 99))})
        print(f"[serve] {fr:.2f} T: p50 {points[-1]['p50_s']:.3f} s  p99 {points[-1]['p99_s']:.3f} s",
              file=log, flush=True)
    for c in clouds:
        c.destroy()
    ctx.close()
    return T, points


def main(args):
    T, points = run(n_requests=256, arena_gb=args.arena_gb)
    head = min(points, key=lambda p: abs(p["fraction_of_saturation"] - 0.7))
    print(json.dumps({
        "metric": "1M×256 mapper-graph seconds, BF16-MFMA vs FP32 path; p99 request latency",
        "value": head["p99_s"], "unit": "s", "n_gpus": 1, "steps": 256, "warmup": 8,
        "ms_per_step": 1e3 / head["graphs_per_s"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic (8 seeded Gaussian-mixture clouds)",
        "config": {"workload": "serving_8clouds_poisson", "requests": 256, "slots": SLOTS,
                   "qps": head["qps"], "saturation_graphs_per_s": T},
        "sweep": points,
    }))
