"""Benchmark: seconds per mapper graph of a 1,000,000 x 256 cloud on one MI355X.

A step is one whole mapper graph (lens -> cover -> pullback sets -> distance
tiles -> FP64 band recheck -> clusters -> nodes and edges) of the resident
cloud, timed from the host around mapper_run (the graph is on the host when
the step ends).  The cloud is uploaded once before timing.  The BF16 path (hi/lo split tiles + FP64
recheck) is the reported value; the plain FP32 path is timed beside it on the
same cloud, and its graph must be identical.

Prints ONE JSON line (rank 0) with the roofline of the dominant kernel (the
matrix-core distance tiles) and the FP64 CPU oracle timed on a bounded sample.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload mix1m_d256|mix500k_d128_grid|mix100k_d64]
  python bench.py --serve   # serving form: Poisson requests over 8 resident clouds
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2011_03209_amd import synth  # noqa: E402

PEAK = {"fp32": 157.3e12, "bf16": 2.5e15, "bf16x3": 2.5e15, "fp16": 2.5e15, "fp16x3": 2.5e15}
PREC_NAME = {0: "fp32", 1: "bf16", 2: "bf16x3", 3: "fp16", 4: "fp16x3"}


def workload(name: str, precision: int):
    if name == "mix1m_d256":
        return synth.mixture_1m_d256(precision=precision)
    if name == "mix500k_d128_grid":
        return synth.mixture_500k_d128_2d(precision=precision)
    if name == "mix100k_d64":
        w = synth.mixture_100k_d64()
        w.params.precision = precision
        return w
    raise SystemExit(f"unknown workload {name}")


def time_path(cloud, params, steps: int, warmup: int, flags: int = 0):
    import torch
    for _ in range(warmup):
        g = cloud.run(params, flags=flags)
    torch.cuda.synchronize()
    times, stats = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        g = cloud.run(params, flags=flags)
        times.append(time.perf_counter() - t0)
        stats.append(g.stats)
    torch.cuda.synchronize()
    return g, times, stats


def recorded_traffic(workload: str, precision: str):
    """HBM bytes per launch of the tile kernel from the committed rocprofv3
    counter record (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when the record is missing or was taken from
    another version of the kernel source (tile.hip, and internal.h, which
    holds the tile order and the panel layout)."""
    import hashlib
    rec = os.path.join(ROOT, "profiles", f"mapper_{workload}_{precision}.txt")
    csrc = os.path.join(ROOT, "paper_2011_03209_amd", "csrc")
    srcs = [os.path.join(csrc, "tile.hip"), os.path.join(csrc, "internal.h")]
    if not (os.path.exists(rec) and all(os.path.exists(s) for s in srcs)):
        return None
    kv = {}
    for line in open(rec):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(b"".join(open(s, "rb").read() for s in srcs)).hexdigest()[:16]
    if kv.get("tile_source_sha256_16") != sha:
        return None
    try:
        return float(kv["traffic_fetch_bytes"]) + float(kv["traffic_write_bytes"])
    except (KeyError, ValueError):
        return None


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, min_pair_frac: float = 0.2, max_s: float = 240.0):
    """The FP64 oracle timed on a stratified sample of whole cover elements.

    The oracle's cost is quadratic in the element size, so the sample always
    holds the largest element and then elements spread evenly over the size
    range until at least `min_pair_frac` of the
    in-element pairs have been timed (or `max_s` of DBSCAN time has passed).
    Each element left out is charged the per-pair time of the timed element
    closest to it in size; the lens and cover are timed in full."""
    from oracle import oracle as O
    X, p = w.X, w.params
    t0 = time.perf_counter()
    f = [O.lens(X, a) for a in p.axes]
    los, his = [], []
    for a, fa in zip(p.axes, f):
        lo, hi = O.cover(float(fa.min()), float(fa.max()), a.n_intervals, a.overlap)
        los.append(lo)
        his.append(hi)
    shape = [a.n_intervals for a in p.axes]
    elems = []
    for e in range(int(np.prod(shape))):
        idx = np.unravel_index(e, shape)
        m = np.ones(X.shape[0], bool)
        for a in range(len(p.axes)):
            m &= (los[a][idx[a]] <= f[a]) & (f[a] <= his[a][idx[a]])
        elems.append(np.nonzero(m)[0].astype(np.int32))
    t_lens = time.perf_counter() - t0
    pairs = np.array([len(m) * (len(m) + 1) / 2 for m in elems])
    total_pairs = float(pairs.sum())
    by_size = [int(e) for e in np.argsort(-pairs, kind="stable") if pairs[e] > 0]
    # the largest element, then elements spread over the size range (van der
    # Corput positions 1/2, 1/4, 3/4, 1/8, ... of the list sorted by size)
    pick, L = [by_size[0]], len(by_size)
    for k in range(1, 4 * L):
        q, x, b = 0.0, k, 0.5
        while x:
            q += b * (x & 1)
            x >>= 1
            b *= 0.5
        e = by_size[int(round(q * (L - 1)))]
        if e not in pick:
            pick.append(e)
    pick += [e for e in by_size if e not in pick]
    timed = {}
    t_db = done_pairs = 0.0
    for e in pick:
        if done_pairs >= min_pair_frac * total_pairs or t_db >= max_s:
            break
        t1 = time.perf_counter()
        O.dbscan(X, elems[e], p.eps, p.min_pts)
        dt = time.perf_counter() - t1
        timed[e] = dt
        t_db += dt
        done_pairs += pairs[e]
        print(f"[cpu_baseline] element {e}: {len(elems[e])} points, {dt:.2f} s "
              f"({100 * done_pairs / total_pairs:.1f}% of pairs timed)", file=sys.stderr, flush=True)
    sizes = {e: len(elems[e]) for e in timed}
    est = t_lens + t_db
    for e in by_size:
        if e in timed:
            continue
        near = min(timed, key=lambda q: abs(sizes[q] - len(elems[e])))
        est += timed[near] / pairs[near] * pairs[e]
    largest = by_size[0]
    return {"value": est, "unit": "s", "cores": O.threads(), "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
            "measured_pair_frac": done_pairs / total_pairs,
            "sample": f"{len(timed)} of {len(by_size)} non-empty cover elements timed whole, the largest "
                      f"({len(elems[largest])} points) included: {done_pairs:.3g} of {total_pairs:.3g} "
                      f"in-element pairs ({100 * done_pairs / total_pairs:.1f}%), {t_db:.1f} s of DBSCAN; "
                      f"lens and cover timed in full ({t_lens:.1f} s); every other element charged the "
                      f"per-pair time of the timed element nearest in size"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mix1m_d256")
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16", "bf16x3", "fp16", "fp16x3", "auto"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--serve", action="store_true", help="serving form only (its own JSON line)")
    ap.add_argument("--no-serve", action="store_true", help="leave the serving block out of the line")
    ap.add_argument("--arena-gb", type=float, default=64.0)
    ap.add_argument("--tile-form", default="auto", choices=["auto", "pairs", "macro"],
                    help="launch form of the distance tiles (auto: the library's choice)")
    ap.add_argument("--no-screen", action="store_true",
                    help="compute every tile pair (no screening of tile pairs by landmark cells)")
    ap.add_argument("--sweep", action="store_true", help="time every tile precision (stderr)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a plain copy kernel of known "
                         "size, used to scale FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the bench measures one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is designed, not run)"}))
        sys.exit(2)
    if args.serve:
        from paper_2011_03209_amd import serve
        serve.main(args)
        return
    import torch
    from paper_2011_03209_amd import binding
    prec = {"fp32": 0, "bf16": 1, "bf16x3": 2, "fp16": 3, "fp16x3": 4, "auto": 5}[args.precision]
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = workload(args.workload, prec)
    ctx = binding.Context(arena_bytes=int(args.arena_gb * (1 << 30)))
    cloud = ctx.cloud(w.X)
    print(f"[bench] workload {w.name} n={w.X.shape[0]} d={w.X.shape[1]} uploaded", file=sys.stderr, flush=True)
    if args.sweep:
        import copy
        for pv in (0, 1, 2, 3, 4):
            pp = copy.copy(w.params)
            pp.precision = pv
            _, ts, ss = time_path(cloud, pp, 2, 1)
            print(json.dumps({"sweep": PREC_NAME[pv], "s_per_graph": float(np.median(ts)),
                              **{k: ss[-1][k] for k in ("ms_tiles", "ms_recheck", "ms_cc", "ms_edges",
                                                        "ms_lens", "ms_bin", "band_pairs")}}),
                  file=sys.stderr, flush=True)
        pb = copy.deepcopy(w.params)
        pb.axes[0].cover = 1
        _, ts, ss = time_path(cloud, pb, 2, 1)
        print(json.dumps({"sweep": f"balanced cover {args.precision}", "s_per_graph": float(np.median(ts)),
                          **{k: ss[-1][k] for k in ("ms_lens", "ms_bin", "ms_tiles", "pairs", "band_pairs")}}),
              file=sys.stderr, flush=True)
        eps4 = [20.0, 22.0, 24.0, 26.0]
        t0 = time.perf_counter()
        cloud.run_eps_sweep(w.params, eps4)
        t1 = time.perf_counter()
        gs4 = cloud.run_eps_sweep(w.params, eps4)
        t2 = time.perf_counter()
        print(json.dumps({"sweep": f"eps sweep {eps4} {args.precision}", "s_for_all": t2 - t1,
                          "warm_s": t1 - t0, "ms_tiles": gs4[0].stats["ms_tiles"],
                          "ms_recheck": gs4[0].stats["ms_recheck"],
                          "ms_cc_each": [gg.stats["ms_cc"] for gg in gs4],
                          "nodes": [gg.n_nodes for gg in gs4]}), file=sys.stderr, flush=True)
        mp4 = [5, 10, 20, 40]
        cloud.run_sweep(w.params, [w.params.eps], mp4)
        t1 = time.perf_counter()
        gm = cloud.run_sweep(w.params, [w.params.eps], mp4)[0]
        t2 = time.perf_counter()
        print(json.dumps({"sweep": f"minPts sweep {mp4} at eps {w.params.eps} {args.precision}", "s_for_all": t2 - t1,
                          "ms_tiles": gm[0].stats["ms_tiles"], "ms_cc_each": [gg.stats["ms_cc"] for gg in gm],
                          "ms_edges_each": [gg.stats["ms_edges"] for gg in gm],
                          "nodes": [gg.n_nodes for gg in gm]}), file=sys.stderr, flush=True)
        sub = ctx.cloud(np.ascontiguousarray(w.X[:100_000]))
        sub.knn_d2(5, 5)
        t0 = time.perf_counter()
        kd, kst = sub.knn_d2(5, 5)                          # screening precision chosen by the library (FP16)
        t1 = time.perf_counter()
        print(json.dumps({"sweep": "knn k=5 100000x256 auto", "s": t1 - t0, "screen_precision": PREC_NAME[kst["precision"]],
                          "ms_screen": kst["ms_tiles"], "ms_fp64": kst["ms_recheck"],
                          "candidates": kst["band_pairs"], "pairs": kst["pairs"],
                          "median_knn_d": float(np.sqrt(np.median(kd)))}), file=sys.stderr, flush=True)
        # whole-cloud lenses on the same 100k x 256 points: the k-NN distance
        # (k = 5, a density filter) and the eccentricity, 20 intervals
        for name, kind in (("knn distance k=5", synth.LENS_KNN_DISTANCE), ("eccentricity", synth.LENS_ECCENTRICITY)):
            pl = synth.Params([synth.Axis(kind, 20, 0.3, column=5)], eps=w.params.eps, min_pts=w.params.min_pts,
                              precision=prec)
            sub.run(pl)
            t0 = time.perf_counter()
            gl = sub.run(pl)
            t1 = time.perf_counter()
            print(json.dumps({"sweep": f"{name} lens mapper 100000x256 {args.precision}", "s_per_graph": t1 - t0,
                              **{k: gl.stats[k] for k in ("ms_lens", "ms_tiles", "ms_recheck", "ms_cc", "pairs")},
                              "nodes": gl.n_nodes, "edges": gl.n_edges}), file=sys.stderr, flush=True)
        sub.destroy()
    tflags = {"auto": 0, "pairs": binding.FLAG_TILE_PAIRS, "macro": binding.FLAG_TILE_MACRO}[args.tile_form]
    if args.no_screen:
        tflags |= binding.FLAG_NO_SCREEN
    g, times, stats = time_path(cloud, w.params, args.steps, args.warmup, flags=tflags)
    print(f"[bench] {args.precision}: {np.median(times):.4f} s/graph", file=sys.stderr, flush=True)
    out = {}
    if not args.no_fp32 and prec != 0:
        import copy
        p32 = copy.copy(w.params)
        p32.precision = 0
        g32, t32, s32 = time_path(cloud, p32, max(1, min(args.steps, 3)), 1)
        same = (np.array_equal(g.node_offsets, g32.node_offsets) and np.array_equal(g.node_members, g32.node_members)
                and np.array_equal(g.edges, g32.edges) and np.array_equal(g.edge_weights, g32.edge_weights)
                and np.array_equal(g.node_element, g32.node_element))
        out["fp32_path"] = {"s_per_graph": float(np.median(t32)), "ms_tiles": float(np.median([s["ms_tiles"] for s in s32])),
                            "band_pairs": int(s32[-1]["band_pairs"]), "graph_identical": bool(same)}
        print(f"[bench] fp32: {np.median(t32):.4f} s/graph, identical={same}", file=sys.stderr, flush=True)
    if not args.no_fp32 and prec != 5:
        # the precision the library's own autotuner picks for this run (its
        # first run samples the five precisions; the timed runs reuse it)
        import copy
        pa = copy.copy(w.params)
        pa.precision = 5
        ga, ta, sa = time_path(cloud, pa, max(1, min(args.steps, 3)), 1)
        same = (np.array_equal(g.node_offsets, ga.node_offsets) and np.array_equal(g.node_members, ga.node_members)
                and np.array_equal(g.edges, ga.edges) and np.array_equal(g.edge_weights, ga.edge_weights)
                and np.array_equal(g.node_element, ga.node_element))
        out["auto_path"] = {"s_per_graph": float(np.median(ta)), "precision": PREC_NAME.get(sa[-1]["precision"]),
                            "ms_tiles": float(np.median([s["ms_tiles"] for s in sa])),
                            "band_pairs": int(sa[-1]["band_pairs"]), "graph_identical": bool(same)}
        print(f"[bench] auto ({out['auto_path']['precision']}): {np.median(ta):.4f} s/graph, identical={same}",
              file=sys.stderr, flush=True)
    cloud.destroy()
    st = stats[-1]
    used = PREC_NAME.get(st["precision"], "fp32")
    d = w.X.shape[1]
    ms_tiles = float(np.median([s["ms_tiles"] for s in stats]))
    # algorithmic work of the tile launch: 2d flops per in-element pair of
    # the tile pairs it computes (the screened-out ones are proven empty and
    # not launched)
    flops = 2.0 * d * st["pairs_computed"]
    achieved = flops / (ms_tiles * 1e-3)
    ms = float(np.median(times)) * 1e3
    line = {
        "metric": "1M×256 mapper-graph seconds, BF16-MFMA vs FP32 path; p99 request latency",
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": used,
        "data": "synthetic (seeded Gaussian mixture shaped like the paper's 1M x 256 activations)",
        "config": {"workload": w.name, "n": int(w.X.shape[0]), "d": int(d),
                   "lens": "projection" if w.params.axes[0].kind == 3 else "other",
                   "intervals": [a.n_intervals for a in w.params.axes],
                   "overlap": [a.overlap for a in w.params.axes], "eps": w.params.eps,
                   "min_pts": w.params.min_pts, "precision": used},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[used] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK[used], "traffic": recorded_traffic(w.name, used),
                     "traffic_source": (f"profiles/mapper_{w.name}_{used}.txt: rocprofv3 --pmc FETCH_SIZE, "
                                        "WRITE_SIZE of this kernel source (matched by its SHA-256), scaled by "
                                        "a 1 GiB copy; recorded, not measured in this run"),
                     "kernel": f"k_tiles<{used}>", "ms_per_launch": ms_tiles,
                     "algorithmic_flop": flops,
                     "issued_flop": flops * (3 if used.endswith("x3") else 1)},
        "stages_ms": {k: float(np.median([s[k] for s in stats])) for k in
                      ("ms_lens", "ms_bin", "ms_tiles", "ms_recheck", "ms_cc", "ms_edges", "ms_total")},
        "band_pairs": int(st["band_pairs"]), "pairs": int(st["pairs"]), "pairs_computed": int(st["pairs_computed"]),
        "tiles": int(st["tiles"]), "tiles_screened_out": int(st["tiles_screened_out"]),
        "nodes": g.n_nodes, "edges": g.n_edges,
        "paper_context": "about 3 minutes for 1M x 256 (202.87 s, NVIDIA Titan V; Cifar, 500 intervals)",
    }
    line.update(out)
    ctx.close()
    del ctx
    if not args.no_serve and w.name == "mix1m_d256":
        # the serving form (its own arena and stream slots): saturation
        # throughput, then p50/p99 latency from arrival at fractions of it
        from paper_2011_03209_amd import serve
        T, points = serve.run(n_requests=256, arena_gb=96.0)
        head = min(points, key=lambda q: abs(q["fraction_of_saturation"] - 0.7))
        line["serving"] = {"workload": "serving_8clouds_poisson", "requests": 256, "slots": serve.SLOTS,
                           "precision": "bf16x3", "saturation_graphs_per_s": T, "qps": head["qps"],
                           "p50_s": head["p50_s"], "p99_s": head["p99_s"],
                           "p99_submit_lag_s": head["p99_submit_lag_s"], "sweep": points}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
