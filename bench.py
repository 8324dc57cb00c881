"""Benchmark of the LBVH search path on one MI355X.

One step = the whole hot path over one batch: build the LBVH of n primitives,
answer m radius queries (two-pass count-and-fill CSR) and m k-nearest
queries (k = 10), all through the C-ABI.  Inputs are resident in HBM before
the timed region; W untimed warm-up steps, then exactly K timed steps
bracketed by device synchronisation.

Prints ONE JSON line: value = queries answered per second over the timed
steps (radius + nearest); the build rate, per-phase rates, the dominant
kernel's roofline (algorithmic bytes per launch / its mean HIP-event
duration) and the CPU oracle timed on a bounded sample ride along.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C3", choices=["C1", "C2", "C3"])
    ap.add_argument("--nodes", default="q16", choices=["fp32", "q16"])
    ap.add_argument("--morton-bits", type=int, default=21)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--compare-formats", action="store_true",
                    help="also measure the other node format's query rates (untimed block)")
    return ap.parse_args()


def algorithmic_bytes(stats, node_b, leaf_b, per_query_fixed):
    """Bytes one launch must move: per query a fixed part plus node_b per
    internal node visited and leaf_b per leaf record read."""
    s = stats.astype(np.int64)
    return int(per_query_fixed * s.shape[0] + node_b * s[:, 0].sum() + leaf_b * s[:, 1].sum())


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(each GPU would hold its own share; see the sharding notes). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_11807_amd import abx, datagen

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    cfg = datagen.CONFIGS[args.workload]
    pts_np, q_np = datagen.config_inputs(args.workload)
    n, m, k, r = pts_np.shape[0], q_np.shape[0], args.k, cfg["radius"]
    pts = torch.from_numpy(pts_np).to(dev)
    qs = torch.from_numpy(q_np).to(dev)
    torch.cuda.synchronize()

    def step(rec=None):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if rec is not None else None
        if e: e[0].record()
        t = abx.bvh_build(pts, node_format=args.nodes, morton_bits=args.morton_bits)
        if e: e[1].record()
        off, idx = abx.query_spatial(t, qs, radius=r, capacity=rec.get("cap") if rec else None)
        if e: e[2].record()
        _, ki, kd = abx.query_nearest(t, qs, k)
        if e:
            e[3].record()
            rec.setdefault("ev", []).append(e)
        return t, off, idx, ki, kd

    # warm-up (also sizes the result buffer so timed steps take one pass)
    t = None
    for _ in range(max(args.warmup, 1)):
        t, off, idx, ki, kd = step()
    torch.cuda.synchronize()
    total_hits = int(idx.numel())
    rec = {"cap": total_hits}

    abx.timing_reset()
    abx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t, off, idx, ki, kd = step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    abx.timing_enable(False)

    ms_step = 1e3 * wall / args.steps
    phases = np.array([[a.elapsed_time(b) for a, b in zip(ev[:-1], ev[1:])] for ev in rec["ev"]])
    step_ms = phases.sum(axis=1)
    build_ms, rad_ms, knn_ms = np.median(phases, axis=0)

    kernels = ["morton", "sort_onesweep", "sort_hist", "karras", "refit", "quantise", "scene_partial",
               "query_codes", "spatial_count", "spatial_fill", "scan_tiles", "nearest"]
    ktimes = {}
    for name in kernels:
        ms, cnt = abx.timing_get(name)
        if cnt:
            ktimes[name] = dict(ms_per_launch=ms / cnt, launches_per_step=cnt / args.steps)

    # dominant kernel and its algorithmic bytes per launch
    node_b = 32 if args.nodes == "q16" else 64
    leaf_b = 16 if args.nodes == "q16" else 4
    st_knn = abx.query_nearest_stats(t, qs, k).cpu().numpy()
    st_sp = abx.query_spatial_stats(t, qs, radius=r).cpu().numpy()
    hits = total_hits
    alg = {
        # query point 12 B + order 4 B + k' results (index 4 B + distance 4 B)
        "nearest": algorithmic_bytes(st_knn, node_b, leaf_b, 16 + 8 * min(k, n)),
        # query 12 B + order 4 B + count write 4 B
        "spatial_count": algorithmic_bytes(st_sp, node_b, leaf_b, 20),
        # query 12 B + order 4 B + offsets 8 B, plus 4 B per written index
        "spatial_fill": algorithmic_bytes(st_sp, node_b, leaf_b, 24) + 4 * hits,
    }
    dom = max((kname for kname in ktimes), key=lambda kn: ktimes[kn]["ms_per_launch"] * ktimes[kn]["launches_per_step"])
    if dom in alg:
        per_launch = alg[dom]
        achieved = per_launch / (ktimes[dom]["ms_per_launch"] * 1e-3) / 1e9
        roof = dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    bytes_per_launch=per_launch,
                    ms_per_launch=round(ktimes[dom]["ms_per_launch"], 4))
    else:
        roof = dict(kernel=dom, bound="hbm", achieved=None, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=None, traffic=None)

    out = {
        "metric": "queries/s (kNN k=10, radius) + BVH build Mprims/s at 1e7 pts; p99 batch latency",
        "value": round(2 * m / (ms_step * 1e-3), 1),
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['desc']}", "n": n, "m": m, "k": k,
                   "radius": r, "nodes": args.nodes, "morton_bits": args.morton_bits,
                   "parallelism": "single GPU"},
        "build_mprims_s": round(n / (build_ms * 1e-3) / 1e6, 1),
        "radius_qps": round(m / (rad_ms * 1e-3), 1),
        "knn_qps": round(m / (knn_ms * 1e-3), 1),
        "phase_ms_median": {"build": round(build_ms, 3), "radius": round(rad_ms, 3),
                            "nearest": round(knn_ms, 3)},
        "step_latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                            "p99": round(float(np.percentile(step_ms, 99)), 3)},
        "radius_results": hits,
        "tree_height": t.height,
        "kernels": {kn: {kk: round(v, 4) for kk, v in d.items()} for kn, d in ktimes.items()},
        "roofline": roof,
    }

    if args.compare_formats:
        other = "fp32" if args.nodes == "q16" else "q16"
        t2 = abx.bvh_build(pts, node_format=other, morton_bits=args.morton_bits)
        res = {}
        for name, fn in (("radius", lambda: abx.query_spatial(t2, qs, radius=r, capacity=hits)),
                         ("nearest", lambda: abx.query_nearest(t2, qs, k))):
            fn()
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            res[name + "_qps"] = round(3 * m / (time.perf_counter() - a), 1)
        out["other_format"] = {"nodes": other, **res}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pts_np, q_np, r, k, args.cpu_seconds)

    print(json.dumps(out), flush=True)


def cpu_baseline(pts, q, r, k, budget_s):
    """The oracle (brute force, double precision, all host threads) on a
    seeded sample of the same queries: radius + nearest, rate in queries/s."""
    import oracle
    oracle.build_library()
    rng = np.random.default_rng(7)
    sel = rng.permutation(q.shape[0])
    done, t_used, chunk = 0, 0.0, 16
    while t_used < budget_s and done + chunk <= sel.shape[0]:
        qq = q[sel[done:done + chunk]]
        a = time.perf_counter()
        oracle.spatial(pts, oracle.POINTS, qq, oracle.WITHIN, radius=r)
        oracle.nearest(pts, oracle.POINTS, qq, k)
        t_used += time.perf_counter() - a
        done += chunk
        chunk = min(chunk * 2, 256)
    return {"value": round(2 * done / t_used, 2), "unit": "queries/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{done} seeded queries of the same workload, each answered by brute-force "
                      f"radius and k={k} nearest over all {pts.shape[0]} points ({t_used:.1f} s)"}


if __name__ == "__main__":
    main()
