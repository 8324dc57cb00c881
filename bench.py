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
    ap.add_argument("--workload", default="C3",
                    choices=["C1", "C2", "C3", "C4", "C5", "COPY", "GATHER", "PAPER"])
    ap.add_argument("--nodes", default="q16", choices=["fp32", "q16", "q16w"])
    ap.add_argument("--morton-bits", type=int, default=21)
    ap.add_argument("--hierarchy", default="karras", choices=["karras", "agglomerative"])
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--compare-formats", action="store_true",
                    help="also measure the other node format's query rates (untimed block)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per load level of the serving block (0: skip it)")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95")
    ap.add_argument("--serve-rates", default="700,1400",
                    help="fixed offered request rates (requests/s), comparable across server versions")
    ap.add_argument("--serve-slots", type=int, default=4, help="server streams (C5)")
    ap.add_argument("--serve-merge", type=int, default=0,
                    help="queries per merged launch (0: the library default, <0: no merging)")
    ap.add_argument("--serve-small", type=int, default=0,
                    help="largest small request (0: the library default)")
    ap.add_argument("--serve-merge-large", type=int, default=0,
                    help="queries per merged launch of large requests (0: the library default, <0: none)")
    ap.add_argument("--trees", type=int, default=256, help="forest size (C4)")
    ap.add_argument("--paper-sizes", default="1e4,1e5,1e6,1e7",
                    help="m = n sweep of the paper's filled and hollow cases (PAPER)")
    return ap.parse_args()


def measured_record(kernel, workload, nodes, k):
    """The committed rocprofv3 counter record of this launch (None when there
    is none or the kernel sources changed since it was taken)."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as f:
            rec = json.load(f)
        if (rec.get("kernel"), rec.get("workload"), rec.get("nodes"), rec.get("k")) != \
                (kernel, workload, nodes, k):
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        return rec if h.hexdigest() == rec["sources_sha256"] else None
    return None


# VALU issue of the chip: a wave64 instruction holds a 16-lane SIMD for four
# cycles; 256 CUs x 4 SIMDs at 2.4 GHz
VALU_PEAK_GINST_S = 256 * 4 * 2.4 / 4


def measured_traffic(kernel, workload, nodes, k):
    """HBM bytes per launch from the committed rocprofv3 counter summary:
    (copy-calibrated FETCH_SIZE x 2.0 + WRITE_SIZE, raw FETCH_SIZE + WRITE_SIZE,
    source file), or Nones when no summary covers this launch or the kernel
    sources changed since."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))):
        with open(path) as f:
            rec = json.load(f)
        if (rec.get("kernel"), rec.get("workload"), rec.get("nodes"), rec.get("k")) != \
                (kernel, workload, nodes, k):
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None, None, None
        raw = rec.get("traffic_bytes_per_launch_raw")
        return (int(rec["traffic_bytes_per_launch"]), None if raw is None else int(raw),
                os.path.relpath(path, ROOT))
    return None, None, None


def algorithmic_bytes(stats, node_b, leaf_b, per_query_fixed):
    """Bytes one launch must move: per query a fixed part plus node_b per
    internal node visited and leaf_b per leaf record read."""
    s = stats.astype(np.int64)
    return int(per_query_fixed * s.shape[0] + node_b * s[:, 0].sum() + leaf_b * s[:, 1].sum())


def build_bytes_per_prim(node_format, morton_bits, kind_width=3, depth_first=False, wide_per_prim=0.0):
    """Algorithmic bytes of one Karras build, per point primitive (8-bit radix
    digits; `depth_first`: the tree's nodes were renumbered in depth-first
    order, which Q16 Karras trees of 2^22 primitives and more get by default;
    `wide_per_prim`: 4-wide nodes written per primitive).  The refit writes
    each node once, in its final format; its chunk-crossing staging (a few
    per cent of the nodes) is not counted."""
    keyb = 8 if morton_bits > 10 else 4          # 63- or 30-bit Morton keys
    passes = 8 if morton_bits > 10 else 4        # 8-bit digits
    w = 4 * kind_width                           # 12 B point (24 B box)
    b = w                                        # scene box: read the primitives
    b += w + keyb + 4                            # Morton: read, write key and index
    b += keyb                                    # digit histograms: read the keys once
    b += passes * 2 * (keyb + 4)                 # onesweep passes: read and write (key, index)
    b += keyb + 8 + 8 + 4 + 4                    # hierarchy: keys; parent words of the leaf
    #                                              and the node, range end, arrival counter
    ordered = node_format == "q16w" or (node_format == "q16" and depth_first)
    if ordered:
        b += 8 + 8                               # depth-first order: parent word, first word
        b += 6 * (8 + 8 + 8)                     # 6 pointer-jumping rounds: own, ancestor's, out
        b += 8 + 8 + 4 + 4                       # last round: words, range end, the index
        if node_format == "q16w":
            b += 4                               # and the depth
    b += 4 + 8 + w                               # refit, leaf: permutation, parent word, primitive
    b += 8                                       # refit, node: parent word
    if node_format == "q16":
        b += (4 if depth_first else 0) + 32      # its depth-first slot, the Q16 node
    else:
        b += 64                                  # the FP32 node (staged, for 4-wide trees)
    if node_format == "q16w":
        b += 4 + 4 + 4                           # flags: index, depth, flag
        b += 4 + 4                               # scan of the flags
        b += 64 + 4 + 4 + 4 + 4                  # collapse: every binary node read once, its depth,
        #                                          index, rank, and its rank read by its parent
        b += 64 * wide_per_prim                  # the 4-wide nodes written
    return b


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each GPU would "
              "hold its own share of the queries). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_11807_amd import abx, datagen

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.workload == "C4":
        print(json.dumps(bench_forest(args)), flush=True)
        return
    if args.workload == "C5":
        print(json.dumps(bench_serving(args, standalone=True)), flush=True)
        return
    if args.workload == "PAPER":
        print(json.dumps(bench_paper(args)), flush=True)
        return
    if args.workload == "COPY":
        # plain 1 GiB device copy: the reference for scaling HBM counters
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(max(args.steps, 1)):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"metric": "device copy", "bytes_read_per_copy": x.numel() * 4,
                          "bytes_written_per_copy": x.numel() * 4, "copies": max(args.steps, 1)}))
        return
    if args.workload == "GATHER":
        # random 32-B row gather from a 1 GiB table: the access pattern of a
        # node fetch, for scaling HBM counters of random reads
        rows = 1 << 25
        table = torch.ones((rows, 8), dtype=torch.int32, device="cuda")
        idx = torch.randint(0, rows, (1 << 24,), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
        out = torch.empty((1 << 24, 8), dtype=torch.int32, device="cuda")
        for _ in range(max(args.steps, 1)):
            torch.index_select(table, 0, idx, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"metric": "random 32-B row gather", "rows_gathered": idx.numel(),
                          "bytes_read_per_gather": idx.numel() * (32 + 8),
                          "bytes_written_per_gather": idx.numel() * 32, "gathers": max(args.steps, 1)}))
        return
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
        t = abx.bvh_build(pts, node_format=args.nodes, morton_bits=args.morton_bits,
                          hierarchy=args.hierarchy)
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

    # the timed steps: the library's per-kernel events are off, so nothing
    # but the path itself runs between the synchronisations
    abx.timing_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t, off, idx, ki, kd = step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    ms_step = 1e3 * wall / args.steps
    phases = np.array([[a.elapsed_time(b) for a, b in zip(ev[:-1], ev[1:])] for ev in rec["ev"]])
    step_ms = phases.sum(axis=1)
    build_ms, rad_ms, knn_ms = np.median(phases, axis=0)

    # the same steps again with HIP events around every kernel launch (on the
    # launch stream): per-kernel durations for the roofline
    abx.timing_reset()
    abx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t, off, idx, ki, kd = step()
    torch.cuda.synchronize()
    ms_step_instrumented = 1e3 * (time.perf_counter() - t0) / args.steps
    abx.timing_enable(False)

    kernels = ["morton", "sort_onesweep", "sort_hist", "karras", "refit", "refit_mid", "refit_top", "agglo", "agglo_mid",
               "agglo_top", "quantise", "preorder", "wide_flags", "wide_emit",
               "scene_partial", "query_codes", "spatial_count", "spatial_fill", "scan_tiles", "nearest",
               "nearest_coop"]
    ktimes = {}
    for name in kernels:
        ms, cnt = abx.timing_get(name)
        if cnt:
            ktimes[name] = dict(ms_per_launch=ms / cnt, launches_per_step=cnt / args.steps)
    # the nearest traversal is two launches (one lane per query, then one
    # workgroup per heavy query); the roofline takes them together
    if "nearest" in ktimes and "nearest_coop" in ktimes:
        ktimes["nearest+coop"] = dict(
            ms_per_launch=ktimes["nearest"]["ms_per_launch"] + ktimes["nearest_coop"]["ms_per_launch"],
            launches_per_step=1.0)

    # dominant kernel and its algorithmic bytes per launch
    node_b = int(t.layout.node_bytes)
    leaf_b = int(t.layout.leaf_bytes)
    st_knn = abx.query_nearest_stats(t, qs, k).cpu().numpy()
    st_sp = abx.query_spatial_stats(t, qs, radius=r).cpu().numpy()
    hits = total_hits
    alg = {
        # query point 12 B + order 4 B + k' results (index 4 B + distance 4 B)
        "nearest+coop": algorithmic_bytes(st_knn, node_b, leaf_b, 16 + 8 * min(k, n)),
        # query 12 B + order 4 B + count write 4 B
        "spatial_count": algorithmic_bytes(st_sp, node_b, leaf_b, 20),
        # query 12 B + order 4 B + offsets 8 B, plus 4 B per written index
        "spatial_fill": algorithmic_bytes(st_sp, node_b, leaf_b, 24) + 4 * hits,
    }
    dom = max((kn for kn in ktimes if kn not in ("nearest", "nearest_coop")),
              key=lambda kn: ktimes[kn]["ms_per_launch"] * ktimes[kn]["launches_per_step"])
    if dom in alg:
        per_launch = alg[dom]
        achieved = per_launch / (ktimes[dom]["ms_per_launch"] * 1e-3) / 1e9
        traffic, traffic_raw, tsrc = measured_traffic(dom, args.workload, args.nodes, k)
        roof = dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    traffic_raw=traffic_raw, traffic_source=tsrc,
                    # the measured DRAM bytes over the same launch time: the HBM
                    # fraction the counters support (copy-calibrated and raw)
                    traffic_frac=None if traffic is None else round(
                        traffic / (ktimes[dom]["ms_per_launch"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    traffic_raw_frac=None if traffic_raw is None else round(
                        traffic_raw / (ktimes[dom]["ms_per_launch"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    bytes_per_launch=per_launch,
                    ms_per_launch=round(ktimes[dom]["ms_per_launch"], 4))
        rec = measured_record(dom, args.workload, args.nodes, k)
        if rec and "valu_insts_per_launch" in rec:
            # the same launch against the chip's VALU issue rate: the walk is
            # bound by instruction issue as much as by memory
            insts = sum(rec["valu_insts_per_launch"].values())
            gi = insts / (ktimes[dom]["ms_per_launch"] * 1e-3) / 1e9
            roof["issue"] = dict(valu_insts_per_launch=insts, achieved=round(gi, 1),
                                 peak=VALU_PEAK_GINST_S, unit="G wave64 VALU instructions/s",
                                 frac=round(gi / VALU_PEAK_GINST_S, 4))
    else:
        roof = dict(kernel=dom, bound="hbm", achieved=None, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=None, traffic=None)

    # one-pass radius search (the paper's buffer_size scheme): buffer = the
    # largest row, so one traversal answers the batch
    row_max = int(torch.diff(off).max().item()) if m > 0 else 0
    bsz = max(row_max, 1)
    t1p = []
    for i in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        _, _, trav = abx.query_spatial_1p(t, qs, bsz, radius=r)
        b.record()
        b.synchronize()
        if i:
            t1p.append(a.elapsed_time(b))
    radius_1p = dict(ms=round(float(np.median(t1p)), 3), buffer_size=bsz, traversals=trav,
                     speedup_vs_2p=round(rad_ms / float(np.median(t1p)), 3))

    # the other two phases against the same HBM peak (algorithmic bytes)
    bpp = build_bytes_per_prim(args.nodes, args.morton_bits,
                               depth_first=int(t.layout.node_order) == abx.ORDER_DEPTH_FIRST,
                               wide_per_prim=int(t.layout.node_count) / n if args.nodes == "q16w" else 0.0)
    rad_bytes = alg["spatial_count"] + alg["spatial_fill"]
    phase_rooflines = {
        "build": dict(bytes_per_prim=bpp, achieved=round(bpp * n / (build_ms * 1e-3) / 1e9, 1),
                      peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(bpp * n / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
        "radius_2p": dict(bytes=rad_bytes, achieved=round(rad_bytes / (rad_ms * 1e-3) / 1e9, 1),
                          peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=round(rad_bytes / (rad_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
    }

    # achievable HBM bandwidth: a plain 1 GiB device copy (reads and writes 1 GiB)
    cx = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    cy = torch.empty_like(cx)
    cms = []
    for i in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        cy.copy_(cx)
        b.record()
        b.synchronize()
        if i:
            cms.append(a.elapsed_time(b))
    copy_gbs = 2 * cx.numel() * 4 / (float(np.median(cms)) * 1e-3) / 1e9
    del cx, cy
    roof["copy_gbs"] = round(copy_gbs, 1)
    if roof.get("achieved") is not None:
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)

    out = {
        "metric": "queries/s (kNN k=10, radius) + BVH build Mprims/s at 1e7 pts; p99 batch latency",
        "value": round(2 * m / (ms_step * 1e-3), 1),
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "ms_per_step_instrumented": round(ms_step_instrumented, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['desc']}", "n": n, "m": m, "k": k,
                   "radius": r, "nodes": args.nodes, "morton_bits": args.morton_bits,
                   "hierarchy": args.hierarchy,
                   "parallelism": "single GPU"},
        "build_mprims_s": round(n / (build_ms * 1e-3) / 1e6, 1),
        "radius_qps": round(m / (rad_ms * 1e-3), 1),
        "knn_qps": round(m / (knn_ms * 1e-3), 1),
        "phase_ms_median": {"build": round(build_ms, 3), "radius": round(rad_ms, 3),
                            "nearest": round(knn_ms, 3)},
        "step_latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                            "p99": round(float(np.percentile(step_ms, 99)), 3)},
        "radius_results": hits,
        "phase_rooflines": phase_rooflines,
        "radius_1p": radius_1p,
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
        out["cpu_baseline"] = cpu_baseline(pts_np, q_np, r, k, args.cpu_seconds,
                                           stratify=args.workload == "C3")

    if args.serve_requests > 0 and args.workload == "C3":
        del t, off, idx, ki, kd
        torch.cuda.empty_cache()
        out["serving"] = bench_serving(args, standalone=False)
        out["p99_batch_latency_ms"] = out["serving"]["loads"][-1]["p99_ms"]

    print(json.dumps(out), flush=True)


def bench_paper(args):
    """The paper's two experimental cases (section 3, data sets) over m = n:
    filled (filled-sphere queries in a filled-cube cloud) and hollow
    (hollow-sphere queries in a hollow-cube cloud), kNN k = 10 and radius
    search with r set for 10 neighbours on average in the filled cube, with
    the query ordering on and off.  Reports medians of per-phase HIP-event
    times and the radius neighbour-count statistics the paper quotes."""
    import torch
    from paper_1908_11807_amd import abx, datagen

    dev = torch.device("cuda:0")
    sizes = [int(float(x)) for x in args.paper_sizes.split(",") if x]
    reps = max(args.steps, 1)
    rows = []

    def timed(fn):
        fn()                                   # warm-up
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            out = fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), out

    for case in ("filled", "hollow"):
        for p in sizes:
            if case == "filled":
                prims = datagen.paper_filled_cube(p, 601)
                queries = datagen.paper_filled_sphere(p, 602)
            else:
                prims = datagen.paper_hollow_cube(p, 603)
                queries = datagen.paper_hollow_sphere(p, 604)
            # 10 neighbours on average in the filled cube [-a, a]^3 (volume 8p)
            r = datagen.radius_for_density(p, 10, volume=8.0 * p)
            pts = torch.from_numpy(prims).to(dev)
            qs = torch.from_numpy(queries).to(dev)
            build_ms, t = timed(lambda: abx.bvh_build(pts, node_format=args.nodes))
            row = dict(case=case, n=p, m=p, radius=r, build_ms=round(build_ms, 4),
                       build_mprims_s=round(p / build_ms / 1e3, 1))
            for srt in (True, False):
                tag = "sorted" if srt else "unsorted"
                knn_ms, _ = timed(lambda: abx.query_nearest(t, qs, 10, sort_queries=srt))
                rad_ms, (off, _) = timed(lambda: abx.query_spatial(t, qs, radius=r, sort_queries=srt))
                row[f"knn_ms_{tag}"] = round(knn_ms, 4)
                row[f"knn_qps_{tag}"] = round(p / knn_ms * 1e3, 1)
                row[f"radius_ms_{tag}"] = round(rad_ms, 4)
                row[f"radius_qps_{tag}"] = round(p / rad_ms * 1e3, 1)
            cnt = torch.diff(off).cpu().numpy()
            row["neighbours"] = dict(mean=round(float(cnt.mean()), 3), min=int(cnt.min()),
                                     max=int(cnt.max()))
            # one pass (Morton-ordered queries): buffer = the largest row (one
            # traversal), and a fixed buffer of 16 (overflow: second traversal)
            for tag, bsz in (("1p_max", max(int(cnt.max()), 1)), ("1p_16", 16)):
                ms1, (_, _, trav) = timed(lambda: abx.query_spatial_1p(t, qs, bsz, radius=r))
                row[f"radius_ms_{tag}"] = round(ms1, 4)
                row[f"radius_qps_{tag}"] = round(p / ms1 * 1e3, 1)
                row[f"traversals_{tag}"] = trav
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
            del t, pts, qs
    return {"metric": "paper cases: build Mprims/s, kNN and radius queries/s over m = n",
            "workload": "PAPER", "nodes": args.nodes, "k": 10, "reps": reps,
            "data": "synthetic (the paper's four generators)", "rows": rows}


def bench_forest(args):
    import torch
    from paper_1908_11807_amd import abx, datagen
    k = 16
    pts_np, off, q_np, qoff = datagen.forest_inputs(args.trees)
    N, M = int(off[-1]), int(qoff[-1])
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        pts = torch.from_numpy(pts_np).cuda()
        qs = torch.from_numpy(q_np).cuda()
        plan = abx.ForestPlan(pts, off, qs, qoff, k, node_format=args.nodes)
        plan.check()
        tuned = plan.autotune()
        plan.capture(build=True)
        for _ in range(max(args.warmup, 1)):
            plan.replay()
        torch.cuda.synchronize()
        abx.timing_reset()
        # per-kernel times of three eager steps with events on the launch
        # stream (graph replays carry none), per step
        abx.timing_enable(True)
        for _ in range(3):
            plan.build()
            plan.query()
        torch.cuda.synchronize()
        abx.timing_enable(False)
        ktimes = {}
        for name in ("forest_nearest", "forest_nearest_coop", "refit", "sort_onesweep", "karras",
                     "forest_keys", "forest_qkeys", "quantise", "forest_boxes"):
            ms, cnt = abx.timing_get(name)
            if cnt:
                ktimes[name] = round(ms / 3, 4)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.replay()
        ev[1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev[0].elapsed_time(ev[1]) / args.steps
        # algorithmic bytes of the query launch pair: per query the point
        # (12 B), its order entry (4 B) and its row (8 B per entry), plus
        # node_b per node visited and 32 B per leaf record read (counting walk)
        st = plan.stats().cpu().numpy()
        node_b = 32 if args.nodes == "q16" else 64
        kk = np.repeat(np.minimum(k, np.diff(off)), np.diff(qoff))
        alg = int(16 * M + 8 * int(kk.sum()) + node_b * int(st[:, 0].astype(np.int64).sum())
                  + 32 * int(st[:, 1].astype(np.int64).sum()))
    pair_ms = ktimes.get("forest_nearest", 0.0) + ktimes.get("forest_nearest_coop", 0.0)
    achieved = alg / (pair_ms * 1e-3) / 1e9 if pair_ms > 0 else None
    rec = measured_record("forest_nearest+coop", "C4", args.nodes, k)
    traffic = int(rec["traffic_bytes_per_launch"]) if rec else None
    traffic_raw = int(rec["traffic_bytes_per_launch_raw"]) if rec else None
    roof = {"kernel": "forest_nearest+coop", "bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None, "traffic": traffic,
            "traffic_raw": traffic_raw,
            "traffic_frac": round(traffic / (pair_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            if traffic and pair_ms > 0 else None,
            "traffic_source": "profiles/traffic_forest_c4_q16.json" if rec else None,
            "bytes_per_launch": alg, "ms_per_launch": round(pair_ms, 4),
            "visits_per_query": round(float(st[:, 0].mean()), 1)}
    cpu = None if args.no_cpu_baseline else forest_cpu_baseline(pts_np, off, q_np, qoff, k, args.cpu_seconds)
    return {
        "metric": "forest kNN queries/s (k=16, build + query per step, one HIP graph)",
        "value": round(M / (ms * 1e-3), 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "wall_ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"C4: forest of {args.trees} trees, sizes log-uniform [1e3,1e6], "
                               "uniform cube / Gaussian clusters, equal-count queries",
                   "trees": args.trees, "points": N, "queries": M, "k": k, "nodes": args.nodes,
                   "tuned": tuned},
        "eager_kernel_ms": ktimes,
        "results": plan.total,
        "roofline": roof,
        **({"cpu_baseline": cpu} if cpu else {}),
    }


def forest_cpu_baseline(pts, off, q, qoff, k, budget_s):
    """The oracle on a seeded sample of the forest's queries: rows drawn
    evenly from every tree (each answered by brute force over its own tree's
    points), median of three runs; queries/s."""
    import oracle
    oracle.build_library()
    T = len(off) - 1
    rng = np.random.default_rng(9)

    def sample(per_tree):
        return [(t, rng.choice(int(qoff[t + 1] - qoff[t]), min(per_tree, int(qoff[t + 1] - qoff[t])),
                               replace=False)) for t in range(T)]

    def rate(picks):
        a = time.perf_counter()
        cnt = 0
        for t, rows in picks:
            if rows.size:
                oracle.nearest(pts[off[t]:off[t + 1]], oracle.POINTS, q[qoff[t] + rows], k)
                cnt += rows.size
        return cnt / (time.perf_counter() - a)

    est = rate(sample(1))
    per_tree = int(max(1, min(64, est * budget_s / 3 / T)))
    picks = sample(per_tree)
    runs = [rate(picks) for _ in range(3)]
    n_rows = sum(int(r.size) for _, r in picks)
    return {"value": round(float(np.median(runs)), 2), "unit": "queries/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{n_rows} seeded queries, {per_tree} from each of the {T} trees, each answered by "
                      f"brute-force k={k} nearest over its own tree; median of 3 runs "
                      f"({', '.join(f'{x:.1f}' for x in runs)} queries/s)"}


def bench_serving(args, standalone):
    """4 device-resident trees of 1e7 points (two uniform cubes, two thin
    shells); Poisson stream of requests (m = floor(10^U(0,5)), kind radius /
    k=1 / k=8 / k=32, tree uniform); saturated throughput, then p50/p99
    latency at fractions of it."""
    import torch
    from paper_1908_11807_amd import abx, datagen
    n = 10_000_000
    dev = torch.device("cuda:0")
    trees, radii, pools = [], [], []
    for t in range(4):
        if t < 2:
            p = datagen.uniform_cube(n, 501 + t)
            radii.append(float(np.float32(datagen.radius_for_density(n))))
            pools.append(torch.from_numpy(datagen.uniform_cube(1_000_000, 601 + t)).pin_memory())
        else:
            p = datagen.shell(n, 501 + t)
            radii.append(float(np.float32(datagen.radius_for_shell(n, 1e-3))))
            pools.append(torch.from_numpy(datagen.uniform_cube(1_000_000, 601 + t, -1.0, 1.0)).pin_memory())
        trees.append(abx.bvh_build(torch.from_numpy(p).to(dev), node_format=args.nodes))
        del p
    torch.cuda.synchronize()
    budget = 2 << 30
    srv = abx.Server(slots=args.serve_slots, budget_bytes=budget, host_bytes=2 << 30,
                     merge_queries=args.serve_merge, small_queries=args.serve_small,
                     merge_large=args.serve_merge_large)
    tids = [srv.add_tree(t) for t in trees]
    kinds = ("radius", 1, 8, 32)

    def make(nreq, seed, rate):
        reqs = datagen.request_stream(nreq, seed, rate, 4, kinds=kinds)
        rng = np.random.default_rng(seed + 1)
        for r in reqs:
            o = int(rng.integers(0, 1_000_000 - r["m"] + 1))
            r["q"] = pools[r["tree"]][o:o + r["m"]]
        return reqs

    def run(reqs, t0, paced):
        lat, gpu_t, done, live = [], [], 0, {}
        qsum = 0
        last = t0
        for r in reqs:
            ta = t0 + r["t_arrival"] if paced else t0
            if paced:
                while abx.server_now() < ta:
                    for tk in list(live):
                        res = srv.poll(tk, copy=False)
                        if res is not None:
                            lat.append(res["t_done"] - res["t_arrival"])
                            gpu_t.append(res["t_device"])
                            last = max(last, res["t_done"])
                            srv.release(tk)
                            del live[tk]
            kind = r["kind"]
            if kind == "radius":
                tk = srv.submit(tids[r["tree"]], abx.REQ_RADIUS, r["q"], radius=radii[r["tree"]], t_arrival=ta)
            else:
                tk = srv.submit(tids[r["tree"]], abx.REQ_NEAREST, r["q"], k=kind, t_arrival=ta)
            live[tk] = r
            qsum += r["m"]
        for tk in list(live):
            res = srv.wait(tk, copy=False)
            lat.append(res["t_done"] - res["t_arrival"])
            gpu_t.append(res["t_device"])
            last = max(last, res["t_done"])
            srv.release(tk)
        return np.array(lat), np.array(gpu_t), qsum, last - t0

    nreq = max(args.serve_requests, 20)
    nwarm = min(nreq, 1000)
    run(make(nwarm, 700, 1.0), abx.server_now(), paced=False)   # warm-up
    lat, gpu_t, qsum, span = run(make(nreq, 701, 1.0), abx.server_now(), paced=False)
    sat_rps = nreq / span
    out = {"saturated_requests_per_s": round(sat_rps, 1), "saturated_queries_per_s": round(qsum / span, 1),
           "loads": []}
    def level(seed, rate):
        lat, gpu_t, qsum, span = run(make(nreq, seed, rate), abx.server_now() + 0.01, paced=True)
        return {"requests_per_s": round(nreq / span, 1), "queries_per_s": round(qsum / span, 1),
                "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
                "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
                # the requests' own GPU time (copies + kernels, stream events)
                "device_p50_ms": round(1e3 * float(np.percentile(gpu_t, 50)), 3),
                "device_p99_ms": round(1e3 * float(np.percentile(gpu_t, 99)), 3)}

    # loads relative to this server's saturated rate, then fixed request rates
    # (the same traffic whatever the server's capacity)
    for i, f in enumerate(float(x) for x in args.serve_loads.split(",")):
        out["loads"].append({"offered": f, **level(710 + i, f * sat_rps)})
    out["fixed_rates"] = []
    for i, r in enumerate(float(x) for x in args.serve_rates.split(",") if x):
        if r < sat_rps:
            out["fixed_rates"].append({"offered_requests_per_s": r, **level(730 + i, r)})
    st = srv.stats()
    out["server"] = {"slots": args.serve_slots, "merge_queries": args.serve_merge,
                     "small_queries": args.serve_small, "merge_large": args.serve_merge_large,
                     "budget_bytes": budget,
                     "max_in_flight": st["max_in_flight"], "batches": st["batches"],
                     "requests": st["completed"], "device_high_water": st["device_high_water"],
                     "failed": st["failed"]}
    out["requests_per_level"] = nreq
    srv.close()
    if standalone:
        top = out["loads"][-1]
        return {"metric": "serving p99 batch latency at 95% load (4 x 1e7-point trees)",
                "value": top["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": nreq, "warmup": nwarm,
                "ms_per_step": top["p50_ms"], "higher_is_better": False, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": "C5: 4 device-resident trees of 1e7 points (2 cube, 2 shell), "
                                       "Poisson requests m=floor(10^U(0,5)), radius/k=1/8/32, "
                                       "HBM budget 2 GiB", "nodes": args.nodes},
                "serving": out}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def baseline_sample(q, size, stratify, seed=7):
    """Seeded query rows: uniform, or (C3) stratified like the workload's
    extremes -- 70 % uniform, 10 % nearest the centre (the longest nearest
    walks), 10 % nearest the corners, 10 % within 2e-3 of the shell."""
    rng = np.random.default_rng(seed)
    if not stratify:
        return rng.choice(q.shape[0], size, replace=False)
    nrm = np.linalg.norm(q.astype(np.float64), axis=1)
    tenth = max(size // 10, 1)
    shell = np.nonzero(np.abs(nrm - 1.0) < 2e-3)[0]
    parts = [np.argpartition(nrm, tenth)[:tenth], np.argpartition(-nrm, tenth)[:tenth],
             rng.choice(shell, min(tenth, shell.shape[0]), replace=False)]
    taken = np.concatenate(parts)
    rest = np.setdiff1d(rng.choice(q.shape[0], size, replace=False), taken)[:size - taken.shape[0]]
    return np.concatenate([taken, rest])


def cpu_baseline(pts, q, r, k, budget_s, stratify=False):
    """The oracle (brute force, double precision, all host threads) on a
    seeded sample of the same queries: radius + nearest, rate in queries/s,
    the median of three runs over the same sample (sized so that one run
    takes about a third of the budget); then the same on one thread."""
    import oracle
    oracle.build_library()

    def rate(rows):
        qq = q[rows]
        a = time.perf_counter()
        oracle.spatial(pts, oracle.POINTS, qq, oracle.WITHIN, radius=r)
        oracle.nearest(pts, oracle.POINTS, qq, k)
        return 2 * rows.shape[0] / (time.perf_counter() - a)

    # size the sample from a short probe of random rows
    probe = np.random.default_rng(5).choice(q.shape[0], 32, replace=False)
    est = rate(probe) / 2
    size = int(min(max(est * budget_s / 3, 64), q.shape[0]))
    rows = baseline_sample(q, size, stratify)
    runs = [rate(rows) for _ in range(3)]
    cores = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        rows1 = rows[np.random.default_rng(8).choice(rows.shape[0], max(8, min(rows.shape[0], size // cores)),
                                                     replace=False)]
        runs1 = [rate(rows1) for _ in range(3)]
    finally:
        oracle.set_num_threads(cores)
    kind = "stratified (70 % uniform, 10 % centre, 10 % corners, 10 % shell)" if stratify else "uniform"
    return {"value": round(float(np.median(runs)), 2), "unit": "queries/s", "cores": cores,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{rows.shape[0]} seeded queries of the same workload, {kind}, each answered by "
                      f"brute-force radius and k={k} nearest over all {pts.shape[0]} points; median of "
                      f"3 runs ({', '.join(f'{x:.1f}' for x in runs)} queries/s)",
            "value_1thread": round(float(np.median(runs1)), 2),
            "sample_1thread": f"{rows1.shape[0]} queries of the sample on one thread, median of 3 runs"}


if __name__ == "__main__":
    main()
