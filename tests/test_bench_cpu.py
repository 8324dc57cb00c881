"""Host logic of bench.py, without a GPU: the one-GPU guard, the algorithmic
byte counts behind the roofline figures, the lookup of committed HBM
traffic records (and their invalidation when the kernel sources change),
and the shape of the CPU-oracle baseline."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_counts_visits_and_reads():
    # rows: (internal nodes visited, leaf records read) per query
    stats = np.array([[3, 0], [10, 2], [0, 0]], np.int32)
    got = bench.algorithmic_bytes(stats, node_b=32, leaf_b=32, per_query_fixed=96)
    # 3 queries x 96 + 13 visits x 32 + 2 reads x 32, counted by hand
    assert got == 288 + 416 + 64


def test_build_bytes_differences():
    fp32 = bench.build_bytes_per_prim("fp32", 21)
    q16 = bench.build_bytes_per_prim("q16", 21)
    q16_df = bench.build_bytes_per_prim("q16", 21, depth_first=True)
    # the refit writes each node once in its final format: 32 bytes, not 64
    assert fp32 - q16 == 64 - 32
    # the depth-first renumbering is charged only when it ran: the pointer
    # jumping (init 16, 6 rounds of 24, last round 24) and the refit's slot read
    assert q16_df - q16 == 16 + 6 * 24 + 24 + 4
    # 30-bit keys: half the key bytes and half the sort passes
    assert bench.build_bytes_per_prim("fp32", 10) < fp32
    # box primitives read 24 bytes where points read 12, three times (scene,
    # Morton, refit gather)
    assert bench.build_bytes_per_prim("fp32", 21, kind_width=6) - fp32 == 3 * 12


def _sources_hash(root, sources):
    import hashlib
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(root, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def test_committed_traffic_records():
    # a record is used while the kernel sources hash to its value, and
    # ignored once they have changed (the counters must then be taken again)
    for nodes in ("q16", "fp32"):
        path = os.path.join(ROOT, "profiles", f"traffic_nearest_c3_{nodes}.json")
        if not os.path.exists(path):
            pytest.skip(f"no traffic record for {nodes}")
        rec = json.load(open(path))
        traffic, raw, src = bench.measured_traffic("nearest+coop", "C3", nodes, 10)
        if _sources_hash(ROOT, rec["sources"]) != rec["sources_sha256"]:
            assert (traffic, raw, src) == (None, None, None)
            continue
        assert src == os.path.relpath(path, ROOT)
        assert traffic == rec["traffic_bytes_per_launch"]
        # the figure is the copy-calibrated counters, as recorded
        fetch = sum(rec["fetch_kib_per_launch"].values())
        write = sum(rec["write_kib_per_launch"].values())
        kib = fetch * rec["fetch_scale"] + write * rec["write_scale"]
        assert abs(traffic - 1024 * kib) <= 1
        if raw is not None:
            assert abs(raw - 1024 * (fetch + write)) <= 1
        # the record the issue figure comes from is the same one
        assert bench.measured_record("nearest+coop", "C3", nodes, 10) == rec
        if "valu_insts_per_launch" in rec:
            assert all(v > 0 for v in rec["valu_insts_per_launch"].values())
    assert bench.measured_traffic("nearest+coop", "C3", "q16", 11) == (None, None, None)


def test_traffic_record_is_dropped_when_sources_change(tmp_path, monkeypatch):
    sources = ["src/a.hip", "src/b.h"]
    for i, s in enumerate(sources):
        (tmp_path / s).parent.mkdir(parents=True, exist_ok=True)
        (tmp_path / s).write_text(f"// kernel source {i}\n")
    rec = {"kernel": "nearest+coop", "workload": "C3", "nodes": "q16", "k": 10,
           "sources": sources, "sources_sha256": _sources_hash(str(tmp_path), sources),
           "traffic_bytes_per_launch": 123456789}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_x.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("nearest+coop", "C3", "q16", 10) == \
        (123456789, None, os.path.join("profiles", "traffic_x.json"))
    assert bench.measured_traffic("nearest+coop", "C3", "fp32", 10) == (None, None, None)
    with open(tmp_path / sources[0], "a") as f:
        f.write("// edited\n")
    assert bench.measured_traffic("nearest+coop", "C3", "q16", 10) == (None, None, None)


def test_cpu_baseline_reports_the_oracle_rate():
    from paper_1908_11807_amd import datagen
    pts = datagen.uniform_cube(20000, 1)
    q = datagen.uniform_cube(4000, 2)
    out = bench.cpu_baseline(pts, q, 0.04, 10, 0.5)
    assert out["kind"] == "oracle" and out["unit"] == "queries/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert out["value_1thread"] is not None and out["value_1thread"] > 0
    import oracle
    # the thread count is restored after the one-thread sample
    assert oracle.num_threads() == out["cores"]


def test_baseline_sample_strata():
    from paper_1908_11807_amd import datagen
    q = datagen.uniform_cube(50_000, 3, -1.0, 1.0)
    rows = bench.baseline_sample(q, 1000, True)
    assert rows.shape[0] == 1000 and np.unique(rows).shape[0] == 1000
    nrm = np.linalg.norm(q.astype(np.float64), axis=1)
    # the centre stratum holds the 100 queries nearest the centre
    assert set(np.argsort(nrm)[:100]) <= set(rows.tolist())
    assert set(np.argsort(-nrm)[:100]) <= set(rows.tolist())
    assert np.sum(np.abs(nrm[rows] - 1.0) < 2e-3) >= 100
    # uniform sampling without strata: distinct rows
    r2 = bench.baseline_sample(q, 500, False)
    assert np.unique(r2).shape[0] == 500


def test_cpu_baseline_stratified_reports_cpu_and_runs():
    from paper_1908_11807_amd import datagen
    pts = datagen.shell(20000, 4)
    q = datagen.uniform_cube(5000, 5, -1.0, 1.0)
    out = bench.cpu_baseline(pts, q, 0.02, 10, 0.6, stratify=True)
    assert "median of 3 runs" in out["sample"] and "stratified" in out["sample"]
    assert out["value"] > 0 and "cpu" in out
