"""Host-side logic of the benchmark and the profile summaries (no GPU): the
multi-GPU refusal, the choice of the binding roofline, the source-hash guard
on stored traffic, and the counter arithmetic of the traffic summary on a
synthetic rocprofv3 counter file."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1802_07210_amd import profiling  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_roofline_is_the_larger_floor():
    st = {"support_evals": 2_240_000, "dense_evals": 3_200_000, "n_support_left": 750,
          "n_support_right": 750, "n_tri_left": 1502, "n_tri_right": 1502,
          "lattice": 12065, "lattice_rows": 95}
    dense = bench.roofline_of("dense", 640, 480, st, 0.0125, "k_dense2")
    # 12.3 MB / 8 TB/s = 1.5 us > 51 M / 157.3 T = 0.33 us: HBM binds
    assert dense["bound"] == "hbm" and dense["work_per_launch"] == 2 * 640 * 480 * 20
    assert abs(dense["achieved"] - 12_288_000 / 12.5e-6 / 1e9) < 1e-3
    assert "alu_view" in dense
    support = bench.roofline_of("support", 640, 480, st, 0.0110, "k_support")
    assert support["bound"] == "alu" and support["work_per_launch"] == 64 * 2_240_000


def test_batched_launch_work_scales_with_the_pairs():
    # statistics summed over 8 pairs, lattice sizes per pair
    st = {"support_evals": 8 * 2_240_000, "dense_evals": 8 * 3_200_000, "n_support_left": 8 * 750,
          "n_support_right": 8 * 750, "n_tri_left": 8 * 1502, "n_tri_right": 8 * 1502,
          "lattice": 12065, "lattice_rows": 95}
    dense = bench.roofline_of("dense", 640, 480, st, 0.09, "k_dense2_batch", pairs=8)
    assert dense["work_per_launch"] == 8 * 2 * 640 * 480 * 20
    assert dense["alu_view"]["work_per_launch"] == 16 * 8 * 3_200_000
    sup_bytes, sup_ops = bench.algorithmic_work("support", 640, 480, st, pairs=8)
    assert sup_bytes == 8 * 2 * 2 * 16 * 640 * 95 and sup_ops == 64 * 8 * 2_240_000
    mesh_bytes, _ = bench.algorithmic_work("mesh", 640, 480, st, pairs=8)
    assert mesh_bytes == 8 * (12 * 1500 + 24 * 3004)


def test_workgroup_counts_of_the_bench_shape():
    wg = bench.workgroups(640, 480, 128)
    assert wg["mesh"] == 2 and wg["filter"] == 16 * 12 and wg["rows"] == 95
    assert wg["dense"] == 2 * 240 * 3 and wg["raster"] == 2 * 120


def test_stored_traffic_requires_the_same_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    f = tmp_path / "traffic_k_dense2_batch_640x480_D128_x8.json"
    f.write_text(json.dumps({"kernel": "k_dense2_batch", "bytes_per_launch": 123,
                             "source_sha256_16": bench.source_hash()}))
    assert bench.stored_traffic("k_dense2_batch", "640x480_D128_x8") == 123
    assert bench.stored_traffic("k_dense2_batch", "640x480_D128") is None  # other workload
    assert bench.stored_traffic("k_raster", "640x480_D128_x8") is None
    f.write_text(json.dumps({"kernel": "k_dense2_batch", "bytes_per_launch": 123,
                             "source_sha256_16": "0" * 16}))
    assert bench.stored_traffic("k_dense2_batch", "640x480_D128_x8") is None


def test_stored_valu_issue_requires_the_same_kernel_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    f = tmp_path / "valu_640x480_D128_x8.json"
    rec = {"kernels": {"k_support_batch": {"sq_insts_valu": 24_000_000.0}},
           "source_sha256_16": bench.source_hash()}
    f.write_text(json.dumps(rec))
    assert bench.stored_valu("k_support_batch", "640x480_D128_x8") == 24_000_000.0
    assert bench.stored_valu("k_dense1_batch", "640x480_D128_x8") is None
    st = {"support_evals": 2_240_000, "dense_evals": 3_200_000, "n_support_left": 750,
          "n_support_right": 750, "n_tri_left": 1502, "n_tri_right": 1502,
          "lattice": 12065, "lattice_rows": 95}
    roof = bench.roofline_of("support", 640, 480, st, 0.05, "k_support_batch", pairs=8,
                             workload="640x480_D128_x8")
    # 24 M wavefront instructions in 50 us against 614.4 G per second
    assert abs(roof["valu_issue"]["frac"] - 24e6 / 50e-6 / 614.4e9) < 1e-4
    rec["source_sha256_16"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.stored_valu("k_support_batch", "640x480_D128_x8") is None


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_by_the_copy_kernel(tmp_path):
    d = {k: tmp_path / k for k in ("f", "w", "cf", "cw")}
    for p in d.values():
        p.mkdir()
    kname = "elas::(anonymous namespace)::k_dense2(elas::Frame)"
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda()>(int)"
    _counter_csv(d["f"] / "run_counter_collection.csv",
                 [[1, kname, "FETCH_SIZE", 100.0], [2, kname, "FETCH_SIZE", 300.0]])
    _counter_csv(d["w"] / "run_counter_collection.csv", [[1, kname, "WRITE_SIZE", 50.0]])
    # the copy moves 1 MiB each way; FETCH_SIZE reads half of it
    _counter_csv(d["cf"] / "run_counter_collection.csv", [[1, copy, "FETCH_SIZE", 512.0]])
    _counter_csv(d["cw"] / "run_counter_collection.csv", [[1, copy, "WRITE_SIZE", 1024.0]])
    out_json, out_md = tmp_path / "t.json", tmp_path / "t.md"
    profiling.main(["traffic", "--kernel", "k_dense2", "--workload", "x", "--fetch", str(d["f"]),
                    "--write", str(d["w"]), "--calib-fetch", str(d["cf"]), "--calib-write",
                    str(d["cw"]), "--copy-bytes", str(1 << 20), "--json", str(out_json),
                    "--md", str(out_md), "--cmd", "cmd"])
    rec = json.loads(out_json.read_text())
    # fetch: mean 200 KiB x factor 2; write: 50 KiB x factor 1
    assert rec["fetch_bytes"] == 200 * 1024 * 2 and rec["write_bytes"] == 50 * 1024
    assert rec["bytes_per_launch"] == 200 * 1024 * 2 + 50 * 1024
    assert rec["calib_copy_kernel"] == ["neg_kernel_cuda", "neg_kernel_cuda"]
    assert "HBM traffic per launch" in out_md.read_text()


def test_kernel_short_names():
    assert profiling.short_name("elas::(anonymous namespace)::k_mesh(elas::Frame)") == "k_mesh"
    assert profiling.short_name("k_check") == "k_check"
