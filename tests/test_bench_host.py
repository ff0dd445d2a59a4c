"""Host logic of bench.py that needs no GPU: the counter summary that turns
rocprofv3 FETCH_SIZE / WRITE_SIZE readings into bytes per launch."""
import csv
import json
import os

import bench

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size",
          "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value",
          "Start_Timestamp", "End_Timestamp"]


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, counter, value) in enumerate(rows):
            r = {k: 0 for k in FIELDS}
            r.update(Dispatch_Id=i + 1, Kernel_Name=name, Counter_Name=counter, Counter_Value=value)
            w.writerow(r)


def test_traffic_from_scales_by_the_copy_probe(tmp_path):
    kern = "demap_mfma_w<4, false, true, 6, false>"
    full = f"void air::{kern}(air::DemapArgs, ...)"
    other = "void air::demap_mfma_w<4, false, true, 6, true>(air::DemapArgs, ...)"
    # two dispatches of the kernel (100 and 300 KiB fetched), one of another kernel
    _write(str(tmp_path / "f" / "h" / "1_counter_collection.csv"),
           [(full, "FETCH_SIZE", 100.0), (other, "FETCH_SIZE", 5000.0), (full, "FETCH_SIZE", 300.0)])
    _write(str(tmp_path / "w" / "h" / "1_counter_collection.csv"),
           [(full, "WRITE_SIZE", 50.0), (full, "WRITE_SIZE", 50.0)])
    # the 1 GiB copy reads 2^20 KiB worth of FETCH_SIZE / 2 and writes 2^20 KiB
    _write(str(tmp_path / "cf" / "h" / "1_counter_collection.csv"),
           [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0), ("fill", "FETCH_SIZE", 7.0)])
    _write(str(tmp_path / "cw" / "h" / "1_counter_collection.csv"),
           [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0)])
    d = bench.traffic_from(str(tmp_path), "psk8x8", "fp16x3", kern, ["cmd"])
    assert d["dispatches"] == [2, 2]
    assert d["fetch_size_kib_per_dispatch"] == 200.0
    assert d["copy_probe"]["fetch_factor"] == 2.0 and d["copy_probe"]["write_factor"] == 1.0
    assert d["fetch_bytes_per_launch"] == 200.0 * 1024 * 2
    assert d["write_bytes_per_launch"] == 50.0 * 1024
    assert d["bytes_per_launch"] == 200.0 * 1024 * 2 + 50.0 * 1024
    assert d["source_hash"] == bench.source_hash()
    json.dumps(d)


def test_stored_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    p = tmp_path / "traffic_x_fp16x3.json"
    p.write_text(json.dumps({"bytes_per_launch": 123.0, "source_hash": bench.source_hash()}))
    assert bench.stored_traffic("x", "fp16x3") == 123.0
    p.write_text(json.dumps({"bytes_per_launch": 123.0, "source_hash": "stale"}))
    assert bench.stored_traffic("x", "fp16x3") is None
    assert bench.stored_traffic("y", "fp16x3") is None
