"""Host-side checks of the benchmark's profile summaries on synthetic rocprofv3
output: the finest-level operator applications are found as (shared-DoF
clearing, batch kernel) pairs, and the HBM traffic is scaled by the
calibration copy.  No GPU involved."""
import csv
import json
import os

import pytest

import bench

VMULT = "void mfmg::(anonymous namespace)::vmult_batch_kernel<4, double, double, 4, 0, false>(mfmg::CellMeta const*)"
CLEAR = "void mfmg::(anonymous namespace)::clear_shared_kernel<double>(long, double*)"
OTHER = "void mfmg::(anonymous namespace)::vmult_batch_kernel<4, double, double, 1, 0, false>(mfmg::CellMeta const*)"
COPY = "void at::native::elementwise_kernel<128, 4>(int, Func)"


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _dispatches():
    """(name, grid, duration ns) in launch order: a coarse-level pair, three
    finest-level pairs (clearing grid 1000) and a fused kernel between them."""
    seq = [(CLEAR, 100, 2000), (VMULT, 524288, 90000)]
    for _ in range(3):
        seq += [(CLEAR, 1000, 20000), (VMULT, 524288, 780000), (OTHER, 524288, 1200000)]
    return seq


def test_trace_summary_pairs_clear_and_batch(tmp_path):
    rows, t = [], 0
    for name, grid, dur in _dispatches():
        rows.append({"Kind": "KERNEL_DISPATCH", "Kernel_Name": name, "Grid_Size_X": grid, "Grid_Size_Y": 1,
                     "Grid_Size_Z": 1, "Start_Timestamp": t, "End_Timestamp": t + dur})
        t += dur + 100
    trace = tmp_path / "kernel_trace.csv"
    _write_csv(trace, rows)
    line = {"steps": 3, "roofline": {"avg_launch_ms": 0.8, "alg_bytes_per_launch": 1.6e9, "achieved": 2000.0,
                                      "frac": 0.25},
            "config": {"cells": 10, "hanging_cells": 1, "free_dofs": 100000000}}
    bj = tmp_path / "bench.json"
    bj.write_text("progress line\n" + json.dumps(line) + "\n")
    text = bench.trace_summary(str(trace), str(bj), ["cmd"])
    assert "| clear_shared_kernel<double> | 1000 | 3 | 20.0 us |" in text
    assert "| vmult_batch_kernel<4, double, double, 4, 0, false> | 524288 | 3 | 780.0 us |" in text
    assert "| sum = one operator application | | | 800.0 us |" in text
    assert "(0.0 % from the trace)" in text
    assert "2000 GB/s from the trace" in text


def _pmc_folder(root, counter, values):
    """One rocprofv3 counter-collection csv with one counter per dispatch."""
    os.makedirs(root)
    rows = []
    for i, ((name, grid, _), v) in enumerate(zip(_dispatches() + [(COPY, 4096, 0)], values)):
        rows.append({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                     "Counter_Value": v})
    _write_csv(os.path.join(root, "run_counter_collection.csv"), rows)


def test_pmc_summary_scales_by_the_copy(tmp_path):
    n = 1 << 20  # doubles moved each way by the calibration copy
    copy_kib = 8.0 * n / 1024.0
    # FETCH_SIZE reads half the bytes (scale 2), WRITE_SIZE all of them
    fetch = [1.0, 2.0] + [0.0, 100.0, 7.0] * 3 + [copy_kib / 2]
    write = [1.0, 2.0] + [50.0, 300.0, 7.0] * 3 + [copy_kib]
    _pmc_folder(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _pmc_folder(str(tmp_path / "w"), "WRITE_SIZE", write)
    text = bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), n, ["cmd"])
    assert "factors 2.0000 (FETCH_SIZE) and 1.0000 (WRITE_SIZE)" in text
    traffic = float(text.split("traffic_bytes_per_launch:")[1].split()[0])
    assert traffic == pytest.approx((100.0 * 2.0 + 50.0 + 300.0) * 1024.0)
    assert "source_sha256: " + bench.operator_source_digest() in text


def test_recorded_traffic_follows_the_source_digest(tmp_path, monkeypatch):
    """The bench line reports the committed traffic only while the operator
    sources hash to the digest the summary was taken with."""
    f = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic() is None  # no summary
    f.write_text(f"traffic_bytes_per_launch: 1234\nsource_sha256: {bench.operator_source_digest()}\n")
    assert bench.recorded_traffic() == 1234.0
    f.write_text("traffic_bytes_per_launch: 1234\nsource_sha256: " + "0" * 64 + "\n")
    assert bench.recorded_traffic() is None  # sources changed since
