"""Host-side logic of the benchmark (no GPU): the algorithmic byte models,
the roofline record, the traffic lookup's source check, and the host models
of x access (lines per wavefront gather, stride distributions)."""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_byte_models_count_each_array_once():
    # CRS: val + col per entry, row_ptr, x once, y once (twice with beta)
    assert bench.bytes_crs(10, 4, 5, 8, 8) == 10 * 12 + 4 * 5 + 8 * 5 + 8 * 4
    assert bench.bytes_crs(10, 4, 5, 8, 8, beta=True) == 10 * 12 + 4 * 5 + 8 * 5 + 8 * 8
    assert bench.bytes_crs(10, 4, 5, 4, 8, k=3) == 10 * 8 + 4 * 5 + 3 * 8 * (5 + 4)
    # JDS: entries, jd_ptr, perm, x, y
    assert bench.bytes_jds(10, 4, 5, 3, 8, 8) == 10 * 12 + 4 * 4 + 4 * 4 + 8 * 9
    # blocked: entries, 12 bytes per slice, perm, x, y
    assert bench.bytes_blocked(10, 4, 5, 2, 2, 8) == 10 * 6 + 24 + 16 + 8 * 9


def test_dia_bytes_count_spans():
    class R:
        nnz, n_rows = 3, 6

    class D:
        n_rows, n_cols, offsets, rem, rem_slices = 6, 6, np.array([-2, 0, 5]), R(), None
    # spans 4 + 6 + 1 stored values, the remainder as CRS, x and y
    assert bench.bytes_dia(D, 8, 8) == 11 * 8 + 3 * 12 + 4 * 7 + 8 * 12

    class T:                                        # one slice of depth 2: 128 padded slots
        bl_col, slice_nd, slot_row = np.zeros(128), np.zeros(1), np.zeros(6)

    D.rem_slices = T()
    assert bench.bytes_dia(D, 8, 8) == 11 * 8 + 128 * 12 + 12 + 6 + 8 * 12


def test_roofline_record():
    e = bench.roofline_for("no_such_kernel", 8e9, 2.0, "powerlaw")
    assert e["achieved"] == 4000.0 and e["frac"] == 0.5 and e["peak"] == 8000.0 and e["unit"] == "GB/s"
    assert e["traffic"] is None                     # nothing measured for it


def test_traffic_only_while_sources_match(tmp_path, monkeypatch):
    import json
    srcs = bench.kernel_sources("jds_f64")
    good = {"entries": {"powerlaw:jds_f64": {"source_sha": bench.kernel_source_sha(srcs), "bytes_per_launch": 123}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(p))
    assert bench.measured_traffic("jds_f64", "powerlaw") == 123
    good["entries"]["powerlaw:jds_f64"]["source_sha"] = "0" * 16
    p.write_text(json.dumps(good))
    assert bench.measured_traffic("jds_f64", "powerlaw") is None


def test_lines_per_wave():
    # 64 consecutive columns: 4 lines of 16 FP64; 64 columns 16 apart: 64 lines
    cols = np.concatenate([np.arange(64), np.arange(64) * 16]).astype(np.int32)
    chunk = np.repeat([0, 1], 64)
    r = bench._lines_per_wave(cols, chunk, 16)
    assert r["mean"] == 34.0 and r["frac_ge_32"] == 0.5
    # padding (col < 0) is not a gather
    r = bench._lines_per_wave(np.array([-1, -1, 0, 1], np.int32), np.zeros(4, np.int64), 16)
    assert r["mean"] == 1.0


def test_stride_distribution():
    d = bench._stride_dist(np.array([0, 1, 2, 10, 3, -1, 4, 1000], np.int32))
    # jumps 1, 1, 8, -7, 1, 996 elements (padding skipped): 8 bytes each
    assert d["jumps"] == 6
    assert d["backward_frac"] == round(1 / 6, 4)
    assert d["forward_below_64B_frac"] == round(3 / 6, 4)
    assert d["forward_cdf"]["64"] == round(3 / 6, 4) and d["forward_cdf"]["512"] == round(4 / 6, 4)
    assert d["backward_cdf"]["64"] == round(1 / 6, 4)


def test_row_order_traversal():
    class A:
        row_ptr = torch.tensor([0, 2, 3, 6], dtype=torch.int32)
        col_idx = torch.tensor([5, 6, 1, 7, 8, 9], dtype=torch.int32)
    assert bench._row_order_cols(A, np.array([2, 0, 1])).tolist() == [7, 8, 9, 5, 6, 1]
