"""Host-side logic of bench.py: the sweep kind's byte model and the roofline
object (no GPU)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import bench  # noqa: E402

N = 1_000_000


def test_sweep_kind_bytes_fused_path():
    # x_1 from the noise launch; first launch 116 B/pt (reads x_1, y, spread,
    # col, p; writes x_2), each later iterate 96 B/pt, the tail's finalisation 28 B/pt
    assert bench.sweep_kind_bytes(N, 4, 8, 8, 8, True) == (116 + 2 * 96 + 28) * N
    assert bench.sweep_kind_bytes(N, 4, 8, 8, 8, False) == (116 + 2 * 96) * N
    assert bench.sweep_kind_bytes(N, 2, 8, 8, 8, True) == (116 + 28) * N
    # a selection that stopped at x_1: the first launch only adds the flags and sums
    assert bench.sweep_kind_bytes(N, 1, 8, 8, 8, True) == (16 + 16 + 12 + 8 + 28) * N


def test_sweep_kind_sum_missing_record_is_none():
    rec = {"sweep_first_merged": 117e6, "sweep": 98e6}
    assert bench.sweep_kind_sum(4, 8, False, rec.get) == pytest.approx(117e6 + 2 * 98e6)
    assert bench.sweep_kind_sum(4, 8, True, rec.get) is None  # no tail record


def test_roofline_object_hbm_and_alu():
    k = {"ms_per_step": 0.1, "launches_per_step": 1.0, "us_per_launch": 100.0}
    # 400 MB in 0.1 ms = 4 TB/s = 0.5 of peak; VALU at 0.1 of its peak: HBM view
    low = {"insts_per_launch": 0.1 * bench.VALU_ISSUE_PEAK * 100e-6, "frac": 0.1}
    r = bench.roofline_object("sweep", k, 400e6, 410e6, low)
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(0.5) and r["traffic"] == 410e6
    assert r["valu"] is low
    # 100 MB in 0.1 ms = 0.125 of HBM peak; VALU issue at 0.6: the ALU view
    insts = 0.6 * bench.VALU_ISSUE_PEAK * 100e-6
    r = bench.roofline_object("local_sort", k, 100e6, 120e6, {"insts_per_launch": insts, "frac": 0.6})
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(0.6)
    assert r["achieved"] == pytest.approx(0.6 * r["peak"])
    assert r["hbm"]["frac"] == pytest.approx(0.125) and r["traffic"] == 120e6
    # no counter record: the HBM view
    assert bench.roofline_object("merge", k, 100e6, None, None)["bound"] == "hbm"
