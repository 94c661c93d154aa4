"""The committed HBM-traffic record (profiles/lw_step_traffic.json) against
the bench's own definitions: every tiling the sweep times has an entry, each
entry's bytes follow from its raw counter values and the calibration, and a
tiling outside the record gives no traffic.  CPU only: it reads files."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REC = os.path.join(ROOT, "profiles", "lw_step_traffic.json")


@pytest.fixture(scope="module")
def rec():
    with open(REC) as f:
        return json.load(f)


def test_every_swept_tiling_has_an_entry(rec):
    for prec, tilings in bench.SWEEP_TILINGS.items():
        for rows, order in tilings:
            assert "%d:%d" % (rows, order) in rec["fp%d" % prec], (prec, rows, order)


def test_entries_follow_from_the_counts(rec):
    points = 32768 * 1024                       # the swept workload's grid
    for prec in (64, 32):
        for key, e in rec["fp%d" % prec].items():
            assert e["algorithmic_bytes"] == bench.BYTES_PER_UPDATE[prec] * points, key
            assert e["fetch_bytes"] == round(e["fetch_raw_KiB"] * 1024 * rec["fetch_scale"]), key
            assert e["write_bytes"] == round(e["write_raw_KiB"] * 1024 * rec["write_scale"]), key
            ratio = (e["fetch_bytes"] + e["write_bytes"]) / e["algorithmic_bytes"]
            assert e["ratio_to_algorithmic"] == pytest.approx(ratio, abs=5e-5), key
            # at least the algorithmic bytes move, and not wildly more
            assert 1.0 <= ratio < 1.6, key
            assert e["dispatches"] >= 1 and e["trace_avg_ns"] > 0 and e["sweep_ms_per_launch"] > 0, key


def test_the_calibration_is_the_one_applied(rec):
    # the copy kernel moves 2 GiB each way: fetch counts read half of it
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert "1.0000 GiB" in rec["calibration"] and "2.0000 GiB" in rec["calibration"]


def test_lookup(rec):
    if rec.get("kernel_code_sha256") != bench.kernel_code_hash():
        # counters of other kernel code are never reported
        assert bench.measured_traffic(64, 96, 0) is None
        return
    t = bench.measured_traffic(64, 96, 0)
    e = rec["fp64"]["96:0"]
    assert t["bytes_per_launch"] == e["fetch_bytes"] + e["write_bytes"]
    assert bench.measured_traffic(64, 7, 0) is None      # a tiling outside the record
