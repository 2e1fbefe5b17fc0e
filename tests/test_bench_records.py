"""Host logic of the bench's traffic records: a record is reported only for
the sources it was measured on and for the schedule it names."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def _bytes(t):
    return int((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)


def test_record_per_schedule(monkeypatch):
    monkeypatch.setattr(bench, "SOURCES_SHA256", bench.sources_sha256())
    recs = bench.TRAFFIC["bulk k_lv_rows"]
    assert isinstance(recs, list) and len(recs) >= 2
    for t in recs:
        assert bench.measured_traffic("bulk k_lv_rows", dict(t["schedule"], rounds_per_launch=16)) == _bytes(t)
    assert bench.measured_traffic("bulk k_lv_rows", {"lv_grid": 3}) is None
    assert bench.measured_traffic("bulk k_lv_rows", None) is None
    # a record without a schedule holds for any
    plain = bench.TRAFFIC["plain k_rows"]
    assert bench.measured_traffic("plain k_rows") == _bytes(plain)
    assert bench.measured_traffic("no such kernel") is None
    # a schedule key the record names must match
    probe = bench.TRAFFIC["probe k_rows"]
    assert bench.measured_traffic("probe k_rows", dict(probe["schedule"])) == _bytes(probe)
    assert bench.measured_traffic("probe k_rows", dict(probe["schedule"], probe_slots=512)) is None


def test_no_record_once_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "SOURCES_SHA256", "0" * 64)
    assert bench.measured_traffic("plain k_rows") is None
    monkeypatch.setattr(bench, "SOURCES_SHA256", None)
    assert bench.measured_traffic("plain k_rows") is None
