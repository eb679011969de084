"""Host logic of bench.py: the counted-traffic record is used only for the kernel source and the
schedule (grid form, XCD mapping, staging mode) it was measured on."""
import hashlib
import json

import bench


def _record(tmp_path, src_bytes, records):
    src = tmp_path / "k.hip"
    src.write_bytes(src_bytes)
    rec = tmp_path / "traffic.json"
    rec.write_text(json.dumps({"kernel_source_sha256": hashlib.sha256(src_bytes).hexdigest(), "records": records}))
    return str(src), str(rec)


def test_traffic_record_matches_schedule_and_source(tmp_path, monkeypatch):
    src, rec = _record(tmp_path, b"kernel v1", [
        {"counter_schedule": "1,0,1,2", "traffic_bytes_per_launch": 2.0e9},
        {"counter_schedule": "1,0,0,2", "traffic_bytes_per_launch": 2.5e9},
    ])
    monkeypatch.setattr(bench, "KERNEL_SOURCE", src)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", rec)
    s = dict(waves_per_block=1, blocks_per_cu=0, xcd_remap=1, shared_segments=2)
    assert bench.measured_traffic(s) == 2.0e9
    # waves per workgroup only regroup the same units: the record still applies
    assert bench.measured_traffic(dict(s, waves_per_block=4)) == 2.0e9
    assert bench.measured_traffic(dict(s, xcd_remap=0)) == 2.5e9
    # another grid form, staging mode or no schedule: no record
    assert bench.measured_traffic(dict(s, blocks_per_cu=2)) is None
    assert bench.measured_traffic(dict(s, shared_segments=0)) is None
    assert bench.measured_traffic(None) is None
    # a changed kernel source voids the record
    (tmp_path / "k.hip").write_bytes(b"kernel v2")
    assert bench.measured_traffic(s) is None


def test_traffic_record_missing_or_malformed(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.measured_traffic(dict(waves_per_block=1, blocks_per_cu=0, xcd_remap=1, shared_segments=2)) is None
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(bad))
    assert bench.measured_traffic(dict(waves_per_block=1, blocks_per_cu=0, xcd_remap=1, shared_segments=2)) is None
