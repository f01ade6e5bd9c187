"""Host logic of bench.py's counter-derived roofline fields: the committed
rocprofv3 record is used only while the sources it was taken with are
unchanged and only for the launch shape it was taken with; the gather object
derives from the same record."""
import json
import os
import shutil

import pytest

import bench

LAUNCH = {"algorithm": 1, "samples_per_tile": 64, "waves_per_group": 4, "groups_per_cu": 4, "xcd_queues": 8,
          "chunk": 64, "coherence": 0.5}


def _record():
    return json.load(open(os.path.join(bench.ROOT, "profiles", "traffic_conv_c3.json")))


def _current_or_skip():
    if bench.measured_counters(LAUNCH) is None:
        pytest.skip("the committed counter record was taken with other sources (the bench reports null)")


def test_record_matches_current_sources():
    _current_or_skip()
    rec = _record()
    t = bench.measured_traffic(LAUNCH)
    r8 = next(r for r in rec["records"] if r["launch"]["xcd_queues"] == 8)
    assert t == r8["traffic_bytes_per_launch"]
    # bytes = FETCH KiB x fetch factor + WRITE KiB x write factor, per launch
    cal = r8["copy_calibration"]
    want = 1024 * (r8["fetch_kib_per_launch"] * cal["fetch_factor"] + r8["write_kib_per_launch"] * cal["write_factor"])
    assert t == pytest.approx(want, rel=1e-12)


def test_gather_object_from_the_record():
    _current_or_skip()
    g = bench.gather_roofline(LAUNCH, pairs=1_000_000, k_ms=1.0)
    p = bench.measured_counters(LAUNCH)["pipeline"]
    assert g["achieved"] == pytest.approx(1e6 * 16 / 1e-3 / 1e9)
    assert g["td_busy"] == p["td_busy"] and 0.0 < g["td_busy"] <= 1.0
    c = p["counters"]
    assert g["l1_lines_per_gather"] == pytest.approx(c["TCP_TOTAL_CACHE_ACCESSES_sum"] / c["TA_BUFFER_READ_WAVEFRONTS_sum"])


def test_other_launch_shape_or_changed_source_gives_none(tmp_path, monkeypatch):
    other = dict(LAUNCH, xcd_queues=4)
    assert bench.measured_traffic(other) is None
    assert bench.gather_roofline(other, 1, 1.0) is None
    # a copy of the tree whose kernel source differs by one byte
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    shutil.copy(os.path.join(bench.ROOT, "profiles", "traffic_conv_c3.json"), root / "profiles")
    for f in _record()["sources_sha256"]:
        dst = root / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), dst)
    monkeypatch.setattr(bench, "ROOT", str(root))
    if bench.measured_traffic(LAUNCH) is None:
        pytest.skip("the committed counter record was taken with other sources")
    src = root / next(iter(_record_at(root)["sources_sha256"]))
    src.write_bytes(src.read_bytes() + b"\n")
    assert bench.measured_traffic(LAUNCH) is None
    assert bench.gather_roofline(LAUNCH, 1, 1.0) is None


def _record_at(root):
    return json.load(open(os.path.join(root, "profiles", "traffic_conv_c3.json")))
