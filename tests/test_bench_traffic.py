"""The benchmark reports the measured HBM traffic of the determinant kernel
only while the committed counter summary matches the kernel sources and the
launch plan it was taken with (host logic, no device)."""
import json

import bench

PLAN = [{"walker_tile": 64, "item_exc": 702, "threads": 512},
        {"walker_tile": 64, "item_exc": 679, "threads": 512}]


def _summary(tmp_path, source_hash, plan, nbytes=98765000):
    p = tmp_path / "traffic.md"
    p.write_text("# counters\n\n| a | b |\n\n"
                 f"traffic_bytes_per_launch: {nbytes}\n"
                 f"traffic_source_hash: {source_hash}\n"
                 f"traffic_plan: {json.dumps(plan, sort_keys=True)}\n")
    return str(p)


def test_traffic_reported_when_sources_and_plan_match(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, bench.kernel_source_hash(), PLAN))
    assert bench.measured_traffic(PLAN) == 98765000.0


def test_traffic_null_after_a_source_change(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, "0123456789abcdef", PLAN))
    assert bench.measured_traffic(PLAN) is None


def test_traffic_null_for_another_plan(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, bench.kernel_source_hash(), PLAN))
    other = [dict(PLAN[0], item_exc=351), PLAN[1]]
    assert bench.measured_traffic(other) is None


def test_traffic_null_without_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic(PLAN) is None

