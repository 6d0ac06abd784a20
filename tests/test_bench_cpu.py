"""Host-side helpers of bench.py: the rocprofv3 summary tables and the
recorded-traffic lookup (used only while the kernel source is unchanged)."""
import json
import os
import sqlite3
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_profile_summary_tables(tmp_path):
    db = tmp_path / "r.db"
    con = sqlite3.connect(db)
    con.execute("create table top_kernels (name text, total_calls int, total_duration real, average real, "
                "percentage real)")
    con.execute("insert into top_kernels values ('ctmi::(anonymous namespace)::k_backward_interp(float const*)', "
                "2, 4000000.0, 2000000.0, 90.0)")
    con.execute("create table pmc_events (name text, dispatch_id int, counter_name text, counter_value real)")
    for d in (1, 2):
        con.execute("insert into pmc_events values ('k_forward_interp(float const*)', ?, 'FETCH_SIZE', 10.0)", (d,))
        con.execute("insert into pmc_events values ('k_forward_interp(float const*)', ?, 'FETCH_SIZE', 5.0)", (d,))
    con.commit()
    con.close()
    out = bench.profile_summary(str(db))
    assert "| k_backward_interp | 2 | 2000.000 | 4000.000 | 90.00 |" in out
    assert "| k_forward_interp | 2 | 15 |" in out


def test_recorded_traffic_requires_matching_source(tmp_path, monkeypatch):
    src = tmp_path / "paper_2412_10129_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "backward.hip").write_text("kernel v1")
    (tmp_path / "profiles").mkdir()
    rec = {"calibration": {"fetch_factor": 2.0, "write_factor": 1.0},
           "kernels": {"interp_bwd": {"fetch_kib": 100.0, "write_kib": 10.0,
                                      "source_sha256": bench._sha256(str(src / "backward.hip"))}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("interp_bwd") == 1024 * (100 * 2 + 10)
    assert bench.recorded_traffic("interp_fwd") is None
    (src / "backward.hip").write_text("kernel v2")
    assert bench.recorded_traffic("interp_bwd") is None


def test_more_than_one_gpu_is_refused():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
