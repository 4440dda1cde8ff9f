"""bench.py's command-line contract that can be checked without a GPU."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_is_reported_only_for_current_sources(tmp_path, monkeypatch):
    """The counter-measured bytes of a kernel are used only while the hash
    recorded with them matches its sources; a stale line reads as None."""
    sys.path.insert(0, ROOT)
    import bench
    src = "backproject.hip"
    good = bench.source_hash(src)
    f = tmp_path / "traffic.md"
    f.write_text("traffic: cells %s %s 2000 1000\ntraffic: gather %s %s 30 10\n"
                 % (src, good, src, "0" * 16))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("cells", (0, 1)) == 2000
    assert bench.measured_traffic("cells", (1, 1)) == 1500      # weighted by launches
    assert bench.measured_traffic("gather", (0, 1)) is None     # stale hash
    assert bench.measured_traffic("project", (0, 1)) is None    # no line
    ops = bench.operator_rooflines(_Geom(), 1.0e9, 2.0, 4.0)
    assert "measured_bytes" not in ops["P"] and "measured_bytes" not in ops["PT"]


class _Geom:
    n_vox = 1000
    n_meas = 500
