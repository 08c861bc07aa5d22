"""Host-side checks of bench.py's command line (no GPU needed)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_workload_choices_include_adjoint():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for w in ("plummer", "plummer-imf", "two-clusters", "adjoint", "adjoint-block"):
        assert w in r.stdout
    assert "--accuracy-targets" in r.stdout


def test_vjp_flop_count_is_read_from_the_counter_summary():
    # read only while the VJP traffic record's source hash matches the
    # current VJP sources (the counters were taken with those sources)
    sys.path.insert(0, ROOT)
    import bench

    f = bench._vjp_flops_per_pair()
    t = bench._vjp_traffic_per_launch()
    if os.path.exists(bench.VJP_COUNTER_FILE) and bench._vjp_record() is not None:
        assert f is not None and 100.0 < f < 1000.0
        assert t is not None and t > 0
    else:
        assert f is None and t is None
    json.dumps({"f": f, "t": t})
