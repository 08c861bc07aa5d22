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


def test_committed_counter_records_match_the_current_sources():
    # the traffic and VALU summaries under profiles/ were taken with the
    # kernel sources as they are: bench.py reports them only while the
    # sources hash to the recorded value, so a stale record shows here
    sys.path.insert(0, ROOT)
    import bench

    assert bench._traffic_fields().get("eval_source_sha256") == bench._eval_sources_sha256()
    assert bench._executed_flops_per_interaction() is not None
    assert bench._vjp_record() is not None
    assert bench._vjp_flops_per_pair() is not None


def test_loop_breakdown_sums_both_kernels_per_block():
    # records as h6_profile_read returns them at level 2: evaluation (kind 2)
    # and finishing kernel (kind 4) per active-count bin, prediction slots in
    # bin -2 (their evaluations empty), empty slots in bin -1
    sys.path.insert(0, ROOT)
    import bench
    from paper_1901_08532_amd import h6

    def rec(kind, b, launches, ms, nbytes):
        return {"order": 2, "kind": kind, "block": 0, "ipl": 0, "precision": 0, "nact_log2": b,
                "launches": launches, "interactions": 0.0, "kernel_ms": ms, "bytes": nbytes}

    recs = [rec(2, 1, 10, 0.1, 1e6), rec(2, 12, 2, 4.0, 2e7), rec(4, 1, 10, 0.12, 3e6),
            rec(4, 12, 2, 0.1, 4e7), rec(2, -2, 3, 0.01, 0.0), rec(4, -2, 3, 0.015, 6e6),
            rec(2, -1, 5, 0.02, 0.0), rec(4, -1, 5, 0.02, 0.0)]
    out = bench._loop_breakdown(recs, 12, h6.H6_FP64)
    assert out["blocks"] == 12
    ev, fi, ps = out["k_bl_eval"], out["k_bl_finish"], out["k_bl_finish (prediction slots)"]
    assert ev["launches"] == 12 and fi["launches"] == 12 and ps["launches"] == 3
    assert abs(fi["avg_us"] - 1e3 * 0.22 / 12) < 1e-9
    assert abs(ev["algorithmic_bytes_per_launch"] - 2.1e7 / 12) < 1e-6
    total = 4.1 + 0.22 + 0.015  # empty slots apart
    assert abs(fi["share_of_loop_gpu_time"] - 0.22 / total) < 1e-12
    assert abs(fi["algorithmic_bytes_per_nonempty_launch"] - 4.9e7 / 15) < 1e-6
