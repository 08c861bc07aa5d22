"""The rocprofv3 summaries' host logic on small synthetic CSV files (CPU)."""

import subprocess
import sys


def test_phases_joins_slots_with_the_kernel_trace(tmp_path):
    # three slots: a prediction slot, a 2-target block, an empty slot; times
    # in ns, each slot an evaluation then a finishing dispatch
    rows = [("k_bl_eval<false, false>", 0, 1000), ("k_bl_finish", 3000, 7000),
            ("k_bl_eval<false, false>", 9000, 14000), ("k_bl_finish", 16000, 26000),
            ("k_bl_eval<false, false>", 28000, 29000), ("k_bl_finish", 31000, 32000)]
    trace = tmp_path / "trace.csv"
    with open(trace, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp\n")
        f.write("1,void h6::(anonymous namespace)::k_bl_setup_plan(h6::LoopArgs),0,0\n")
        for i, (k, t0, t1) in enumerate(rows):
            f.write('%d,"void h6::(anonymous namespace)::%s(h6::LoopArgs, long)",%d,%d\n'
                    % (i + 2, k, t0, t1))
    log = tmp_path / "slots.txt"
    log.write_text("# n_act split\n5 -1\n2 64\n0 0\n")
    out = subprocess.run([sys.executable, "-m", "paper_1901_08532_amd.profsum", "phases",
                          str(trace), str(log)], capture_output=True, text=True, check=True).stdout
    lines = {l.split()[0]: l.split() for l in out.splitlines() if not l.startswith("#")}
    # the 2-target block: eval 5 us, gap 2 us, finish 10 us, gap 2 us, slot 19 us
    assert lines["2"][1:7] == ["1", "5.00", "2.00", "10.00", "2.00", "19.00"]
    # the prediction slot: eval 1, gap 2, finish 4, gap 2, slot 9 of 32 us
    pred = [l for l in out.splitlines() if l.startswith("prediction slot")][0].split()
    assert pred[2:8] == ["1", "1.00", "2.00", "4.00", "2.00", "9.00"]
    assert pred[8] == "28.1%"
