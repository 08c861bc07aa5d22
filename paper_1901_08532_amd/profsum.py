"""Summaries of rocprofv3 CSV output for the measurement records.

  python -m paper_1901_08532_amd.profsum stats <kernel_stats.csv> [--match SUBSTR]
      per-kernel calls, average and total duration

  python -m paper_1901_08532_amd.profsum counters <counter_collection.csv> --match K
      --interactions I
      the largest dispatches of kernel K: each counter, VALU/LDS instructions
      per interaction (for I interactions per dispatch), executed FP64 flops
      and the clock from GRBM_GUI_ACTIVE

  python -m paper_1901_08532_amd.profsum traffic <fetch counter_collection.csv>
      <write counter_collection.csv> --copy-bytes B [--match SUBSTR] [--sources eval|vjp]
      [--min-kib K]
      HBM bytes per dispatch of each matching kernel from FETCH_SIZE and
      WRITE_SIZE (KiB per dispatch), each scaled by the ratio of the known
      bytes a plain device copy of B bytes moves to what the same counter
      reports for it, averaged over the dispatches that fetched at least K
      KiB (default 64: the loop's launches with nothing to do read a few
      descriptor lines); the i-th dispatch of a kernel in the write run is
      taken for the i-th of the fetch run (the runs are deterministic).
      Prints key = value lines.

  python -m paper_1901_08532_amd.profsum phases <kernel_trace.csv> <slot log>
      the device loop's slots (bench.py --slot-log) joined with the kernel
      trace of the same process (slot k: the k-th k_bl_eval and k_bl_finish
      dispatches): per class of active count, the mean evaluation time, the
      gap to the finishing kernel, the finishing time, the gap to the next
      slot's evaluation, and the classes' shares of the interval
"""

import argparse
import csv
import hashlib
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1901_08532_amd", "csrc")
# the evaluation kernels' sources (the same list as bench.py checks), and
# the evaluation VJP kernel's
EVAL_SOURCES = ("eval_body.h", "eval_mixed_body.h", "device_math.h", "steps_body.h",
                "blockloop.hip", "eval.hip", "eval_mixed.hip")
VJP_SOURCES = ("adjoint.hip", "device_math.h")


def eval_sources_sha256(sources=EVAL_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def _short(name):
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"\(.*\)$", "", name)  # drop the parameter list
    return name.replace("void ", "").strip()


def stats(path, match=None):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        nm = _short(r["Name"])
        if match and match not in nm:
            continue
        out.append((nm, int(r["Calls"]), float(r["AverageNs"]), float(r["TotalDurationNs"]),
                    float(r["Percentage"])))
    out.sort(key=lambda t: -t[3])
    print("%-60s %8s %14s %14s %7s" % ("kernel", "calls", "avg_us", "total_ms", "pct"))
    for nm, calls, avg, tot, pct in out:
        print("%-60s %8d %14.3f %14.3f %7.2f" % (nm[:60], calls, avg / 1e3, tot / 1e6, pct))


def _counter_per_dispatch(path, counter):
    """{kernel short name: [value per dispatch, in dispatch order]} for one
    counter (summed over the per-instance rows of a dispatch)."""
    per = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        d = int(r["Dispatch_Id"])
        per[d] += float(r["Counter_Value"])
        names[d] = _short(r["Kernel_Name"])
    by_kernel = defaultdict(list)
    for d in sorted(per):
        by_kernel[names[d]].append(per[d])
    return by_kernel


def _tag(k):
    m = re.search(r"k_eval_f64<2, (\d+), (\d+), false>", k)
    if m:
        return "b%s_i%s" % (m.group(1), m.group(2))
    for pat, tag in (("k_bl_eval<false, false>", "bl_eval_fp64"),
                     ("k_bl_eval<true, false>", "bl_eval_mixed"),
                     ("k_bl_finish", "bl_finish"),
                     ("k_eval_vjp<2, 128, 0>", "eval_vjp")):
        if pat in k:
            return tag
    return re.sub(r"\W+", "_", k)[:60]


def traffic(fetch_csv, write_csv, copy_bytes, match=None, sources="eval", min_kib=64.0):
    fetch = _counter_per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _counter_per_dispatch(write_csv, "WRITE_SIZE")
    # the calibration copy is the largest dispatch of a copy kernel in each run
    cf = max(max(v) for k, v in fetch.items() if "copy" in k.lower())
    cw = max(max(v) for k, v in write.items() if "copy" in k.lower())
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    print("# rocprofv3 FETCH_SIZE / WRITE_SIZE, KiB per dispatch, scaled by a %d-byte copy" % copy_bytes)
    print("copy_fetch_kib = %.1f" % cf)
    print("copy_write_kib = %.1f" % cw)
    print("fetch_scale = %.6f" % f_scale)
    print("write_scale = %.6f" % w_scale)
    if sources == "vjp":
        print("vjp_source_sha256 = %s" % eval_sources_sha256(VJP_SOURCES))
    else:
        print("eval_source_sha256 = %s" % eval_sources_sha256())
    for k in sorted(fetch):
        if match and match not in k:
            continue
        fv = fetch[k]
        wv = write.get(k, [])
        keep = [i for i, v in enumerate(fv) if v >= min_kib]
        if not keep:
            continue
        fb = sum(fv[i] for i in keep) / len(keep) * 1024.0 * f_scale
        if len(wv) == len(fv):
            wb = sum(wv[i] for i in keep) / len(keep) * 1024.0 * w_scale
        else:  # runs not aligned: every write dispatch
            wb = sum(wv) / max(1, len(wv)) * 1024.0 * w_scale
        tag = _tag(k)
        print("# %s: %d dispatches, %d below %.0f KiB fetched (nothing to do) excluded"
              % (k, len(fv), len(fv) - len(keep), min_kib))
        print("dispatches_%s = %d" % (tag, len(keep)))
        print("fetch_bytes_per_launch_%s = %.1f" % (tag, fb))
        print("write_bytes_per_launch_%s = %.1f" % (tag, wb))
        print("hbm_bytes_per_launch_%s = %.1f" % (tag, fb + wb))


def _slot_class(n_act, split):
    if split < 0:
        return "prediction slot"
    if n_act == 0:
        return "empty (after the last block)"
    for hi, name in ((1, "1"), (2, "2"), (3, "3"), (15, "4-15"), (63, "16-63"), (511, "64-511"),
                     (4095, "512-4095")):
        if n_act <= hi:
            return name
    return "4096+"


def phases(trace_csv, slot_log):
    disp = []
    for r in csv.DictReader(open(trace_csv)):
        disp.append((int(r["Dispatch_Id"]), _short(r["Kernel_Name"]), int(r["Start_Timestamp"]),
                     int(r["End_Timestamp"])))
    disp.sort()
    evals = [d for d in disp if d[1].startswith("h6::k_bl_eval")]
    fins = [d for d in disp if d[1] == "h6::k_bl_finish"]
    slots = [tuple(int(t) for t in line.split()) for line in open(slot_log)
             if line.strip() and not line.startswith("#")]
    if not (len(evals) == len(fins) == len(slots)):
        raise SystemExit("dispatches (%d evaluations, %d finishing) and slots (%d) differ"
                         % (len(evals), len(fins), len(slots)))
    order = ["1", "2", "3", "4-15", "16-63", "64-511", "512-4095", "4096+", "prediction slot",
             "empty (after the last block)"]
    acc = {c: [0, 0.0, 0.0, 0.0, 0.0, 0.0] for c in order}
    t_first, t_last = evals[0][2], fins[-1][3]
    for k, ((na, sp), e, f) in enumerate(zip(slots, evals, fins)):
        nxt = evals[k + 1][2] if k + 1 < len(evals) else f[3]
        a = acc[_slot_class(na, sp)]
        a[0] += 1
        a[1] += (e[3] - e[2]) * 1e-3
        a[2] += (f[2] - e[3]) * 1e-3
        a[3] += (f[3] - f[2]) * 1e-3
        a[4] += (nxt - f[3]) * 1e-3
        a[5] += (nxt - e[2]) * 1e-3
    total = (t_last - t_first) * 1e-3
    print("# %d slots, %.3f ms from the first evaluation's start to the last finishing "
          "kernel's end" % (len(slots), total * 1e-3))
    print("%-28s %7s %9s %9s %9s %9s %9s %7s" % ("active count", "slots", "eval_us", "gap1_us",
                                                  "finish_us", "gap2_us", "slot_us", "share"))
    for c in order:
        a = acc[c]
        if not a[0]:
            continue
        m = [v / a[0] for v in a[1:]]
        print("%-28s %7d %9.2f %9.2f %9.2f %9.2f %9.2f %6.1f%%" % (c, a[0], *m, 100 * a[5] / total))
    print("# eval: k_bl_eval duration; gap1: its end to the finishing kernel's start; finish:")
    print("# k_bl_finish duration; gap2: its end to the next slot's evaluation start; slot: from")
    print("# this slot's evaluation start to the next one's (all means per slot, microseconds)")


def counters(path, match, interactions):
    """Per-dispatch counters of the largest dispatches of a kernel (by
    SQ_INSTS_VALU_FMA_F64), as instructions per interaction for a dispatch
    of `interactions` pair interactions, and the clock from GRBM_GUI_ACTIVE."""
    per = defaultdict(dict)
    meta = {}
    for r in csv.DictReader(open(path)):
        if match not in r["Kernel_Name"]:
            continue
        d = r["Dispatch_Id"]
        per[d][r["Counter_Name"]] = per[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        meta[d] = (int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
    # rank dispatches by their FMA count (FP64, or FP32 for the mixed kernels)
    tot = defaultdict(float)
    for v in per.values():
        for name in ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_FMA_F32"):
            tot[name] += v.get(name, 0.0)
    key = max(tot, key=tot.get) if tot else None
    top = sorted(per, key=lambda d: -per[d].get(key, 0.0) if key else 0.0)[:3]
    for d in top:
        c = per[d]
        dur = (meta[d][1] - meta[d][0]) * 1e-9
        print("# dispatch %s: %.3f ms" % (d, dur * 1e3))
        for name in sorted(c):
            v = c[name]
            line = "%-28s %16.0f" % (name, v)
            if name.startswith("SQ_INSTS_VALU") or name.startswith("SQ_INSTS_LDS"):
                line += "   %8.3f wave-instr x64 / interaction" % (v * 64.0 / interactions)
            if name == "GRBM_GUI_ACTIVE" and dur > 0:
                line += "   %.3f GHz" % (v / dur * 1e-9)
            print(line)
        for prec in ("F64", "F32"):
            names = ["SQ_INSTS_VALU_%s_%s" % (op, prec) for op in ("FMA", "ADD", "MUL", "TRANS")]
            if not all(k in c for k in names):
                continue
            ex = 64.0 * (2 * c[names[0]] + c[names[1]] + c[names[2]] + c[names[3]])
            print("executed %s flops per interaction (FMA 2, ADD/MUL/TRANS 1) = %.2f"
                  % (prec.replace("F", "FP"), ex / interactions))
            if dur > 0:
                print("executed %s rate = %.2f TFLOP/s" % (prec.replace("F", "FP"), ex / dur * 1e-12))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--match")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--match")
    b.add_argument("--sources", choices=("eval", "vjp"), default="eval",
                   help="which kernels' sources the record's hash covers")
    b.add_argument("--min-kib", type=float, default=64.0)
    ph = sub.add_parser("phases")
    ph.add_argument("trace_csv")
    ph.add_argument("slot_log")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--match", required=True)
    c.add_argument("--interactions", type=float, required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        stats(args.csv, args.match)
    elif args.cmd == "counters":
        counters(args.csv, args.match, args.interactions)
    elif args.cmd == "phases":
        phases(args.trace_csv, args.slot_log)
    else:
        traffic(args.fetch_csv, args.write_csv, args.copy_bytes, args.match, args.sources,
                args.min_kib)


if __name__ == "__main__":
    main()
