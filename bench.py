"""Benchmark of the Hermite-6 block-step hot path on one MI355X.

Workload: Plummer sphere, N = 65536 equal masses, Henon units, Plummer
softening eps = 1e-4, FP64, block time steps (power-of-two steps from the
6th-order generalized Aarseth criterion, eta = 0.4, largest step 1/16).

One "step" is one pass of the whole hot path over one synchronisation
interval: every block step (scheduler, predictor of all particles, a/j/s
evaluation of the active ones, slice reduction, corrector with
interpolation and step assignment) until all particles reach the next
multiple of 1/16, then the energy / angular-momentum diagnostic at that
sync time. The default 16 steps integrate one time unit. Warm-up steps run
first from the start-up state, which is then restored, so the timed steps
always integrate [0, K/16].

value = sum over blocks of N_active * N (the self pair counted, as the
kernel evaluates it branch-free) divided by the wall time of the K steps.
roofline: the dominant evaluation-kernel instantiation, 78 flops per
interaction divided by its HIP-event-measured duration, against the FP64
vector peak.
cpu_baseline: the FP64 CPU oracle, timed on a bounded sample of the same
workload (its a/j/s evaluation of sampled targets against all sources).

--workload adjoint measures the differentiable shared-step path instead
(loss and full gradient through 64 shared steps, N = 16384); its JSON line
names its own metric.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "a/j/s pair interactions/s, % of vector FP peak, at stated rel. error vs FP64"
FLOPS_PER_INTERACTION = 78  # FMA 2, rsqrt 1, potential excluded
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBPS = 8000.0
MIXED_N = 262144
MIXED_ACCURACY_TARGETS = 256
TRAFFIC_INTERVALS = 16  # sync intervals the committed HBM-traffic record covers (the default --steps)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blockloop_n65536_hbm_traffic.txt")
CSRC = os.path.join(ROOT, "paper_1901_08532_amd", "csrc")
# the evaluation kernels' sources: the traffic record is void once any changes
EVAL_SOURCES = ("eval_body.h", "eval_mixed_body.h", "device_math.h", "steps_body.h",
                "blockloop.hip", "eval.hip", "eval_mixed.hip")


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _kernel_name(rec, mixed):
    """Kernel symbol (as rocprofv3 shows it) of an evaluation timing record."""
    if rec["kind"] == 2:
        return "k_bl_eval<%s, false>" % ("true" if mixed else "false")
    if rec["kind"] == 1:
        return "k_eval_small%s<%d, false>" % ("_mixed" if mixed else "", rec["ipl"])
    if mixed:
        return "k_eval_mixed<%d, %d, false>" % (rec["block"], rec["ipl"])
    return "k_eval_f64<2, %d, %d, false>" % (rec["block"], rec["ipl"])


def _traffic_tag(rec, mixed):
    if rec["kind"] == 2:
        return "bl_eval_%s" % ("mixed" if mixed else "fp64")
    return "b%d_i%d" % (rec["block"], rec["ipl"])


def _traffic_per_launch(tag):
    """HBM bytes per launch of the given kernel from the committed rocprofv3
    counter summary, or None when the evaluation sources changed since the
    counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = _traffic_fields()
    if fields.get("eval_source_sha256") != _eval_sources_sha256():
        return None
    key = "hbm_bytes_per_launch_" + tag
    return float(fields[key]) if key in fields else None


def _traffic_fields():
    """key = value lines of the committed traffic record."""
    fields = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            fields[k.strip()] = v.strip()
    return fields


def _executed_flops_per_interaction():
    """Executed FP64 flops per interaction of the block-loop evaluation
    (FMA 2, ADD/MUL/TRANS 1) from the committed counter summary, or None
    once the evaluation sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "bl_eval_fp64_valu_counters.md")
    if not os.path.exists(path) or not os.path.exists(TRAFFIC_FILE):
        return None
    # the counter summary and the traffic record are taken for the same sources
    if _traffic_fields().get("eval_source_sha256") != _eval_sources_sha256():
        return None
    for line in open(path):
        if line.startswith("executed FP64 flops per interaction"):
            return float(line.rsplit("=", 1)[1])
    return None


def _eval_sources_sha256():
    h = hashlib.sha256()
    for f in EVAL_SOURCES:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None,
                    help="particles (default 65536; 16384 for the adjoint workload)")
    ap.add_argument("--seed", type=int, default=None,
                    help="initial-condition seed (default 2; 4 for the adjoint workload)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--workload", choices=("plummer", "plummer-imf", "two-clusters", "adjoint",
                                           "adjoint-block"),
                    default="plummer",
                    help="equal-mass Plummer sphere; Plummer with dN/dm ~ m^-2.35 masses "
                         "(mass seed 10*seed+seed); two Plummer spheres of n/2 on a head-on "
                         "approach (seeds seed, 10*seed+seed); adjoint: gradient of a loss on "
                         "the final positions of 64 shared steps (one step = forward + backward); "
                         "adjoint-block: the same loss through 1/16 time unit of block steps")
    ap.add_argument("--accuracy-targets", type=int, default=256,
                    help="sampled targets of the last block checked against the FP64 oracle")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--host-loop", action="store_true",
                    help="one host round trip per block instead of the device-resident loop")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-vs-FP64 leg (power-law Plummer N = 262144, one sync interval each)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--timed-only", action="store_true",
                    help="only the timed window (for a profiler's per-kernel averages): no "
                         "accuracy, single-pass, CPU-baseline, breakdown or mixed legs")
    ap.add_argument("--slot-log", default=None, metavar="PATH",
                    help="instead of the benchmark: one sync interval of the device loop with no "
                         "event timing (for a kernel tracer), its slot log (n_act, split per "
                         "slot) written to PATH")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1901_08532_amd import h6, ics

    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        _log("copy calibration: %d bytes" % nbytes)
        del src, dst
    if args.workload == "adjoint":
        return run_adjoint(args)
    if args.workload == "adjoint-block":
        return run_adjoint_block(args)
    args.n = 65536 if args.n is None else args.n
    args.seed = 2 if args.seed is None else args.seed
    n, eps, eta, lev_min, lev_max = args.n, 1e-4, 0.4, 4, 30
    prec = h6.H6_FP64 if args.precision == "fp64" else h6.H6_MIXED
    sync_ticks = 1 << (h6.TICK_BITS - lev_min)

    seed2 = 10 * args.seed + args.seed
    _log("inputs: %s N=%d seed=%d" % (args.workload, n, args.seed))
    if args.workload == "plummer":
        x, v, m = ics.plummer(n, args.seed)
    elif args.workload == "plummer-imf":
        x, v, _ = ics.plummer(n, args.seed)
        m = ics.salpeter_masses(n, seed2)
    else:
        x, v, m = ics.two_clusters(n // 2, args.seed, seed2)
    sysg = h6.System(x, v, m, eps)
    sysg.startup(eta_s=0.1, lev_min=lev_min, lev_max=lev_max)
    rc = sysg.ctx.h6_check_status()
    if rc != h6.H6_OK:
        raise h6.H6Error(rc, "start-up")
    if args.slot_log:
        return _slot_log_interval(args, sysg, sync_ticks, eta, lev_min, lev_max, prec)
    S0, T0 = sysg.S.clone(), sysg.T.clone()
    e_start = sysg.energy()
    E0 = e_start[0] + e_start[1]

    def one_step(k):
        rc, stats = sysg.run_blocks((k + 1) * sync_ticks, eta, lev_min, lev_max, prec, check=False,
                                    host_loop=args.host_loop)
        if rc != h6.H6_OK:
            raise h6.H6Error(rc, "h6_run_blocks", h6.lib().h6_last_error(sysg.ctx.handle).decode())
        e = sysg.energy()
        return stats, e

    for w in range(args.warmup):
        st, _ = one_step(w)
        _log("warmup step %d: %d blocks" % (w, st.blocks))
    sysg.S.copy_(S0)
    sysg.T.copy_(T0)
    # both kernels of every slot timed: each dispatch carries one event, at
    # its end, so timing the finishing kernels too costs nothing more
    sysg.ctx.h6_profile_enable(2)
    torch.cuda.synchronize()

    blocks = psteps = 0
    inter = 0.0
    drift = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        st, e = one_step(k)
        blocks += st.blocks
        psteps += st.particle_steps
        inter += st.interactions
        drift = max(drift, abs(e[0] + e[1] - E0) / abs(E0))
        _log("step %d: %d blocks" % (k, st.blocks))  # after the step's own synchronising read
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sysg.ctx.h6_profile_read()
    sysg.ctx.h6_profile_enable(False)
    wall = t1 - t0
    value = inter / wall if wall > 0 else 0.0
    _log("timed %d steps: %d blocks, %.3e interactions, %.3f s" % (args.steps, blocks, inter, wall))

    # per instantiation (summed over active-set bins) and per active-set bin;
    # bin -1 holds the evaluation launches of empty blocks (device loop)
    evals = [p for p in prof if p["order"] == 2 and p["kind"] != 4]  # not the finishing kernel
    inst = {}
    bins = {}
    empty_launches = 0
    empty_ms = 0.0
    for p in evals:
        b = bins.setdefault(p["nact_log2"], {"launches": 0, "interactions": 0.0, "kernel_ms": 0.0})
        for f in ("launches", "interactions", "kernel_ms"):
            b[f] += p[f]
        if p["nact_log2"] < 0:
            # launches enqueued past the last due block (bin -1) and those of
            # prediction slots (bin -2): nothing evaluated
            empty_launches += p["launches"]
            empty_ms += p["kernel_ms"]
            continue
        key = (p["kind"], p["block"], p["ipl"])
        d = inst.setdefault(key, {"kind": p["kind"], "block": p["block"], "ipl": p["ipl"],
                                  "launches": 0, "interactions": 0.0, "kernel_ms": 0.0,
                                  "bytes": 0.0})
        for f in ("launches", "interactions", "kernel_ms", "bytes"):
            d[f] += p[f]
    dom = max(inst.values(), key=lambda p: p["kernel_ms"])
    eval_ms = sum(p["kernel_ms"] for p in evals)
    by_active = []
    for b in sorted(bins):
        if b < 0:
            continue
        d = bins[b]
        rate = d["interactions"] / (d["kernel_ms"] * 1e-3)
        by_active.append({"n_act_from": 1 << b, "n_act_below": 1 << (b + 1), "launches": d["launches"],
                          "interactions": d["interactions"], "eval_ms": d["kernel_ms"],
                          "eval_interactions_per_s": rate,
                          "eval_pct_fp64_peak": 100.0 * rate * FLOPS_PER_INTERACTION / (FP64_PEAK_TFLOPS * 1e12)})
    achieved = FLOPS_PER_INTERACTION * dom["interactions"] / (dom["kernel_ms"] * 1e-3) / 1e12
    traffic = _traffic_per_launch(_traffic_tag(dom, prec == h6.H6_MIXED))
    roofline = {
        "bound": "alu",
        "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": traffic,
        "kernel": _kernel_name(dom, prec == h6.H6_MIXED),
        "launches": dom["launches"],
        "empty_launches_excluded": empty_launches,
        "avg_launch_us": 1e3 * dom["kernel_ms"] / max(1, dom["launches"]),
        # every dispatch of the kernel in the timed window, empty ones too (what
        # a profiler's per-kernel average over the same window counts)
        "dispatches_all": dom["launches"] + empty_launches,
        "avg_dispatch_us_all": 1e3 * (dom["kernel_ms"] + empty_ms)
                               / max(1, dom["launches"] + empty_launches),
        "flops_per_launch": FLOPS_PER_INTERACTION * dom["interactions"] / max(1, dom["launches"]),
        "algorithmic_bytes_per_launch": dom["bytes"] / max(1, dom["launches"]),
        "traffic_window": "per dispatch over %d timed sync intervals" % TRAFFIC_INTERVALS,
    }
    xfl = _executed_flops_per_interaction() if prec == h6.H6_FP64 else None
    if xfl is not None:
        roofline["executed_flops_per_interaction"] = xfl
        roofline["executed_tflops"] = achieved * xfl / FLOPS_PER_INTERACTION

    # the two kernels of every block over the timed window
    step_roofs = None if args.host_loop else _loop_breakdown(prof, blocks, prec)
    acc = timings = cpu = mixed = None
    if not args.timed_only:
        # accuracy of the timed kernel itself: one more sync interval of the
        # same loop (untimed), whose last block (every particle active)
        # leaves its a, j, s in the state; the oracle evaluates sampled
        # targets from that block's predicted arrays
        rng = np.random.Generator(np.random.PCG64(7))
        acc = _loop_accuracy(sysg, (args.steps + 1) * sync_ticks, eta, lev_min, lev_max, prec, m, eps,
                             args.accuracy_targets, rng)
        _log("accuracy of the loop's last block: a %.2e j %.2e s %.2e" % (
            acc["max_rel_err_a"], acc["max_rel_err_j"], acc["max_rel_err_s"]))

        # timings of single passes on the final, synchronised state, HIP events
        # on the library's stream (torch's current one), mean of 10: (i) the
        # a/j/s evaluation of all n particles with its slice reduction, (ii) a
        # whole step of all n particles (predict, evaluate, reduce, correct)
        reps = 10
        Pt = sysg.S[0:9].contiguous()
        Ft = torch.empty((9, n), dtype=torch.float64, device="cuda")
        St = sysg.S.clone()
        Pw = torch.empty((9, n), dtype=torch.float64, device="cuda")

        def _events(fn):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return 1e3 * e0.elapsed_time(e1) / reps

        t_eval = _events(lambda: sysg.ctx.h6_evaluate(Pt, sysg.m, None, n, prec, Ft))
        t_step = _events(lambda: sysg.ctx.h6_shared_steps(St, sysg.m, Pw, Ft, 2.0 ** -12, 1, prec))
        timings = {
            "eval_reduce_all_n_us": t_eval,
            "eval_reduce_all_n_pct_fp64_peak": 100.0 * FLOPS_PER_INTERACTION * float(n) * n
                                                 / (t_eval * 1e-6) / (FP64_PEAK_TFLOPS * 1e12),
            "step_all_n_us": t_step,
            "block_step_avg_us": 1e6 * wall / max(1, blocks),
            "run_s": wall,
            "repeats": reps,
        }
        _log("eval+reduce of all %d: %.1f us; full step %.1f us" % (n, t_eval, t_step))

        import oracle

        P = sysg.S[0:9].contiguous()
        xs, vs, as_ = (P[3 * k:3 * k + 3].T.cpu().numpy().copy() for k in range(3))

        if not args.no_cpu_baseline:
            # the oracle's a/j/s evaluation of sampled targets against all n sources
            probe = np.arange(0, n, max(1, n // 256))[:256]
            tp = time.perf_counter()
            oracle.forces(xs, vs, m, eps * eps, a=as_, idx=probe, order=2)
            tp = time.perf_counter() - tp
            n_i = int(min(n, max(256, len(probe) * args.cpu_seconds / max(tp, 1e-6))))
            sample = np.sort(rng.choice(n, n_i, replace=False))
            tc = time.perf_counter()
            oracle.forces(xs, vs, m, eps * eps, a=as_, idx=sample, order=2)
            tc = time.perf_counter() - tc
            cpu = {
                "value": n_i * n / tc,
                "unit": "interactions/s",
                "cores": oracle.num_threads(),
                "kind": "oracle",
                "sample": "FP64 oracle a/j/s evaluation of %d sampled targets against all %d sources "
                          "of the final synchronised state (%.1f s)" % (n_i, n, tc),
            }
            _log("cpu baseline: %.3e interactions/s on %d threads" % (cpu["value"], cpu["cores"]))

        if not args.no_mixed:
            mixed = _mixed_vs_fp64(args, h6, ics, oracle)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == h6.H6_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": "%s_n%d_eps1e-4_blocksteps_eta0.4_dtmax1/16_%gtu_%s" % (
                args.workload.replace("-", "_"), n, args.steps / 16, args.precision),
            "n": n, "eps": eps, "eta": eta, "dt_max": 2.0 ** -lev_min, "lev_max": lev_max,
            "time_units": args.steps / 16.0, "precision": args.precision, "seed": args.seed,
            "flops_per_interaction": FLOPS_PER_INTERACTION,
        },
        "pct_fp64_vector_peak": 100.0 * value * FLOPS_PER_INTERACTION / (FP64_PEAK_TFLOPS * 1e12),
        "pct_fp32_vector_peak": 100.0 * value * FLOPS_PER_INTERACTION / (FP32_PEAK_TFLOPS * 1e12),
        "blocks": blocks,
        "block_us_avg": 1e6 * wall / max(1, blocks),
        "particle_steps": psteps,
        "interactions": inter,
        "eval_kernel_share_of_wall": 1e-3 * eval_ms / wall if wall > 0 else None,
        "eval_by_active_set": by_active,
        "timings": timings,
        "energy_rel_err_max": drift,
        "accuracy": acc,
        "roofline": roofline,
        "step_rooflines": step_roofs,
        "mixed_vs_fp64": mixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def _slot_log_interval(args, sysg, sync_ticks, eta, lev_min, lev_max, prec):
    """One sync interval of the device loop under the slot log alone (no
    events on the dispatches): writes one line "n_act split" per slot, in
    launch order (each slot is one k_bl_eval and one k_bl_finish dispatch),
    and prints a JSON line with the interval's blocks and wall time. The
    first k_bl_eval dispatch of the process is this interval's first slot."""
    import torch

    from paper_1901_08532_amd import h6

    sysg.ctx.h6_profile_enable(3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = sysg.run_blocks(sync_ticks, eta, lev_min, lev_max, prec, check=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if rc != h6.H6_OK:
        raise h6.H6Error(rc, "h6_run_blocks (slot log)")
    slots = sysg.ctx.h6_profile_slots()
    sysg.ctx.h6_profile_enable(False)
    with open(args.slot_log, "w") as f:
        f.write("# n_act split, one line per device-loop slot in launch order (split -1: "
                "prediction slot; n_act 0: after the last due block)\n")
        for na, sp in slots:
            f.write("%d %d\n" % (na, sp))
    print(json.dumps({"slot_log": args.slot_log, "slots": int(len(slots)), "blocks": st.blocks,
                      "particle_steps": st.particle_steps, "wall_s": wall,
                      "workload": args.workload, "n": sysg.n}), flush=True)


def _loop_accuracy(sysg, t_end, eta, lev_min, lev_max, prec, m, eps, n_targets, rng):
    """Largest per-particle relative error of the a, j, s that the device
    loop's block at t_end (a sync time: every particle active) leaves in
    the state, against the FP64 oracle evaluated from that block's predicted
    arrays, on n_targets sampled particles. The loop runs to one tick before
    t_end, the library's predictor takes every particle to t_end (the code
    of the loop's own prediction slot), then the loop runs the block."""
    import numpy as np
    import torch

    import oracle
    from paper_1901_08532_amd import h6

    rc, _ = sysg.run_blocks(t_end - 1, eta, lev_min, lev_max, prec, check=False)
    if rc != h6.H6_OK:
        raise h6.H6Error(rc, "h6_run_blocks (accuracy interval)")
    Pt = torch.zeros_like(sysg.P)
    sysg.ctx.h6_predict(sysg.S, sysg.m, sysg.T, t_end, Pt)
    rc, st = sysg.run_blocks(t_end, eta, lev_min, lev_max, prec, check=False)
    if rc != h6.H6_OK or st.particle_steps != sysg.n:
        raise h6.H6Error(rc, "h6_run_blocks (accuracy block)")
    n = sysg.n
    idx = np.sort(rng.choice(n, min(n, n_targets), replace=False))
    P = Pt.cpu().numpy()
    xp, vp, ap = P[0:3].T.copy(), P[3:6].T.copy(), P[6:9].T.copy()
    want = oracle.forces(xp, vp, m, eps * eps, a=ap, idx=idx, order=2)[:3]
    acc = {}
    for k, name in enumerate("ajs"):
        got = sysg.field(name)[idx]
        err = np.linalg.norm(got - want[k], axis=1) / np.linalg.norm(want[k], axis=1)
        acc["max_rel_err_" + name] = float(err.max())
    acc["sample_targets"] = len(idx)
    acc["source"] = ("a, j, s that the loop's evaluation kernel left at a sync block (all "
                     "particles active), one untimed interval after the timed ones")
    return acc


def _loop_breakdown(recs, blocks, prec):
    """The evaluation and finishing kernels of every block over the timed
    window (profile level 2 records; the finishing kernels of the
    prediction slots apart, their evaluations are empty): launches, time,
    algorithmic bytes (each datum moved once, from the block's active count
    and slice count) and the resulting fraction of the 8 TB/s HBM bound
    per kernel. A dispatch is timed from the end of the one before it, so
    its launch latency (a few microseconds) is in its time, which dominates
    the smallest blocks' kernels."""
    from paper_1901_08532_amd import h6

    names = {2: "k_bl_eval", 4: "k_bl_finish", -4: "k_bl_finish (prediction slots)"}
    agg = {k: {"launches": 0, "kernel_ms": 0.0, "bytes": 0.0} for k in names}
    for r in recs:
        if r["kind"] not in (2, 4) or r["nact_log2"] == -1:
            continue
        key = r["kind"] if r["nact_log2"] >= 0 else -r["kind"]
        if key not in agg:
            continue  # empty evaluations of prediction slots
        a = agg[key]
        a["launches"] += r["launches"]
        a["kernel_ms"] += r["kernel_ms"]
        a["bytes"] += r["bytes"]
    total_ms = sum(a["kernel_ms"] for a in agg.values())
    out = {"blocks": blocks, "window": "the timed window, an end event on every dispatch"}
    for k, name in names.items():
        a = agg[k]
        secs = a["kernel_ms"] * 1e-3
        gbs = a["bytes"] / secs / 1e9 if secs > 0 else 0.0
        out[name] = {
            "bound": "hbm" if k != 2 else "alu",
            "launches": a["launches"],
            "avg_us": 1e3 * a["kernel_ms"] / max(1, a["launches"]),
            "share_of_loop_gpu_time": a["kernel_ms"] / total_ms if total_ms > 0 else None,
            "algorithmic_bytes_per_launch": a["bytes"] / max(1, a["launches"]),
            "achieved_GBps": gbs,
            "peak_GBps": HBM_PEAK_GBPS,
            "frac_of_hbm": gbs / HBM_PEAK_GBPS,
        }
    # measured HBM traffic of the finishing kernel (rocprofv3 counters over
    # the default timed window, launches with nothing to do excluded: blocks
    # and prediction slots alike) beside the algorithmic bytes of the same set
    fin = [agg[4], agg[-4]]
    n_fin = sum(a["launches"] for a in fin)
    out["k_bl_finish"]["algorithmic_bytes_per_nonempty_launch"] = (
        sum(a["bytes"] for a in fin) / max(1, n_fin))
    out["k_bl_finish"]["traffic_per_nonempty_launch"] = _traffic_per_launch(
        "bl_finish" + ("_mixed" if prec == h6.H6_MIXED else ""))
    out["k_bl_finish"]["traffic_window"] = "per dispatch over %d timed sync intervals" % TRAFFIC_INTERVALS
    return out


def _mixed_vs_fp64(args, h6, ics, oracle):
    """The power-law-mass workload (Plummer N = 262144, seeds 3 and 33,
    eps 1e-4): one sync interval from the same start-up state in FP64 and
    in the mixed form; rate of each, the mixed form's speedup, each run's
    a, j, s error (the evaluation kernel's own output at the interval's
    last block, against the FP64 oracle on sampled targets) and energy
    drift over the interval."""
    import numpy as np
    import torch

    n, eps, eta, lev_min, lev_max = MIXED_N, 1e-4, 0.4, 4, 30
    sync = 1 << (h6.TICK_BITS - lev_min)
    x, v, _ = ics.plummer(n, 3)
    m = ics.salpeter_masses(n, 33)
    base = h6.System(x, v, m, eps)
    base.startup(eta_s=0.1, lev_min=lev_min, lev_max=lev_max)
    S0, T0 = base.S.clone(), base.T.clone()
    e0 = sum(base.energy()[:2])
    res = {"workload": "plummer_imf_n%d_eps1e-4_seed3_masses33_blocksteps_1/16tu" % n}
    for tag, prec in (("fp64", h6.H6_FP64), ("mixed", h6.H6_MIXED)):
        base.S.copy_(S0)
        base.T.copy_(T0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = base.run_blocks(sync, eta, lev_min, lev_max, prec, check=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if rc != h6.H6_OK:
            raise h6.H6Error(rc, "h6_run_blocks (%s)" % tag)
        e1 = sum(base.energy()[:2])
        rng = np.random.Generator(np.random.PCG64(333))
        acc = _loop_accuracy(base, 2 * sync, eta, lev_min, lev_max, prec, m, eps,
                             MIXED_ACCURACY_TARGETS, rng)
        rate = st.interactions / wall
        res[tag] = {
            "interactions_per_s": rate,
            "pct_fp64_vector_peak": 100.0 * rate * FLOPS_PER_INTERACTION / (FP64_PEAK_TFLOPS * 1e12),
            "pct_fp32_vector_peak": 100.0 * rate * FLOPS_PER_INTERACTION / (FP32_PEAK_TFLOPS * 1e12),
            "blocks": st.blocks,
            "wall_s": wall,
            "max_rel_err_a": acc["max_rel_err_a"],
            "max_rel_err_j": acc["max_rel_err_j"],
            "max_rel_err_s": acc["max_rel_err_s"],
            "energy_rel_err": abs(e1 - e0) / abs(e0),
        }
        _log("mixed_vs_fp64 %s: %.3e interactions/s, %d blocks, a/j/s err %.1e %.1e %.1e" % (
            tag, rate, st.blocks, acc["max_rel_err_a"], acc["max_rel_err_j"], acc["max_rel_err_s"]))
    res["speedup"] = res["mixed"]["interactions_per_s"] / res["fp64"]["interactions_per_s"]
    res["energy_drift_ratio"] = res["mixed"]["energy_rel_err"] / max(res["fp64"]["energy_rel_err"], 1e-300)
    res["sample_targets"] = MIXED_ACCURACY_TARGETS
    return res


VJP_COUNTER_FILE = os.path.join(ROOT, "profiles", "eval_vjp_valu_counters.md")
VJP_FLOPS_PER_PAIR = 235  # algorithmic flops of one pair's order-2 VJP (FMA 2, rsqrt 1)
ADJ_METRIC = "pair-sum passes x N^2 per second, forward sums and their vector-Jacobian products"


VJP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "eval_vjp_hbm_traffic.txt")
VJP_SOURCES = ("adjoint.hip", "device_math.h")


def _vjp_record():
    """key = value lines of the VJP kernel's traffic record if it was taken
    for the current VJP sources (the VALU counter summary was taken with
    them too), else None."""
    if not os.path.exists(VJP_TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(VJP_TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in VJP_SOURCES:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return fields if fields.get("vjp_source_sha256") == h.hexdigest() else None


def _vjp_flops_per_pair():
    """Executed FP64 flops per pair of the evaluation VJP kernel (FMA 2,
    ADD/MUL/TRANS 1) from the committed counter summary, or None once the
    VJP sources changed since it was taken."""
    if not os.path.exists(VJP_COUNTER_FILE) or _vjp_record() is None:
        return None
    for line in open(VJP_COUNTER_FILE):
        if line.startswith("executed FP64 flops per interaction"):
            return float(line.rsplit("=", 1)[1])
    return None


def _vjp_traffic_per_launch():
    rec = _vjp_record()
    key = "hbm_bytes_per_launch_eval_vjp"
    return float(rec[key]) if rec and key in rec else None


def run_adjoint_block(args):
    """Block-step adjoint workload: Plummer N = 16384, eps = 1e-3, start-up
    then every block step to 1/16 time unit (eta 0.4, levels 4..30), loss
    and targets as the shared-step adjoint workload. One bench step is one
    loss evaluation plus its full gradient with respect to the initial
    positions, velocities and masses, the step lengths held fixed (forward
    blocks, then the backward pass: segment replay from the checkpoints and
    the transposes of each block's corrector, active-set evaluation and
    predictor). value counts, per bench step, the forward blocks' pair
    interactions (sum of N_act N) and the VJP's (twice that: the active
    targets against all sources and every source against the active
    targets); the replay inside the backward pass is not counted. The
    block sequence's active counts come from the same start-up run through
    the host loop (the same kernels, the same blocks)."""
    import numpy as np
    import torch

    from paper_1901_08532_amd import h6, ics
    from paper_1901_08532_amd.adjoint import hermite_block_run

    n = 16384 if args.n is None else args.n
    seed = 4 if args.seed is None else args.seed
    eps, eta, lev_min, lev_max = 1e-3, 0.4, 4, 30
    t_end = 1 << (h6.TICK_BITS - lev_min)
    torch.cuda.set_device(0)
    _log("inputs: adjoint-block plummer N=%d seed=%d" % (n, seed))
    x, v, m = ics.plummer(n, seed)
    rng = np.random.Generator(np.random.PCG64(10 * seed + seed))
    xt = x + 0.01 * rng.normal(0, 1, (n, 3))
    probe = h6.System(x, v, m, eps)
    probe.startup(eta_s=0.1, lev_min=lev_min, lev_max=lev_max)
    rc, st = probe.run_blocks(t_end, eta, lev_min, lev_max, host_loop=True, check=False)
    if rc not in (h6.H6_OK, h6.H6_EDTMIN):
        raise h6.H6Error(rc, "block sequence")
    del probe
    ctx = h6.Context(n, eps)
    X0, V0, M0, XT = (torch.from_numpy(a).cuda() for a in (x, v, m, xt))

    def forward():
        with torch.no_grad():
            return hermite_block_run(X0, V0, M0, ctx, t_end, eta, lev_min, lev_max)

    def one():
        x0, v0, m0 = (a.clone().requires_grad_(True) for a in (X0, V0, M0))
        xT, _ = hermite_block_run(x0, v0, m0, ctx, t_end, eta, lev_min, lev_max)
        loss = ((xT - XT) ** 2).sum()
        return loss.detach(), torch.autograd.grad(loss, (x0, v0, m0))

    for w in range(args.warmup):
        one()
        torch.cuda.synchronize()
        _log("warmup step %d done" % w)
    reps = max(1, args.steps // 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        forward()
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, grads = one()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    finite = all(bool(torch.isfinite(g).all()) for g in grads) and bool(torch.isfinite(loss))
    pairs = float(st.particle_steps) * n
    value = args.steps * 3.0 * pairs / wall
    out = {
        "metric": "block-step pair interactions per second, forward blocks and their VJPs",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plummer_n%d_eps1e-3_seed%d_blocksteps_eta0.4_1/16tu_adjoint" % (n, seed),
                   "n": n, "eps": eps, "eta": eta, "lev_min": lev_min, "lev_max": lev_max,
                   "time_units": 1.0 / 16},
        "blocks": st.blocks,
        "particle_steps": st.particle_steps,
        "forward_s": t_fwd,
        "gradient_s": wall / max(1, args.steps),
        "gradient_over_forward": (wall / max(1, args.steps)) / t_fwd if t_fwd > 0 else None,
        "gradient_finite": finite,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_adjoint(args):
    """Adjoint workload: Plummer N = 16384, eps = 1e-3, start-up then 64
    shared steps of 1/256 with a checkpoint every 8 steps; loss = sum of
    squared distances of the final positions from perturbed targets. One
    bench step is one loss evaluation plus its full gradient with respect to
    the initial positions, velocities and masses (forward integration, then
    the backward pass: segment replay from the checkpoints and the
    hand-written transposes). value counts, per bench step, the pair-sum
    passes of the method (2 start-up passes + one per shared step) and their
    VJPs (one each), times N^2; the replay of the forward steps inside the
    backward pass is not counted."""
    import numpy as np
    import torch

    from paper_1901_08532_amd import h6, ics
    from paper_1901_08532_amd.adjoint import hermite_shared_run

    n = 16384 if args.n is None else args.n
    seed = 4 if args.seed is None else args.seed
    eps, dt, nsteps, ckpt = 1e-3, 1.0 / 256, 64, 8
    torch.cuda.set_device(0)
    _log("inputs: adjoint plummer N=%d seed=%d" % (n, seed))
    x, v, m = ics.plummer(n, seed)
    rng = np.random.Generator(np.random.PCG64(10 * seed + seed))
    xt = x + 0.01 * rng.normal(0, 1, (n, 3))
    ctx = h6.Context(n, eps)
    X0, V0, M0, XT = (torch.from_numpy(a).cuda() for a in (x, v, m, xt))

    def one():
        x0, v0, m0 = (a.clone().requires_grad_(True) for a in (X0, V0, M0))
        xT = hermite_shared_run(x0, v0, m0, ctx, dt, nsteps, ckpt)
        loss = ((xT - XT) ** 2).sum()
        g = torch.autograd.grad(loss, (x0, v0, m0))
        return loss.detach(), g

    for w in range(args.warmup):
        one()
        torch.cuda.synchronize()
        _log("warmup step %d done" % w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        loss, grads = one()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    passes = 2 * nsteps + 4
    value = args.steps * passes * float(n) * n / wall
    _log("timed %d loss+gradient evaluations: %.3f s" % (args.steps, wall))
    finite = all(bool(torch.isfinite(g).all()) for g in grads) and bool(torch.isfinite(loss))

    # the evaluation and its VJP alone, on the predicted state of the first
    # step, timed with events on the library's stream (torch's current one)
    S = torch.zeros((18, n), dtype=torch.float64, device="cuda")
    S[0:3] = X0.T
    S[3:6] = V0.T
    ctx.h6_init_forces(S, M0)
    P = torch.empty((9, n), dtype=torch.float64, device="cuda")
    ctx.h6_predict_dt(S, M0, dt, P)
    F = torch.empty((9, n), dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    CF = torch.randn((9, n), dtype=torch.float64, device="cuda", generator=gen)
    CP = torch.empty((9, n), dtype=torch.float64, device="cuda")
    gm = torch.zeros(n, dtype=torch.float64, device="cuda")
    reps = 10

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    t_eval = timed(lambda: ctx.h6_evaluate(P, M0, None, n, h6.H6_FP64, F))
    t_vjp = timed(lambda: ctx.h6_evaluate_vjp(P, M0, CF, CP, gm))
    pairs = float(n) * n
    achieved = VJP_FLOPS_PER_PAIR * pairs / t_vjp / 1e12
    fpp = _vjp_flops_per_pair()
    roofline = {
        "bound": "alu",
        "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": _vjp_traffic_per_launch(),  # of the k_eval_vjp dispatch alone
        "kernel": "k_eval_vjp<2, 128, 0> + slice reduction (one h6_evaluate_vjp call)",
        "flops_per_pair": VJP_FLOPS_PER_PAIR,
        "flops_convention": "algorithmic: the operations of the factored reverse sweep of one "
                            "pair (forward recompute 44, six dot products and G, G_alpha per "
                            "cotangent 2 x 43, mass weights 9, scalars 12, gradient sums 36, "
                            "source-cotangent terms 42, target scalar sums 6); FMA 2, rsqrt 1",
        "executed_flops_per_pair": fpp,
        "executed_tflops": fpp * pairs / t_vjp / 1e12 if fpp is not None else None,
        "avg_call_us": 1e6 * t_vjp,
    }

    cpu = None
    if not args.no_cpu_baseline:
        # the autograd CPU reference on a small system of the same kind: its
        # all-pairs tensors and graph do not fit N = 16384
        import oracle.adjoint_ref as ar

        n_c = 256
        xc, vc, mc = ics.plummer(n_c, seed)
        xtc = xc + 0.01 * rng.normal(0, 1, (n_c, 3))
        tp = time.perf_counter()
        ar.loss_and_grad(xc, vc, mc, xtc, eps * eps, dt, 2)
        tp = time.perf_counter() - tp
        steps_c = int(max(2, min(nsteps, 2 * args.cpu_seconds / max(tp, 1e-6))))
        tc = time.perf_counter()
        ar.loss_and_grad(xc, vc, mc, xtc, eps * eps, dt, steps_c)
        tc = time.perf_counter() - tc
        cpu = {
            "value": (2 * steps_c + 4) * float(n_c) * n_c / tc,
            "unit": "pair-sum passes x N^2 per second",
            "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": "FP64 autograd reference, loss and gradient of Plummer N=%d through %d shared "
                      "steps of 1/256 (%.1f s)" % (n_c, steps_c, tc),
        }
        _log("cpu baseline: %.3e on %d threads" % (cpu["value"], cpu["cores"]))

    out = {
        "metric": ADJ_METRIC,
        "value": value,
        "unit": "pair-sum passes x N^2 per second",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "adjoint_plummer_n%d_eps1e-3_64_shared_steps_dt1/256_checkpoint8" % n,
            "n": n, "eps": eps, "dt": dt, "shared_steps": nsteps, "checkpoint": ckpt,
            "seed": seed, "passes_per_step": passes,
        },
        "gradient_finite": finite,
        "eval_call_us": 1e6 * t_eval,
        "vjp_call_us": 1e6 * t_vjp,
        "vjp_over_eval_time": t_vjp / t_eval,
        "eval_pct_fp64_peak": 100.0 * FLOPS_PER_INTERACTION * pairs / t_eval / (FP64_PEAK_TFLOPS * 1e12),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
