"""Conservation study of the evaluation arithmetic (Sec. 3 item 6, Eq. (1), Fig. 1).

The paper integrates a 4096-body system with each of its arithmetics and
follows the relative errors of energy and angular momentum,

    dE/E = |E_start - E(t)| / |E_start|,    dL/L = |L_start - L(t)| / |L_start|,

to show that round-off accumulates with single precision but not with
double or the extended (double-single) type. This module runs the same
study with libh6: one Plummer sphere, the a/j/s evaluation in the chosen
arithmetic (H6_FP64, H6_EX, H6_SP, or the mixed form), FP64 predictor,
corrector and diagnostics, and E and L sampled every 1/16 time unit. L is
the norm of the total angular momentum vector.

Two integration modes:
  shared (default): the paper's shared-step scheme, with one fixed step for
      every arithmetic (default 1/2048) and a softening (default 1/64) at
      which the FP64 truncation error stays near 1e-14 per time unit, far
      below what single-precision round-off adds, so that the curves differ
      by arithmetic only;
  block: the block time steps of the hot path (eta = 0.4, steps 2^-4 down
      to 2^-30, eps = 1e-4 by default). Single precision is refused here:
      its evaluation noise, differentiated by the corrector's interpolation
      (crackle and higher derivatives scale as noise / dt^3 and beyond),
      makes the sixth-order step criterion ask for ever smaller steps once a
      step is below about 2^-12, so the steps collapse to the smallest level
      and the run does not finish.

    python -m paper_1901_08532_amd.conservation [--mode shared|block]
        [--n 4096] [--time-units 8] [--precisions fp64,ex,sp,mixed]
        [--eps E] [--dt H] [--seed 2] [--out FILE]

Prints one JSON object per line: a header, then one record per precision
with the sampled times and errors. Needs the built HIP library and a GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import torch

from . import h6, ics

PRECISIONS = {"fp64": h6.H6_FP64, "mixed": h6.H6_MIXED, "ex": h6.H6_EX, "sp": h6.H6_SP}


def _e_l(sysg):
    k, w, lv = sysg.energy()
    return k + w, lv


def run(n=4096, time_units=8.0, precision="fp64", mode="shared", eps=None, dt=1.0 / 2048,
        seed=2, eta=0.4, lev_min=4, lev_max=30, eta_s=0.1, progress=None):
    """Integrates one Plummer sphere for time_units and returns a dict with
    the sample times and dE/E, dL/L at each (including t = 0)."""
    prec = PRECISIONS[precision]
    if mode not in ("shared", "block"):
        raise ValueError("mode must be 'shared' or 'block'")
    if mode == "block" and prec == h6.H6_SP:
        raise ValueError("single precision with block steps: the step criterion collapses the "
                         "steps to the smallest level (see the module documentation)")
    if eps is None:
        eps = 1.0 / 64 if mode == "shared" else 1e-4
    sample = 1.0 / (1 << lev_min)
    steps_per_sample = sample / dt
    if mode == "shared" and (steps_per_sample < 1 or steps_per_sample != int(steps_per_sample)):
        raise ValueError("dt must divide 1/16")
    x, v, m = ics.plummer(n, seed)
    sysg = h6.System(x, v, m, eps)
    sysg.startup(eta_s=eta_s if mode == "block" else None, lev_min=lev_min, lev_max=lev_max)
    rc = sysg.ctx.h6_check_status()
    if rc != h6.H6_OK:
        raise h6.H6Error(rc, "start-up")
    e0, l0 = _e_l(sysg)
    l0n = math.sqrt(sum(c * c for c in l0))
    sync = 1 << (h6.TICK_BITS - lev_min)
    n_sync = int(round(time_units * (1 << lev_min)))
    times, de, dl = [0.0], [0.0], [0.0]
    blocks = 0
    t0 = time.perf_counter()
    for k in range(n_sync):
        if mode == "shared":
            sysg.shared_steps(dt, int(steps_per_sample), prec)
            blocks += int(steps_per_sample)
        else:
            rc, st = sysg.run_blocks((k + 1) * sync, eta, lev_min, lev_max, prec, check=False)
            if rc != h6.H6_OK:
                raise h6.H6Error(rc, "h6_run_blocks")
            blocks += st.blocks
        e, lv = _e_l(sysg)
        times.append((k + 1) * sample)
        de.append(abs(e0 - e) / abs(e0))
        dl.append(math.sqrt(sum((a - b) ** 2 for a, b in zip(l0, lv))) / l0n)
        if progress is not None and (k + 1) % (1 << lev_min) == 0:
            progress("%s t=%g dE/E=%.3e dL/L=%.3e" % (precision, times[-1], de[-1], dl[-1]))
    torch.cuda.synchronize()
    return {
        "precision": precision,
        "mode": mode,
        "n": n,
        "eps": eps,
        "dt": dt if mode == "shared" else None,
        "seed": seed,
        "E_start": e0,
        "L_start": l0n,
        "steps_or_blocks": blocks,
        "seconds": time.perf_counter() - t0,
        "t": times,
        "dE_over_E": de,
        "dL_over_L": dl,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--mode", choices=("shared", "block"), default="shared")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--time-units", type=float, default=8.0)
    ap.add_argument("--precisions", default=None,
                    help="comma-separated from fp64, ex, sp, mixed (default: all that the "
                         "mode allows)")
    ap.add_argument("--eps", type=float, default=None,
                    help="softening (default 1/64 shared, 1e-4 block)")
    ap.add_argument("--dt", type=float, default=1.0 / 2048, help="shared step (divides 1/16)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--out", default=None, help="also write the JSON lines to this file")
    args = ap.parse_args(argv)
    default = "fp64,ex,sp,mixed" if args.mode == "shared" else "fp64,ex,mixed"
    names = [p.strip() for p in (args.precisions or default).split(",") if p.strip()]
    for p in names:
        if p not in PRECISIONS:
            ap.error("unknown precision %r (choose from %s)" % (p, ", ".join(PRECISIONS)))
        if p == "sp" and args.mode == "block":
            ap.error("sp is not available with block steps (see --help)")
    torch.cuda.set_device(0)

    def progress(msg):
        print("[conservation] " + msg, file=sys.stderr, flush=True)

    eps = args.eps if args.eps is not None else (1.0 / 64 if args.mode == "shared" else 1e-4)
    lines = [json.dumps({"study": "energy and angular momentum conservation", "mode": args.mode,
                         "n": args.n, "time_units": args.time_units, "eps": eps,
                         "dt": args.dt if args.mode == "shared" else None, "seed": args.seed,
                         "precisions": names})]
    print(lines[0], flush=True)
    for p in names:
        r = run(args.n, args.time_units, p, args.mode, eps, args.dt, args.seed,
                progress=progress)
        progress("%s: %d steps/blocks, %.1f s, final dE/E %.3e, max dE/E %.3e, final dL/L %.3e"
                 % (p, r["steps_or_blocks"], r["seconds"], r["dE_over_E"][-1],
                    max(r["dE_over_E"]), r["dL_over_L"][-1]))
        lines.append(json.dumps(r))
        print(lines[-1], flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
