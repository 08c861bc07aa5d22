"""GPU double-single (H6_EX) and single-precision (H6_SP) evaluation against
the FP64 oracle, and the conservation study built on them.

Stated bounds, per target particle (vector norms), from the arithmetic:
* EX: unit roundoff of double-single u = 2^-48 = 3.6e-15. A pair term takes
  about 30 double-single operations (each within a few u) after the input
  split, whose error (u |x|) grows to u |x| / |r| in a difference r; with
  |x| / |r| up to ~100 for close pairs and the cancellation of the sums,
  the bound is 2e-12 (a), 4e-12 (j), 1e-11 (s), about 500-3000 u. The
  largest errors measured on these inputs are 1.9e-13, 2.3e-13 and 9.4e-13
  (the sums of products and the accumulations in the "sloppy" double-single
  addition, whose operand-relative error is that of the terms it adds).
* SP: u = 2^-24 = 6.0e-8; same reasoning, bound 1e-4 (a), 2e-4 (j), 5e-4
  (s), against 7.9e-6, 1.1e-5, 4.1e-5 measured.
The typical (median) EX error is that of SP times about 2^-24: the test
requires a factor below 1e-6, which fails if the low halves of the
double-single values were lost anywhere.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1901_08532_amd import conservation, h6, ics
from _gpu import gpu_evaluate, vec_rel_err

pytestmark = pytest.mark.gpu

BOUND = {
    h6.H6_EX: {"a": 2e-12, "j": 4e-12, "s": 1e-11},
    h6.H6_SP: {"a": 1e-4, "j": 2e-4, "s": 5e-4},
}
PRECS = [pytest.param(h6.H6_EX, id="ex"), pytest.param(h6.H6_SP, id="sp")]


def _case(n, seed, eps, imf=False):
    x, v, m = ics.plummer(n, seed)
    if imf:
        m = ics.salpeter_masses(n, 10 * seed + seed)
    a, _, _, _ = oracle.forces(x, v, m, eps * eps, order=1)
    return x, v, a, m


def _check(prec, got, want):
    for name, g, w in zip("ajs", got, want):
        assert np.all(np.isfinite(g)), name
        rel = vec_rel_err(g, w)
        assert rel.max() <= BOUND[prec][name], (name, float(rel.max()))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,seed,eps,imf", [(1000, 1, 1e-4, False), (4096, 3, 1e-4, True),
                                            (2000, 6, 0.0, False), (33, 7, 1e-4, False)])
def test_all_targets_against_oracle(prec, n, seed, eps, imf):
    x, v, a, m = _case(n, seed, eps, imf)
    ctx = h6.Context(n, eps)
    got = gpu_evaluate(ctx, x, v, a, m, precision=prec)
    again = gpu_evaluate(ctx, x, v, a, m, precision=prec)
    for g1, g2 in zip(got, again):
        assert np.array_equal(g1, g2)
    want = oracle.forces(x, v, m, eps * eps, a=a, order=2)[:3]
    _check(prec, got, want)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n_act", [1, 3, 17, 300])
def test_active_subsets(prec, n_act):
    n = 5000
    x, v, a, m = _case(n, 5, 1e-4, imf=True)
    rng = np.random.Generator(np.random.PCG64(n_act))
    act = rng.choice(n, n_act, replace=False).astype(np.int32)
    ctx = h6.Context(n, 1e-4)
    got = gpu_evaluate(ctx, x, v, a, m, active=act, precision=prec)
    want = oracle.forces(x, v, m, 1e-8, a=a, idx=act.astype(np.int64), order=2)[:3]
    _check(prec, got, want)


def test_ex_error_is_single_precision_error_times_2_to_minus_24():
    n = 4096
    x, v, a, m = _case(n, 3, 1e-4, imf=True)
    ctx = h6.Context(n, 1e-4)
    want = oracle.forces(x, v, m, 1e-8, a=a, order=2)[:3]
    ex = gpu_evaluate(ctx, x, v, a, m, precision=h6.H6_EX)
    sp = gpu_evaluate(ctx, x, v, a, m, precision=h6.H6_SP)
    for name, ge, gs, w in zip("ajs", ex, sp, want):
        me, ms = np.median(vec_rel_err(ge, w)), np.median(vec_rel_err(gs, w))
        assert 0 < me < 1e-6 * ms, (name, float(me), float(ms))


def test_bad_precision_is_rejected():
    n = 64
    x, v, a, m = _case(n, 1, 1e-4)
    ctx = h6.Context(n, 1e-4)
    with pytest.raises(h6.H6Error):
        gpu_evaluate(ctx, x, v, a, m, precision=4)


def test_ex_block_steps_run_the_host_loop_and_follow_fp64():
    # H6_EX in h6_run_blocks always takes the host loop; over 1/16 time unit
    # its trajectory stays within the EX evaluation error of the FP64 one
    n = 1024
    x, v, m = ics.plummer(n, 8)
    runs = {}
    for prec in (h6.H6_FP64, h6.H6_EX):
        s = h6.System(x, v, m, 1e-4)
        s.startup(eta_s=0.1, lev_min=4, lev_max=30)
        rc, st = s.run_blocks(1 << (h6.TICK_BITS - 4), 0.4, 4, 30, prec)
        assert rc == h6.H6_OK
        runs[prec] = (st.blocks, s.field("x"), s.field("v"))
    assert runs[h6.H6_EX][0] == runs[h6.H6_FP64][0]
    for k in (1, 2):
        d = np.abs(runs[h6.H6_EX][k] - runs[h6.H6_FP64][k]).max()
        assert d <= 1e-9 * np.abs(runs[h6.H6_FP64][k]).max(), d


def test_sp_shared_steps_follow_fp64_within_single_precision():
    n = 1024
    x, v, m = ics.plummer(n, 9)
    out = {}
    for prec in (h6.H6_FP64, h6.H6_SP):
        s = h6.System(x, v, m, 1.0 / 64)
        s.startup()
        s.shared_steps(1.0 / 256, 16, prec)
        torch.cuda.synchronize()
        out[prec] = s.field("x")
    d = np.abs(out[h6.H6_SP] - out[h6.H6_FP64]).max()
    assert 0 < d <= 1e-6, d


def test_conservation_study_single_precision_accumulates():
    # the paper's qualitative result on a small system (fixed shared step
    # 1/2048, eps 1/64, one time unit): EX follows FP64 (measured: both
    # dE/E 2.4e-14, dL/L 1.6e-15) while SP accumulates round-off (2.3e-9,
    # 6.4e-10)
    res = {p: conservation.run(n=1024, time_units=1.0, precision=p) for p in ("fp64", "ex", "sp")}
    de = {p: np.array(r["dE_over_E"]) for p, r in res.items()}
    dl = {p: np.array(r["dL_over_L"]) for p, r in res.items()}
    assert all(np.all(np.isfinite(d)) for d in list(de.values()) + list(dl.values()))
    assert de["fp64"].max() < 1e-12
    assert np.max(np.abs(de["ex"] - de["fp64"])) <= 1e-13
    assert np.max(np.abs(dl["ex"] - dl["fp64"])) <= 1e-13
    assert de["sp"][-1] > 1e3 * max(de["fp64"].max(), 1e-16)
    assert dl["sp"][-1] > 1e3 * max(dl["fp64"].max(), 1e-16)
    with pytest.raises(ValueError):
        conservation.run(n=64, time_units=0.0625, precision="sp", mode="block")


@pytest.mark.parametrize("prec", PRECS)
def test_single_particle_and_empty_active_set(prec):
    # one particle: no other source, all sums exactly zero; n_act = 0 is a no-op
    x, v, a, m = _case(1, 3, 1e-4)
    ctx = h6.Context(1, 1e-4)
    for g in gpu_evaluate(ctx, x, v, a, m, precision=prec):
        assert np.array_equal(g, np.zeros((1, 3)))
    x, v, a, m = _case(100, 3, 1e-4)
    ctx = h6.Context(100, 1e-4)
    got = gpu_evaluate(ctx, x, v, a, m, active=np.zeros(0, dtype=np.int32), precision=prec)
    assert all(g.shape == (0, 3) for g in got)
