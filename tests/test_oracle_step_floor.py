"""The smallest-step clamp of the block-step rule (Sec. 2 block steps; the
time-step criterion of Sec. 3 item 3): a particle whose criterion asks for
a step below 2^-lev_max gets exactly 2^-lev_max, the call reports -5, and
the run goes on with every time a multiple of its step.

Pinned on a circular binary, where both criteria have closed forms (the
6th-order one gives eta / omega, the start-up one eta_s / omega; see the
circular-orbit tests of the criteria), so the level the criterion asks for
is known without the oracle: a clamp to lev_max + 1, no clamp, a clamp at
the wrong tick or a lost return code each fails a check below.
"""

import math

import numpy as np

import oracle

TB = oracle.TICK_BITS
ETA, ETA_S = 0.4, 0.1
LEV_MIN, LEV_MAX = 4, 12
EPS = 1e-6


def floor_system():
    """Equal-mass circular binary (total mass 1) whose angular frequency
    puts log2(omega / eta) at 12.2 (criterion level 13) and log2(omega /
    eta_s) at 14.2 (start-up level 15); clamped to 2^-12 its steps are
    omega h = 0.46, a little longer than the criterion's 0.4 (much longer
    ones would break the binary up within the run). Returns x, v, m,
    omega."""
    omega = ETA * 2.0 ** 12.2
    # softened relative orbit: omega^2 = M / (d^2 + eps^2)^(3/2), M = 1
    d = math.sqrt(omega ** (-4.0 / 3.0) - EPS ** 2)
    half = 0.5 * d
    x = np.array([[half, 0.0, 0.0], [-half, 0.0, 0.0]])
    vb = omega * half
    v = np.array([[0.0, vb, 0.0], [0.0, -vb, 0.0]])
    m = np.array([0.5, 0.5])
    return x, v, m, omega


def test_closed_form_levels():
    _, _, _, omega = floor_system()
    assert math.ceil(math.log2(omega / ETA)) == 13
    assert math.ceil(math.log2(omega / ETA_S)) == 15


def test_initial_levels_clamp_at_lev_max():
    x, v, m, omega = floor_system()
    a, j, s, c = oracle.startup(x, v, m, EPS ** 2)
    # without the floor the binary gets the closed-form level 15
    rc, dt = oracle.initial_levels(a, j, s, c, ETA_S, LEV_MIN, 30)
    assert rc == 0
    assert list(dt) == [1 << (TB - 15)] * 2
    # with lev_max = 12: exactly 2^-12, and -5
    rc, dt = oracle.initial_levels(a, j, s, c, ETA_S, LEV_MIN, LEV_MAX)
    assert rc == -5
    assert list(dt) == [1 << (TB - LEV_MAX)] * 2


def test_block_steps_clamp_and_continue():
    x, v, m, omega = floor_system()
    st = oracle.State(x, v, m, EPS ** 2)
    assert st.startup(eta_s=ETA_S, lev_min=LEV_MIN, lev_max=LEV_MAX) == -5
    e0 = sum(st.energy()[:2])
    t_end = 1 << (TB - LEV_MIN)
    clamped = blocks = 0
    while st.t[0] < t_end:
        # the same block without the floor (lev_max 30): the step rule is the
        # same except for the clamp, so the clamped run takes exactly
        # min(level asked for, lev_max) and returns -5 iff the level asked
        # for is deeper; on the first block the level is the closed-form 13
        free = st.copy()
        rc_free, tn_free, _ = free.block_step(ETA, LEV_MIN, 30)
        assert rc_free == 0
        lev_free = TB - np.log2(free.dt).astype(int)
        if blocks == 0:
            assert list(lev_free) == [13, 13]
        due = st.t[0] + st.dt[0]
        rc, tn, na = st.block_step(ETA, LEV_MIN, LEV_MAX)
        assert (tn, na) == (due, 2) and tn == tn_free
        want_clamp = bool(np.any(lev_free > LEV_MAX))
        assert rc == (-5 if want_clamp else 0), blocks
        assert list(st.dt) == [1 << (TB - min(int(q), LEV_MAX)) for q in lev_free]
        assert np.all((st.dt & (st.dt - 1)) == 0)
        assert np.all(st.dt >= 1 << (TB - LEV_MAX)) and np.all(st.dt <= t_end)
        assert np.all(st.t % st.dt == 0)
        assert np.all(np.isfinite(st.x)) and np.all(np.isfinite(st.v))
        clamped += want_clamp
        blocks += 1
    # the run reaches the next multiple of 2^-lev_min, every block clamped
    assert np.all(st.t == t_end) and blocks == 256
    assert clamped == blocks
    # the clamped (too long) steps still integrate the binary: its
    # separation stays near d and the energy moves little
    sep = np.linalg.norm(st.x[0] - st.x[1])
    d = np.linalg.norm(x[0] - x[1])
    assert abs(sep - d) < 1e-2 * d
    assert abs(sum(st.energy()[:2]) - e0) < 1e-2 * abs(e0)
