"""The device-resident block loop (h6_run_blocks, host_loop = 0).

It must take the same blocks as the host-sequenced loop and as the oracle
(block times and active counts bit-exact, steps bit-exact), and agree with
them on the state to rounding; empty runs and awkward sizes included.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_1901_08532_amd import h6, ics
from _gpu import DEV, vec_rel_err

pytestmark = pytest.mark.gpu

TB = h6.TICK_BITS
EPS = 1e-4
SYNC = 1 << (TB - 4)


def _predicted(s, t_tick):
    """The host-sequenced predictor's arrays: every particle of s to t_tick."""
    P = torch.zeros_like(s.P)
    s.ctx.h6_predict(s.S, s.m, s.T, t_tick, P)
    torch.cuda.synchronize()
    return P


def _assert_speculative_prediction(s, t_block, lv_hi_dt):
    # after a block at t_block, the finishing kernel left every particle
    # predicted to t_block plus the step of the block's highest occupied
    # level (the next block's time unless a correction changed that level):
    # bit for bit the predictor's result on the stored state
    t_spec = int(t_block) + int(lv_hi_dt)
    want = _predicted(s, t_spec)
    assert torch.equal(s.P, want)


def _from_oracle(st):
    sysg = h6.System(st.x, st.v, st.m, math.sqrt(st.eps2))
    for k, name in enumerate(("x", "v", "a", "j", "s", "c")):
        sysg.S[3 * k:3 * k + 3] = torch.from_numpy(np.ascontiguousarray(getattr(st, name).T)).to(DEV)
    sysg.T[0] = torch.from_numpy(st.t).to(DEV)
    sysg.T[1] = torch.from_numpy(st.dt).to(DEV)
    return sysg


@pytest.mark.parametrize("n,eps", [(33, EPS), (1000, EPS), (5000, EPS), (200, 0.0)])
def test_device_loop_matches_oracle_blocks(n, eps):
    x, v, m = ics.plummer(n, 100 + n)
    st = oracle.State(x, v, m, eps ** 2)
    assert st.startup(eta_s=0.1, lev_min=4, lev_max=30) == 0
    sysg = _from_oracle(st)
    nblk = psteps = 0
    while True:
        rc, tn, na = st.block_step(0.4, 4, 30)
        assert rc == 0
        nblk += 1
        psteps += na
        if tn == SYNC and np.all(st.t == SYNC):
            break
    rc, stats = sysg.run_blocks(SYNC, 0.4, 4, 30)
    assert rc == h6.H6_OK
    assert (stats.blocks, stats.particle_steps) == (nblk, psteps)
    assert stats.interactions == float(psteps) * n
    assert np.array_equal(sysg.T.cpu().numpy(), np.stack([st.t, st.dt]))
    for name in ("x", "v", "a", "j", "s"):
        assert vec_rel_err(sysg.field(name), getattr(st, name)).max() < 1e-9, name


@pytest.mark.parametrize("precision", [h6.H6_FP64, h6.H6_MIXED])
def test_device_loop_matches_host_loop(precision):
    n = 20000
    x, v, m = ics.plummer(n, 7)
    a = h6.System(x, v, m, EPS)
    a.startup(eta_s=0.1, lev_min=4, lev_max=30)
    b = h6.System(x, v, m, EPS)
    b.S.copy_(a.S)
    b.T.copy_(a.T)
    for k in range(2):
        ra, sa = a.run_blocks((k + 1) * SYNC, 0.4, 4, 30, precision)
        rb, sb = b.run_blocks((k + 1) * SYNC, 0.4, 4, 30, precision, host_loop=True)
        assert ra == rb == h6.H6_OK
        if precision == h6.H6_FP64:
            assert (sa.blocks, sa.particle_steps) == (sb.blocks, sb.particle_steps)
        else:
            # FP32 partial sums group differently under the two launch shapes;
            # forces then differ at ~1e-7 and a step decision within that of a
            # power of two may flip for a handful of particles
            assert abs(sa.particle_steps - sb.particle_steps) <= 1e-4 * sb.particle_steps
    if precision == h6.H6_FP64:
        assert torch.equal(a.T, b.T)
        for name in ("x", "v", "a", "j", "s"):
            assert vec_rel_err(a.field(name), b.field(name)).max() < 1e-9, name
    else:
        assert (a.T != b.T).any(dim=0).sum().item() <= 1e-3 * n
        for name in ("x", "v"):
            assert np.median(vec_rel_err(a.field(name), b.field(name))) < 1e-6, name
        ea, eb = sum(a.energy()[:2]), sum(b.energy()[:2])
        assert abs(ea - eb) < 1e-9 * abs(eb)


def test_device_loop_nothing_due_and_repeat():
    n = 3000
    x, v, m = ics.plummer(n, 9)
    s = h6.System(x, v, m, EPS)
    s.startup(eta_s=0.1, lev_min=4, lev_max=30)
    rc, st = s.run_blocks(SYNC, 0.4, 4, 30)
    assert rc == h6.H6_OK and st.blocks > 0
    T1 = s.T.clone()
    S1 = s.S.clone()
    rc, st = s.run_blocks(SYNC, 0.4, 4, 30)  # already there: no block
    assert rc == h6.H6_OK and st.blocks == 0 and st.particle_steps == 0
    assert torch.equal(s.T, T1) and torch.equal(s.S, S1)


def test_device_loop_profile_records():
    n = 8192
    x, v, m = ics.plummer(n, 11)
    s = h6.System(x, v, m, EPS)
    s.startup(eta_s=0.1, lev_min=4, lev_max=30)
    s.ctx.h6_profile_enable(True)
    rc, st = s.run_blocks(SYNC, 0.4, 4, 30)
    recs = s.ctx.h6_profile_read()
    s.ctx.h6_profile_enable(False)
    assert rc == h6.H6_OK
    loop = [r for r in recs if r["kind"] == 2]
    real = [r for r in loop if r["nact_log2"] >= 0]
    assert sum(r["launches"] for r in real) == st.blocks
    assert sum(r["interactions"] for r in real) == pytest.approx(st.interactions)
    assert all(r["kernel_ms"] > 0 for r in real)


def test_device_loop_profile_records_of_both_kernels():
    # level 2: the finishing kernel of every slot too, with the algorithmic
    # bytes of each record from the slot's (n_act, split); prediction slots
    # (bin -2) apart
    n = 8192
    x, v, m = ics.plummer(n, 12)
    s = h6.System(x, v, m, EPS)
    s.startup(eta_s=0.1, lev_min=4, lev_max=30)
    s.ctx.h6_profile_enable(2)
    rc, st = s.run_blocks(SYNC, 0.4, 4, 30)
    recs = s.ctx.h6_profile_read()
    s.ctx.h6_profile_enable(False)
    assert rc == h6.H6_OK
    assert not [r for r in recs if r["kind"] == 3]  # no separate predictor
    by_kind, slots = {}, {}
    for r in recs:
        if r["kind"] not in (2, 4):
            continue
        if r["nact_log2"] >= 0:
            d = by_kind.setdefault(r["kind"], [0, 0.0, 0.0])
            d[0] += r["launches"]
            d[1] += r["interactions"]
            d[2] += r["bytes"]
        elif r["nact_log2"] == -2:
            d = slots.setdefault(r["kind"], [0, 0.0, 0.0])
            d[0] += r["launches"]
            d[1] += r["interactions"]
            d[2] += r["bytes"]
    for kind in (2, 4):
        assert by_kind[kind][0] == st.blocks, kind
        assert by_kind[kind][1] == pytest.approx(st.interactions), kind
    # the run's first slot predicts (its set-up makes no guess); each
    # prediction slot: an empty evaluation, a prediction of all n
    n_slots = slots[4][0]
    assert 1 <= n_slots <= st.blocks and slots[2][0] == n_slots
    assert slots[2][1] == slots[4][1] == 0.0 and slots[2][2] == 0.0
    assert slots[4][2] == 224.0 * n * n_slots
    # finishing kernel: 368 B per active particle plus 72 B per slice, and
    # the prediction of every inactive particle (224 B)
    inactive = 224.0 * (n * st.blocks - st.particle_steps)
    assert by_kind[4][2] >= (368.0 + 72.0) * st.particle_steps + inactive
    assert by_kind[4][2] <= (368.0 + 72.0 * 4096) * st.particle_steps + inactive
    # evaluation: at least every source and target once per block
    assert by_kind[2][2] >= 80.0 * n * st.blocks + 76.0 * st.particle_steps


def test_device_loop_end_events_across_runs():
    # level 2 over two consecutive runs: each loop dispatch carries one event,
    # at its end, and is timed from the end of the work before it (the other
    # kernel, the run's start or a plan readback). Every block of both runs
    # is timed once per kernel with a positive span, and the spans, which
    # tile the stream's time without overlapping, sum to no more than the
    # wall time of the two runs
    import time

    n = 8192
    x, v, m = ics.plummer(n, 14)
    s = h6.System(x, v, m, EPS)
    s.startup(eta_s=0.1, lev_min=4, lev_max=30)
    s.ctx.h6_profile_enable(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc1, st1 = s.run_blocks(SYNC // 2, 0.4, 4, 30)
    rc2, st2 = s.run_blocks(SYNC, 0.4, 4, 30)
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0)
    recs = s.ctx.h6_profile_read()
    s.ctx.h6_profile_enable(False)
    assert rc1 == rc2 == h6.H6_OK and st1.blocks > 0 and st2.blocks > 0
    loop = [r for r in recs if r["kind"] in (2, 4)]
    for kind in (2, 4):
        real = [r for r in loop if r["kind"] == kind and r["nact_log2"] >= 0]
        assert sum(r["launches"] for r in real) == st1.blocks + st2.blocks, kind
        assert all(r["kernel_ms"] > 0 for r in real), kind
    assert sum(r["kernel_ms"] for r in loop) <= wall_ms


def test_slot_log_accounts_for_every_block():
    # profile level 3: no events, the slot log only. Every block appears once
    # with its active count, prediction slots carry the count of the block
    # they precede, and the run's first slot is one (its set-up makes no guess)
    n = 8192
    x, v, m = ics.plummer(n, 13)
    s = h6.System(x, v, m, EPS)
    s.startup(eta_s=0.1, lev_min=4, lev_max=30)
    s.ctx.h6_profile_enable(3)
    rc, st = s.run_blocks(SYNC, 0.4, 4, 30)
    slots = s.ctx.h6_profile_slots()
    assert s.ctx.h6_profile_read() == []  # no event records at this level
    s.ctx.h6_profile_enable(False)
    assert rc == h6.H6_OK
    na, sp = slots[:, 0], slots[:, 1]
    blocks = (na > 0) & (sp > 0)
    assert int(blocks.sum()) == st.blocks
    assert int(na[blocks].sum()) == st.particle_steps
    assert sp[0] == -1 and na[0] > 0
    pslots = np.nonzero(sp < 0)[0]
    assert np.all(pslots + 1 < len(slots))
    assert np.array_equal(na[pslots], na[pslots + 1]) and np.all(sp[pslots + 1] > 0)
    # after the last block only empty slots (batch overshoot)
    last = np.nonzero(blocks)[0][-1]
    assert np.all(na[last + 1:] == 0)


def _host_vs_device(s_dev, s_host, t_end, lev_min, lev_max):
    rd, sd = s_dev.run_blocks(t_end, 0.4, lev_min, lev_max)
    rh, sh = s_host.run_blocks(t_end, 0.4, lev_min, lev_max, host_loop=True)
    assert rd == rh == h6.H6_OK
    assert (sd.blocks, sd.particle_steps) == (sh.blocks, sh.particle_steps)
    assert torch.equal(s_dev.T, s_host.T) and torch.equal(s_dev.S, s_host.S)


def _pair(n, seed):
    x, v, m = ics.plummer(n, seed)
    a = h6.System(x, v, m, EPS)
    a.startup(eta_s=0.1, lev_min=4, lev_max=30)
    b = h6.System(x, v, m, EPS)
    b.S.copy_(a.S)
    b.T.copy_(a.T)
    return a, b


def test_device_loop_off_grid_state_uses_host_loop():
    # a particle time that is not a multiple of its step: the level lists do
    # not apply, and the call runs the host-sequenced loop (bitwise the same)
    a, b = _pair(2000, 21)
    for s in (a, b):
        s.T[0, 7] = s.T[1, 7] // 2
    _host_vs_device(a, b, SYNC, 4, 30)


def test_device_loop_levels_outside_run_range_use_host_loop():
    # start-up steps taken with lev_max 30; a run limited to two levels below
    # the deepest one cannot list those particles and falls back to the host
    # loop (which clamps their steps and reports H6_EDTMIN)
    a, b = _pair(2000, 22)
    lev = h6.TICK_BITS - torch.log2(a.T[1].double()).round().long()
    top = int(lev.max()) - 2
    assert top > 4
    ra, _ = a.run_blocks(SYNC, 0.4, 4, top, check=False)
    rb, _ = b.run_blocks(SYNC, 0.4, 4, top, check=False, host_loop=True)
    assert ra == rb
    assert torch.equal(a.T, b.T) and torch.equal(a.S, b.S)


def test_device_loop_single_particle_and_tiny_systems():
    for n in (1, 2, 3):
        x, v, m = ics.plummer(max(n, 2), 30 + n)
        x, v, m = x[:n], v[:n], m[:n]
        s = h6.System(x, v, m, EPS)
        s.startup(eta_s=0.1, lev_min=4, lev_max=30)
        rc, st = s.run_blocks(SYNC, 0.4, 4, 30)
        assert rc == h6.H6_OK and st.blocks > 0
        assert bool((s.T[0] == SYNC).all())


def _one_block_against_host_loop_and_oracle(n, n_act, precision, seed=21, samples=128):
    # the first block has exactly n_act of n particles active (levels 5 and
    # 4 at t = 0): the device loop's state after it must match the host
    # loop's, and the forces it left must match the oracle evaluated on the
    # host loop's predicted arrays (the same predictor code, bit for bit)
    x, v, m = ics.plummer(n, seed)
    rng = np.random.Generator(np.random.PCG64(n_act))
    act = np.sort(rng.choice(n, n_act, replace=False))
    dt = np.full(n, 1 << (TB - 4), dtype=np.int64)
    dt[act] = 1 << (TB - 5)
    systems = []
    for host_loop in (False, True):
        s = h6.System(x, v, m, EPS)
        s.startup()
        s.T[0].zero_()
        s.T[1].copy_(torch.from_numpy(dt).to(DEV))
        rc, st = s.run_blocks(1 << (TB - 5), 0.4, 4, 30, precision, host_loop=host_loop)
        assert rc == h6.H6_OK
        assert (st.blocks, st.particle_steps) == (1, n_act)
        systems.append(s)
    a, b = systems
    bound = ({"a": 1e-12, "j": 1e-12, "s": 1e-12} if precision == h6.H6_FP64
             else {"a": 2e-5, "j": 5e-5, "s": 2e-4})
    if precision == h6.H6_FP64:
        assert torch.equal(a.T, b.T)
    # FP64: compensated sums over different slicings agree to rounding; mixed:
    # the FP32 partial sums group differently, and the force differences
    # (within twice the stated bound) move x and v after one step
    xv_tol = 1e-12 if precision == h6.H6_FP64 else 1e-6
    for name in ("x", "v"):
        assert vec_rel_err(a.field(name), b.field(name)).max() < xv_tol, name
    for name in "ajs":  # two evaluations, each within the bound of the oracle's
        assert vec_rel_err(a.field(name), b.field(name)).max() < 2 * bound[name], name
    # the device loop's prediction of the active (corrected) and inactive
    # particles to the guessed next block time: level 5 was the highest
    _assert_speculative_prediction(a, 1 << (TB - 5), 1 << (TB - 5))
    P = b.P.cpu().numpy()
    xp, vp, ap = P[0:3].T.copy(), P[3:6].T.copy(), P[6:9].T.copy()
    idx = act if n_act <= samples else np.sort(rng.choice(act, samples, replace=False))
    want = oracle.forces(xp, vp, m, EPS ** 2, a=ap, idx=idx, order=2)[:3]
    for k, name in enumerate("ajs"):
        err = vec_rel_err(a.field(name)[idx], want[k])
        assert err.max() <= bound[name], (name, float(err.max()))


@pytest.mark.parametrize("precision", [h6.H6_FP64, h6.H6_MIXED])
@pytest.mark.parametrize("n_act", [24000, 44000])
def test_device_loop_tile_units_beyond_the_grid(precision, n_act):
    # one block of n_act of 65536 particles: the device loop cuts the sources
    # into more tile units (target group x slice) than it launches workgroups
    # (3008 and 7912 units for 2048 workgroups), which take them in rounds.
    # Every unit must be evaluated exactly once.
    _one_block_against_host_loop_and_oracle(65536, n_act, precision)


@pytest.mark.parametrize("precision", [h6.H6_FP64, h6.H6_MIXED])
@pytest.mark.parametrize("n_act", [1, 16, 17, 48, 49, 64, 65, 512, 513])
def test_device_loop_evaluation_kind_boundaries(precision, n_act):
    # the device loop's evaluation kinds change at 16 / 17 (one or two
    # targets per wave), 48 / 49 (source-parallel to one target per lane in
    # 64-target tiles) and 512 / 513 (to two per lane in 128-target tiles);
    # 64 / 65 fill one tile group exactly and spill into a second
    _one_block_against_host_loop_and_oracle(20000, n_act, precision)


@pytest.mark.parametrize("precision", [h6.H6_FP64, h6.H6_MIXED])
def test_device_loop_two_clusters_full_activity_block(precision):
    # the largest blocks of the two-cluster workload (2 x 524288, seeds 5 and
    # 55, eps 1e-4) in the device loop's own launch shape: every particle on
    # level 4 at t = 0, so the first block evaluates all 1048576 targets
    # against all sources. Seeded a, j, s, c stand in for the start-up (any
    # state is a valid input of the evaluation); sampled targets against the
    # oracle on the loop's predicted arrays
    x, v, m = ics.two_clusters(524288, 5, 55)
    n = len(m)
    rng = np.random.Generator(np.random.PCG64(555))
    s = h6.System(x, v, m, EPS)
    for k, scale in ((6, 1.0), (9, 0.1), (12, 0.01), (15, 0.001)):
        s.S[k:k + 3] = torch.from_numpy(rng.normal(0.0, scale, (3, n))).to(DEV)
    s.T[0].zero_()
    s.T[1].fill_(1 << (TB - 4))
    # the arrays the block evaluates from (its prediction slot's, bit for bit)
    P = _predicted(s, 1 << (TB - 4)).cpu().numpy()
    rc, st = s.run_blocks(1 << (TB - 4), 0.4, 4, 30, precision, check=False)
    assert rc in (h6.H6_OK, h6.H6_EDTMIN)  # random derivatives may ask for tiny steps
    assert (st.blocks, st.particle_steps) == (1, n)
    xp, vp, ap = P[0:3].T.copy(), P[3:6].T.copy(), P[6:9].T.copy()
    idx = np.sort(rng.choice(n, 256, replace=False))
    want = oracle.forces(xp, vp, m, EPS ** 2, a=ap, idx=idx, order=2)[:3]
    bound = ({"a": 1e-12, "j": 1e-12, "s": 1e-12} if precision == h6.H6_FP64
             else {"a": 2e-5, "j": 5e-5, "s": 2e-4})
    for k, name in enumerate("ajs"):
        err = vec_rel_err(s.field(name)[idx], want[k])
        assert err.max() <= bound[name], (name, float(err.max()))


@pytest.mark.parametrize("n,precision,imf", [(65536, h6.H6_FP64, False),
                                              (262144, h6.H6_MIXED, True)])
def test_device_loop_full_size_sync_block_against_oracle(n, precision, imf):
    # the workloads the benchmark times (N = 65536 FP64; N = 262144 power-law
    # masses, mixed), one sync interval on the device loop. The block at the
    # sync time has every particle active: its evaluation, in the launch
    # shape of the loop, left a, j, s in the state and the predicted x, v, a
    # in the work array, so sampled targets can be checked one by one
    x, v, m = ics.plummer(n, 2 if not imf else 3)
    if imf:
        m = ics.salpeter_masses(n, 33)
    s = h6.System(x, v, m, EPS)
    s.startup(eta_s=0.1, lev_min=4, lev_max=30)
    # every block before the sync time (t_end one tick short of it), then
    # the sync block alone, from the state it starts from
    rc, st = s.run_blocks(SYNC - 1, 0.4, 4, 30, precision)
    assert rc == h6.H6_OK and st.blocks > 100
    pre = {name: s.field(name) for name in ("x", "v", "a", "j", "s", "c")}
    t_pre = s.T[0].cpu().numpy()
    dt_hi = int(s.T[1].min())  # step of the highest occupied level
    assert np.all(t_pre < SYNC)
    # the arrays the sync block evaluates from: the run's first slot
    # predicts every particle to SYNC with this same code
    Pt = _predicted(s, SYNC)
    rc, st = s.run_blocks(SYNC, 0.4, 4, 30, precision)
    assert rc == h6.H6_OK and (st.blocks, st.particle_steps) == (1, n)
    assert bool((s.T[0] == SYNC).all())
    P = Pt.cpu().numpy()
    xp, vp, ap = P[0:3].T.copy(), P[3:6].T.copy(), P[6:9].T.copy()
    order = ("x", "v", "a", "j", "s", "c")

    def against_oracle_predict(st_in, delta, got):
        # the predictor (every particle over its own interval) against the
        # oracle's: the sum of the absolute Taylor terms bounds the rounding
        # of both
        want_p = oracle.predict(*(st_in[q] for q in order), delta)
        D = delta[:, None]
        for k in range(3):
            scale = sum(np.abs(st_in[q]) * D ** (i - k) for i, q in enumerate(order) if i >= k)
            assert np.all(np.abs(got[:, 3 * k:3 * k + 3] - want_p[k]) <= 8e-16 * scale), k

    against_oracle_predict(pre, (SYNC - t_pre) * 2.0 ** -TB, P.T)
    # the loop's own prediction after the block, of the corrected state to
    # SYNC plus the step of the highest level: bit for bit the predictor's,
    # and against the oracle's
    _assert_speculative_prediction(s, SYNC, dt_hi)
    post = {name: s.field(name) for name in order}
    against_oracle_predict(post, np.full(n, dt_hi * 2.0 ** -TB), s.P.cpu().numpy().T)
    rng = np.random.Generator(np.random.PCG64(77))
    idx = np.sort(rng.choice(n, 256 if not imf else 1024, replace=False))
    want = oracle.forces(xp, vp, m, EPS ** 2, a=ap, idx=idx, order=2)[:3]
    bound = ({"a": 1e-12, "j": 1e-12, "s": 1e-12} if precision == h6.H6_FP64
             else {"a": 2e-5, "j": 5e-5, "s": 2e-4})
    for k, name in enumerate("ajs"):
        got = s.field(name)[idx]
        err = vec_rel_err(got, want[k])
        assert err.max() <= bound[name], (name, float(err.max()))


def test_two_contexts_run_concurrently_from_two_threads():
    # distinct contexts are independent: two device-loop runs, each context
    # on its own stream and driven from its own host thread, give bit for
    # bit the state of the same runs made one after the other on the
    # default stream
    import threading

    n = 4096
    made = {}
    for tag in ("a", "b", "a_ref", "b_ref"):
        x, v, m = ics.plummer(n, 41 if tag.startswith("a") else 42)
        s = h6.System(x, v, m, EPS)
        s.startup(eta_s=0.1, lev_min=4, lev_max=30)
        made[tag] = s
    torch.cuda.synchronize()
    for tag in ("a_ref", "b_ref"):
        rc, _ = made[tag].run_blocks(SYNC, 0.4, 4, 30)
        assert rc == h6.H6_OK
    torch.cuda.synchronize()
    streams = {"a": torch.cuda.Stream(), "b": torch.cuda.Stream()}
    for tag, st in streams.items():
        made[tag].ctx.set_stream(st)
    rcs = {}

    def run(tag):
        rcs[tag] = made[tag].run_blocks(SYNC, 0.4, 4, 30)[0]

    threads = [threading.Thread(target=run, args=(tag,)) for tag in streams]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert rcs == {"a": h6.H6_OK, "b": h6.H6_OK}
    for tag in streams:
        assert torch.equal(made[tag].T, made[tag + "_ref"].T), tag
        assert torch.equal(made[tag].S, made[tag + "_ref"].S), tag
