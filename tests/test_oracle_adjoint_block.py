"""Pins of the oracle parts behind the block-step adjoint and energy losses
(CPU only): the per-particle potential, the torch reference's energy, and
its block-step forward unrolled along the C oracle's block sequence."""

import numpy as np
import pytest
import torch

import oracle
import oracle.adjoint_ref as ar
from paper_1901_08532_amd import ics

TICK_SYNC = 1 << 36  # 1/16 time unit in ticks of 2^-40


def test_potential_sums_to_the_potential_energy():
    x, v, m = ics.plummer(300, 3)
    m = ics.salpeter_masses(300, 33)
    for eps2 in (1e-8, 0.0):
        phi = oracle.potential(x, m, eps2)
        _, w, _ = oracle.energy(x, v, m, eps2)
        assert 0.5 * np.dot(m, phi) == pytest.approx(w, rel=1e-13)
        assert np.all(phi < 0)


def test_potential_gradient_is_minus_the_acceleration():
    # d phi_i / d x_i = -a_i (softened), checked by a central difference
    x, v, m = ics.plummer(64, 4)
    eps2 = 1e-4
    a = oracle.forces(x, v, m, eps2, order=1)[0]
    h = 1e-6
    for i in (0, 17, 63):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            fd = (oracle.potential(xp, m, eps2)[i] - oracle.potential(xm, m, eps2)[i]) / (2 * h)
            assert fd == pytest.approx(-a[i, c], rel=1e-6, abs=1e-8)


def test_potential_of_two_bodies_is_closed_form():
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    m = np.array([2.0, 5.0])
    phi = oracle.potential(x, m, 0.0)
    assert phi[0] == pytest.approx(-5.0 / 5.0, rel=1e-15)
    assert phi[1] == pytest.approx(-2.0 / 5.0, rel=1e-15)


def test_reference_energy_equals_the_c_oracle():
    x, v, m = ics.plummer(128, 5)
    k, w, _ = oracle.energy(x, v, m, 1e-6)
    e = ar.energy(torch.from_numpy(x), torch.from_numpy(v), torch.from_numpy(m), 1e-6)
    assert float(e) == pytest.approx(k + w, rel=1e-14)


def _tensors(x, v, m):
    return torch.from_numpy(x), torch.from_numpy(v), torch.from_numpy(m)


def test_block_run_on_one_forced_level_is_the_shared_run():
    # lev_min = lev_max: every particle steps 2^-7 in every block
    x, v, m = ics.plummer(32, 6)
    eps2 = 1e-2
    sched = ar.block_schedule(x, v, m, eps2, TICK_SYNC, lev_min=7, lev_max=7)
    assert len(sched) == 8 and all(len(act) == 32 for _, act, _, _ in sched)
    xb = ar.block_run(*_tensors(x, v, m), eps2, sched)
    xs = ar.run(*_tensors(x, v, m), eps2, 2.0 ** -7, 8)
    for qb, qs in zip(xb, xs):
        assert torch.allclose(qb, qs, rtol=1e-13, atol=1e-15)


def test_block_run_follows_the_c_oracle_block_steps():
    # the unrolled torch forward reproduces the C oracle's own block run
    x, v, m = ics.plummer(48, 7)
    eps2 = 1e-6
    sched = ar.block_schedule(x, v, m, eps2, TICK_SYNC)
    assert len(sched) > 16
    assert len({len(a) for _, a, _, _ in sched}) > 1  # several active-set sizes
    st = oracle.State(x, v, m, eps2)
    st.startup(0.1, 4, 30)
    for _ in sched:
        st.block_step(0.4, 4, 30)
    got = ar.block_run(*_tensors(x, v, m), eps2, sched)
    for name, g, w in zip("xvajsc", got, (st.x, st.v, st.a, st.j, st.s, st.c)):
        g = g.numpy()
        assert np.max(np.abs(g - w)) <= 1e-10 * np.max(np.abs(w)), name


def test_block_run_gradient_matches_central_differences_of_the_c_oracle():
    # loss sum |x_T|^2 over one sync interval; perturbations small enough
    # that the C oracle takes the same block sequence
    x, v, m = ics.plummer(24, 8)
    eps2 = 1e-4
    sched = ar.block_schedule(x, v, m, eps2, TICK_SYNC)
    xt, vt, mt = (t.clone().requires_grad_(True) for t in _tensors(x, v, m))
    loss = (ar.block_run(xt, vt, mt, eps2, sched)[0] ** 2).sum()
    gx, gv, gm = torch.autograd.grad(loss, (xt, vt, mt))

    def c_loss(xx, vv, mm):
        s2 = ar.block_schedule(xx, vv, mm, eps2, TICK_SYNC)
        assert [(t, tuple(a)) for t, a, _, _ in s2] == [(t, tuple(a)) for t, a, _, _ in sched]
        st = oracle.State(xx, vv, mm, eps2)
        st.startup(0.1, 4, 30)
        for _ in sched:
            st.block_step(0.4, 4, 30)
        return float((st.x ** 2).sum())

    for kind, i, c in (("x", 3, 0), ("x", 11, 2), ("v", 5, 1), ("v", 20, 0), ("m", 9, 0)):
        arrs = {"x": x.copy(), "v": v.copy(), "m": m.copy()}
        h = 1e-3 * m[i] if kind == "m" else 1e-6
        vals = []
        for sgn in (1, -1):
            q = {k2: a.copy() for k2, a in arrs.items()}
            if kind == "m":
                q["m"][i] += sgn * h
            else:
                q[kind][i, c] += sgn * h
            vals.append(c_loss(q["x"], q["v"], q["m"]))
        fd = (vals[0] - vals[1]) / (2 * h)
        g = {"x": gx, "v": gv}[kind][i, c] if kind != "m" else gm[i]
        assert float(g) == pytest.approx(fd, rel=1e-5, abs=1e-7), (kind, i, c)
