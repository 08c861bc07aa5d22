"""Pins of the oracle's pair terms and sums against mathematics, not itself.

* Two-body Kepler motion: a, j, s, c from the start-up passes equal the
  time derivatives (orders 2..5) of the closed-form orbit.
* A single softened pair: J, S, C equal the 1st..3rd time derivatives of
  the softened Newtonian acceleration m r (|r|^2+eps^2)^(-3/2) along
  r(t) = r + v t + a t^2/2 + jr t^3/6, taken numerically at 40 digits.
* Newton's third law: sum_i m_i F_i = 0 for F = a, j, s, c.
* Self exclusion: a particle's own mass never enters its own sum.
* The potential energy's gradient is minus the force (softening consistent).
* Energy and angular momentum of a Kepler pair match the closed forms.
"""

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_1901_08532_amd import ics
from _kepler import Kepler


@pytest.mark.parametrize("m1,m2,e,t", [(0.6, 0.4, 0.5, 0.3), (0.5, 0.5, 0.9, 0.05),
                                       (0.999, 0.001, 0.2, 2.0), (0.3, 0.7, 0.7, 4.5)])
def test_kepler_startup_matches_orbit_derivatives(m1, m2, e, t):
    k = Kepler(m1, m2, 1.0, e)
    b1, b2 = k.bodies(t, 5)
    x = np.array([b1[0], b2[0]])
    v = np.array([b1[1], b2[1]])
    m = np.array([m1, m2])
    got = oracle.startup(x, v, m, 0.0)
    for body, ref in ((0, b1), (1, b2)):
        for order, q in enumerate(got):
            want = np.array(ref[order + 2])
            err = np.abs(q[body] - want).max() / np.abs(want).max()
            assert err < 2e-13, (body, order, err)


def _mp_softened_acc_derivs(r, v, a, jr, m, eps2, kmax):
    """Time derivatives 0..kmax at t=0 of m r(t) (|r(t)|^2+eps2)^(-3/2)."""
    mp.mp.dps = 40
    r, v, a, jr = ([mp.mpf(float(q)) for q in vec] for vec in (r, v, a, jr))
    m = mp.mpf(float(m))
    e2 = mp.mpf(float(eps2))

    def comp(c):
        def f(t):
            rt = [r[k] + v[k] * t + a[k] * t ** 2 / 2 + jr[k] * t ** 3 / 6 for k in range(3)]
            R2 = sum(q * q for q in rt) + e2
            return m * rt[c] / R2 ** mp.mpf(1.5)
        return f

    return [np.array([float(mp.diff(comp(c), 0, k)) for c in range(3)]) for k in range(kmax + 1)]


@pytest.mark.parametrize("seed", range(6))
def test_pair_terms_are_time_derivatives_of_softened_force(seed):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    r = rng.normal(0, 1, 3)
    v = rng.normal(0, 1, 3)
    a = rng.normal(0, 1, 3)
    jr = rng.normal(0, 1, 3)
    m = rng.uniform(0.1, 2.0)
    eps2 = [0.0, 1e-4, 0.3][seed % 3]
    ref = _mp_softened_acc_derivs(r, v, a, jr, m, eps2, 3)
    got = oracle.pair(r, v, a, jr, m, eps2, order=3)
    for k in range(4):
        err = np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()
        assert err < 1e-13, (k, err)


def test_pair_orders_leave_unrequested_outputs():
    r, v, a, jr = np.ones(3), np.ones(3) * 0.5, np.ones(3) * 0.2, np.ones(3)
    A1, J1, S1, C1 = oracle.pair(r, v, a, jr, 1.0, 0.0, order=1)
    assert np.all(S1 == 0) and np.all(C1 == 0)
    A3, J3, S3, C3 = oracle.pair(r, v, a, jr, 1.0, 0.0, order=3)
    assert np.array_equal(A1, A3) and np.array_equal(J1, J3)


def test_third_law_all_orders():
    n = 512
    x, v, m = ics.plummer(n, 7)
    m = ics.salpeter_masses(n, 77)  # unequal masses make the check sharper
    eps2 = 1e-4 ** 2
    a, j, s, c = oracle.startup(x, v, m, eps2)
    for name, F in (("a", a), ("j", j), ("s", s), ("c", c)):
        tot = np.abs((m[:, None] * F).sum(axis=0)).max()
        scale = (m[:, None] * np.abs(F)).sum()
        assert tot <= 10 * n * np.finfo(float).eps * scale, (name, tot, scale)


def test_self_mass_does_not_enter_own_sum():
    x, v, m = ics.plummer(64, 3)
    eps2 = 1e-2
    A, J, _, _ = oracle.forces(x, v, m, eps2, order=1)
    m2 = m.copy()
    m2[5] *= 1000.0
    A2, J2, _, _ = oracle.forces(x, v, m2, eps2, order=1)
    assert np.array_equal(A[5], A2[5]) and np.array_equal(J[5], J2[5])
    assert not np.array_equal(A[6], A2[6])


def test_subset_targets_equal_full_sum():
    x, v, m = ics.plummer(200, 11)
    a, j, _, _ = oracle.forces(x, v, m, 1e-6, order=1)
    idx = np.array([199, 0, 57, 57, 3])
    A, J, S, _ = oracle.forces(x, v, m, 1e-6, a=a, idx=idx, order=2)
    Af, Jf, Sf, _ = oracle.forces(x, v, m, 1e-6, a=a, order=2)
    assert np.array_equal(A, Af[idx]) and np.array_equal(S, Sf[idx])


def test_potential_gradient_is_minus_force():
    x, v, m = ics.plummer(40, 5)
    eps2 = 0.01
    A, _, _, _ = oracle.forces(x, v, m, eps2, order=1)
    h = 1e-6
    for i in (0, 17, 39):
        for c in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            dE = (oracle.energy(xp, v, m, eps2)[1] - oracle.energy(xm, v, m, eps2)[1]) / (2 * h)
            assert abs(-dE - m[i] * A[i, c]) < 1e-8 * m[i] * np.abs(A[i]).max() + 1e-12


def test_kepler_energy_and_angular_momentum():
    k = Kepler(0.7, 0.3, 1.3, 0.6)
    for t in (0.0, 1.1, 3.0):
        b1, b2 = k.bodies(t, 1)
        x = np.array([b1[0], b2[0]])
        v = np.array([b1[1], b2[1]])
        ek, ep, L = oracle.energy(x, v, np.array([0.7, 0.3]), 0.0)
        assert abs(ek + ep - k.energy()) < 1e-14
        assert abs(L[2] - k.ang_mom()) < 1e-14 and abs(L[0]) < 1e-16 and abs(L[1]) < 1e-16


def test_absolute_sums_bound_the_sums():
    x, v, m = ics.plummer(300, 12)
    a, _, _, _ = oracle.forces(x, v, m, 1e-6, order=1)
    F = oracle.forces(x, v, m, 1e-6, a=a, order=2)
    Fa = oracle.forces(x, v, m, 1e-6, a=a, order=2, absolute=True)
    for f, fa in zip(F[:3], Fa[:3]):
        assert np.all(fa >= np.abs(f) * (1 - 1e-14))
    # a single source: the absolute sum is the absolute value
    Fs = oracle.forces(x[:2], v[:2], m[:2], 1e-6, a=a[:2], order=2)
    Fsa = oracle.forces(x[:2], v[:2], m[:2], 1e-6, a=a[:2], order=2, absolute=True)
    for f, fa in zip(Fs[:3], Fsa[:3]):
        assert np.array_equal(np.abs(f), fa)
