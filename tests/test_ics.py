"""Properties of the seeded input generators (CPU only)."""

import numpy as np

import oracle
from paper_1901_08532_amd import ics


def test_plummer_is_seeded_and_centred():
    x1, v1, m1 = ics.plummer(4096, 1)
    x2, v2, m2 = ics.plummer(4096, 1)
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
    x3, _, _ = ics.plummer(4096, 2)
    assert not np.array_equal(x1, x3)
    assert abs(m1.sum() - 1.0) < 1e-14
    assert np.abs((m1[:, None] * x1).sum(0)).max() < 1e-14
    assert np.abs((m1[:, None] * v1).sum(0)).max() < 1e-14
    assert np.sqrt((x1 ** 2).sum(1)).max() < 22.9  # mass cut 0.999


def test_plummer_henon_units():
    x, v, m = ics.plummer(4096, 3)
    ek, ep, _ = oracle.energy(x, v, m, 0.0)
    # virial equilibrium and E = -1/4 up to sampling noise
    assert abs(2 * ek / abs(ep) - 1.0) < 0.08
    assert abs(ek + ep + 0.25) < 0.02


def test_salpeter_masses():
    m = ics.salpeter_masses(200000, 33)
    assert abs(m.sum() - 1.0) < 1e-12
    raw = m / m.min() * 0.1
    assert raw.max() <= 100.0 * 1.0001
    # maximum-likelihood slope of a truncated power law, checked loosely
    lo = m.min()
    sel = m[m < 50 * lo]
    alpha = 1 + sel.size / np.log(sel / lo).sum()
    assert 2.2 < alpha < 2.5


def test_two_clusters_geometry():
    x, v, m = ics.two_clusters(2048, 5, 55)
    n = 2048
    assert abs(m.sum() - 1.0) < 1e-14
    assert np.abs((m[:, None] * v).sum(0)).max() < 1e-14
    ca = (m[:n, None] * x[:n]).sum(0) / m[:n].sum()
    cb = (m[n:, None] * x[n:]).sum(0) / m[n:].sum()
    va = (m[:n, None] * v[:n]).sum(0) / m[:n].sum()
    vb = (m[n:, None] * v[n:]).sum(0) / m[n:].sum()
    assert abs((cb - ca)[0] - 10.0) < 0.2
    assert abs((va - vb)[0] - 0.5) < 0.05
