"""Seeded synthetic initial conditions for the direct N-body workloads.

This module only draws particle positions, velocities and masses. It holds
none of the integrator's arithmetic and imports nothing else from the
package, so both the GPU path and the CPU oracle can take their inputs from
it.

The paper measures a Plummer-type star cluster (Sec. 3, the N=4096
conservation run behind Fig. 1); these generators stand in for such inputs:

* ``plummer``: the Aarseth-Henon-Wielen rejection sampler for the Plummer
  model, scaled to Henon units (G = M = 1, virial radius 1, so the analytic
  total energy is -1/4) and moved to the centre-of-mass frame. No exact
  energy rescaling is applied; the measured energy of a sample differs from
  -1/4 by its sampling noise.
* ``salpeter_masses``: masses with dN/dm ~ m^-2.35 on [0.1, 100], drawn
  independently of the phase-space sample and normalised to total mass 1.
* ``two_clusters``: two Plummer spheres of mass 1/2 each on a head-on
  approach.

Every generator takes an integer seed and uses numpy's PCG64 bit generator,
so the same seed gives the same arrays on every machine.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = ["plummer", "salpeter_masses", "two_clusters", "random_state"]

# Length scale of the Plummer model whose virial radius is 1 (Henon units).
_PLUMMER_A = 3.0 * math.pi / 16.0


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """Unit vectors uniform on the sphere, shape (n, 3)."""
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)


def _plummer_speed_fraction(rng: np.random.Generator, n: int) -> np.ndarray:
    """q = v / v_escape drawn from g(q) ~ q^2 (1 - q^2)^(7/2) by rejection."""
    out = np.empty(n)
    filled = 0
    while filled < n:
        want = n - filled
        batch = max(1024, int(want * 10.5))  # acceptance is about 1/10
        q = rng.uniform(0.0, 1.0, batch)
        y = rng.uniform(0.0, 0.1, batch)
        keep = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(keep.size, want)
        out[filled:filled + take] = keep[:take]
        filled += take
    return out


def plummer(n: int, seed: int, mass_cut: float = 0.999):
    """Plummer sphere of ``n`` equal-mass particles in Henon units.

    Returns (x, v, m): float64 arrays of shape (n, 3), (n, 3), (n,), with
    total mass 1 and the centre of mass at rest at the origin.

    ``mass_cut`` truncates the cumulative mass fraction, which bounds the
    radius at (mass_cut^(-2/3) - 1)^(-1/2) Plummer lengths (about 22.8 in
    Henon units for 0.999).
    """
    if n < 1:
        raise ValueError("n must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    frac = rng.uniform(0.0, mass_cut, n)
    frac = np.maximum(frac, 1e-300)
    r = 1.0 / np.sqrt(frac ** (-2.0 / 3.0) - 1.0)
    x = r[:, None] * _isotropic(rng, n)
    q = _plummer_speed_fraction(rng, n)
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** -0.25
    v = speed[:, None] * _isotropic(rng, n)
    x *= _PLUMMER_A
    v *= 1.0 / math.sqrt(_PLUMMER_A)
    m = np.full(n, 1.0 / n)
    x -= (m[:, None] * x).sum(axis=0) / m.sum()
    v -= (m[:, None] * v).sum(axis=0) / m.sum()
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


def salpeter_masses(n: int, seed: int, m_lo: float = 0.1, m_hi: float = 100.0,
                    slope: float = 2.35) -> np.ndarray:
    """Masses with dN/dm ~ m^-slope on [m_lo, m_hi], normalised to sum 1.

    Inverse-CDF sampling of the truncated power law.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(0.0, 1.0, n)
    k = 1.0 - slope
    m = (m_lo ** k + u * (m_hi ** k - m_lo ** k)) ** (1.0 / k)
    return m / m.sum()


def two_clusters(n_each: int, seed_a: int, seed_b: int, separation: float = 10.0,
                 rel_speed: float = 0.5):
    """Two Plummer spheres of mass 1/2 each, approaching head-on along x.

    Each sphere keeps the Henon length scale and has its velocities scaled
    by sqrt(1/2), so it stays in virial equilibrium at half the mass. The
    centres start at -separation/2 and +separation/2 and move towards each
    other with relative speed ``rel_speed``; the result is in the
    centre-of-mass frame. Returns (x, v, m) for 2*n_each particles.
    """
    xa, va, ma = plummer(n_each, seed_a)
    xb, vb, mb = plummer(n_each, seed_b)
    s = math.sqrt(0.5)
    va = va * s
    vb = vb * s
    xa = xa + np.array([-0.5 * separation, 0.0, 0.0])
    xb = xb + np.array([+0.5 * separation, 0.0, 0.0])
    va = va + np.array([+0.5 * rel_speed, 0.0, 0.0])
    vb = vb + np.array([-0.5 * rel_speed, 0.0, 0.0])
    x = np.concatenate([xa, xb])
    v = np.concatenate([va, vb])
    m = np.concatenate([ma, mb]) * 0.5
    x -= (m[:, None] * x).sum(axis=0) / m.sum()
    v -= (m[:, None] * v).sum(axis=0) / m.sum()
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


def random_state(n: int, seed: int, scale: float = 1.0):
    """Generic seeded arrays for unit tests of elementwise steps.

    Returns a dict of float64 (n, 3) arrays ``x, v, a, j, s, c`` drawn from
    N(0, scale^2) and masses in (0.5/n, 1.5/n). These have no physical
    meaning; they exercise the predictor and corrector on arbitrary data.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {k: rng.normal(0.0, scale, (n, 3)) for k in ("x", "v", "a", "j", "s", "c")}
    out["m"] = rng.uniform(0.5, 1.5, n) / n
    return out
