"""Closed-form two-body (Kepler) motion in mpmath, for pinning the oracle.

Relative orbit r(t) = x2 - x1 of two point masses with G = 1, total mass
M = m1 + m2, semi-major axis ``sma`` and eccentricity ``e``, pericentre at
t = 0 on the +x axis, motion in the xy plane. Positions come from Kepler's
equation E - e sin E = n t (n = sqrt(M / sma^3)); every time derivative is
taken numerically from that closed form at 40 significant digits, so the
values are independent of any force-law formula.
"""

import mpmath as mp

DPS = 40


class Kepler:
    def __init__(self, m1, m2, sma=1.0, e=0.5):
        mp.mp.dps = DPS
        self.m1 = mp.mpf(m1)
        self.m2 = mp.mpf(m2)
        self.M = self.m1 + self.m2
        self.a = mp.mpf(sma)
        self.e = mp.mpf(e)
        self.n = mp.sqrt(self.M / self.a ** 3)
        self.period = 2 * mp.pi / self.n

    def ecc_anomaly(self, t):
        mean = self.n * t
        E = mean + self.e * mp.sin(mean)
        for _ in range(200):
            f = E - self.e * mp.sin(E) - mean
            E1 = E - f / (1 - self.e * mp.cos(E))
            if abs(E1 - E) < mp.mpf(10) ** (-DPS + 3):
                E = E1
                break
            E = E1
        return E

    def rel(self, t, comp):
        E = self.ecc_anomaly(t)
        if comp == 0:
            return self.a * (mp.cos(E) - self.e)
        if comp == 1:
            return self.a * mp.sqrt(1 - self.e ** 2) * mp.sin(E)
        return mp.mpf(0)

    def rel_deriv(self, t, k):
        """k-th time derivative of the relative position vector at t."""
        mp.mp.dps = DPS
        t = mp.mpf(t)
        return [mp.diff(lambda tt: self.rel(tt, c), t, k) if c < 2 else mp.mpf(0)
                for c in range(3)]

    def bodies(self, t, kmax):
        """Derivatives 0..kmax of both bodies' positions (centre of mass at rest).

        Returns two lists of [x, y, z] float triples: body1[k], body2[k].
        """
        b1, b2 = [], []
        for k in range(kmax + 1):
            d = self.rel_deriv(t, k)
            b1.append([float(-self.m2 / self.M * q) for q in d])
            b2.append([float(self.m1 / self.M * q) for q in d])
        return b1, b2

    def energy(self):
        return float(-self.m1 * self.m2 / (2 * self.a))

    def ang_mom(self):
        mu = self.m1 * self.m2 / self.M
        return float(mu * mp.sqrt(self.M * self.a * (1 - self.e ** 2)))
