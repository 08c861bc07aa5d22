"""Python access to the FP64 CPU oracle (``h6_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may use this module. The HIP library and its
binding never import it, and it imports nothing from them.

``build()`` compiles the C file with gcc (-O2, no FMA contraction, OpenMP)
into ``oracle/liboracle.so``; ``lib()`` loads it, building first when the
library is missing or older than its source. The wrappers below take and
return numpy float64 arrays of shape (n, 3) for vectors.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "h6_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
TICK_BITS = 40

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle; returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        L.orc_pair.argtypes = [dp, dp, dp, dp, C.c_double, C.c_double, C.c_int, dp, dp, dp, dp]
        L.orc_pair.restype = None
        L.orc_forces.argtypes = [C.c_int64, dp, dp, dp, dp, dp, C.c_double, C.c_int64, ip, C.c_int,
                                 dp, dp, dp, dp]
        L.orc_forces.restype = C.c_int
        L.orc_forces_abs.argtypes = L.orc_forces.argtypes
        L.orc_forces_abs.restype = C.c_int
        L.orc_predict.argtypes = [C.c_int64] + [dp] * 10
        L.orc_predict.restype = None
        L.orc_correct.argtypes = [C.c_int64] + [dp] * 14
        L.orc_correct.restype = None
        L.orc_dt_crit6.argtypes = [dp] * 6 + [C.c_double]
        L.orc_dt_crit6.restype = C.c_double
        L.orc_dt_crit4.argtypes = [dp] * 4 + [C.c_double]
        L.orc_dt_crit4.restype = C.c_double
        L.orc_level_of.argtypes = [C.c_double, C.c_int, C.c_int]
        L.orc_level_of.restype = C.c_int
        L.orc_next_level.argtypes = [C.c_int, C.c_int, C.c_int64]
        L.orc_next_level.restype = C.c_int
        L.orc_startup.argtypes = [C.c_int64, dp, dp, dp, C.c_double, dp, dp, dp, dp]
        L.orc_startup.restype = C.c_int
        L.orc_initial_levels.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_double, C.c_int, C.c_int, ip]
        L.orc_initial_levels.restype = C.c_int
        L.orc_next_block.argtypes = [C.c_int64, ip, ip, ip, ip]
        L.orc_next_block.restype = C.c_int64
        L.orc_block_step_flat.argtypes = [C.c_int64] + [dp] * 7 + [ip, ip, C.c_double, C.c_double,
                                                                   C.c_int, C.c_int, ip, ip]
        L.orc_block_step_flat.restype = C.c_int
        L.orc_shared_steps.argtypes = [C.c_int64] + [dp] * 7 + [C.c_double, C.c_double, C.c_int64]
        L.orc_shared_steps.restype = C.c_int
        L.orc_energy.argtypes = [C.c_int64, dp, dp, dp, C.c_double, dp]
        L.orc_energy.restype = C.c_int
        L.orc_potential.argtypes = [C.c_int64, dp, dp, C.c_double, dp]
        L.orc_potential.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "need C-contiguous float64"
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int64 and a.flags.c_contiguous, "need C-contiguous int64"
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _v(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def pair(r, v, a, jr, m, eps2, order=3):
    """Single pair terms (A, J, S, C) of source relative to target."""
    out = [np.zeros(3) for _ in range(4)]
    lib().orc_pair(_d(_v(r)), _d(_v(v)), _d(_v(a)), _d(_v(jr)), float(m), float(eps2), int(order),
                   *[_d(o) for o in out])
    return tuple(out)


def forces(x, v, m, eps2, a=None, jk=None, idx=None, order=2, absolute=False):
    """Sums over j != i of the pair terms for targets idx (default: all).

    Returns (A, J, S, C) arrays of shape (n_i, 3); S is None for order 1 and
    C is None below order 3. absolute=True sums |pair term| per component.
    """
    x, v, m = _v(x), _v(v), _v(m)
    n = x.shape[0]
    if idx is None:
        n_i, ip = n, None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        n_i, ip = idx.shape[0], idx
    A = np.zeros((n_i, 3))
    J = np.zeros((n_i, 3))
    S = np.zeros((n_i, 3)) if order >= 2 else None
    Cc = np.zeros((n_i, 3)) if order >= 3 else None
    fn = lib().orc_forces_abs if absolute else lib().orc_forces
    rc = fn(n, _d(x), _d(v), _d(_v(a)) if a is not None else None,
                          _d(_v(jk)) if jk is not None else None, _d(m), float(eps2), n_i, _i(ip),
                          int(order), _d(A), _d(J), _d(S), _d(Cc))
    if rc:
        raise ValueError("orc_forces failed (%d)" % rc)
    return A, J, S, Cc


def predict(x, v, a, j, s, c, delta):
    x, v, a, j, s, c = (_v(q) for q in (x, v, a, j, s, c))
    n = x.shape[0]
    delta = np.ascontiguousarray(np.broadcast_to(np.asarray(delta, dtype=np.float64), (n,)))
    xp, vp, ap = (np.zeros((n, 3)) for _ in range(3))
    lib().orc_predict(n, _d(x), _d(v), _d(a), _d(j), _d(s), _d(c), _d(delta), _d(xp), _d(vp), _d(ap))
    return xp, vp, ap


def correct(x0, v0, a0, j0, s0, a1, j1, s1, h):
    """Returns (x1, v1, c1, p1, d5a)."""
    arrs = [_v(q) for q in (x0, v0, a0, j0, s0, a1, j1, s1)]
    n = arrs[0].shape[0]
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (n,)))
    outs = [np.zeros((n, 3)) for _ in range(5)]
    lib().orc_correct(n, *[_d(q) for q in arrs], _d(h), *[_d(o) for o in outs])
    return tuple(outs)


def dt_crit6(a, j, s, c, p, d5a, eta):
    return float(lib().orc_dt_crit6(*[_d(_v(q)) for q in (a, j, s, c, p, d5a)], float(eta)))


def dt_crit4(a, j, s, c, eta_s):
    return float(lib().orc_dt_crit4(*[_d(_v(q)) for q in (a, j, s, c)], float(eta_s)))


def level_of(dt, lev_min, lev_cap):
    return int(lib().orc_level_of(float(dt), int(lev_min), int(lev_cap)))


def next_level(lev_old, lev_crit, t1_ticks):
    return int(lib().orc_next_level(int(lev_old), int(lev_crit), int(t1_ticks)))


def startup(x, v, m, eps2):
    """Start-up passes: returns (a, j, s, c) at t = 0."""
    x, v, m = _v(x), _v(v), _v(m)
    n = x.shape[0]
    outs = [np.zeros((n, 3)) for _ in range(4)]
    rc = lib().orc_startup(n, _d(x), _d(v), _d(m), float(eps2), *[_d(o) for o in outs])
    if rc:
        raise ValueError("orc_startup failed (%d)" % rc)
    return tuple(outs)


def initial_levels(a, j, s, c, eta_s, lev_min, lev_max):
    """Returns (rc, dt_ticks[n])."""
    a, j, s, c = (_v(q) for q in (a, j, s, c))
    n = a.shape[0]
    dt = np.zeros(n, dtype=np.int64)
    rc = lib().orc_initial_levels(n, _d(a), _d(j), _d(s), _d(c), float(eta_s), int(lev_min),
                                  int(lev_max), _i(dt))
    return int(rc), dt


def next_block(t, dt):
    t = np.ascontiguousarray(t, dtype=np.int64)
    dt = np.ascontiguousarray(dt, dtype=np.int64)
    n = t.shape[0]
    act = np.zeros(n, dtype=np.int64)
    na = np.zeros(1, dtype=np.int64)
    tn = lib().orc_next_block(n, _i(t), _i(dt), _i(act), _i(na))
    return int(tn), act[: int(na[0])].copy()


class State:
    """Oracle integrator state: numpy arrays, updated in place."""

    def __init__(self, x, v, m, eps2):
        self.x = _v(x).copy()
        self.v = _v(v).copy()
        self.m = _v(m).copy()
        self.eps2 = float(eps2)
        n = self.x.shape[0]
        self.a = np.zeros((n, 3))
        self.j = np.zeros((n, 3))
        self.s = np.zeros((n, 3))
        self.c = np.zeros((n, 3))
        self.t = np.zeros(n, dtype=np.int64)
        self.dt = np.zeros(n, dtype=np.int64)

    @property
    def n(self):
        return self.x.shape[0]

    def copy(self):
        o = State.__new__(State)
        for k, val in self.__dict__.items():
            o.__dict__[k] = val.copy() if isinstance(val, np.ndarray) else val
        return o

    def startup(self, eta_s=None, lev_min=4, lev_max=30):
        self.a, self.j, self.s, self.c = startup(self.x, self.v, self.m, self.eps2)
        if eta_s is not None:
            rc, self.dt = initial_levels(self.a, self.j, self.s, self.c, eta_s, lev_min, lev_max)
            return rc
        return 0

    def shared_steps(self, h, nsteps):
        rc = lib().orc_shared_steps(self.n, _d(self.x), _d(self.v), _d(self.a), _d(self.j),
                                    _d(self.s), _d(self.c), _d(self.m), self.eps2, float(h),
                                    int(nsteps))
        if rc:
            raise ValueError("orc_shared_steps failed (%d)" % rc)

    def block_step(self, eta, lev_min, lev_max):
        """One block step; returns (rc, t_next_ticks, n_act)."""
        tn = np.zeros(1, dtype=np.int64)
        na = np.zeros(1, dtype=np.int64)
        rc = lib().orc_block_step_flat(self.n, _d(self.x), _d(self.v), _d(self.a), _d(self.j),
                                       _d(self.s), _d(self.c), _d(self.m), _i(self.t), _i(self.dt),
                                       self.eps2, float(eta), int(lev_min), int(lev_max), _i(tn),
                                       _i(na))
        return int(rc), int(tn[0]), int(na[0])

    def energy(self):
        return energy(self.x, self.v, self.m, self.eps2)


def potential(x, m, eps2):
    """phi[i] = -sum_{j != i} m_j / sqrt(r_ij^2 + eps2), shape (n,)."""
    x, m = _v(x), _v(m)
    phi = np.zeros(x.shape[0])
    lib().orc_potential(x.shape[0], _d(x), _d(m), float(eps2), _d(phi))
    return phi


def energy(x, v, m, eps2):
    """Returns (ekin, epot, L[3])."""
    x, v, m = _v(x), _v(v), _v(m)
    out = np.zeros(5)
    rc = lib().orc_energy(x.shape[0], _d(x), _d(v), _d(m), float(eps2), _d(out))
    if rc:
        raise ValueError("orc_energy failed (%d)" % rc)
    return float(out[0]), float(out[1]), out[2:5].copy()
