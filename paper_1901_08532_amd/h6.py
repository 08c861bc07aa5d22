"""ctypes binding of libh6 (include/h6.h), with the same call names.

Argument marshalling only: every step of the method runs in the HIP
kernels of libh6.so. PyTorch supplies device memory and the stream. If the
library has not been built, importing works but every call raises
``H6Error``; there is no fallback path.

Device layout used by the helpers here (structure of arrays, float64):
  state ``S``: shape (18, n), rows x0 x1 x2 v0 v1 v2 a0.. j0.. s0.. c0..
  masses ``m``: (n,); times ``T``: int64 (2, n), rows t, dt (ticks)
  predicted ``P``: (9, n), rows x, v, a; forces ``F``: (9, n), rows a, j, s
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh6.so")

H6_OK, H6_EINVAL, H6_ENOMEM, H6_EHIP, H6_ESTATE, H6_EDTMIN, H6_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
H6_FP64, H6_MIXED, H6_EX, H6_SP = 0, 1, 2, 3
TICK_BITS = 40
TICKS_PER_UNIT = 1 << TICK_BITS

_P3 = C.c_void_p * 3


class h6_state(C.Structure):
    _fields_ = [("x", _P3), ("v", _P3), ("a", _P3), ("j", _P3), ("s", _P3), ("c", _P3),
                ("m", C.c_void_p), ("t", C.c_void_p), ("dt", C.c_void_p)]


class h6_pred(C.Structure):
    _fields_ = [("x", _P3), ("v", _P3), ("a", _P3)]


class h6_force(C.Structure):
    _fields_ = [("a", _P3), ("j", _P3), ("s", _P3)]


class h6_params(C.Structure):
    _fields_ = [("eta", C.c_double), ("lev_min", C.c_int), ("lev_max", C.c_int),
                ("precision", C.c_int), ("host_loop", C.c_int)]


class h6_run_stats(C.Structure):
    _fields_ = [("blocks", C.c_int64), ("particle_steps", C.c_int64),
                ("interactions", C.c_double), ("t_end", C.c_int64)]


class h6_eval_timing(C.Structure):
    _fields_ = [("order", C.c_int), ("kind", C.c_int), ("block", C.c_int), ("ipl", C.c_int),
                ("precision", C.c_int), ("nact_log2", C.c_int),
                ("launches", C.c_int64), ("interactions", C.c_double), ("kernel_ms", C.c_double),
                ("bytes", C.c_double)]


class H6Error(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        super().__init__("%s failed: %s (%d)%s" % (where, _strerror(code), code,
                                                   (": " + detail) if detail else ""))


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "h6_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int64, C.c_double, C.c_void_p]),
    "h6_destroy": (C.c_int, [C.c_void_p]),
    "h6_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "h6_set_eval_config": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]),
    "h6_predict": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_int64,
                             C.POINTER(h6_pred)]),
    "h6_predict_dt": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_double,
                                C.POINTER(h6_pred)]),
    "h6_evaluate": (C.c_int, [C.c_void_p, C.POINTER(h6_pred), C.c_void_p, C.c_int64, C.c_void_p,
                              C.c_int64, C.c_int, C.POINTER(h6_force)]),
    "h6_correct": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_void_p, C.c_int64,
                             C.POINTER(h6_force), C.c_int64, C.POINTER(h6_params)]),
    "h6_correct_shared": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64,
                                    C.POINTER(h6_force), C.c_double]),
    "h6_init_forces": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64]),
    "h6_initial_steps": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_double,
                                   C.c_int, C.c_int]),
    "h6_next_block": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_void_p,
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "h6_block_step": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.POINTER(h6_pred),
                                C.POINTER(h6_force), C.c_void_p, C.POINTER(h6_params),
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "h6_run_blocks": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.POINTER(h6_pred),
                                C.POINTER(h6_force), C.c_void_p, C.POINTER(h6_params), C.c_int64,
                                C.POINTER(h6_run_stats)]),
    "h6_shared_steps": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.POINTER(h6_pred),
                                  C.POINTER(h6_force), C.c_double, C.c_int64, C.c_int]),
    "h6_energy": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.POINTER(C.c_double)]),
    "h6_check_status": (C.c_int, [C.c_void_p]),
    "h6_evaluate_vjp": (C.c_int, [C.c_void_p, C.POINTER(h6_pred), C.c_void_p, C.c_int64,
                                  C.POINTER(h6_force), C.POINTER(h6_pred), C.c_void_p]),
    "h6_correct_shared_vjp": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64,
                                        C.POINTER(h6_force), C.c_double]),
    "h6_predict_dt_vjp": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64,
                                    C.POINTER(h6_pred), C.c_double]),
    "h6_init_forces_vjp": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64,
                                     C.POINTER(h6_state)]),
    "h6_evaluate_vjp_active": (C.c_int, [C.c_void_p, C.POINTER(h6_pred), C.c_void_p, C.c_int64,
                                         C.c_void_p, C.c_int64, C.POINTER(h6_force),
                                         C.POINTER(h6_pred), C.c_void_p]),
    "h6_correct_vjp": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_void_p,
                                 C.c_int64, C.c_void_p, C.POINTER(h6_force)]),
    "h6_predict_vjp": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_void_p,
                                 C.c_int64, C.POINTER(h6_pred)]),
    "h6_potential": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_void_p]),
    "h6_evaluate_noalloc": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(h6_pred), C.c_void_p,
                                      C.c_int64, C.c_void_p, C.c_int64, C.c_int,
                                      C.POINTER(h6_force)]),
    "h6_energy_vjp": (C.c_int, [C.c_void_p, C.POINTER(h6_state), C.c_int64, C.c_void_p,
                                C.POINTER(h6_state)]),
    "h6_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "h6_profile_read": (C.c_int, [C.c_void_p, C.POINTER(h6_eval_timing), C.c_int,
                                  C.POINTER(C.c_int)]),
    "h6_profile_slots": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "h6_strerror": (C.c_char_p, [C.c_int]),
    "h6_self_pair_masked": (C.c_int, [C.c_double, C.c_int]),
    "h6_last_error": (C.c_char_p, [C.c_void_p]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libh6.so (raises H6Error if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise H6Error(H6_ESTATE, "load", "%s not built (run python -m paper_1901_08532_amd.build)" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().h6_strerror(int(code)).decode()
    except Exception:  # library missing: still give a message
        return "error"


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _rows(t: torch.Tensor, first: int):
    return _P3(t[first].data_ptr(), t[first + 1].data_ptr(), t[first + 2].data_ptr())


def _check_dev(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise H6Error(H6_EINVAL, name, "tensor must be on the GPU")
    if t.dtype != dtype:
        raise H6Error(H6_EINVAL, name, "dtype must be %s" % dtype)
    if not t.is_contiguous():
        raise H6Error(H6_EINVAL, name, "tensor must be contiguous")


def make_state(S: torch.Tensor, m: torch.Tensor, T: torch.Tensor | None) -> h6_state:
    st = h6_state()
    st.x, st.v, st.a = _rows(S, 0), _rows(S, 3), _rows(S, 6)
    st.j, st.s, st.c = _rows(S, 9), _rows(S, 12), _rows(S, 15)
    st.m = m.data_ptr()
    if T is not None:
        st.t = T[0].data_ptr()
        st.dt = T[1].data_ptr()
    return st


def make_pred(P: torch.Tensor) -> h6_pred:
    p = h6_pred()
    p.x, p.v, p.a = _rows(P, 0), _rows(P, 3), _rows(P, 6)
    return p


def make_force(F: torch.Tensor) -> h6_force:
    f = h6_force()
    f.a, f.j, f.s = _rows(F, 0), _rows(F, 3), _rows(F, 6)
    return f


class Context:
    """Owns an h6_ctx: scratch for systems of up to n_max particles."""

    def __init__(self, n_max: int, eps: float, stream: torch.cuda.Stream | None = None):
        self._h = C.c_void_p()
        self.n_max = int(n_max)
        self.eps = float(eps)
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = lib().h6_create(C.byref(self._h), self.n_max, self.eps, C.c_void_p(s.cuda_stream))
        if rc != H6_OK:
            raise H6Error(rc, "h6_create")

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().h6_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, where):
        if rc != H6_OK:
            raise H6Error(rc, where, lib().h6_last_error(self._h).decode())
        return rc

    def set_stream(self, stream: torch.cuda.Stream):
        self._check(lib().h6_set_stream(self._h, C.c_void_p(stream.cuda_stream)), "h6_set_stream")

    def set_eval_config(self, block=0, ipl=0, n_split=0, small_max=-1):
        self._check(lib().h6_set_eval_config(self._h, int(block), int(ipl), int(n_split),
                                             int(small_max)), "h6_set_eval_config")

    # ---- single stages -------------------------------------------------
    def h6_evaluate(self, P, m, active, n_act, precision, F):
        _check_dev(P, torch.float64, "h6_evaluate")
        _check_dev(F, torch.float64, "h6_evaluate")
        n = P.shape[1]
        pr, fo = make_pred(P), make_force(F)
        act = _ptr(active) if active is not None else None
        return self._check(lib().h6_evaluate(self._h, C.byref(pr), _ptr(m), n, act, int(n_act),
                                             int(precision), C.byref(fo)), "h6_evaluate")

    def h6_predict(self, S, m, T, t_tick, P):
        st, pr = make_state(S, m, T), make_pred(P)
        return self._check(lib().h6_predict(self._h, C.byref(st), S.shape[1], int(t_tick),
                                            C.byref(pr)), "h6_predict")

    def h6_predict_dt(self, S, m, dt, P):
        st, pr = make_state(S, m, None), make_pred(P)
        return self._check(lib().h6_predict_dt(self._h, C.byref(st), S.shape[1], float(dt),
                                               C.byref(pr)), "h6_predict_dt")

    def h6_correct(self, S, m, T, active, n_act, F, t_next, eta, lev_min, lev_max,
                   precision=H6_FP64):
        st, fo = make_state(S, m, T), make_force(F)
        prm = h6_params(float(eta), int(lev_min), int(lev_max), int(precision), 0)
        return self._check(lib().h6_correct(self._h, C.byref(st), _ptr(active), int(n_act),
                                            C.byref(fo), int(t_next), C.byref(prm)), "h6_correct")

    def h6_correct_shared(self, S, m, F, dt):
        st, fo = make_state(S, m, None), make_force(F)
        return self._check(lib().h6_correct_shared(self._h, C.byref(st), S.shape[1], C.byref(fo),
                                                   float(dt)), "h6_correct_shared")

    def h6_init_forces(self, S, m):
        st = make_state(S, m, None)
        return self._check(lib().h6_init_forces(self._h, C.byref(st), S.shape[1]), "h6_init_forces")

    def h6_initial_steps(self, S, m, T, eta_s, lev_min, lev_max):
        st = make_state(S, m, T)
        return self._check(lib().h6_initial_steps(self._h, C.byref(st), S.shape[1], float(eta_s),
                                                  int(lev_min), int(lev_max)), "h6_initial_steps")

    def h6_next_block(self, S, m, T, active):
        st = make_state(S, m, T)
        tn, na = C.c_int64(), C.c_int64()
        self._check(lib().h6_next_block(self._h, C.byref(st), S.shape[1], _ptr(active),
                                        C.byref(tn), C.byref(na)), "h6_next_block")
        return tn.value, na.value

    def h6_block_step(self, S, m, T, P, F, active, eta, lev_min, lev_max, precision=H6_FP64):
        st, pr, fo = make_state(S, m, T), make_pred(P), make_force(F)
        prm = h6_params(float(eta), int(lev_min), int(lev_max), int(precision), 0)
        tn, na = C.c_int64(), C.c_int64()
        self._check(lib().h6_block_step(self._h, C.byref(st), S.shape[1], C.byref(pr), C.byref(fo),
                                        _ptr(active), C.byref(prm), C.byref(tn), C.byref(na)),
                    "h6_block_step")
        return tn.value, na.value

    def h6_run_blocks(self, S, m, T, P, F, active, eta, lev_min, lev_max, t_end,
                      precision=H6_FP64, check=True, host_loop=False):
        st, pr, fo = make_state(S, m, T), make_pred(P), make_force(F)
        prm = h6_params(float(eta), int(lev_min), int(lev_max), int(precision),
                        1 if host_loop else 0)
        stats = h6_run_stats()
        rc = lib().h6_run_blocks(self._h, C.byref(st), S.shape[1], C.byref(pr), C.byref(fo),
                                 _ptr(active), C.byref(prm), int(t_end), C.byref(stats))
        if check:
            self._check(rc, "h6_run_blocks")
        return rc, stats

    def h6_shared_steps(self, S, m, P, F, dt, nsteps, precision=H6_FP64):
        st, pr, fo = make_state(S, m, None), make_pred(P), make_force(F)
        return self._check(lib().h6_shared_steps(self._h, C.byref(st), S.shape[1], C.byref(pr),
                                                 C.byref(fo), float(dt), int(nsteps),
                                                 int(precision)), "h6_shared_steps")

    def h6_energy(self, S, m):
        st = make_state(S, m, None)
        out = (C.c_double * 5)()
        self._check(lib().h6_energy(self._h, C.byref(st), S.shape[1], out), "h6_energy")
        return float(out[0]), float(out[1]), [float(out[2]), float(out[3]), float(out[4])]

    # ---- adjoint -------------------------------------------------------
    def h6_evaluate_vjp(self, P, m, CF, GP, gm):
        pr, cf, gp = make_pred(P), make_force(CF), make_pred(GP)
        return self._check(lib().h6_evaluate_vjp(self._h, C.byref(pr), _ptr(m), P.shape[1],
                                                 C.byref(cf), C.byref(gp), _ptr(gm)),
                           "h6_evaluate_vjp")

    def h6_correct_shared_vjp(self, CS, gm, CF, dt):
        cs, cf = make_state(CS, gm, None), make_force(CF)
        return self._check(lib().h6_correct_shared_vjp(self._h, C.byref(cs), CS.shape[1],
                                                       C.byref(cf), float(dt)),
                           "h6_correct_shared_vjp")

    def h6_predict_dt_vjp(self, CS, gm, CP, dt):
        cs, cp = make_state(CS, gm, None), make_pred(CP)
        return self._check(lib().h6_predict_dt_vjp(self._h, C.byref(cs), CS.shape[1], C.byref(cp),
                                                   float(dt)), "h6_predict_dt_vjp")

    def h6_evaluate_vjp_active(self, P, m, active, n_act, CF, GP, gm):
        """Adds to GP (9, n) and gm (n) the VJP of the evaluation of the
        active set; CF holds the cotangents by rank, (9, >= n_act)."""
        _check_dev(P, torch.float64, "h6_evaluate_vjp_active")
        pr, cf, gp = make_pred(P), make_force(CF), make_pred(GP)
        return self._check(lib().h6_evaluate_vjp_active(self._h, C.byref(pr), _ptr(m), P.shape[1],
                                                        _ptr(active), int(n_act), C.byref(cf),
                                                        C.byref(gp), _ptr(gm)),
                           "h6_evaluate_vjp_active")

    def h6_correct_vjp(self, CS, gm, active, n_act, dt_old, CF):
        cs, cf = make_state(CS, gm, None), make_force(CF)
        return self._check(lib().h6_correct_vjp(self._h, C.byref(cs), CS.shape[1], _ptr(active),
                                                int(n_act), _ptr(dt_old), C.byref(cf)),
                           "h6_correct_vjp")

    def h6_predict_vjp(self, CS, gm, t_old, t_tick, CP):
        cs, cp = make_state(CS, gm, None), make_pred(CP)
        return self._check(lib().h6_predict_vjp(self._h, C.byref(cs), CS.shape[1], _ptr(t_old),
                                                int(t_tick), C.byref(cp)), "h6_predict_vjp")

    def h6_potential(self, S, m, phi):
        st = make_state(S, m, None)
        return self._check(lib().h6_potential(self._h, C.byref(st), S.shape[1], _ptr(phi)),
                           "h6_potential")

    def h6_energy_vjp(self, S, m, cot_e, GS, gm):
        """Energy gradient: rows 0-5 of GS (x, v) and gm, scaled by the
        0-d device tensor cot_e (None: 1)."""
        st, gs = make_state(S, m, None), make_state(GS, gm, None)
        ce = _ptr(cot_e) if cot_e is not None else None
        return self._check(lib().h6_energy_vjp(self._h, C.byref(st), S.shape[1], ce, C.byref(gs)),
                           "h6_energy_vjp")

    def h6_init_forces_vjp(self, S, m, CS, gm):
        st, cs = make_state(S, m, None), make_state(CS, gm, None)
        return self._check(lib().h6_init_forces_vjp(self._h, C.byref(st), S.shape[1], C.byref(cs)),
                           "h6_init_forces_vjp")

    def h6_check_status(self):
        return lib().h6_check_status(self._h)

    def h6_profile_enable(self, on=True):
        """on: False/0 off, True/1 evaluation kernels, 2 also the device
        loop's finishing kernels, 3 no events (the device loop's slot log
        only)."""
        level = int(on) if not isinstance(on, bool) else (1 if on else 0)
        self._check(lib().h6_profile_enable(self._h, level), "h6_profile_enable")

    def h6_profile_read(self):
        """List of dicts, one per evaluation-kernel instantiation launched."""
        cap = 1024
        buf = (h6_eval_timing * cap)()
        cnt = C.c_int()
        self._check(lib().h6_profile_read(self._h, buf, cap, C.byref(cnt)), "h6_profile_read")
        return [{k: getattr(buf[q], k) for k, _ in h6_eval_timing._fields_}
                for q in range(min(cnt.value, cap))]

    def h6_profile_slots(self):
        """(n_act, split) of every slot of the last device-loop run (profile
        hook on), as an (S, 2) int32 array; split -1: a prediction slot."""
        cnt = C.c_int()
        self._check(lib().h6_profile_slots(self._h, None, 0, C.byref(cnt)), "h6_profile_slots")
        out = np.zeros((max(cnt.value, 1), 2), dtype=np.int32)
        self._check(lib().h6_profile_slots(self._h, out.ctypes.data, cnt.value, C.byref(cnt)),
                    "h6_profile_slots")
        return out[:cnt.value]


class System:
    """Device-resident particle system driven through libh6.

    Holds the state, masses, times, predicted and force work arrays as
    torch tensors on one GPU, and a Context sized for them.
    """

    def __init__(self, x, v, m, eps, device="cuda", ctx: Context | None = None):
        x = torch.as_tensor(x, dtype=torch.float64)
        v = torch.as_tensor(v, dtype=torch.float64)
        n = x.shape[0]
        self.n = n
        self.eps = float(eps)
        self.device = torch.device(device)
        self.S = torch.zeros((18, n), dtype=torch.float64, device=self.device)
        self.S[0:3] = x.T.to(self.device)
        self.S[3:6] = v.T.to(self.device)
        self.m = torch.as_tensor(m, dtype=torch.float64).to(self.device).contiguous()
        self.T = torch.zeros((2, n), dtype=torch.int64, device=self.device)
        self.P = torch.zeros((9, n), dtype=torch.float64, device=self.device)
        self.F = torch.zeros((9, n), dtype=torch.float64, device=self.device)
        self.active = torch.zeros(n, dtype=torch.int32, device=self.device)
        self.ctx = ctx if ctx is not None else Context(n, eps)

    # views as (n, 3) host arrays for tests and diagnostics
    def field(self, name):
        k = {"x": 0, "v": 3, "a": 6, "j": 9, "s": 12, "c": 15}[name]
        return self.S[k:k + 3].T.cpu().numpy().copy()

    def startup(self, eta_s=None, lev_min=4, lev_max=30):
        self.ctx.h6_init_forces(self.S, self.m)
        if eta_s is not None:
            self.ctx.h6_initial_steps(self.S, self.m, self.T, eta_s, lev_min, lev_max)

    def shared_steps(self, dt, nsteps, precision=H6_FP64):
        self.ctx.h6_shared_steps(self.S, self.m, self.P, self.F, dt, nsteps, precision)

    def block_step(self, eta, lev_min, lev_max, precision=H6_FP64):
        return self.ctx.h6_block_step(self.S, self.m, self.T, self.P, self.F, self.active, eta,
                                      lev_min, lev_max, precision)

    def run_blocks(self, t_end_ticks, eta, lev_min, lev_max, precision=H6_FP64, check=True,
                   host_loop=False):
        return self.ctx.h6_run_blocks(self.S, self.m, self.T, self.P, self.F, self.active, eta,
                                      lev_min, lev_max, t_end_ticks, precision, check, host_loop)

    def energy(self):
        return self.ctx.h6_energy(self.S, self.m)
