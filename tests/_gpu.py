"""Shared helpers of the GPU parity tests (inputs, error measures)."""

import numpy as np
import torch

import oracle
from paper_1901_08532_amd import h6, ics

DEV = "cuda"


def to_rows(*arrs):
    """(n,3) host arrays -> one (3k, n) float64 device tensor."""
    return torch.from_numpy(np.concatenate([np.ascontiguousarray(a.T) for a in arrs])).to(DEV).contiguous()


def from_rows(t, k):
    """Rows 3k..3k+2 of a (., n) device tensor as an (n, 3) host array."""
    return t[3 * k:3 * k + 3].T.cpu().numpy().copy()


def vec_rel_err(got, want):
    """Per-particle |got - want| / |want| (vector norms), shape (n,)."""
    num = np.linalg.norm(got - want, axis=1)
    den = np.linalg.norm(want, axis=1)
    return num / np.where(den > 0, den, 1.0)


def plummer_pred(n, seed, eps2):
    """Plummer x, v and the oracle's start-up acceleration as predicted a."""
    x, v, m = ics.plummer(n, seed)
    a, _, _, _ = oracle.forces(x, v, m, eps2, order=1)
    return x, v, a, m


def gpu_evaluate(ctx, x, v, a, m, active=None, n_act=None, precision=h6.H6_FP64):
    n = x.shape[0]
    P = to_rows(x, v, a)
    mt = torch.from_numpy(np.ascontiguousarray(m)).to(DEV)
    if active is None:
        n_act = n if n_act is None else n_act
        act_t = None
    else:
        act_t = torch.from_numpy(np.ascontiguousarray(active, dtype=np.int32)).to(DEV)
        n_act = len(active)
    F = torch.full((9, max(n_act, 1)), np.nan, dtype=torch.float64, device=DEV)
    ctx.h6_evaluate(P, mt, act_t, n_act, precision, F)
    torch.cuda.synchronize()
    return from_rows(F, 0)[:n_act], from_rows(F, 1)[:n_act], from_rows(F, 2)[:n_act]
