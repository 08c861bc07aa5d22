"""h6_evaluate_noalloc (the allocation-free evaluation) against h6_evaluate
through the C ABI: two calls in a row on one GPU, the second smaller, each
within the FP64 bar of the context-based call on the same inputs (the two
share kernels and, at these sizes, launch shapes)."""

import ctypes as C

import numpy as np
import pytest
import torch

from paper_1901_08532_amd import h6, ics
from _gpu import DEV, to_rows, vec_rel_err

pytestmark = pytest.mark.gpu

EPS = 1e-4


def _inputs(n, n_act, seed):
    x, v, m = ics.plummer(n, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    a = rng.normal(0.0, 1.0, (n, 3))
    P = to_rows(x, v, a)
    mt = torch.from_numpy(np.ascontiguousarray(m)).to(DEV)
    act = torch.from_numpy(np.sort(rng.choice(n, n_act, replace=False)).astype(np.int32)).to(DEV)
    return P, mt, act


def _noalloc(P, mt, act, n_act, precision, F):
    pr, fo = h6.make_pred(P), h6.make_force(F)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return h6.lib().h6_evaluate_noalloc(stream, EPS, C.byref(pr), C.c_void_p(mt.data_ptr()),
                                        P.shape[1], C.c_void_p(act.data_ptr()), n_act,
                                        precision, C.byref(fo))


# FP64: the bar against the oracle; mixed: two evaluations, each within the
# mixed form's bounds against FP64 (their slicings may group the FP32
# partial sums differently)
BOUNDS = {h6.H6_FP64: (1e-12, 1e-12, 1e-12), h6.H6_MIXED: (4e-5, 1e-4, 4e-4)}


@pytest.mark.parametrize("precision", [h6.H6_FP64, h6.H6_MIXED])
def test_noalloc_matches_evaluate_on_two_calls(precision):
    for n, n_act, seed in ((20000, 5000, 3), (3000, 700, 4)):
        P, mt, act = _inputs(n, n_act, seed)
        F0 = torch.full((9, n_act), float("nan"), dtype=torch.float64, device=DEV)
        F1 = torch.full((9, n_act), float("nan"), dtype=torch.float64, device=DEV)
        assert _noalloc(P, mt, act, n_act, precision, F1) == h6.H6_OK
        ctx = h6.Context(n, EPS)
        ctx.h6_evaluate(P, mt, act, n_act, precision, F0)
        torch.cuda.synchronize()
        for k in range(3):
            got = F1[3 * k:3 * k + 3].T.cpu().numpy()
            want = F0[3 * k:3 * k + 3].T.cpu().numpy()
            assert np.all(np.isfinite(got))
            assert vec_rel_err(got, want).max() <= BOUNDS[precision][k], (n, k)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    n = 1000
    P, mt, act = _inputs(n, 10, 5)
    F = torch.zeros((9, n), dtype=torch.float64, device=DEV)
    too_many = (32 << 20) // 72 + 1
    assert _noalloc(P, mt, act, too_many, h6.H6_FP64, F) == h6.H6_EINVAL
    assert _noalloc(P, mt, act, 0, h6.H6_FP64, F) == h6.H6_OK
