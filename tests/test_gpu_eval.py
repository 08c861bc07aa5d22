"""GPU parity of the a/j/s evaluation against the FP64 oracle.

Bound: per target particle, |F_gpu - F_oracle| / |F_oracle| <= 1e-12 for
F = a, j, s (FP64 path), on seeded Plummer inputs. Small systems are
compared on every target; full-size systems on sampled targets that the
oracle evaluates one by one. Launch shapes are swept and each shape is
checked for bitwise reproducibility.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1901_08532_amd import h6
from _gpu import DEV, gpu_evaluate, plummer_pred, to_rows, vec_rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12
EPS = 1e-4


def _check(got, want, tol=TOL):
    for name, g, w in zip("ajs", got, want):
        err = vec_rel_err(g, w)
        assert np.all(np.isfinite(g)), name
        assert err.max() <= tol, (name, float(err.max()), int(err.argmax()))


@pytest.mark.parametrize("n", [1, 2, 63, 255, 1024, 3001])
def test_all_targets_small(n):
    x, v, a, m = plummer_pred(n, 10 + n, EPS ** 2)
    ctx = h6.Context(n, EPS)
    got = gpu_evaluate(ctx, x, v, a, m)
    if n == 1:  # a lone particle feels nothing
        for g in got:
            assert np.array_equal(g, np.zeros((1, 3)))
        return
    want = oracle.forces(x, v, m, EPS ** 2, a=a, order=2)[:3]
    _check(got, want)


@pytest.mark.parametrize("n,n_act", [(1000, 1), (1000, 7), (4099, 300), (4099, 4099)])
def test_active_subsets(n, n_act):
    x, v, a, m = plummer_pred(n, 20 + n_act, EPS ** 2)
    rng = np.random.Generator(np.random.PCG64(n_act))
    act = np.sort(rng.choice(n, n_act, replace=False)).astype(np.int32)
    ctx = h6.Context(n, EPS)
    got = gpu_evaluate(ctx, x, v, a, m, active=act)
    want = oracle.forces(x, v, m, EPS ** 2, a=a, idx=act.astype(np.int64), order=2)[:3]
    _check(got, want)


def test_unequal_masses_zero_softening():
    # eps = 0 takes the explicit self-exclusion path
    n = 2000
    x, v, a, _ = plummer_pred(n, 31, 0.0)
    from paper_1901_08532_amd import ics
    m = ics.salpeter_masses(n, 32)
    ctx = h6.Context(n, 0.0)
    got = gpu_evaluate(ctx, x, v, a, m)
    want = oracle.forces(x, v, m, 0.0, a=a, order=2)[:3]
    _check(got, want)


@pytest.mark.parametrize("block,ipl,split", [(64, 1, 1), (64, 2, 3), (128, 1, 5), (128, 2, 1),
                                             (256, 1, 2), (256, 2, 7), (256, 1, 64)])
def test_launch_shapes_agree_and_are_deterministic(block, ipl, split):
    n = 2500
    x, v, a, m = plummer_pred(n, 40, EPS ** 2)
    ctx = h6.Context(n, EPS)
    ctx.set_eval_config(block, ipl, split)
    got1 = gpu_evaluate(ctx, x, v, a, m)
    got2 = gpu_evaluate(ctx, x, v, a, m)
    for g1, g2 in zip(got1, got2):
        assert np.array_equal(g1, g2)
    want = oracle.forces(x, v, m, EPS ** 2, a=a, order=2)[:3]
    _check(got1, want)


@pytest.mark.parametrize("n_act", [1, 2, 3, 5, 8, 13, 32, 33])
@pytest.mark.parametrize("small_max", [0, 64])
def test_small_active_sets_both_kernels(n_act, small_max):
    # small_max 64: source-parallel kernel; 0: LDS-tiled kernel with many slices
    n = 5000
    x, v, a, m = plummer_pred(n, 200 + n_act, EPS ** 2)
    rng = np.random.Generator(np.random.PCG64(300 + n_act))
    act = rng.choice(n, n_act, replace=False).astype(np.int32)  # unsorted on purpose
    ctx = h6.Context(n, EPS)
    ctx.set_eval_config(small_max=small_max)
    got = gpu_evaluate(ctx, x, v, a, m, active=act)
    again = gpu_evaluate(ctx, x, v, a, m, active=act)
    for g1, g2 in zip(got, again):
        assert np.array_equal(g1, g2)
    want = oracle.forces(x, v, m, EPS ** 2, a=a, idx=act.astype(np.int64), order=2)[:3]
    _check(got, want)


def test_small_kernel_zero_softening():
    n = 3000
    x, v, a, _ = plummer_pred(n, 33, 0.0)
    from paper_1901_08532_amd import ics
    m = ics.salpeter_masses(n, 34)
    act = np.array([0, 1, 2999, 1500, 7], dtype=np.int32)
    ctx = h6.Context(n, 0.0)
    got = gpu_evaluate(ctx, x, v, a, m, active=act)
    want = oracle.forces(x, v, m, 0.0, a=a, idx=act.astype(np.int64), order=2)[:3]
    _check(got, want)


def test_empty_active_set_is_noop():
    n = 100
    x, v, a, m = plummer_pred(n, 41, EPS ** 2)
    ctx = h6.Context(n, EPS)
    P = torch.zeros((9, n), dtype=torch.float64, device="cuda")
    F = torch.full((9, 4), 7.0, dtype=torch.float64, device="cuda")
    act = torch.zeros(4, dtype=torch.int32, device="cuda")
    mt = torch.ones(n, dtype=torch.float64, device="cuda")
    ctx.h6_evaluate(P, mt, act, 0, h6.H6_FP64, F)
    torch.cuda.synchronize()
    assert torch.all(F == 7.0)


@pytest.mark.parametrize("n", [65536, 262144])
def test_full_size_sampled_targets(n):
    x, v, m = __import__("paper_1901_08532_amd.ics", fromlist=["plummer"]).plummer(n, 2)
    rng = np.random.Generator(np.random.PCG64(5))
    a = rng.normal(0.0, 1.0, (n, 3))  # any predicted acceleration
    ctx = h6.Context(n, EPS)
    got = gpu_evaluate(ctx, x, v, a, m)
    idx = np.sort(rng.choice(n, 256, replace=False))
    want = oracle.forces(x, v, m, EPS ** 2, a=a, idx=idx, order=2)[:3]
    _check([g[idx] for g in got], want)


def test_bad_arguments_rejected():
    ctx = h6.Context(16, EPS)
    P = torch.zeros((9, 32), dtype=torch.float64, device="cuda")
    F = torch.zeros((9, 32), dtype=torch.float64, device="cuda")
    mt = torch.ones(32, dtype=torch.float64, device="cuda")
    with pytest.raises(h6.H6Error) as ei:
        ctx.h6_evaluate(P, mt, None, 32, h6.H6_FP64, F)  # n = 32 > n_max
    assert ei.value.code == h6.H6_EINVAL
    with pytest.raises(h6.H6Error):
        ctx.h6_evaluate(P[:, :16].contiguous(), mt, None, 16, 7, F)


def test_context_on_side_streams():
    # a context made on one side stream, then moved to another with
    # h6_set_stream, enqueues its work there: a copy ordered on that stream
    # alone reads the finished sums, equal bit for bit to the default
    # stream's (streams at the default priority)
    n = 3000
    x, v, a, m = plummer_pred(n, 31, EPS ** 2)
    ref = gpu_evaluate(h6.Context(n, EPS), x, v, a, m)
    P = to_rows(x, v, a)
    mt = torch.from_numpy(np.ascontiguousarray(m)).to(DEV)
    torch.cuda.synchronize()  # inputs complete before other streams read them
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ctx = h6.Context(n, EPS, stream=s1)
    for k, s in enumerate((s1, s2)):
        if k:
            ctx.set_stream(s)
        with torch.cuda.stream(s):
            F = torch.full((9, n), np.nan, dtype=torch.float64, device=DEV)
            ctx.h6_evaluate(P, mt, None, n, h6.H6_FP64, F)
            out = F.cpu().numpy()
        for c in range(3):
            assert np.array_equal(out[3 * c:3 * c + 3].T, ref[c]), (k, c)


def test_evaluate_rejects_bad_sizes_before_any_launch():
    # sizes are validated on the host: n_act above n without an active
    # list, negative n_act, n or n_act above the context's n_max
    n = 100
    x, v, a, m = plummer_pred(n, 33, EPS ** 2)
    P = to_rows(x, v, a)
    mt = torch.from_numpy(np.ascontiguousarray(m)).to(DEV)
    F = torch.zeros((9, 2 * n), dtype=torch.float64, device=DEV)
    ctx = h6.Context(2 * n, EPS)
    for n_act in (n + 1, -1, 2 * n + 1):
        with pytest.raises(h6.H6Error) as e:
            ctx.h6_evaluate(P, mt, None, n_act, h6.H6_FP64, F)
        assert e.value.code == h6.H6_EINVAL
    small = h6.Context(n - 1, EPS)
    with pytest.raises(h6.H6Error) as e:
        small.h6_evaluate(P, mt, None, 1, h6.H6_FP64, F)
    assert e.value.code == h6.H6_EINVAL
    assert torch.count_nonzero(F).item() == 0  # nothing was written
