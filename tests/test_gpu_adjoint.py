"""GPU adjoint (hand-written VJPs behind torch.autograd.Function) against
the PyTorch-CPU FP64 reference gradient and central finite differences.

* Pair VJP of the per-step evaluation, and of the two start-up passes,
  against autograd of the reference pair sums (N = 300): 1e-11 relative.
* One shared step's transposes against autograd of the reference step.
* Whole chain, N = 256, 64 shared steps of 1/256, eps = 1e-3, checkpoint
  every 8 steps: gradient w.r.t. x0, v0, m against the reference gradient.
* N = 16384 (same run): 32 random coordinates (11 of x, 11 of v, 10
  masses) against finite differences of the GPU forward loss: a
  fourth-order central stencil (step 1e-5 for x, v; 1e-3 relative for m)
  to 1e-6 relative, and for x, v also the plain central difference with
  h = 1e-6 to 1e-6 relative plus its rounding-noise floor of 1e-7.
"""

import math

import numpy as np
import pytest
import torch

from oracle import adjoint_ref as ar
from paper_1901_08532_amd import h6, ics
from paper_1901_08532_amd.adjoint import hermite_shared_run
from _gpu import DEV, from_rows, to_rows

pytestmark = pytest.mark.gpu

EPS = 1e-3
DT = 1.0 / 256


def _close(got, want, rtol):
    scale = np.abs(want).max()
    err = np.abs(got - want).max()
    assert err <= rtol * scale, (err, scale, err / scale)


def _rand(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x, v, _ = ics.plummer(n, seed)
    m = rng.uniform(0.5, 1.5, n) / n
    a = rng.normal(0, 1, (n, 3))
    return rng, x, v, a, m


def test_evaluate_vjp_matches_autograd():
    n = 300
    rng, x, v, a, m = _rand(n, 1)
    cot = [rng.normal(0, 1, (n, 3)) for _ in range(3)]
    ref = ar.pair_sums_vjp(x, v, m, EPS ** 2, cot, a=a, order=2)
    ctx = h6.Context(n, EPS)
    P = to_rows(x, v, a)
    CF = to_rows(*cot)
    GP = torch.full((9, n), np.nan, dtype=torch.float64, device=DEV)
    gm = torch.full((n,), 0.25, dtype=torch.float64, device=DEV)  # accumulated into
    ctx.h6_evaluate_vjp(P, torch.from_numpy(m).to(DEV), CF, GP, gm)
    torch.cuda.synchronize()
    _close(from_rows(GP, 0), ref["x"], 1e-11)
    _close(from_rows(GP, 1), ref["v"], 1e-11)
    _close(from_rows(GP, 2), ref["a"], 1e-11)
    _close(gm.cpu().numpy() - 0.25, ref["m"], 1e-11)


def test_init_forces_vjp_matches_autograd():
    n = 300
    rng, x, v, _, m = _rand(n, 2)
    cots = [rng.normal(0, 1, (n, 3)) for _ in range(4)]  # of a, j, s, c
    leaves = [torch.from_numpy(q).clone().requires_grad_(True) for q in (x, v, m)]
    outs = ar.startup(*leaves, EPS ** 2)
    total = sum((o * torch.from_numpy(c)).sum() for o, c in zip(outs, cots))
    gx, gv, gmr = (g.numpy() for g in torch.autograd.grad(total, leaves))
    ctx = h6.Context(n, EPS)
    sysg = h6.System(x, v, m, EPS, ctx=ctx)
    sysg.startup()
    CS = torch.zeros((18, n), dtype=torch.float64, device=DEV)
    CS[6:18] = to_rows(*cots)
    gm = torch.zeros(n, dtype=torch.float64, device=DEV)
    ctx.h6_init_forces_vjp(sysg.S, sysg.m, CS, gm)
    torch.cuda.synchronize()
    _close(from_rows(CS, 0), gx, 1e-11)
    _close(from_rows(CS, 1), gv, 1e-11)
    _close(gm.cpu().numpy(), gmr, 1e-11)


def test_one_shared_step_transposes():
    n = 200
    rng, x, v, _, m = _rand(n, 3)
    st = [torch.from_numpy(q) for q in (x, v)] + [torch.from_numpy(rng.normal(0, s, (n, 3)))
                                                  for s in (1.0, 3.0, 10.0, 30.0)]
    leaves = [t.clone().requires_grad_(True) for t in st] + [torch.from_numpy(m).clone().requires_grad_(True)]
    out = ar.shared_step(*leaves[:6], leaves[6], EPS ** 2, DT)
    cots = [rng.normal(0, 1, (n, 3)) for _ in range(6)]
    total = sum((o * torch.from_numpy(c)).sum() for o, c in zip(out, cots))
    want = [g.numpy() for g in torch.autograd.grad(total, leaves)]
    ctx = h6.Context(n, EPS)
    S = to_rows(*[t.numpy() for t in st])
    mt = torch.from_numpy(m).to(DEV)
    P = torch.empty((9, n), dtype=torch.float64, device=DEV)
    ctx.h6_predict_dt(S, mt, DT, P)
    cot = to_rows(*cots)
    gm = torch.zeros(n, dtype=torch.float64, device=DEV)
    CF = torch.empty((9, n), dtype=torch.float64, device=DEV)
    CP = torch.empty((9, n), dtype=torch.float64, device=DEV)
    ctx.h6_correct_shared_vjp(cot, gm, CF, DT)
    ctx.h6_evaluate_vjp(P, mt, CF, CP, gm)
    ctx.h6_predict_dt_vjp(cot, gm, CP, DT)
    torch.cuda.synchronize()
    # the crackle cotangent enters scaled by 60 / h^3 (about 1e9), so these
    # sums cancel at that scale: 1e-9 of the largest entry
    for k in range(6):
        _close(from_rows(cot, k), want[k], 1e-9)
    _close(gm.cpu().numpy(), want[6], 1e-9)


def _c4_case(n):
    x, v, m = ics.plummer(n, 4)
    rng = np.random.Generator(np.random.PCG64(44))
    xt = x + 0.01 * rng.normal(0, 1, (n, 3))
    return x, v, m, xt


def _gpu_loss_grad(ctx, x, v, m, xt, nsteps, checkpoint=8):
    x0 = torch.from_numpy(x).to(DEV).requires_grad_(True)
    v0 = torch.from_numpy(v).to(DEV).requires_grad_(True)
    mt = torch.from_numpy(m).to(DEV).requires_grad_(True)
    xT = hermite_shared_run(x0, v0, mt, ctx, DT, nsteps, checkpoint)
    loss = ((xT - torch.from_numpy(xt).to(DEV)) ** 2).sum()
    gx, gv, gm = torch.autograd.grad(loss, (x0, v0, mt))
    return float(loss.detach()), gx.cpu().numpy(), gv.cpu().numpy(), gm.cpu().numpy()


def test_full_gradient_n256_matches_reference():
    n = 256
    x, v, m, xt = _c4_case(n)
    ctx = h6.Context(n, EPS)
    loss, gx, gv, gm = _gpu_loss_grad(ctx, x, v, m, xt, 64)
    rloss, rx, rv, rm = ar.loss_and_grad(x, v, m, xt, EPS ** 2, DT, 64)
    assert loss == pytest.approx(rloss, rel=1e-12)
    _close(gx, rx, 1e-9)
    _close(gv, rv, 1e-9)
    _close(gm, rm, 1e-9)
    # checkpoint spacing does not change the result
    _, gx2, gv2, gm2 = _gpu_loss_grad(ctx, x, v, m, xt, 64, checkpoint=5)
    assert np.array_equal(gx, gx2) and np.array_equal(gv, gv2) and np.array_equal(gm, gm2)


def _gpu_loss(ctx, x, v, m, xt, nsteps):
    with torch.no_grad():
        xT = hermite_shared_run(torch.from_numpy(x).to(DEV), torch.from_numpy(v).to(DEV),
                                torch.from_numpy(m).to(DEV), ctx, DT, nsteps)
        d = (xT.cpu().numpy() - xt).ravel()
    return math.fsum(d * d)


def test_c4_gradient_matches_central_differences():
    # Plummer N = 16384, eps = 1e-3, 64 shared steps of 1/256, checkpoint 8
    n = 16384
    x, v, m, xt = _c4_case(n)
    ctx = h6.Context(n, EPS)
    _, gx, gv, gm = _gpu_loss_grad(ctx, x, v, m, xt, 64)
    rng = np.random.Generator(np.random.PCG64(444))
    picks = [("x", int(rng.integers(n)), int(rng.integers(3))) for _ in range(11)]
    picks += [("v", int(rng.integers(n)), int(rng.integers(3))) for _ in range(11)]
    picks += [("m", int(rng.integers(n)), 0) for _ in range(10)]
    arrs = {"x": x, "v": v, "m": m}

    def loss_at(kind, k, c, delta):
        q = {name: a.copy() for name, a in arrs.items()}
        if kind == "m":
            q["m"][k] += delta
        else:
            q[kind][k, c] += delta
        return _gpu_loss(ctx, q["x"], q["v"], q["m"], xt, 64)

    bad = []
    for kind, k, c in picks:
        # fourth-order central stencil: relative step 1e-3 for the masses
        # (m ~ 6e-5), absolute 1e-5 for positions and velocities; truncation
        # and rounding noise both stay near 1e-9 of the derivative
        h = 1e-3 * m[k] if kind == "m" else 1e-5
        fd4 = (8 * (loss_at(kind, k, c, h) - loss_at(kind, k, c, -h))
               - (loss_at(kind, k, c, 2 * h) - loss_at(kind, k, c, -2 * h))) / (12 * h)
        g = {"x": gx, "v": gv}[kind][k, c] if kind != "m" else gm[k]
        if abs(fd4 - g) > 1e-6 * abs(g):
            bad.append(("fd4", kind, k, c, fd4, g, abs(fd4 - g) / abs(g)))
        if kind != "m":
            # plain central difference with h = 1e-6: its rounding noise is
            # about (loss rounding ~4e-14) / 2h = 2e-8, hence the floor
            fd2 = (loss_at(kind, k, c, 1e-6) - loss_at(kind, k, c, -1e-6)) / 2e-6
            if abs(fd2 - g) > 1e-6 * abs(g) + 1e-7:
                bad.append(("fd2", kind, k, c, fd2, g, abs(fd2 - g) / abs(g)))
    assert not bad, bad
