"""GPU adjoint of the block-step path (steps held fixed) and energy losses.

* h6_evaluate_vjp_active (2 n_act n pairs) against h6_evaluate_vjp with the
  same cotangents spread over all particles (zero off the active set);
* h6_correct_vjp / h6_predict_vjp against the shared-step transposes when
  every particle has the same step, and untouched off the active set;
* h6_potential against the oracle;
* system_energy and its gradient against the torch reference;
* hermite_block_run: equal to the shared-step adjoint when every particle
  is held on one level; against the torch reference unrolled along the C
  oracle's block sequence (the GPU takes the same sequence); against
  fourth-order central differences at N = 512 (perturbations that keep the
  block sequence);
* an energy loss (energies at both ends) through shared and block runs
  against the reference.
"""

import numpy as np
import pytest
import torch

import oracle
import oracle.adjoint_ref as ar
from paper_1901_08532_amd import h6, ics
from paper_1901_08532_amd.adjoint import hermite_block_run, hermite_shared_run, system_energy
from _gpu import DEV

pytestmark = pytest.mark.gpu

SYNC = 1 << 36  # 1/16 time unit in ticks


def _rel(got, want):
    got, want = np.asarray(got), np.asarray(want)
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))


def _dev(*arrs):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in arrs)


@pytest.mark.parametrize("eps", [1e-4, 0.0])
@pytest.mark.parametrize("n_act", [1, 37, 300, 1000])
def test_active_set_vjp_equals_the_full_vjp(eps, n_act):
    n = 1000
    x, v, m = ics.plummer(n, 11)
    a = oracle.forces(x, v, m, eps * eps, order=1)[0]
    rng = np.random.Generator(np.random.PCG64(n_act))
    act = np.sort(rng.choice(n, n_act, replace=False)).astype(np.int32)
    cot = rng.normal(0, 1, (9, n_act))
    ctx = h6.Context(n, eps)
    P = torch.from_numpy(np.concatenate([x.T, v.T, a.T])).to(DEV).contiguous()
    mt, act_t = _dev(m, act)
    CF = torch.from_numpy(cot).to(DEV).contiguous()
    dense = torch.zeros((9, n), dtype=torch.float64, device=DEV)
    dense[:, act_t.long()] = CF
    G_full = torch.empty((9, n), dtype=torch.float64, device=DEV)
    gm_full = torch.zeros(n, dtype=torch.float64, device=DEV)
    ctx.h6_evaluate_vjp(P, mt, dense, G_full, gm_full)
    G = torch.zeros((9, n), dtype=torch.float64, device=DEV)
    gm = torch.zeros(n, dtype=torch.float64, device=DEV)
    ctx.h6_evaluate_vjp_active(P, mt, act_t, n_act, CF, G, gm)
    torch.cuda.synchronize()
    # the same pair terms, summed in different groupings (the self pair is
    # excluded exactly by both)
    for r in range(3):
        assert _rel(G[3 * r:3 * r + 3].cpu(), G_full[3 * r:3 * r + 3].cpu()) <= 1e-11, r
    assert _rel(gm.cpu(), gm_full.cpu()) <= 1e-11


def test_block_transposes_reduce_to_the_shared_ones():
    n = 777
    rng = np.random.Generator(np.random.PCG64(5))
    ctx = h6.Context(n, 1e-4)
    lev = 9
    dt_ticks = 1 << (40 - lev)
    T = torch.zeros((2, n), dtype=torch.int64, device=DEV)
    T[0] = 3 * dt_ticks
    T[1] = dt_ticks
    cot0 = torch.from_numpy(rng.normal(0, 1, (18, n))).to(DEV)
    gm = torch.zeros(n, dtype=torch.float64, device=DEV)
    act = torch.arange(n, dtype=torch.int32, device=DEV)
    # corrector, all particles active
    c1, c2 = cot0.clone(), cot0.clone()
    F1 = torch.empty((9, n), dtype=torch.float64, device=DEV)
    F2 = torch.empty((9, n), dtype=torch.float64, device=DEV)
    ctx.h6_correct_vjp(c1, gm, act, n, T[1], F1)
    ctx.h6_correct_shared_vjp(c2, gm, F2, 2.0 ** -lev)
    torch.cuda.synchronize()
    assert torch.allclose(c1, c2, rtol=1e-14, atol=0) and torch.allclose(F1, F2, rtol=1e-14, atol=0)
    # predictor over one step from t_old = t - dt
    CP = torch.from_numpy(rng.normal(0, 1, (9, n))).to(DEV)
    p1, p2 = cot0.clone(), cot0.clone()
    ctx.h6_predict_vjp(p1, gm, T[0], 4 * dt_ticks, CP)
    ctx.h6_predict_dt_vjp(p2, gm, CP, 2.0 ** -lev)
    torch.cuda.synchronize()
    assert torch.allclose(p1, p2, rtol=1e-14, atol=0)
    # a subset: other particles untouched, active ones as in the full call
    sub = torch.from_numpy(np.sort(rng.choice(n, 100, replace=False)).astype(np.int32)).to(DEV)
    c3 = cot0.clone()
    F3 = torch.empty((9, 100), dtype=torch.float64, device=DEV)
    ctx.h6_correct_vjp(c3, gm, sub, 100, T[1], F3)
    torch.cuda.synchronize()
    mask = torch.zeros(n, dtype=torch.bool, device=DEV)
    mask[sub.long()] = True
    assert torch.equal(c3[:, ~mask], cot0[:, ~mask])
    assert torch.equal(c3[:, mask], c1[:, mask])
    assert torch.equal(F3, F1[:, sub.long()])


@pytest.mark.parametrize("eps", [1e-4, 0.0])
def test_potential_matches_the_oracle(eps):
    n = 1000
    x, v, m = ics.plummer(n, 12)
    m = ics.salpeter_masses(n, 122)
    ctx = h6.Context(n, eps)
    S = torch.zeros((18, n), dtype=torch.float64, device=DEV)
    S[0:3] = torch.from_numpy(x.T).to(DEV)
    (mt,) = _dev(m)
    phi = torch.empty(n, dtype=torch.float64, device=DEV)
    ctx.h6_potential(S, mt, phi)
    want = oracle.potential(x, m, eps * eps)
    assert _rel(phi.cpu().numpy(), want) <= 1e-13


def test_system_energy_and_its_gradient():
    n = 256
    x, v, m = ics.plummer(n, 13)
    m = ics.salpeter_masses(n, 133)
    eps = 1e-3
    ctx = h6.Context(n, eps)
    xt, vt, mt = (t.requires_grad_(True) for t in _dev(x, v, m))
    e = system_energy(xt, vt, mt, ctx)
    gx, gv, gm = torch.autograd.grad(e, (xt, vt, mt))
    xr, vr, mr = (torch.from_numpy(a).clone().requires_grad_(True) for a in (x, v, m))
    er = ar.energy(xr, vr, mr, eps * eps)
    rx, rv, rm = torch.autograd.grad(er, (xr, vr, mr))
    assert float(e.detach()) == pytest.approx(float(er.detach()), rel=1e-13)
    for g, r in ((gx, rx), (gv, rv), (gm, rm)):
        assert _rel(g.cpu().numpy(), r.numpy()) <= 1e-11


@pytest.mark.parametrize("n,cot", [(1, None), (257, None), (1000, 2.5)])
def test_energy_vjp_call_against_the_reference(n, cot):
    # the ABI call itself: every gradient component on the device, scaled by
    # a cotangent held in device memory (NULL: 1), against the autograd
    # gradient of the torch reference energy (n = 257: a ragged tile)
    x, v, m = ics.plummer(max(n, 2), 17 + n)
    x, v, m = x[:n], v[:n], m[:n]
    eps = 1e-3
    ctx = h6.Context(n, eps)
    S = torch.zeros((18, n), dtype=torch.float64, device=DEV)
    S[0:3] = torch.from_numpy(np.ascontiguousarray(x.T)).to(DEV)
    S[3:6] = torch.from_numpy(np.ascontiguousarray(v.T)).to(DEV)
    mt = torch.from_numpy(np.ascontiguousarray(m)).to(DEV)
    GS = torch.full((18, n), float("nan"), dtype=torch.float64, device=DEV)
    gm = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    ce = None if cot is None else torch.tensor(cot, dtype=torch.float64, device=DEV)
    ctx.h6_energy_vjp(S, mt, ce, GS, gm)
    xr, vr, mr = (torch.from_numpy(a).clone().requires_grad_(True) for a in (x, v, m))
    rx, rv, rm = torch.autograd.grad(ar.energy(xr, vr, mr, eps * eps), (xr, vr, mr))
    g = 1.0 if cot is None else cot
    assert _rel(GS[0:3].T.cpu().numpy(), g * rx.numpy()) <= 1e-11
    assert _rel(GS[3:6].T.cpu().numpy(), g * rv.numpy()) <= 1e-15
    assert _rel(gm.cpu().numpy(), g * rm.numpy()) <= 1e-11
    assert torch.isnan(GS[6:]).all()  # only x, v (and m) are written


def _block_grads(ctx, x, v, m, t_end, loss_fn, **kw):
    xt, vt, mt = (t.requires_grad_(True) for t in _dev(x, v, m))
    xT, vT = hermite_block_run(xt, vt, mt, ctx, t_end, **kw)
    loss = loss_fn(xT, vT, xt, vt, mt)
    grads = torch.autograd.grad(loss, (xt, vt, mt))
    return (float(loss.detach()),) + tuple(g.cpu().numpy() for g in grads)


def _sq_loss(xT, vT, *_):
    return (xT ** 2).sum() + 0.5 * (vT ** 2).sum()


def test_block_adjoint_on_one_level_equals_the_shared_adjoint():
    n = 256
    x, v, m = ics.plummer(n, 14)
    ctx = h6.Context(n, 1e-2)
    lb, gxb, gvb, gmb = _block_grads(ctx, x, v, m, SYNC, _sq_loss, lev_min=8, lev_max=8)
    xt, vt, mt = (t.requires_grad_(True) for t in _dev(x, v, m))
    xT, vT = hermite_shared_run(xt, vt, mt, ctx, 2.0 ** -8, 16, checkpoint=5,
                                return_velocities=True)
    ls = _sq_loss(xT, vT)
    gxs, gvs, gms = (g.cpu().numpy() for g in torch.autograd.grad(ls, (xt, vt, mt)))
    assert lb == pytest.approx(float(ls.detach()), rel=1e-13)
    for gb, gs in ((gxb, gxs), (gvb, gvs), (gmb, gms)):
        assert _rel(gb, gs) <= 1e-10


def _gpu_sequence(ctx, x, v, m, t_end, eta=0.4, lev_min=4, lev_max=30):
    s = h6.System(x, v, m, ctx.eps, ctx=ctx)
    s.startup(eta_s=0.1, lev_min=lev_min, lev_max=lev_max)
    seq = []
    while True:
        tn, na = ctx.h6_next_block(s.S, s.m, s.T, s.active)
        if tn > t_end:
            return seq
        seq.append((tn, tuple(sorted(s.active[:na].cpu().numpy().tolist()))))
        s.block_step(eta, lev_min, lev_max)


def test_block_adjoint_matches_the_reference_along_the_oracle_sequence():
    n = 64
    x, v, m = ics.plummer(n, 15)
    eps = 1e-3
    ctx = h6.Context(n, eps)
    sched = ar.block_schedule(x, v, m, eps * eps, SYNC)
    assert len(sched) > 8
    assert _gpu_sequence(ctx, x, v, m, SYNC) == [(t, tuple(sorted(a.tolist()))) for t, a, _, _ in sched]
    lg, gx, gv, gm = _block_grads(ctx, x, v, m, SYNC, _sq_loss)
    xr, vr, mr = (torch.from_numpy(a).clone().requires_grad_(True) for a in (x, v, m))
    out = ar.block_run(xr, vr, mr, eps * eps, sched)
    lr = _sq_loss(out[0], out[1])
    rx, rv, rm = torch.autograd.grad(lr, (xr, vr, mr))
    assert lg == pytest.approx(float(lr.detach()), rel=1e-12)
    for g, r in ((gx, rx), (gv, rv), (gm, rm)):
        assert _rel(g, r.numpy()) <= 1e-9


def test_block_adjoint_matches_central_differences():
    n = 512
    x, v, m = ics.plummer(n, 16)
    eps = 1e-3
    ctx = h6.Context(n, eps)
    _, gx, gv, gm = _block_grads(ctx, x, v, m, SYNC, _sq_loss)
    base = _gpu_sequence(ctx, x, v, m, SYNC)
    assert len(set(len(a) for _, a in base)) > 1

    def loss_at(q):
        with torch.no_grad():
            xT, vT = hermite_block_run(*_dev(q["x"], q["v"], q["m"]), ctx, SYNC)
        return float(_sq_loss(xT, vT)), _gpu_sequence(ctx, q["x"], q["v"], q["m"], SYNC)

    rng = np.random.Generator(np.random.PCG64(166))
    picks = [("x", int(rng.integers(n)), int(rng.integers(3))) for _ in range(4)]
    picks += [("v", int(rng.integers(n)), int(rng.integers(3))) for _ in range(4)]
    picks += [("m", int(rng.integers(n)), 0) for _ in range(3)]
    checked = 0
    for kind, i, c in picks:
        h = 1e-3 * m[i] if kind == "m" else 1e-5
        vals, same = [], True
        for k in (1, -1, 2, -2):
            q = {"x": x.copy(), "v": v.copy(), "m": m.copy()}
            if kind == "m":
                q["m"][i] += k * h
            else:
                q[kind][i, c] += k * h
            val, seq = loss_at(q)
            same = same and seq == base
            vals.append(val)
        if not same:  # the perturbation moved a step: not a frozen-step derivative
            continue
        fd = (8 * (vals[0] - vals[1]) - (vals[2] - vals[3])) / (12 * h)
        g = {"x": gx, "v": gv}[kind][i, c] if kind != "m" else gm[i]
        assert g == pytest.approx(fd, rel=1e-6, abs=1e-9), (kind, i, c)
        checked += 1
    assert checked >= 8


@pytest.mark.parametrize("mode", ["shared", "block"])
def test_energy_loss_matches_the_reference(mode):
    # loss E(t) - E(0) / 2 over one sync interval: energies at both ends
    n = 64
    x, v, m = ics.plummer(n, 17)
    eps = 1e-3
    ctx = h6.Context(n, eps)
    xt, vt, mt = (t.requires_grad_(True) for t in _dev(x, v, m))
    if mode == "shared":
        xT, vT = hermite_shared_run(xt, vt, mt, ctx, 2.0 ** -8, 16, return_velocities=True)
    else:
        xT, vT = hermite_block_run(xt, vt, mt, ctx, SYNC)
    loss = system_energy(xT, vT, mt, ctx) - 0.5 * system_energy(xt, vt, mt, ctx)
    g = [t.cpu().numpy() for t in torch.autograd.grad(loss, (xt, vt, mt))]
    xr, vr, mr = (torch.from_numpy(a).clone().requires_grad_(True) for a in (x, v, m))
    if mode == "shared":
        out = ar.run(xr, vr, mr, eps * eps, 2.0 ** -8, 16)
    else:
        out = ar.block_run(xr, vr, mr, eps * eps, ar.block_schedule(x, v, m, eps * eps, SYNC))
    lr = ar.energy(out[0], out[1], mr, eps * eps) - 0.5 * ar.energy(xr, vr, mr, eps * eps)
    r = [t.numpy() for t in torch.autograd.grad(lr, (xr, vr, mr))]
    assert float(loss.detach()) == pytest.approx(float(lr.detach()), rel=1e-12)
    for gg, rr in zip(g, r):
        assert _rel(gg, rr) <= 1e-9


def test_edge_cases_of_the_block_adjoint_calls():
    n = 2
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    v = np.zeros((2, 3))
    m = np.array([2.0, 5.0])
    ctx = h6.Context(n, 0.0)
    S = torch.zeros((18, n), dtype=torch.float64, device=DEV)
    S[0:3] = torch.from_numpy(x.T).to(DEV)
    (mt,) = _dev(m)
    phi = torch.empty(n, dtype=torch.float64, device=DEV)
    ctx.h6_potential(S, mt, phi)
    assert np.allclose(phi.cpu().numpy(), [-1.0, -0.4], rtol=1e-15, atol=0)
    # empty active set: the VJP and the corrector transpose change nothing
    P = S[0:9].contiguous()
    G = torch.zeros((9, n), dtype=torch.float64, device=DEV)
    gm = torch.zeros(n, dtype=torch.float64, device=DEV)
    none = torch.zeros(1, dtype=torch.int32, device=DEV)
    CF = torch.zeros((9, 1), dtype=torch.float64, device=DEV)
    ctx.h6_evaluate_vjp_active(P, mt, none, 0, CF, G, gm)
    cot = torch.ones((18, n), dtype=torch.float64, device=DEV)
    dt = torch.full((n,), 1 << 30, dtype=torch.int64, device=DEV)
    ctx.h6_correct_vjp(cot, gm, none, 0, dt, CF)
    torch.cuda.synchronize()
    assert not G.any() and not gm.any() and bool((cot == 1).all())
    # bad sizes are refused
    with pytest.raises(h6.H6Error):
        ctx.h6_evaluate_vjp_active(P, mt, none, 3, CF, G, gm)
    with pytest.raises(h6.H6Error):
        ctx.h6_correct_vjp(cot, gm, none, -1, dt, CF)


def test_block_run_with_no_block_before_the_end_time():
    # t_end before the first block: the result is the initial state, and the
    # gradient of sum |x|^2 + |v|^2 / 2 is (2 x0, v0, 0)
    n = 32
    x, v, m = ics.plummer(n, 18)
    ctx = h6.Context(n, 1e-3)
    loss, gx, gv, gm = _block_grads(ctx, x, v, m, 0, _sq_loss)
    assert loss == pytest.approx(float((x ** 2).sum() + 0.5 * (v ** 2).sum()), rel=1e-14)
    assert np.allclose(gx, 2 * x, rtol=1e-15, atol=0)
    assert np.allclose(gv, v, rtol=1e-15, atol=0)
    assert not np.any(gm)
