"""Pins of the PyTorch-CPU reference gradient (oracle/adjoint_ref.py).

* Its forward pass (start-up and shared steps) equals the C oracle's.
* Its autograd gradient equals central finite differences of the C
  oracle's loss (an independent forward implementation).
* Its autograd gradient equals complex-step derivatives of its own forward
  pass (exact to rounding; independent of autograd).
* The pair-sum VJP helper equals complex-step derivatives, orders 1-3.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint_ref as ar
from paper_1901_08532_amd import ics

EPS2 = 1e-3 ** 2
H = 1.0 / 256


def _case(n, seed, steps):
    x, v, m = ics.plummer(n, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    m = m * rng.uniform(0.5, 1.5, n)
    xt = x + 0.01 * rng.normal(0, 1, (n, 3))
    return x, v, m, xt


def _c_oracle_loss(x, v, m, xt, steps):
    st = oracle.State(x, v, m, EPS2)
    st.startup()
    st.shared_steps(H, steps)
    d = (st.x - xt).ravel()
    return float(np.sum(d * d))


def test_forward_matches_c_oracle():
    x, v, m, _ = _case(24, 3, 8)
    t = [torch.from_numpy(q) for q in (x, v, m)]
    a, j, s, c = ar.startup(*t, EPS2)
    want = oracle.startup(x, v, m, EPS2)
    for got, w in zip((a, j, s, c), want):
        assert np.abs(got.numpy() - w).max() <= 1e-13 * np.abs(w).max()
    fin = ar.run(*t, EPS2, H, 8)
    st = oracle.State(x, v, m, EPS2)
    st.startup()
    st.shared_steps(H, 8)
    for got, w in zip(fin[:5], (st.x, st.v, st.a, st.j, st.s)):
        assert np.abs(got.numpy() - w).max() <= 1e-11 * np.abs(w).max()
    # crackle is a difference quotient 60 (a1 - a0) / h^3 + ...: rounding of
    # a is amplified by about 60 / h^3
    assert np.abs(fin[5].numpy() - st.c).max() <= 1e-13 * 60 * np.abs(st.a).max() / H ** 3


def test_gradient_matches_finite_differences_of_c_oracle():
    n, steps = 12, 6
    x, v, m, xt = _case(n, 4, steps)
    loss, gx, gv, gm = ar.loss_and_grad(x, v, m, xt, EPS2, H, steps)
    assert loss == pytest.approx(_c_oracle_loss(x, v, m, xt, steps), rel=1e-12)
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(6):
        k, c = int(rng.integers(n)), int(rng.integers(3))
        for arr, g in ((x, gx), (v, gv)):
            h = 1e-6
            p, q = arr.copy(), arr.copy()
            p[k, c] += h
            q[k, c] -= h
            args_p = (p, v, m) if arr is x else (x, p, m)
            args_q = (q, v, m) if arr is x else (x, q, m)
            fd = (_c_oracle_loss(*args_p, xt, steps) - _c_oracle_loss(*args_q, xt, steps)) / (2 * h)
            assert abs(fd - g[k, c]) <= 1e-6 * max(1.0, np.abs(g).max()), (k, c, fd, g[k, c])
        h = 1e-6 * m[k]
        p, q = m.copy(), m.copy()
        p[k] += h
        q[k] -= h
        fd = (_c_oracle_loss(x, v, p, xt, steps) - _c_oracle_loss(x, v, q, xt, steps)) / (2 * h)
        assert abs(fd - gm[k]) <= 1e-5 * np.abs(gm).max(), (k, fd, gm[k])


def test_gradient_matches_complex_step():
    n, steps = 10, 5
    x, v, m, xt = _case(n, 6, steps)
    _, gx, gv, gm = ar.loss_and_grad(x, v, m, xt, EPS2, H, steps)
    xtc = torch.from_numpy(xt).to(torch.complex128)

    def cs(which, k, c):
        hh = 1e-30
        xs = [torch.from_numpy(q).to(torch.complex128) for q in (x, v, m)]
        if which == 2:
            xs[2][k] += 1j * hh
        else:
            xs[which][k, c] += 1j * hh
        xT = ar.run(xs[0], xs[1], xs[2], EPS2, H, steps)[0]
        return float(((xT - xtc) ** 2).sum().imag) / hh

    for k in range(n):
        for c in range(3):
            assert cs(0, k, c) == pytest.approx(gx[k, c], rel=1e-9, abs=1e-12)
            assert cs(1, k, c) == pytest.approx(gv[k, c], rel=1e-9, abs=1e-12)
        assert cs(2, k, 0) == pytest.approx(gm[k], rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_pair_sum_vjp_matches_complex_step(order):
    n = 9
    rng = np.random.Generator(np.random.PCG64(10 + order))
    x, v, a, jk = (rng.normal(0, 1, (n, 3)) for _ in range(4))
    m = rng.uniform(0.5, 1.5, n)
    nout = 2 if order != 2 else 3
    cot = [rng.normal(0, 1, (n, 3)) for _ in range(nout)]
    g = ar.pair_sums_vjp(x, v, m, 0.01, cot, a=a, jk=jk, order=order)
    names = ["x", "v", "m"] + (["a"] if order >= 2 else []) + (["jk"] if order == 3 else [])
    base = {"x": x, "v": v, "m": m, "a": a, "jk": jk}
    hh = 1e-30
    for name in names:
        for k in (0, 4, 8):
            for c in (range(3) if name != "m" else [0]):
                ins = {kk: torch.from_numpy(vv).to(torch.complex128) for kk, vv in base.items()}
                if name == "m":
                    ins["m"][k] += 1j * hh
                else:
                    ins[name][k, c] += 1j * hh
                outs = ar.pair_sums(ins["x"], ins["v"], ins["m"], 0.01, a=ins["a"], jk=ins["jk"],
                                    order=order)
                tot = sum((o * torch.from_numpy(cc)).sum() for o, cc in zip(outs, cot))
                d = float(tot.imag) / hh
                want = g[name][k] if name == "m" else g[name][k, c]
                assert d == pytest.approx(want, rel=1e-10, abs=1e-12), (name, k, c)
