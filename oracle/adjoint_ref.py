"""Plain PyTorch CPU float64 reference of the shared-step Hermite-6
integrator, differentiated by autograd.

TEST INFRASTRUCTURE ONLY (as the C oracle): it gives the reference
gradient of a loss on final positions with respect to initial positions,
velocities and masses, through the start-up passes and the unrolled
predict / evaluate / correct steps. Dense all-pairs tensors, so it is meant
for a few hundred particles. Written independently of both the C oracle
and the HIP library; its forward pass is pinned to the C oracle and its
gradient to finite differences of the C oracle and to complex-step
derivatives of itself.

The arithmetic follows the same statement of the method as the C oracle:
softened pair acceleration and its time derivatives summed over all other
particles (self term excluded), Taylor predictor, 6th-order Hermite
corrector with crackle from the quintic interpolant, start-up passes for
a, j then s, c.
"""

from __future__ import annotations

import torch


def pair_sums(x, v, m, eps2, a=None, jk=None, order=2):
    """Sums over j != i of the pair terms, all targets.

    order 1 -> (A, J); order 2 -> (A, J, S); order 3 -> (S, C).
    Tensors are (n, 3) (x, v, a, jk) and (n,) (m); float64 or complex128.
    """
    n = x.shape[0]
    eye = torch.eye(n, dtype=torch.float64)
    off = 1.0 - eye
    r = x[None, :, :] - x[:, None, :]  # r[i, j] = x_j - x_i
    vv = v[None, :, :] - v[:, None, :]
    R2 = (r * r).sum(-1) + eps2 + eye  # diagonal made harmless, then masked
    Rinv = R2 ** -0.5
    Rinv2 = Rinv * Rinv
    mR3 = m[None, :] * Rinv * Rinv2 * off
    alpha = (r * vv).sum(-1) * Rinv2
    A = mR3[..., None] * r
    J = mR3[..., None] * vv - 3.0 * alpha[..., None] * A
    if order == 1:
        return A.sum(1), J.sum(1)
    aa = a[None, :, :] - a[:, None, :]
    beta = ((vv * vv).sum(-1) + (r * aa).sum(-1)) * Rinv2 + alpha * alpha
    S = mR3[..., None] * aa - 6.0 * alpha[..., None] * J - 3.0 * beta[..., None] * A
    if order == 2:
        return A.sum(1), J.sum(1), S.sum(1)
    jj = jk[None, :, :] - jk[:, None, :]
    gamma = (3.0 * (vv * aa).sum(-1) + (r * jj).sum(-1)) * Rinv2 + alpha * (3.0 * beta - 4.0 * alpha * alpha)
    C = (mR3[..., None] * jj - 9.0 * alpha[..., None] * S - 9.0 * beta[..., None] * J
         - 3.0 * gamma[..., None] * A)
    return S.sum(1), C.sum(1)


def startup(x, v, m, eps2):
    a, j = pair_sums(x, v, m, eps2, order=1)
    s, c = pair_sums(x, v, m, eps2, a=a, jk=j, order=3)
    return a, j, s, c


def shared_step(x, v, a, j, s, c, m, eps2, h):
    # predictor: Taylor series over the step
    xp = x + h * v + h ** 2 / 2 * a + h ** 3 / 6 * j + h ** 4 / 24 * s + h ** 5 / 120 * c
    vp = v + h * a + h ** 2 / 2 * j + h ** 3 / 6 * s + h ** 4 / 24 * c
    ap = a + h * j + h ** 2 / 2 * s + h ** 3 / 6 * c
    a1, j1, s1 = pair_sums(xp, vp, m, eps2, a=ap, order=2)
    # corrector (two-point Hermite quadrature) and crackle at the step end
    v1 = v + h / 2 * (a + a1) - h ** 2 / 10 * (j1 - j) + h ** 3 / 120 * (s + s1)
    x1 = x + h / 2 * (v + v1) - h ** 2 / 10 * (a1 - a) + h ** 3 / 120 * (j + j1)
    c1 = (60.0 * (a1 - a) - h * (24.0 * j + 36.0 * j1) + h ** 2 * (9.0 * s1 - 3.0 * s)) / h ** 3
    return x1, v1, a1, j1, s1, c1


def run(x0, v0, m, eps2, h, nsteps):
    """Start-up plus nsteps shared steps; returns the final state tuple."""
    a, j, s, c = startup(x0, v0, m, eps2)
    x, v = x0, v0
    for _ in range(nsteps):
        x, v, a, j, s, c = shared_step(x, v, a, j, s, c, m, eps2, h)
    return x, v, a, j, s, c


TICK = 2.0 ** -40


def block_schedule(x0, v0, m, eps2, t_end, eta=0.4, lev_min=4, lev_max=30, eta_s=0.1):
    """The block sequence the C oracle takes from the start-up to t_end
    (ticks): a list of (t_next, active indices, particle times before the
    block, particle steps before the block). Used to unroll block_run."""
    from . import State, next_block

    st = State(x0, v0, m, eps2)
    st.startup(eta_s, lev_min, lev_max)
    sched = []
    while True:
        tn, act = next_block(st.t, st.dt)
        if tn > t_end:
            break
        sched.append((tn, act.copy(), st.t.copy(), st.dt.copy()))
        rc, _, _ = st.block_step(eta, lev_min, lev_max)
        if rc < 0 and rc != -5:  # -5: a step clamped at 2^-lev_max (run continues)
            raise ValueError("oracle block step failed (%d)" % rc)
    return sched


def block_run(x0, v0, m, eps2, schedule):
    """Start-up, then the blocks of `schedule` with their steps held fixed:
    per block, every particle predicted over its own interval to t_next,
    a, j, s evaluated at the predicted states, and the active particles
    corrected over their own steps. Returns the final (x, v, a, j, s, c)."""
    a, j, s, c = startup(x0, v0, m, eps2)
    x, v = x0, v0
    n = x.shape[0]
    for tn, act, t_old, dt_old in schedule:
        d = torch.as_tensor((tn - t_old) * TICK, dtype=torch.float64)[:, None]
        xp = x + d * v + d ** 2 / 2 * a + d ** 3 / 6 * j + d ** 4 / 24 * s + d ** 5 / 120 * c
        vp = v + d * a + d ** 2 / 2 * j + d ** 3 / 6 * s + d ** 4 / 24 * c
        ap = a + d * j + d ** 2 / 2 * s + d ** 3 / 6 * c
        a1, j1, s1 = pair_sums(xp, vp, m, eps2, a=ap, order=2)
        h = torch.as_tensor(dt_old * TICK, dtype=torch.float64)[:, None]
        v1 = v + h / 2 * (a + a1) - h ** 2 / 10 * (j1 - j) + h ** 3 / 120 * (s + s1)
        x1 = x + h / 2 * (v + v1) - h ** 2 / 10 * (a1 - a) + h ** 3 / 120 * (j + j1)
        c1 = (60.0 * (a1 - a) - h * (24.0 * j + 36.0 * j1) + h ** 2 * (9.0 * s1 - 3.0 * s)) / h ** 3
        mask = torch.zeros(n, dtype=torch.bool)
        mask[torch.as_tensor(act, dtype=torch.int64)] = True
        mk = mask[:, None]
        x, v = torch.where(mk, x1, x), torch.where(mk, v1, v)
        a, j, s, c = (torch.where(mk, new, old) for new, old in ((a1, a), (j1, j), (s1, s), (c1, c)))
    return x, v, a, j, s, c


def energy(x, v, m, eps2):
    """Kinetic plus softened potential energy (pairs i < j), a 0-d tensor."""
    n = x.shape[0]
    r = x[None, :, :] - x[:, None, :]
    R = ((r * r).sum(-1) + eps2) ** -0.5
    iu = torch.triu_indices(n, n, offset=1)
    pot = -(m[iu[0]] * m[iu[1]] * R[iu[0], iu[1]]).sum()
    return 0.5 * (m * (v * v).sum(-1)).sum() + pot


def loss_and_grad(x0, v0, m, x_target, eps2, h, nsteps):
    """Loss sum |x_T - x_target|^2 and its gradient w.r.t. (x0, v0, m)."""
    x0 = torch.as_tensor(x0, dtype=torch.float64).clone().requires_grad_(True)
    v0 = torch.as_tensor(v0, dtype=torch.float64).clone().requires_grad_(True)
    m = torch.as_tensor(m, dtype=torch.float64).clone().requires_grad_(True)
    xt = torch.as_tensor(x_target, dtype=torch.float64)
    xT = run(x0, v0, m, eps2, h, nsteps)[0]
    loss = ((xT - xt) ** 2).sum()
    gx, gv, gm = torch.autograd.grad(loss, (x0, v0, m))
    return float(loss.detach()), gx.numpy(), gv.numpy(), gm.numpy()


def pair_sums_vjp(x, v, m, eps2, cot, a=None, jk=None, order=2):
    """Autograd VJP of pair_sums: gradient of sum(outputs * cot) w.r.t. the
    inputs; returns dict with keys x, v, m (and a, jk when used)."""
    ins = {"x": x, "v": v, "m": m}
    if order >= 2:
        ins["a"] = a
    if order == 3:
        ins["jk"] = jk
    leaves = {k: torch.as_tensor(t, dtype=torch.float64).clone().requires_grad_(True)
              for k, t in ins.items()}
    outs = pair_sums(leaves["x"], leaves["v"], leaves["m"], eps2, a=leaves.get("a"),
                     jk=leaves.get("jk"), order=order)
    total = sum((o * torch.as_tensor(c, dtype=torch.float64)).sum() for o, c in zip(outs, cot))
    grads = torch.autograd.grad(total, list(leaves.values()))
    return {k: g.numpy() for k, g in zip(leaves, grads)}
