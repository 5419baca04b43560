"""Oracle reverse-mode gradients through a shared-step leapfrog run and through a run on a
fixed block schedule (the second half of this module).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward map is the self-starting leapfrog of Section 2 with one shared step h:
    a_0     = F(r_0, m)
    r_{n+1} = r_n + h v_n + h^2 a_n / 2
    a_{n+1} = F(r_{n+1}, m)
    v_{n+1} = v_n + h (a_n + a_{n+1}) / 2
and the loss is L = sum |r_S - r_target|^2.  The gradient is the chain rule applied to
these equations in reverse order, storing every forward state (no checkpointing), with
the force's vector-Jacobian product taken from ``oracle.force_backward``.
"""
from __future__ import annotations

import numpy as np

from . import force, force_backward


def forward(r0, v0, m, eps, h, nsteps):
    """Return (r_S, states) with states[n] = (r_n, v_n, a_n) for n = 0..S."""
    r = np.array(r0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    a, _ = force(r, m, eps)
    states = [(r, v, a)]
    for _ in range(nsteps):
        r = r + h * v + 0.5 * h * h * a
        a_new, _ = force(r, m, eps)
        v = v + 0.5 * h * (a + a_new)
        a = a_new
        states.append((r, v, a))
    return r, states


def loss(r0, v0, m, eps, h, nsteps, r_target):
    r, _ = forward(r0, v0, m, eps, h, nsteps)
    return float(((r - r_target) ** 2).sum())


def gradient(r0, v0, m, eps, h, nsteps, r_target):
    """(L, dL/dr0 [3,N], dL/dv0 [3,N], dL/dm [N])."""
    m = np.asarray(m, dtype=np.float64)
    n = m.size
    every = np.arange(n, dtype=np.int32)
    r_end, states = forward(r0, v0, m, eps, h, nsteps)
    L = float(((r_end - r_target) ** 2).sum())
    rbar = 2.0 * (r_end - r_target)     # adjoint of r_{n+1}
    vbar = np.zeros_like(rbar)          # adjoint of v_{n+1}
    abar = np.zeros_like(rbar)          # adjoint of a_{n+1} from later steps
    mbar = np.zeros(n)
    for k in range(nsteps - 1, -1, -1):
        r_next = states[k + 1][0]
        # v_{k+1} = v_k + h (a_k + a_{k+1}) / 2 feeds a_{k+1}
        abar_next = abar + 0.5 * h * vbar
        # a_{k+1} = F(r_{k+1}, m)
        gr, gm = force_backward(r_next, m, eps, every, abar_next)
        rbar = rbar + gr
        mbar = mbar + gm
        # step k's inputs: r_k, v_k, a_k
        abar = 0.5 * h * vbar + 0.5 * h * h * rbar
        vbar = vbar + h * rbar
    gr, gm = force_backward(states[0][0], m, eps, every, abar)
    rbar = rbar + gr
    mbar = mbar + gm
    return L, rbar, vbar, mbar


# ----------------------------------------------------------------------------------------
# Fixed block schedule (Section 2's individual power-of-two steps, one pass, Taylor
# prediction of every particle to the block time).  Particle i keeps its step dt_i for the
# whole run; all particles start together at t = 0 with a_0 = F(r_0, m).  At a block time
# t_b the active set is {i : t_last_i + dt_i = t_b}; every particle is predicted with
# h_j = t_b - t_last_j,
#     p_j = r_j + h_j v_j + h_j^2 a_j / 2,
# the active particles get an_i = F_i(p, m) and are corrected
#     r_i <- p_i,  v_i <- v_i + dt_i (a_i + an_i) / 2,  a_i <- an_i,  t_last_i <- t_b,
# and the others keep their state.  With every dt_i equal this is ``forward`` above.


def block_times(dt, t_end):
    """Block times of the schedule: multiples of the smallest step up to t_end."""
    dt = np.asarray(dt, dtype=np.float64)
    hmin = float(dt.min())
    k = int(round(t_end / hmin))
    assert k * hmin == t_end, "t_end must be a multiple of the smallest step"
    return [hmin * (s + 1) for s in range(k)]


def block_forward(r0, v0, m, eps, dt, t_end):
    """(r_end, v_end, trace); trace[s] = (t_b, active, r, v, a, t_last) before block s."""
    r = np.array(r0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    dt = np.asarray(dt, dtype=np.float64)
    n = dt.size
    a, _ = force(r, m, eps)
    t_last = np.zeros(n)
    trace = []
    for t_b in block_times(dt, t_end):
        act = np.nonzero(t_last + dt == t_b)[0].astype(np.int32)
        trace.append((t_b, act, r.copy(), v.copy(), a.copy(), t_last.copy()))
        hh = t_b - t_last
        p = r + v * hh + 0.5 * a * hh * hh
        an, _ = force(p, m, eps, act)
        r[:, act] = p[:, act]
        v[:, act] = v[:, act] + 0.5 * dt[act] * (a[:, act] + an)
        a[:, act] = an
        t_last[act] = t_b
    return r, v, trace


def block_loss(r0, v0, m, eps, dt, t_end, r_target, v_target):
    """L = |r_end - r_target|^2 + |v_end - v_target|^2."""
    r, v, _ = block_forward(r0, v0, m, eps, dt, t_end)
    return float(((r - r_target) ** 2).sum() + ((v - v_target) ** 2).sum())


def block_gradient(r0, v0, m, eps, dt, t_end, r_target, v_target):
    """(L, dL/dr0, dL/dv0, dL/dm) by the chain rule through the block steps in reverse,
    from every stored pre-step state (no checkpointing)."""
    m = np.asarray(m, dtype=np.float64)
    dt = np.asarray(dt, dtype=np.float64)
    n = m.size
    r_end, v_end, trace = block_forward(r0, v0, m, eps, dt, t_end)
    L = float(((r_end - r_target) ** 2).sum() + ((v_end - v_target) ** 2).sum())
    rbar = 2.0 * (r_end - r_target)
    vbar = 2.0 * (v_end - v_target)
    abar = np.zeros_like(rbar)
    mbar = np.zeros(n)
    for (t_b, act, r, v, a, t_last) in reversed(trace):
        hh = t_b - t_last
        p = r + v * hh + 0.5 * a * hh * hh
        # corrector of the active particles: an_i feeds a_i' and v_i'
        seed = abar[:, act] + 0.5 * dt[act] * vbar[:, act]
        pbar = np.zeros_like(rbar)
        pbar[:, act] = rbar[:, act]            # r_i' = p_i
        abar[:, act] = 0.5 * dt[act] * vbar[:, act]  # a_i enters v_i'
        rbar[:, act] = 0.0                      # r_i enters only through p_i
        # an = F(p, m) on the active set
        gr, gm = force_backward(p, m, eps, act, seed)
        pbar += gr
        mbar += gm
        # predictor of every particle
        rbar += pbar
        vbar += hh * pbar
        abar += 0.5 * hh * hh * pbar
    gr, gm = force_backward(np.asarray(r0, dtype=np.float64), m, eps,
                            np.arange(n, dtype=np.int32), abar)
    return L, rbar + gr, vbar, mbar + gm
