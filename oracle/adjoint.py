"""Oracle reverse-mode gradient through a shared-step leapfrog run.

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
