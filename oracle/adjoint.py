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

from . import force, force_backward, hermite


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


# ----------------------------------------------------------------------------------------
# Block schedules with eras and passes (Section 2's time-symmetric scheme on a given
# schedule).  A schedule lists the initial steps and, per era and pass, the block steps
# (t_b, active set, the active particles' steps after the step), and optionally the
# steps of all particles when each pass starts (a later pass may choose the first step
# of the era again).  Each era is integrated once per listed pass from its start state
# (positions, velocities, accelerations, times and steps).  A pass records, per particle, its era-start state and the state after each
# of its steps (t, r, v, a).  In the first pass every particle is Taylor-predicted to the
# block time; from the second pass on the active particles are still Taylor-predicted from
# their own state (their leapfrog position) and every other particle is taken from the
# previous pass's records: the record itself at a stored time, otherwise the cubic Hermite
# interpolant between the two records that bracket the block time, otherwise (no record
# after the block time) its Taylor prediction.  The era ends with the last pass's state.
# The steps are taken as given (a recorded schedule is replayed; its choice by the
# criterion is not differentiated).  The fixed schedule (every particle keeps dt_i, eras
# of a multiple of the largest step) is one such schedule; with one pass per era it is
# ``block_forward``.


def _records_new(r, v, a, t_last):
    """Per-particle lists of (t, r, v, a), starting with the era-start state."""
    return [[(float(t_last[j]), r[:, j].copy(), v[:, j].copy(), a[:, j].copy())]
            for j in range(r.shape[1])]


def _bracket(recs_j, t):
    """Index of the last record with time <= t (at least 0)."""
    k = 0
    while k + 1 < len(recs_j) and recs_j[k + 1][0] <= t:
        k += 1
    return k


def fixed_schedule(dt, t_end, era, passes):
    """The fixed block schedule (particle i due at every multiple of dt_i) cut into eras of
    length `era` (a multiple of the largest step), `passes` passes per era."""
    dt = np.asarray(dt, dtype=np.float64)
    hmin = float(dt.min())
    assert era % float(dt.max()) == 0.0, "the era must be a multiple of the largest step"
    n_era = int(round(t_end / era))
    assert n_era * era == t_end, "t_end must be a multiple of the era"
    per = int(round(era / hmin))
    eras = []
    for e in range(n_era):
        steps = []
        for s in range(per):
            t_b = e * era + hmin * (s + 1)
            act = np.nonzero(np.mod(t_b, dt) == 0.0)[0].astype(np.int32)
            steps.append((t_b, act, dt[act].copy()))
        eras.append({"passes": [steps] * passes})
    return {"dt0": dt.copy(), "eras": eras}


def _pass(state, m, eps, steps, prev):
    """One pass over an era's block steps from `state` = (r, v, a, t_last, dt), modified in
    place; prev = the previous pass's records or None.  Returns (records, log) with
    log[s] = (t_b, act, pre-step r, v, a, t_last, interpolated: list of (j, k, exact))."""
    r, v, a, t_last, dt = state
    recs = _records_new(r, v, a, t_last)
    log = []
    for (t_b, act, dt_new) in steps:
        act = np.asarray(act, dtype=np.int32)
        due = np.nonzero(t_last + dt == t_b)[0]
        assert np.array_equal(np.sort(act), due), "schedule inconsistent with the steps"
        hh = t_b - t_last
        p = r + v * hh + 0.5 * a * hh * hh
        interp = []
        if prev is not None:
            is_act = np.zeros(dt.size, dtype=bool)
            is_act[act] = True
            for j in np.nonzero(~is_act)[0]:
                k = _bracket(prev[j], t_b)
                tk, rk, vk, ak = prev[j][k]
                if tk == t_b:
                    p[:, j] = rk
                    interp.append((j, k, True))
                elif k + 1 < len(prev[j]):
                    t1, r1, v1, a1 = prev[j][k + 1]
                    p[:, j] = hermite(tk, rk, vk, ak, t1, r1, v1, a1, t_b)[0]
                    interp.append((j, k, False))
        log.append((t_b, act, r.copy(), v.copy(), a.copy(), t_last.copy(), interp))
        an, _ = force(p, m, eps, act)
        h = hh[act]
        r[:, act] = p[:, act]
        v[:, act] = v[:, act] + 0.5 * h * (a[:, act] + an)
        a[:, act] = an
        t_last[act] = t_b
        dt[act] = dt_new
        for i in act:
            recs[i].append((t_b, r[:, i].copy(), v[:, i].copy(), a[:, i].copy()))
    return recs, log


def schedule_forward(r0, v0, m, eps, schedule):
    """(r_end, v_end, eras); eras[e] = (era-start state, [(records, log) per pass])."""
    m = np.asarray(m, dtype=np.float64)
    r = np.array(r0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    a, _ = force(r, m, eps)
    dt = np.array(schedule["dt0"], dtype=np.float64)
    t_last = np.zeros(dt.size)
    out = []
    for era in schedule["eras"]:
        start = (r.copy(), v.copy(), a.copy(), t_last.copy(), dt.copy())
        prev = None
        passes_log = []
        for p, steps in enumerate(era["passes"]):
            r, v, a, t_last, dt = (x.copy() for x in start)
            if "dt_start" in era:
                # steps of the particles when the pass starts (later passes choose the
                # first step of the era again)
                dt = np.array(era["dt_start"][p], dtype=np.float64)
            recs, log = _pass((r, v, a, t_last, dt), m, eps, steps, prev)
            passes_log.append((recs, log))
            prev = recs
        out.append((start, passes_log))
    return r, v, out


def schedule_loss(r0, v0, m, eps, schedule, r_target, v_target):
    r, v, _ = schedule_forward(r0, v0, m, eps, schedule)
    return float(((r - r_target) ** 2).sum() + ((v - v_target) ** 2).sum())


def era_forward(r0, v0, m, eps, dt, t_end, era, passes):
    """The fixed schedule cut into eras (see ``fixed_schedule``)."""
    return schedule_forward(r0, v0, m, eps, fixed_schedule(dt, t_end, era, passes))


def era_loss(r0, v0, m, eps, dt, t_end, era, passes, r_target, v_target):
    return schedule_loss(r0, v0, m, eps, fixed_schedule(dt, t_end, era, passes), r_target,
                         v_target)


def hermite_weights(t0, t1, t):
    """Weights of (r0, v0, r1, v1) in the interpolated position: the interpolant is
    linear in the stored values, so each weight is the interpolant of a unit value."""
    one, zero = np.ones(1), np.zeros(1)
    return tuple(float(hermite(t0, *ends[:3], t1, *ends[3:], t)[0][0]) for ends in (
        (one, zero, zero, zero, zero, zero), (zero, one, zero, zero, zero, zero),
        (zero, zero, zero, one, zero, zero), (zero, zero, zero, zero, one, zero)))


def era_gradient(r0, v0, m, eps, dt, t_end, era, passes, r_target, v_target):
    """``schedule_gradient`` on the fixed schedule cut into eras."""
    return schedule_gradient(r0, v0, m, eps, fixed_schedule(dt, t_end, era, passes),
                             r_target, v_target)


def schedule_gradient(r0, v0, m, eps, schedule, r_target, v_target):
    """(L, dL/dr0, dL/dv0, dL/dm) for L = |r_end - r_target|^2 + |v_end - v_target|^2, by
    the chain rule in reverse: eras last to first, within an era passes last to first.
    A pass's end state only reaches later passes through its records, so the reverse of
    pass p starts from the adjoints of pass p's records (added to the state adjoint at the
    block step that wrote each record) and hands the adjoints of the previous pass's
    records on to it; every pass starts from the era-start state, whose adjoint is the sum
    over the passes (plus the adjoints of the era-start records)."""
    m = np.asarray(m, dtype=np.float64)
    n = m.size
    r_end, v_end, eras = schedule_forward(r0, v0, m, eps, schedule)
    L = float(((r_end - r_target) ** 2).sum() + ((v_end - v_target) ** 2).sum())
    rbar = 2.0 * (r_end - r_target)
    vbar = 2.0 * (v_end - v_target)
    abar = np.zeros_like(rbar)
    mbar = np.zeros(n)
    for start, passes_log in reversed(eras):
        sr, sv, sa = np.zeros_like(rbar), np.zeros_like(rbar), np.zeros_like(rbar)
        rec_bar = None  # adjoints [(R, V)] of the records of the pass being reversed
        for p in range(len(passes_log) - 1, -1, -1):
            recs, steps = passes_log[p]
            prev = passes_log[p - 1][0] if p > 0 else None
            prev_bar = None if prev is None else [
                [[np.zeros(3), np.zeros(3)] for _ in rj] for rj in prev]
            if p < len(passes_log) - 1:
                rb, vb, ab = np.zeros_like(rbar), np.zeros_like(rbar), np.zeros_like(rbar)
            else:
                rb, vb, ab = rbar, vbar, abar
            for (t_b, act, r, v, a, t_last, interp) in reversed(steps):
                if rec_bar is not None:
                    for i in act:
                        k = [q for q, rec in enumerate(recs[i]) if rec[0] == t_b][0]
                        rb[:, i] += rec_bar[i][k][0]
                        vb[:, i] += rec_bar[i][k][1]
                hh = t_b - t_last
                p_pos = r + v * hh + 0.5 * a * hh * hh
                if prev is not None:
                    for (j, k, exact) in interp:
                        if exact:
                            p_pos[:, j] = prev[j][k][1]
                        else:
                            tk, rk, vk, ak = prev[j][k]
                            t1, r1, v1, a1 = prev[j][k + 1]
                            p_pos[:, j] = hermite(tk, rk, vk, ak, t1, r1, v1, a1, t_b)[0]
                h = hh[act]  # the active particles' steps
                seed = ab[:, act] + 0.5 * h * vb[:, act]
                pbar = np.zeros_like(rb)
                pbar[:, act] = rb[:, act]
                ab[:, act] = 0.5 * h * vb[:, act]
                rb[:, act] = 0.0
                gr, gm = force_backward(p_pos, m, eps, act, seed)
                pbar += gr
                mbar += gm
                for (j, k, exact) in interp:
                    if exact:
                        prev_bar[j][k][0] += pbar[:, j]
                    else:
                        w_r0, w_v0, w_r1, w_v1 = hermite_weights(prev[j][k][0],
                                                                  prev[j][k + 1][0], t_b)
                        prev_bar[j][k][0] += w_r0 * pbar[:, j]
                        prev_bar[j][k][1] += w_v0 * pbar[:, j]
                        prev_bar[j][k + 1][0] += w_r1 * pbar[:, j]
                        prev_bar[j][k + 1][1] += w_v1 * pbar[:, j]
                    pbar[:, j] = 0.0
                rb += pbar
                vb += hh * pbar
                ab += 0.5 * hh * hh * pbar
            if rec_bar is not None:
                for j in range(n):
                    rb[:, j] += rec_bar[j][0][0]
                    vb[:, j] += rec_bar[j][0][1]
            sr += rb
            sv += vb
            sa += ab
            rec_bar = prev_bar
        rbar, vbar, abar = sr, sv, sa
    gr, gm = force_backward(np.asarray(r0, dtype=np.float64), m, eps,
                            np.arange(n, dtype=np.int32), abar)
    return L, rbar + gr, vbar, mbar + gm
