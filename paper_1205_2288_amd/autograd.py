"""torch.autograd Functions over the HIP force adjoint.

* ``TsbtsForce``: acceleration and potential of an active set for explicit positions and
  masses; backward calls ``tsbts_force_backward`` (tidal-tensor products).
* ``TsbtsLeapfrog``: a shared-step leapfrog run (Section 2's self-starting leapfrog with
  one step h for all particles) from (r0, v0, m) to (r_S, v_S).  The forward pass keeps
  only era-start checkpoints (r, v, a every `era` steps); the backward pass recomputes
  each era from its checkpoint and sweeps it in reverse with the element-wise leapfrog
  adjoint kernel and the force adjoint kernel.

* ``TsbtsBlockLeapfrog``: a run on a fixed block schedule (Section 2's individual
  power-of-two steps, one pass, every particle predicted by its Taylor polynomial to each
  block time, force and leapfrog corrector on the active set), all particles starting
  together at t = 0.  Same checkpointing; the reverse sweep restores each block step's
  pre-step state, predicts, and runs ``tsbts_block_adjoint`` around the force adjoint.
* ``TsbtsScheduleLeapfrog``: a run on a given block schedule with eras and several passes
  (Section 2's time-symmetric scheme: from the second pass on the non-active particles
  are interpolated from the previous pass's stored states), e.g. the schedule the
  criterion chose in a run of ``driver.TSBTS(record_schedule=True)``, replayed; or the
  fixed schedule cut into eras (``tsbts_era_leapfrog``).  The reverse sweep of a pass
  also moves the adjoints of interpolated positions into the adjoints of the previous
  pass's records (``tsbts_interp_adjoint``) and adds those back at the block steps that
  wrote them (``tsbts_record_adjoint``).

All arithmetic runs in libtsbts kernels; torch provides the tensors and the graph.
"""
from __future__ import annotations

import numpy as np
import torch

from .context import Context


class TsbtsForce(torch.autograd.Function):
    """acc[3, k], pot[k] = force(r[3, N], m[N]) on the targets idx (int32 device tensor)."""

    @staticmethod
    def forward(fctx, r, m, idx, ctx: Context):
        r = r.detach().contiguous()
        m = m.detach().contiguous()
        ctx.load_positions(r, m, 0.0)
        acc, pot = ctx.force(idx, 0.0)
        fctx.save_for_backward(r, m, idx)
        fctx.tsbts = ctx
        return acc, pot

    @staticmethod
    def backward(fctx, g_acc, g_pot):
        r, m, idx = fctx.saved_tensors
        ctx = fctx.tsbts
        ctx.load_positions(r, m, 0.0)
        if g_acc is None:
            g_acc = torch.zeros((3, idx.numel()), dtype=torch.float64, device=r.device)
        gr, gm = ctx.force_backward(idx, 0.0, g_acc.contiguous(),
                                    None if g_pot is None else g_pot.contiguous())
        return gr, gm, None, None


def tsbts_force(r, m, idx, ctx: Context):
    return TsbtsForce.apply(r, m, idx, ctx)


class TsbtsLeapfrog(torch.autograd.Function):
    """(r_S, v_S) after `steps` shared leapfrog steps of size h, with era checkpoints."""

    @staticmethod
    def forward(fctx, r0, v0, m, ctx: Context, h: float, steps: int, era: int):
        n = ctx.n
        dev = ctx.device
        r0, v0, m = (x.detach().contiguous() for x in (r0, v0, m))
        ctx.bind(r0.clone(), v0.clone(), m.clone(), t_last=torch.zeros(n, dtype=torch.float64,
                                                                        device=dev),
                 dt=torch.full((n,), h, dtype=torch.float64, device=dev))
        every = ctx.idx(torch.arange(n, dtype=torch.int32))
        acc = torch.empty((3, n), dtype=torch.float64, device=dev)
        ctx.predict(0.0)
        ctx.force(every, 0.0, with_pot=False, acc=acc)
        ctx.a.copy_(acc)
        checkpoints = []
        for s in range(steps):
            if s % era == 0:
                checkpoints.append((s, ctx.r.clone(), ctx.v.clone(), ctx.a.clone()))
            _step(ctx, every, acc, s, h)
        fctx.tsbts = ctx
        fctx.meta = (h, steps, era)
        fctx.checkpoints = checkpoints
        fctx.save_for_backward(m)
        fctx.every = every
        return ctx.r.clone(), ctx.v.clone()

    @staticmethod
    def backward(fctx, g_r, g_v):
        ctx = fctx.tsbts
        (m,) = fctx.saved_tensors
        h, steps, era = fctx.meta
        n = ctx.n
        dev = ctx.device
        every = fctx.every
        z = lambda: torch.zeros((3, n), dtype=torch.float64, device=dev)  # noqa: E731
        rbar = z() if g_r is None else g_r.contiguous().clone()
        vbar = z() if g_v is None else g_v.contiguous().clone()
        abar = z()
        g = z()
        mbar = torch.zeros(n, dtype=torch.float64, device=dev)
        acc = torch.empty((3, n), dtype=torch.float64, device=dev)
        ctx.bind(ctx.r, ctx.v, m, a=ctx.a, t_last=ctx.t_last, dt=ctx.dt)
        for (s0, r_c, v_c, a_c) in reversed(fctx.checkpoints):
            s1 = min(s0 + era, steps)
            # recompute the era from its checkpoint, keeping the positions of every step
            ctx.r.copy_(r_c)
            ctx.v.copy_(v_c)
            ctx.a.copy_(a_c)
            ctx.t_last.fill_(s0 * h)
            pos = []
            for s in range(s0, s1):
                _step(ctx, every, acc, s, h)
                pos.append(ctx.r.clone())
            for s in range(s1 - 1, s0 - 1, -1):
                ctx.leapfrog_adjoint(0, h, rbar, vbar, abar, g)      # g = abar + h vbar / 2
                ctx.load_positions(pos[s - s0], m, 0.0)
                ctx.force_backward(every, 0.0, g, None, rbar, mbar)  # through a_{s+1}
                ctx.leapfrog_adjoint(1, h, rbar, vbar, abar, g)      # adjoints of step s
        ctx.load_positions(fctx.checkpoints[0][1], m, 0.0)
        ctx.force_backward(every, 0.0, abar, None, rbar, mbar)      # through a_0
        return rbar, vbar, mbar, None, None, None, None


def _step(ctx: Context, every, acc, s: int, h: float):
    tb = (s + 1) * h
    ctx.predict(tb)
    ctx.force(every, tb, with_pot=False, acc=acc)
    ctx.correct(every, tb, acc)


def tsbts_leapfrog(r0, v0, m, ctx: Context, h: float, steps: int, era: int = 16):
    return TsbtsLeapfrog.apply(r0, v0, m, ctx, h, steps, era)


class BlockSchedule:
    """Fixed block schedule: step dt_i = hmin * 2^level_i per particle, block times
    (s + 1) * hmin for s = 0 .. K-1, K = t_end / hmin.  At block s the active set is
    {i : level_i <= trailing zeros of s + 1} (particle i is due at every multiple of dt_i)."""

    def __init__(self, ctx: Context, dt, t_end: float):
        dt = np.asarray(dt.cpu().numpy() if isinstance(dt, torch.Tensor) else dt,
                        dtype=np.float64).reshape(-1)
        if dt.size != ctx.n or not np.all(dt > 0):
            raise ValueError("dt must hold one positive step per particle")
        self.hmin = float(dt.min())
        lev = np.log2(dt / self.hmin)
        self.level = np.rint(lev).astype(np.int64)
        if not np.array_equal(self.hmin * 2.0 ** self.level, dt):
            raise ValueError("every step must be the smallest step times a power of two")
        k = t_end / self.hmin
        self.K = int(round(k))
        if self.K < 1 or self.K * self.hmin != t_end:
            raise ValueError("t_end must be a positive multiple of the smallest step")
        self.dt = dt
        self.lmax = int(self.level.max())
        self.sets = [ctx.idx(np.nonzero(self.level <= L)[0].astype(np.int32))
                     for L in range(self.lmax + 1)]

    def time(self, s: int) -> float:
        return (s + 1) * self.hmin

    def active(self, s: int):
        b = s + 1
        tz = (b & -b).bit_length() - 1
        return self.sets[min(tz, self.lmax)]


def _block_step(ctx: Context, sched: BlockSchedule, s: int, buf, use_history=False):
    tb = sched.time(s)
    idx = sched.active(s)
    k = idx.numel()
    acc = buf[:3 * k].view(3, k)
    ctx.predict(tb, use_history)
    ctx.force(idx, tb, with_pot=False, acc=acc)
    ctx.correct(idx, tb, acc)


class TsbtsBlockLeapfrog(torch.autograd.Function):
    """(r, v) at t_end after a run on the fixed block schedule given by dt (per-particle
    power-of-two steps), with a checkpoint every `era` block steps."""

    @staticmethod
    def forward(fctx, r0, v0, m, ctx: Context, dt, t_end: float, era: int):
        n = ctx.n
        dev = ctx.device
        sched = BlockSchedule(ctx, dt, t_end)
        r0, v0, m = (x.detach().contiguous() for x in (r0, v0, m))
        ctx.bind(r0.clone(), v0.clone(), m.clone(),
                 t_last=torch.zeros(n, dtype=torch.float64, device=dev),
                 dt=torch.tensor(sched.dt, dtype=torch.float64, device=dev))
        every = ctx.idx(torch.arange(n, dtype=torch.int32))
        buf = torch.empty(3 * n, dtype=torch.float64, device=dev)
        acc = buf.view(3, n)
        ctx.predict(0.0)
        ctx.force(every, 0.0, with_pot=False, acc=acc)
        ctx.a.copy_(acc)
        checkpoints = []
        for s in range(sched.K):
            if s % era == 0:
                checkpoints.append((s, ctx.r.clone(), ctx.v.clone(), ctx.a.clone(),
                                    ctx.t_last.clone()))
            _block_step(ctx, sched, s, buf)
        fctx.tsbts = ctx
        fctx.sched = sched
        fctx.era = era
        fctx.checkpoints = checkpoints
        fctx.every = every
        fctx.save_for_backward(m)
        return ctx.r.clone(), ctx.v.clone()

    @staticmethod
    def backward(fctx, g_r, g_v):
        ctx, sched, era = fctx.tsbts, fctx.sched, fctx.era
        (m,) = fctx.saved_tensors
        n = ctx.n
        dev = ctx.device
        z = lambda: torch.zeros((3, n), dtype=torch.float64, device=dev)  # noqa: E731
        rbar = z() if g_r is None else g_r.contiguous().clone()
        vbar = z() if g_v is None else g_v.contiguous().clone()
        abar = z()
        pbar = z()
        mbar = torch.zeros(n, dtype=torch.float64, device=dev)
        buf = torch.empty(3 * n, dtype=torch.float64, device=dev)
        seeds = torch.empty(3 * n, dtype=torch.float64, device=dev)
        first = fctx.checkpoints[0]
        ctx.bind(first[1].clone(), first[2].clone(), m, a=first[3].clone(),
                 t_last=first[4].clone(), dt=torch.tensor(sched.dt, dtype=torch.float64,
                                                          device=dev))
        state = (ctx.r, ctx.v, ctx.a, ctx.t_last)
        for (s0, *ck) in reversed(fctx.checkpoints):
            s1 = min(s0 + era, sched.K)
            for dst, src in zip(state, ck):
                dst.copy_(src)
            pre = []
            for s in range(s0, s1):
                pre.append([x.clone() for x in state])
                _block_step(ctx, sched, s, buf)
            for s in range(s1 - 1, s0 - 1, -1):
                for dst, src in zip(state, pre[s - s0]):
                    dst.copy_(src)
                tb = sched.time(s)
                idx = sched.active(s)
                k = idx.numel()
                sd = seeds[:3 * k].view(3, k)
                ctx.predict(tb)
                ctx.block_adjoint(0, idx, tb, rbar, vbar, abar, pbar, sd)
                ctx.force_backward(idx, tb, sd, None, pbar, mbar)
                ctx.block_adjoint(1, None, tb, rbar, vbar, abar, pbar, None)
        ctx.load_positions(first[1], m, 0.0)
        ctx.force_backward(fctx.every, 0.0, abar, None, rbar, mbar)   # through a_0
        return rbar, vbar, mbar, None, None, None, None


def tsbts_block_leapfrog(r0, v0, m, ctx: Context, dt, t_end: float, era: int = 16):
    return TsbtsBlockLeapfrog.apply(r0, v0, m, ctx, dt, t_end, era)


def _state(ctx: Context):
    return (ctx.r, ctx.v, ctx.a, ctx.t_last, ctx.dt)


def _restore(ctx: Context, saved):
    for dst, src in zip(_state(ctx), saved):
        dst.copy_(src)


def fixed_schedule(dt, t_end: float, era: float, passes: int):
    """The fixed block schedule (particle i due at every multiple of dt_i, steps kept) cut
    into eras of length `era` (a multiple of the largest step that divides t_end), as a
    schedule for tsbts_schedule_leapfrog."""
    dt = np.asarray(dt.cpu().numpy() if isinstance(dt, torch.Tensor) else dt,
                    dtype=np.float64).reshape(-1)
    if dt.size == 0 or not np.all(dt > 0):
        raise ValueError("dt must hold one positive step per particle")
    hmin = float(dt.min())
    level = np.rint(np.log2(dt / hmin))
    if not np.array_equal(hmin * 2.0 ** level, dt):
        raise ValueError("every step must be the smallest step times a power of two")
    per = era / hmin
    n_era = t_end / era if era > 0 else 0.0
    if (passes < 1 or era <= 0 or era % float(dt.max()) != 0.0 or per != int(per)
            or n_era != int(n_era) or n_era < 1):
        raise ValueError("era must be a multiple of the largest step and divide t_end; "
                         "passes >= 1")
    eras = []
    for e in range(int(n_era)):
        steps = []
        for k in range(int(per)):
            tb = e * era + hmin * (k + 1)
            act = np.flatnonzero(np.mod(tb, dt) == 0.0).astype(np.int32)
            steps.append((tb, act, dt[act].copy()))
        eras.append({"passes": [steps] * passes})
    return {"dt0": dt.copy(), "eras": eras}


class _DeviceSchedule:
    """A schedule ({"dt0": steps, "eras": [{"passes": [[(t_b, active, new steps), ...]],
    "dt_start": [steps of all particles when each pass starts] (optional)}]},
    as recorded by driver.TSBTS(record_schedule=True)) with its index and step arrays on the
    device."""

    def __init__(self, ctx: Context, schedule):
        dev = ctx.device
        self.dt0 = torch.tensor(np.asarray(schedule["dt0"], dtype=np.float64), device=dev)
        if self.dt0.numel() != ctx.n:
            raise ValueError("the schedule's initial steps must cover every particle")
        cache = {}
        self.eras = []
        self.pass_dt = []  # per era and pass: the steps when the pass starts, or None
        for era in schedule["eras"]:
            starts = era.get("dt_start")
            self.pass_dt.append([
                None if starts is None else
                torch.tensor(np.asarray(starts[p], dtype=np.float64), device=dev)
                for p in range(len(era["passes"]))])
            passes = []
            for steps in era["passes"]:
                dev_steps = []
                for (tb, act, dtn) in steps:
                    key = id(act)
                    if key not in cache:
                        cache[key] = (ctx.idx(np.asarray(act, dtype=np.int32)), act)
                    dev_steps.append((float(tb), cache[key][0],
                                      torch.tensor(np.asarray(dtn, dtype=np.float64),
                                                   device=dev)))
                passes.append(dev_steps)
            if not passes:
                raise ValueError("every era needs at least one pass")
            self.eras.append(passes)


def _sched_pass(ctx: Context, steps, buf, use_history: bool, record: bool, pre=None,
                dt_start=None):
    """One pass over the listed block steps; record = keep its states as the next pass's
    interpolation source; pre = list receiving each step's pre-step state; dt_start =
    the steps of all particles when the pass starts (None: those of the state)."""
    if dt_start is not None:
        ctx.dt.copy_(dt_start)
    if record:
        ctx.history_begin()
    for (tb, idx, dtn) in steps:
        if pre is not None:
            pre.append([x.clone() for x in _state(ctx)])
        k = idx.numel()
        acc = buf[:3 * k].view(3, k)
        ctx.predict(tb, use_history)
        ctx.force(idx, tb, with_pot=False, acc=acc)
        ctx.correct(idx, tb, acc)
        ctx.set_dt(idx, dtn)
    if record:
        ctx.history_end()


class TsbtsScheduleLeapfrog(torch.autograd.Function):
    """(r, v) at the end of a run on a given block schedule with eras and passes (Section
    2's time-symmetric scheme): each era is integrated once per listed pass from its start
    state; the first pass Taylor-predicts every particle, later passes take the non-active
    particles from the previous pass's stored states (cubic Hermite interpolation).  The
    schedule (block times, active sets, steps) is replayed, not re-chosen: its choice by
    the criterion is piecewise constant and not differentiated.  The forward keeps the
    era-start states; the backward sweeps each era's passes in reverse, recomputing the
    interpolation source of each pass from the era start."""

    @staticmethod
    def forward(fctx, r0, v0, m, ctx: Context, sched: _DeviceSchedule):
        n = ctx.n
        dev = ctx.device
        r0, v0, m = (x.detach().contiguous() for x in (r0, v0, m))
        ctx.bind(r0.clone(), v0.clone(), m.clone(),
                 t_last=torch.zeros(n, dtype=torch.float64, device=dev),
                 dt=sched.dt0.clone())
        every = ctx.idx(torch.arange(n, dtype=torch.int32))
        buf = torch.empty(3 * n, dtype=torch.float64, device=dev)
        acc = buf.view(3, n)
        ctx.predict(0.0)
        ctx.force(every, 0.0, with_pot=False, acc=acc)
        ctx.a.copy_(acc)
        starts = []
        for passes in sched.eras:
            start = [x.clone() for x in _state(ctx)]
            starts.append(start)
            ctx.history_clear()
            for p, steps in enumerate(passes):
                if p:
                    _restore(ctx, start)
                _sched_pass(ctx, steps, buf, p > 0, p < len(passes) - 1,
                            dt_start=sched.pass_dt[len(starts) - 1][p])
        ctx.history_clear()
        fctx.tsbts = ctx
        fctx.sched = sched
        fctx.starts = starts
        fctx.every = every
        fctx.save_for_backward(m)
        return ctx.r.clone(), ctx.v.clone()

    @staticmethod
    def backward(fctx, g_r, g_v):
        ctx, sched = fctx.tsbts, fctx.sched
        (m,) = fctx.saved_tensors
        n = ctx.n
        dev = ctx.device
        z = lambda: torch.zeros((3, n), dtype=torch.float64, device=dev)  # noqa: E731
        rbar = z() if g_r is None else g_r.contiguous().clone()
        vbar = z() if g_v is None else g_v.contiguous().clone()
        abar = z()
        pbar = z()
        mbar = torch.zeros(n, dtype=torch.float64, device=dev)
        buf = torch.empty(3 * n, dtype=torch.float64, device=dev)
        seeds = torch.empty(3 * n, dtype=torch.float64, device=dev)
        first = fctx.starts[0]
        ctx.bind(first[0].clone(), first[1].clone(), m, a=first[2].clone(),
                 t_last=first[3].clone(), dt=first[4].clone())
        for e in range(len(sched.eras) - 1, -1, -1):
            passes, start = sched.eras[e], fctx.starts[e]
            P = len(passes)
            # each particle's first record of a pass is its era-start state, at its own time
            t_start = start[3].cpu().numpy()
            groups = [(float(t), ctx.idx(np.flatnonzero(t_start == t).astype(np.int32)))
                      for t in np.unique(t_start)]
            acc_r, acc_v, acc_a = z(), z(), z()
            later = None   # (layout, record adjoint) of the pass after the one reversed
            for p in range(P - 1, -1, -1):
                # interpolation source of pass p: pass p-1, rebuilt from the era start
                ctx.history_clear()
                for q in range(p):
                    _restore(ctx, start)
                    _sched_pass(ctx, passes[q], buf, q > 0, True,
                                dt_start=sched.pass_dt[e][q])
                if p:
                    layout = ctx.history_layout()
                    hbar = torch.zeros((6, layout[0]), dtype=torch.float64, device=dev)
                _restore(ctx, start)
                pre = []
                _sched_pass(ctx, passes[p], buf, p > 0, False, pre,
                            dt_start=sched.pass_dt[e][p])
                rb, vb, ab = (rbar, vbar, abar) if p == P - 1 else (z(), z(), z())
                for s in range(len(passes[p]) - 1, -1, -1):
                    _restore(ctx, pre[s])
                    tb, idx, _ = passes[p][s]
                    k = idx.numel()
                    sd = seeds[:3 * k].view(3, k)
                    if later is not None:
                        ctx.record_adjoint(idx, tb, later[0], later[1], rb, vb)
                    ctx.predict(tb, p > 0)
                    ctx.block_adjoint(0, idx, tb, rb, vb, ab, pbar, sd)
                    ctx.force_backward(idx, tb, sd, None, pbar, mbar)
                    if p:
                        ctx.interp_adjoint(tb, pbar, hbar)
                    ctx.block_adjoint(1, None, tb, rb, vb, ab, pbar, None)
                if later is not None:
                    for (t0, gidx) in groups:
                        ctx.record_adjoint(gidx, t0, later[0], later[1], rb, vb)
                ctx.adjoint_accumulate(rb, vb, ab, acc_r, acc_v, acc_a)
                later = (layout, hbar) if p else None
            rbar, vbar, abar = acc_r, acc_v, acc_a
            _restore(ctx, start)
        ctx.history_clear()
        ctx.load_positions(first[0], m, 0.0)
        ctx.force_backward(fctx.every, 0.0, abar, None, rbar, mbar)   # through a_0
        return rbar, vbar, mbar, None, None


def tsbts_schedule_leapfrog(r0, v0, m, ctx: Context, schedule):
    """Differentiable run on a recorded block schedule (see TsbtsScheduleLeapfrog)."""
    return TsbtsScheduleLeapfrog.apply(r0, v0, m, ctx, _DeviceSchedule(ctx, schedule))


def tsbts_era_leapfrog(r0, v0, m, ctx: Context, dt, t_end: float, era: float,
                       passes: int = 3):
    """Differentiable run on the fixed block schedule dt cut into eras of length `era`
    with `passes` passes each (see fixed_schedule)."""
    return tsbts_schedule_leapfrog(r0, v0, m, ctx, fixed_schedule(dt, t_end, era, passes))
