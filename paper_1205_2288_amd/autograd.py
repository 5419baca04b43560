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
* ``TsbtsEraLeapfrog``: the same fixed schedule cut into eras, each integrated with
  several passes (Section 2's time-symmetric scheme: from the second pass on the
  non-active particles are interpolated from the previous pass's stored states).  The
  reverse sweep of a pass also moves the adjoints of interpolated positions into the
  adjoints of the previous pass's records (``tsbts_interp_adjoint``) and adds those back
  at the block steps that wrote them (``tsbts_record_adjoint``).

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
    return (ctx.r, ctx.v, ctx.a, ctx.t_last)


def _restore(ctx: Context, saved):
    for dst, src in zip(_state(ctx), saved):
        dst.copy_(src)


def _era_pass(ctx: Context, sched: BlockSchedule, s0: int, s1: int, buf, use_history: bool,
              record: bool, pre=None):
    """Block steps s0 .. s1-1 of one pass; record = keep its states as the next pass's
    interpolation source; pre = list receiving each step's pre-step state."""
    if record:
        ctx.history_begin()
    for s in range(s0, s1):
        if pre is not None:
            pre.append([x.clone() for x in _state(ctx)])
        _block_step(ctx, sched, s, buf, use_history)
    if record:
        ctx.history_end()


class TsbtsEraLeapfrog(torch.autograd.Function):
    """(r, v) at t_end after a run on a fixed block schedule cut into eras of length `era`
    (a multiple of the largest step), each era integrated `passes` times from its start
    state: the first pass Taylor-predicts every particle, later passes take the
    non-active particles from the previous pass's stored states by cubic Hermite
    interpolation (Section 2's time-symmetric scheme on a given schedule).  The forward
    keeps the era-start states; the backward sweeps each era's passes in reverse,
    recomputing the interpolation source of each pass from the era start."""

    @staticmethod
    def forward(fctx, r0, v0, m, ctx: Context, dt, t_end: float, era: float, passes: int):
        n = ctx.n
        dev = ctx.device
        sched = BlockSchedule(ctx, dt, t_end)
        per = era / sched.hmin
        if passes < 1:
            raise ValueError("passes must be >= 1")
        if era % float(sched.dt.max()) != 0.0 or per != int(per) or sched.K % int(per):
            raise ValueError("era must be a multiple of the largest step and divide t_end")
        per = int(per)
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
        starts = []
        for s0 in range(0, sched.K, per):
            start = [x.clone() for x in _state(ctx)]
            starts.append(start)
            ctx.history_clear()
            for p in range(passes):
                if p:
                    _restore(ctx, start)
                _era_pass(ctx, sched, s0, s0 + per, buf, p > 0, p < passes - 1)
        ctx.history_clear()
        fctx.tsbts = ctx
        fctx.sched = sched
        fctx.per = per
        fctx.passes = passes
        fctx.starts = starts
        fctx.every = every
        fctx.save_for_backward(m)
        return ctx.r.clone(), ctx.v.clone()

    @staticmethod
    def backward(fctx, g_r, g_v):
        ctx, sched, per, passes = fctx.tsbts, fctx.sched, fctx.per, fctx.passes
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
                 t_last=first[3].clone(),
                 dt=torch.tensor(sched.dt, dtype=torch.float64, device=dev))
        for e in range(len(fctx.starts) - 1, -1, -1):
            start = fctx.starts[e]
            s0 = e * per
            t0 = s0 * sched.hmin
            acc_r, acc_v, acc_a = z(), z(), z()
            later = None   # (layout, record adjoint) of the pass after the one reversed
            for p in range(passes - 1, -1, -1):
                # interpolation source of pass p: pass p-1, rebuilt from the era start
                ctx.history_clear()
                for q in range(p):
                    _restore(ctx, start)
                    _era_pass(ctx, sched, s0, s0 + per, buf, q > 0, True)
                if p:
                    layout = ctx.history_layout()
                    hbar = torch.zeros((6, layout[0]), dtype=torch.float64, device=dev)
                _restore(ctx, start)
                pre = []
                _era_pass(ctx, sched, s0, s0 + per, buf, p > 0, False, pre)
                rb, vb, ab = (rbar, vbar, abar) if p == passes - 1 else (z(), z(), z())
                for s in range(s0 + per - 1, s0 - 1, -1):
                    _restore(ctx, pre[s - s0])
                    tb = sched.time(s)
                    idx = sched.active(s)
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
                    ctx.record_adjoint(fctx.every, t0, later[0], later[1], rb, vb)
                ctx.adjoint_accumulate(rb, vb, ab, acc_r, acc_v, acc_a)
                later = (layout, hbar) if p else None
            rbar, vbar, abar = acc_r, acc_v, acc_a
            _restore(ctx, start)
        ctx.history_clear()
        ctx.load_positions(first[0], m, 0.0)
        ctx.force_backward(fctx.every, 0.0, abar, None, rbar, mbar)   # through a_0
        return rbar, vbar, mbar, None, None, None, None, None


def tsbts_era_leapfrog(r0, v0, m, ctx: Context, dt, t_end: float, era: float,
                       passes: int = 3):
    return TsbtsEraLeapfrog.apply(r0, v0, m, ctx, dt, t_end, era, passes)
