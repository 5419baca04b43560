"""Host-side TSBTS scheduler driving the HIP kernels (eras, passes, block steps).

The device holds the particle state and does all arithmetic (prediction / interpolation,
force, corrector with history recording, criterion, energy).  The host keeps integer
copies of each particle's last time and block step, picks the block time and active set,
and applies the step-size rules, vectorised over the active set:

* block times are integers in ticks of 2^-20; steps are powers of two of ticks;
* Eq. (blockcondition): the admissible step for a candidate is the largest power of two
  not above the mean of the criterion at the start of the step and at its end, within
  [dt_min, dt_max];
* first pass (Section 2, "standard block step"): drop to the admissible step (several
  halvings allowed), or double at times that are multiples of twice the step;
* later passes, Algorithm 1 as described in its prose: at even times double if admissible,
  else keep if admissible, else halve once; at odd times keep if admissible, else halve
  once.  The end-of-step criterion comes from the previous pass's values of the same
  particle, linear in time between stored values (the start value beyond the last one);
* Algorithm 2: every pass of an era restarts from the era-start state; passes after the
  first interpolate the non-active particles from the previous pass's stored states;
* Algorithm 3 (dynamic era): era size = last minus first next block time, clamped to
  [dt_max / 8, dt_max], rounded up to a power of two, and dt_max when that is below the
  largest step in use (Section 4); the era ends at the next multiple.  A particle whose
  next time is past the era end is not advanced in that era.
* From the second pass on, the step of each particle at the era start is chosen again by
  Algorithm 1 with the previous pass's end values.
"""
from __future__ import annotations

import json
import time

import numpy as np
import torch

from .context import Context

TICK_BITS = 20
TICK = 2.0 ** -TICK_BITS
_KEY_SHIFT = 40


def to_ticks(t: float) -> int:
    k = t / TICK
    if k != int(k):
        raise ValueError(f"{t} is not a multiple of 2^-{TICK_BITS}")
    return int(k)


def admissible(begin, end, dt_min: int, dt_max: int):
    """Largest power of two (ticks) not above (begin + end) / 2, clipped to [dt_min, dt_max]."""
    avg = 0.5 * (np.asarray(begin, dtype=np.float64) + np.asarray(end, dtype=np.float64))
    x = avg / TICK
    big = ~np.isfinite(x) | (x >= dt_max)
    mant, ex = np.frexp(np.where(big, 1.0, x))      # x = mant * 2^ex, mant in [0.5, 1)
    p2 = np.where(x >= 1.0, np.ldexp(1.0, ex - 1), 0.0).astype(np.int64)
    out = np.clip(p2, dt_min, dt_max)
    return np.where(big, dt_max, out)


class CriterionHistory:
    """Criterion values of one pass (start values per particle plus one per step), grouped
    by particle in time order for the end-of-step lookups of the next pass."""

    def __init__(self):
        self._pid, self._t, self._c = [], [], []

    def add(self, pid, t, c):
        # copies: the caller keeps updating its own arrays in place
        self._pid.append(np.array(pid, dtype=np.int64))
        self._t.append(np.array(np.broadcast_to(np.asarray(t, dtype=np.int64), np.shape(pid))))
        self._c.append(np.array(c, dtype=np.float64))

    def close(self, n: int):
        pid = np.concatenate(self._pid)
        order = np.argsort(pid, kind="stable")
        self.pid = pid[order]
        self.t = np.concatenate(self._t)[order]
        self.c = np.concatenate(self._c)[order]
        self.key = (self.pid << _KEY_SHIFT) + self.t
        self.end = np.zeros(n, dtype=np.int64)  # one past each particle's last value
        np.cumsum(np.bincount(self.pid, minlength=n), out=self.end)
        self._pid = self._t = self._c = None
        return self

    def value_at(self, pid, t, fallback):
        """Criterion of particles pid at times t (linear between stored values)."""
        k = np.searchsorted(self.key, (pid << _KEY_SHIFT) + t, side="right") - 1
        tk = self.t[k]
        has_next = k + 1 < self.end[pid]
        k1 = np.where(has_next, k + 1, k)
        t1 = self.t[k1]
        w = np.where(has_next, (t - tk) / np.where(has_next, t1 - tk, 1), 0.0)
        lin = (1.0 - w) * self.c[k] + w * self.c[k1]
        return np.where(tk == t, self.c[k], np.where(has_next, lin, fallback))


def _run_loop(sim, t_end: float, energy_every, log):
    """Run loop of both schedulers: eras up to t_end, the float64 energy at every era end
    that is a multiple of energy_every (default dt_max), where all particles are
    synchronised.  A non-finite energy stops the run with the time and era.  With a log
    stream, each energy sample also writes one JSON line: t, E, the energy error relative
    to the first energy this scheduler measured, block steps, force calls, interactions,
    eras, particle-eras left out of their era since the previous sample, the number of
    particles per step size 2^-k and the wall time of this call."""
    stop = to_ticks(t_end)
    every = sim.dt_max if energy_every is None else to_ticks(energy_every)
    t0 = time.perf_counter()
    excluded = 0

    def sample(T, E):
        if not np.isfinite(E):
            raise FloatingPointError(f"energy is not finite at t = {T * TICK} "
                                     f"(after era {sim.stats['eras']})")
        if not hasattr(sim, "_e_first"):
            sim._e_first = E
        if log is not None:
            st = sim.stats
            ks, counts = np.unique(TICK_BITS - np.log2(sim.dt).astype(np.int64),
                                   return_counts=True)
            rec = {"t": T * TICK, "E": E,
                   "rel_dE": (E - sim._e_first) / abs(sim._e_first),
                   "block_steps": st["block_steps"], "force_calls": st["force_calls"],
                   "interactions": st["interactions"], "eras": st["eras"],
                   "excluded": excluded,
                   "levels": {str(int(k)): int(c) for k, c in zip(ks, counts)},
                   "wall_s": time.perf_counter() - t0}
            log.write(json.dumps(rec) + "\n")
            log.flush()
        return (T * TICK, E)

    out = [sample(sim.time, sim.energy())]
    while sim.time < stop:
        T1 = sim.era_step()
        if log is not None:
            excluded += int(np.count_nonzero(sim.t != T1))
        if T1 % every == 0:
            if not np.all(sim.t == T1):
                raise RuntimeError("particles not synchronised at a dt_max multiple")
            out.append(sample(T1, sim.energy()))
            excluded = 0
    sim.ctx.synchronize()
    return out


def _count_era(sizes: dict, ticks: int):
    key = repr(ticks * TICK)
    sizes[key] = sizes.get(key, 0) + 1


class TSBTS:
    """Dynamic- or fixed-era TSBTS integration on the GPU.

    r, v: (3, N) float64; m: (N,).  era=None selects the dynamic era size.
    precision / separation / newton select the force kernel (see Context)."""

    def __init__(self, r, v, m, eps, eta=0.1, passes=3, dt_max=1.0 / 64, dt_min=2.0 ** -20,
                 era=None, precision="mixed", separation="f64", newton=False, context=None,
                 record_schedule=False):
        """record_schedule: keep the block steps taken in ``self.schedule`` (initial steps
        and, per era, the steps of all particles when each pass starts and, per pass,
        (t_b, active set, new steps of the active set), in time units), the input of
        autograd.tsbts_schedule_leapfrog."""
        self.n = n = int(np.asarray(m).size)
        self.schedule = {"dt0": None, "eras": []} if record_schedule else None
        self._log = None
        self.eta = float(eta)
        self.passes = int(passes)
        self.dt_max = to_ticks(dt_max)
        self.dt_min = to_ticks(dt_min)
        self.era = None if era is None else to_ticks(era)
        # `context` lets a caller supply an object with the Context interface
        self.ctx = context if context is not None else Context(
            n, eps, precision=precision, separation=separation, newton=newton)
        self.ctx.bind(r, v, m)
        dev = self.ctx.device
        # staging: host buffers (pinned by the context) and device buffers
        self._idx_h = self.ctx.host_buffer(n, torch.int32)
        self._dtc_h = self.ctx.host_buffer(n, torch.float64)
        self._dtn_h = self.ctx.host_buffer(n, torch.float64)
        self._idx_d = torch.empty(n, dtype=torch.int32, device=dev)
        self._acc_d = torch.empty(3 * n, dtype=torch.float64, device=dev)
        self._dtc_d = torch.empty(n, dtype=torch.float64, device=dev)
        self._dtn_d = torch.empty(n, dtype=torch.float64, device=dev)
        self._ek_d = torch.empty(2, dtype=torch.float64, device=dev)
        # host mirrors (ticks) and last criterion values
        self.t = np.zeros(n, dtype=np.int64)
        self.dt = np.zeros(n, dtype=np.int64)
        self.dtp = np.zeros(n, dtype=np.int64)  # step that brought each particle to t
        self.dtc = np.zeros(n)
        self.time = 0
        # era_sizes: number of eras of each size (time units, as text)
        self.stats = {"block_steps": 0, "force_calls": 0, "interactions": 0, "eras": 0,
                      "era_sizes": {}, "wall_s": 0.0}
        self._initialise()

    # ------------------------------------------------------------------ device plumbing
    def _upload_idx(self, idx: np.ndarray) -> torch.Tensor:
        k = idx.size
        self._idx_h[:k].numpy()[:] = idx
        d = self._idx_d[:k]
        d.copy_(self._idx_h[:k], non_blocking=True)
        return d

    def _initialise(self):
        c = self.ctx
        every = self._upload_idx(np.arange(self.n, dtype=np.int32))
        c.predict(0.0)  # t_last = dt = 0: every particle is predicted to itself
        acc = self._acc_d.view(3, self.n)
        c.force(every, 0.0, with_pot=False, acc=acc)
        c.a.copy_(acc)
        dtc = c.timestep(every, self.eta, dtc=self._dtc_d)
        self.dtc[:] = dtc.cpu().numpy()
        self.dt[:] = admissible(self.dtc, self.dtc, self.dt_min, self.dt_max)
        c.dt.copy_(torch.from_numpy(self.dt * TICK))
        c.synchronize()
        if self.schedule is not None:
            self.schedule["dt0"] = self.dt * TICK

    # ------------------------------------------------------------------ step rules
    def _new_steps(self, idx, tb, begin, prev: CriterionHistory | None):
        dt = self.dt[idx]
        if prev is None:
            lvl = admissible(begin, begin, self.dt_min, self.dt_max)
            new = np.minimum(dt, lvl)
            grow = (lvl >= 2 * dt) & (tb % (2 * dt) == 0)
            return np.where(grow, 2 * dt, new)
        pid = idx.astype(np.int64)
        even = (tb // dt) % 2 == 0
        end2 = prev.value_at(pid, tb + 2 * dt, begin)
        end1 = prev.value_at(pid, tb + dt, begin)
        ok2 = even & (2 * dt <= self.dt_max) & \
            (2 * dt <= admissible(begin, end2, self.dt_min, self.dt_max))
        ok1 = dt <= admissible(begin, end1, self.dt_min, self.dt_max)
        return np.where(ok2, 2 * dt, np.where(ok1, dt, np.maximum(dt // 2, self.dt_min)))

    # ------------------------------------------------------------------ era / pass
    def _era_end(self, t0: int) -> int:
        if self.era is not None:
            return t0 + self.era
        nxt = self.t + self.dt
        size = int(np.clip(nxt.max() - nxt.min(), self.dt_max // 8, self.dt_max))
        size = 1 << (size - 1).bit_length()  # smallest power of two >= size
        if size < int(self.dt.max()):
            size = self.dt_max  # an era shorter than a step would leave it unsymmetrized
        return (t0 // size + 1) * size

    def _pass(self, p: int, T1: int, prev: CriterionHistory | None) -> CriterionHistory:
        c = self.ctx
        hist = CriterionHistory()
        hist.add(np.arange(self.n), self.t, self.dtc)
        c.history_begin()
        while True:
            nxt = self.t + self.dt
            tb = int(nxt.min())
            if tb > T1:
                break
            idx = np.flatnonzero(nxt == tb).astype(np.int32)
            k = idx.size
            tbs = tb * TICK
            d_idx = self._upload_idx(idx)
            c.predict(tbs, use_history=p > 0)
            acc = self._acc_d[:3 * k].view(3, k)
            c.force(d_idx, tbs, with_pot=False, acc=acc)
            c.correct(d_idx, tbs, acc)
            dtc = c.timestep(d_idx, self.eta, dtc=self._dtc_d[:k])
            self._dtc_h[:k].copy_(dtc, non_blocking=True)
            c.synchronize()
            begin = self._dtc_h[:k].numpy().copy()
            self.dtc[idx] = begin
            self.dtp[idx] = tb - self.t[idx]
            self.t[idx] = tb
            hist.add(idx, tb, begin)
            new = self._new_steps(idx, tb, begin, prev)
            self.dt[idx] = new
            self._dtn_h[:k].numpy()[:] = new * TICK
            dtn = self._dtn_d[:k]
            dtn.copy_(self._dtn_h[:k], non_blocking=True)
            c.set_dt(d_idx, dtn)
            if self._log is not None:
                self._log.append((tbs, idx.copy(), new * TICK))
            self.stats["block_steps"] += 1
            self.stats["force_calls"] += 1
            self.stats["interactions"] += k * self.n
        c.history_end()
        return hist.close(self.n)

    def _first_steps(self, T0: int, prev: CriterionHistory):
        """Later passes: the step of every particle at the era start chosen again by
        Algorithm 1 (from the step that brought it there) with the previous pass's end
        values, so that the first step of an era is symmetrized like the others;
        particles that have not taken a step yet keep their initial step."""
        idx = np.flatnonzero((self.t == T0) & (self.dtp > 0)).astype(np.int32)
        if idx.size == 0:
            return
        self.dt[idx] = self.dtp[idx]
        self.dt[idx] = self._new_steps(idx, T0, self.dtc[idx], prev)
        self.ctx.dt.copy_(torch.from_numpy(self.dt * TICK))

    def era_step(self) -> int:
        c = self.ctx
        T0 = self.time
        T1 = self._era_end(T0)
        saved_dev = [x.clone() for x in (c.r, c.v, c.a, c.t_last, c.dt)]
        saved_host = [x.copy() for x in (self.t, self.dt, self.dtc, self.dtp)]
        prev = None
        era_rec = None
        if self.schedule is not None:
            era_rec = {"passes": [], "dt_start": []}
            self.schedule["eras"].append(era_rec)
        for p in range(self.passes):
            if p > 0:
                for dst, src in zip((c.r, c.v, c.a, c.t_last, c.dt), saved_dev):
                    dst.copy_(src)
                for dst, src in zip((self.t, self.dt, self.dtc, self.dtp), saved_host):
                    dst[...] = src
                self._first_steps(T0, prev)
            if era_rec is not None:
                self._log = []
                era_rec["passes"].append(self._log)
                era_rec["dt_start"].append(self.dt * TICK)
            prev = self._pass(p, T1, prev)
        self._log = None
        self.time = T1
        self.stats["eras"] += 1
        _count_era(self.stats["era_sizes"], T1 - T0)
        return T1

    def energy(self) -> float:
        kw = self.ctx.energy(out=self._ek_d).cpu().numpy()
        return float(kw[0] + kw[1])

    def run(self, t_end: float, energy_every: float | None = None, log=None):
        """Integrate to t_end; return [(t, E)] at era ends that are multiples of
        energy_every (default dt_max), where every particle is synchronised.  log: a
        text stream receiving one JSON line of run metrics per energy sample."""
        t0 = time.perf_counter()
        out = _run_loop(self, t_end, energy_every, log)
        self.stats["wall_s"] += time.perf_counter() - t0
        return out

    def state(self):
        c = self.ctx
        c.synchronize()
        return {"r": c.r.cpu().numpy(), "v": c.v.cpu().numpy(), "a": c.a.cpu().numpy(),
                "t": self.t.copy(), "dt": self.dt.copy(), "dtc": self.dtc.copy(),
                "dtp": self.dtp.copy(), "time": self.time}

    def close(self):
        self.ctx.close()


class NativeTSBTS:
    """The same integration with the block-step loop in the library's native scheduler
    (tsbts_sched_*): one host/device synchronisation per block step and no Python in
    the loop.  Same readings and results as TSBTS."""

    def __init__(self, r, v, m, eps, eta=0.1, passes=3, dt_max=1.0 / 64, dt_min=2.0 ** -20,
                 era=None, precision="mixed", separation="f64", newton=False,
                 criterion="after", tune=None, predict_on_load=True, rule_threads=None):
        """criterion: "after" the corrector (the paper's order) or "before" it, with the
        predicted velocities, in the same pass over the pairs as the force.  tune: keyword
        arguments of Context.tune, applied before the first force evaluation.
        predict_on_load: small active sets predict their sources inside the force kernel,
        and on few particles take the criterion in it too (fewer launches per block step,
        same results).  rule_threads: host threads sharing the step rule of block steps
        with at least 8192 active particles (default 4; the same results for any
        number)."""
        from . import _lib as L
        if criterion not in ("after", "before"):
            raise ValueError("criterion must be 'after' or 'before'")
        self._L = L
        self.n = n = int(np.asarray(m).size)
        self.dt_max = to_ticks(dt_max)
        self.ctx = Context(n, eps, precision=precision, separation=separation, newton=newton)
        if tune:
            self.ctx.tune(**tune)
        self.ctx.bind(r, v, m)
        L.tsbts_sched_init(self.ctx.ctx, eta, passes, dt_min, dt_max,
                           0.0 if era is None else era)
        if criterion == "before":
            L.tsbts_sched_option(self.ctx.ctx, L.TSBTS_SCHED_CRITERION_BEFORE_CORRECTOR, 1)
        L.tsbts_sched_option(self.ctx.ctx, L.TSBTS_SCHED_PREDICT_ON_LOAD,
                             1 if predict_on_load and criterion == "after" else 0)
        if rule_threads is not None:
            L.tsbts_sched_option(self.ctx.ctx, L.TSBTS_SCHED_RULE_THREADS, int(rule_threads))
        self._ek = torch.empty(2, dtype=torch.float64, device=self.ctx.device)
        self._host()
        self.wall_s = 0.0
        self.era_sizes = {}  # eras of each size run by this object (time units, as text)

    def _host(self):
        t, dt, dtc, st, time_ = self._L.tsbts_sched_state(self.ctx.ctx, self.n)
        self.t, self.dt, self.dtc = t, dt, dtc
        self.time = to_ticks(time_)
        self._stats = st

    @property
    def stats(self):
        st = self._stats
        return {"block_steps": int(st[0]), "force_calls": int(st[1]),
                "interactions": int(st[2]), "eras": int(st[3]),
                "era_sizes": dict(self.era_sizes), "wall_s": self.wall_s}

    def step_timing(self) -> dict:
        """Mean wall time per block step (microseconds) in each phase (issue of the
        launches, wait for the GPU's results, host step rule, whole step), by active-set
        class, with the class's block steps and mean active-set size."""
        sec, cnt = self._L.tsbts_sched_timing(self.ctx.ctx)
        out = {}
        for c, name in enumerate(("k<=32", "k<=256", "k<=1024", "k>1024")):
            n = int(cnt[c, 0])
            if n == 0:
                continue
            us = sec[c] / n * 1e6
            out[name] = {"block_steps": n, "mean_k": float(cnt[c, 1]) / n,
                         "issue_us": float(us[0]), "wait_us": float(us[1]),
                         "rule_us": float(us[2]), "step_us": float(us[3])}
        return out

    def era_step(self) -> int:
        T0 = self.time
        end = self._L.tsbts_sched_era(self.ctx.ctx)
        self._host()
        T1 = to_ticks(end)
        _count_era(self.era_sizes, T1 - T0)
        return T1

    def energy(self) -> float:
        kw = self.ctx.energy(out=self._ek).cpu().numpy()
        return float(kw[0] + kw[1])

    def run(self, t_end: float, energy_every: float | None = None, log=None):
        """As TSBTS.run."""
        t0 = time.perf_counter()
        out = _run_loop(self, t_end, energy_every, log)
        self.wall_s += time.perf_counter() - t0
        return out

    def state(self):
        c = self.ctx
        c.synchronize()
        return {"r": c.r.cpu().numpy(), "v": c.v.cpu().numpy(), "a": c.a.cpu().numpy(),
                "t": self.t.copy(), "dt": self.dt.copy(), "dtc": self.dtc.copy(),
                "time": self.time}

    def checkpoint(self) -> dict:
        """Era-end checkpoint (host arrays; times and steps in ticks): continuing it with
        restore() in a scheduler built with the same parameters gives the same run, bit
        for bit.  The dict can be saved with numpy.savez."""
        ck = self.state()
        ck["dtp"] = self._L.tsbts_sched_prev_steps(self.ctx.ctx, self.n)
        ck["stats"] = np.array(self._stats, dtype=np.int64)
        return ck

    def restore(self, ck) -> None:
        """Continue from a checkpoint() of a run with the same parameters.  A checkpoint
        that is not an era-end state is refused before anything changes."""
        c = self.ctx
        xs = {}
        for name in ("r", "v", "a"):
            xs[name] = np.ascontiguousarray(ck[name], dtype=np.float64)
            if xs[name].shape != (3, self.n):
                raise ValueError(f"checkpoint {name} must have shape (3, {self.n})")
        # validates the times and steps, then sets them (and the bound t_last, dt)
        self._L.tsbts_sched_restore(c.ctx, self.n, ck["t"], ck["dt"], ck["dtp"], ck["dtc"],
                                    ck.get("stats"), int(ck["time"]) * TICK)
        for name, x in xs.items():
            getattr(c, name).copy_(torch.from_numpy(x))
        self._host()

    def close(self):
        self.ctx.close()
