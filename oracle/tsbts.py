"""Oracle TSBTS integrator: eras, passes ("iterations") and block steps.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Algorithm 2 (sequential TSBTS), Algorithm 1 (symmetrization of block steps),
Eq. (blockcondition) and Algorithm 3 (dynamic era size) of the paper, in their order.
Where the text is silent or garbled the following readings are taken (they are listed,
with the reasons, in the design notes of the repository):

* Times are integers in ticks of 2^-20; every block step is a power of two of ticks.
* Eq. (blockcondition): the admissible level for a candidate step is the largest power of
  two not exceeding the mean of the criterion value at the beginning and at the end of
  that step, capped at dt_max and floored at dt_min.
* First pass (plain block steps): a step may halve any number of times; it doubles when
  the block time is a multiple of twice the step and twice the step is admissible.
* Later passes, Algorithm 1 read as in its prose (an else-if chain): at an odd time keep
  the step if it is admissible, else halve once; at an even time try doubling, then
  keeping, else halve once.  The end-of-step criterion value comes from the previous
  pass's criterion history of the same particle, linear in time between its stored
  values, and falls back to the beginning value past the last stored time.
* Prediction to a block time (Algorithm 2 step 4): active particles use their own Taylor
  prediction (which is their leapfrog position); in later passes the other particles are
  interpolated (cubic Hermite) from the previous pass's stored points when those bracket
  the block time, otherwise Taylor-predicted.
* A particle whose next time lies beyond the era end is not advanced in that era.
* The step that leaves the era start is a new step of the era: a particle at the era
  start keeps the step chosen when it arrived there in the first pass, and from the
  second pass on that step is chosen again by Algorithm 1 (from the step that brought
  the particle to the era start) with the end values of the previous pass, so that the
  first step of every era is symmetrized like the others.
* Dynamic era (Algorithm 3): size = last - first next block time, clamped to
  [dt_max / 8, dt_max] and rounded up to a power of two; when that is still smaller than
  the largest step in use the era takes dt_max (Section 4's remedy: an era shorter than
  a step leaves that particle out, with no past information to symmetrize it); the era
  then ends at the next multiple of that size.
* Iterations = passes: one pass is the classical block-step scheme (no symmetrization).
"""
from __future__ import annotations

import math

import numpy as np

from . import force, taylor, hermite, timestep, energy

TICK_EXP = 20
TICK = 2.0 ** -TICK_EXP
_KEY = 1 << 40  # record key = particle * _KEY + time in ticks


def ticks(t: float) -> int:
    k = t / TICK
    if k != math.floor(k):
        raise ValueError(f"time {t} is not a multiple of 2^-{TICK_EXP}")
    return int(k)


def level_from_criterion(dt_begin: float, dt_end: float, dt_min_ticks: int,
                         dt_max_ticks: int) -> int:
    """Eq. (blockcondition): Delta t_n = 2^-(n-1) with n the smallest k >= 1 such that
    2^-(k-1) <= (dt_begin + dt_end) / 2; capped at dt_max, floored at dt_min (ticks)."""
    avg = 0.5 * (dt_begin + dt_end)
    k = 1
    # smallest k >= 1 with 2^-(k-1) <= avg, searched upward (the equation as printed)
    while k <= TICK_EXP + 1 and 2.0 ** (-(k - 1)) > avg:
        k += 1
    level_ticks = 1 << (TICK_EXP - (k - 1)) if k - 1 <= TICK_EXP else 0
    return max(dt_min_ticks, min(dt_max_ticks, level_ticks))


class History:
    """Stored data of one pass (Section 2: positions, velocities and accelerations of
    every step of the era) plus the criterion values used for symmetrization.

    Blocks are appended in block-step order; ``freeze`` groups them by particle with a
    stable sort, which keeps each particle's records in time order."""

    def __init__(self):
        self.blocks = []

    def append(self, idx, t, r, v, a, dtc):
        idx = np.asarray(idx, dtype=np.int64)
        tt = np.broadcast_to(np.asarray(t, dtype=np.int64), idx.shape).copy()
        self.blocks.append((idx, tt, np.array(r), np.array(v), np.array(a),
                            np.array(dtc, dtype=np.float64)))

    def freeze(self, n):
        pid = np.concatenate([b[0] for b in self.blocks])
        order = np.argsort(pid, kind="stable")
        self.pid = pid[order]
        self.T = np.concatenate([b[1] for b in self.blocks])[order]
        self.R = np.concatenate([b[2] for b in self.blocks], axis=1)[:, order]
        self.V = np.concatenate([b[3] for b in self.blocks], axis=1)[:, order]
        self.A = np.concatenate([b[4] for b in self.blocks], axis=1)[:, order]
        self.C = np.concatenate([b[5] for b in self.blocks])[order]
        self.key = self.pid * _KEY + self.T
        self.off = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(self.pid, minlength=n), out=self.off[1:])
        self.blocks = None
        return self

    def last_at_or_before(self, j, t):
        """Record index of particle j's last stored time <= t (arrays j, t)."""
        return np.searchsorted(self.key, np.asarray(j) * _KEY + np.asarray(t),
                               side="right") - 1


class OracleTSBTS:
    """Plain FP64 TSBTS integration (oracle).  State arrays are (3, N) / (N,)."""

    def __init__(self, r, v, m, eps, eta=0.1, passes=3, dt_max=1.0 / 64, dt_min=2.0 ** -20,
                 era=None, criterion=None, record_schedule=False):
        """record_schedule: keep the block steps taken (``self.schedule``: initial steps
        and, per era, the steps of all particles when each pass starts and, per pass,
        (t_b, active set, new steps of the active set), in time units) so that the same
        schedule can be replayed."""
        self.n = int(np.asarray(m).size)
        self.m = np.array(m, dtype=np.float64)
        self.eps = float(eps)
        self.eta = float(eta)
        self.passes = int(passes)
        self.dt_max = ticks(dt_max)
        self.dt_min = ticks(dt_min)
        self.era = None if era is None else ticks(era)
        self.criterion = criterion  # optional override (tests): f(r, v, idx) -> dt values
        self.r = np.array(r, dtype=np.float64)
        self.v = np.array(v, dtype=np.float64)
        # Algorithm 2, step 1: forces, time-steps and next block times of all particles.
        self.a, _ = force(self.r, self.m, self.eps)
        self.dtc = self._criterion(self.r, self.v, np.arange(self.n, dtype=np.int32))
        self.t = np.zeros(self.n, dtype=np.int64)
        self.dt = np.array([level_from_criterion(c, c, self.dt_min, self.dt_max)
                            for c in self.dtc], dtype=np.int64)
        # the step that brought each particle to its current time (0: none yet)
        self.dtp = np.zeros(self.n, dtype=np.int64)
        self.time = 0
        # era_sizes: number of eras of each size (time units, as text)
        self.stats = {"block_steps": 0, "force_calls": 0, "interactions": 0, "eras": 0,
                      "era_sizes": {}}
        self.schedule = ({"dt0": self.dt * TICK, "eras": []} if record_schedule else None)
        self._log = None

    # ------------------------------------------------------------------ criterion
    def _criterion(self, r, v, idx):
        if self.criterion is not None:
            return np.asarray(self.criterion(r, v, idx), dtype=np.float64)
        return timestep(r, v, self.m, self.eps, self.eta, idx)

    # ------------------------------------------------------------------ era size
    def _era_end(self, t0: int) -> int:
        if self.era is not None:
            return t0 + self.era
        # Algorithm 3: last block time minus first block time, clamped, power of two
        nxt = self.t + self.dt
        size = int(nxt.max() - nxt.min())
        size = max(self.dt_max // 8, min(self.dt_max, size))
        size = 1 << (size - 1).bit_length()  # smallest power of two >= size
        if size < int(self.dt.max()):
            size = self.dt_max
        return (t0 // size + 1) * size

    # ------------------------------------------------------------------ prediction
    def _predict(self, tb: int, active: np.ndarray, prev: History | None):
        h = (tb - self.t) * TICK
        rp, vp = taylor(self.r, self.v, self.a, h)
        if prev is None:
            return rp, vp
        # later passes: interpolate non-active particles from the previous pass
        j = np.nonzero(~active)[0]
        k = prev.last_at_or_before(j, tb)
        exact = prev.T[k] == tb
        je, ke = j[exact], k[exact]
        rp[:, je] = prev.R[:, ke]
        vp[:, je] = prev.V[:, ke]
        inner = ~exact & (k + 1 < prev.off[j + 1])
        ji, k0 = j[inner], k[inner]
        k1 = k0 + 1
        rr, vv = hermite(prev.T[k0] * TICK, prev.R[:, k0], prev.V[:, k0], prev.A[:, k0],
                         prev.T[k1] * TICK, prev.R[:, k1], prev.V[:, k1], prev.A[:, k1],
                         tb * TICK)
        rp[:, ji] = rr
        vp[:, ji] = vv
        return rp, vp

    # ------------------------------------------------------------------ new steps
    def _dtc_end(self, prev: History, i: int, t_end: int, dtc_begin: float) -> float:
        k = int(prev.last_at_or_before(i, t_end))
        if prev.T[k] == t_end:
            return float(prev.C[k])
        if k + 1 >= prev.off[i + 1]:
            return dtc_begin  # beyond the stored history
        w = (t_end - prev.T[k]) / (prev.T[k + 1] - prev.T[k])
        return float((1.0 - w) * prev.C[k] + w * prev.C[k + 1])

    def _new_step(self, i: int, tb: int, dtc_begin: float, prev: History | None) -> int:
        dt = int(self.dt[i])
        if prev is None:
            # first pass: standard block step
            lvl = level_from_criterion(dtc_begin, dtc_begin, self.dt_min, self.dt_max)
            new = dt
            while new > lvl and new > self.dt_min:
                new //= 2
            if new == dt and 2 * dt <= lvl and tb % (2 * dt) == 0:
                new = 2 * dt
            return new

        def admissible(c):
            end = self._dtc_end(prev, i, tb + c, dtc_begin)
            return c <= level_from_criterion(dtc_begin, end, self.dt_min, self.dt_max)

        even = (tb // dt) % 2 == 0
        if even and 2 * dt <= self.dt_max and admissible(2 * dt):
            return 2 * dt
        if admissible(dt):
            return dt
        return max(dt // 2, self.dt_min)

    # ------------------------------------------------------------------ one pass
    def _pass(self, T1: int, prev: History | None) -> History:
        hist = History()
        every = np.arange(self.n)
        hist.append(every, self.t, self.r, self.v, self.a, self.dtc)  # era-start points
        while True:
            nxt = self.t + self.dt
            tb = int(nxt.min())
            if tb > T1:
                break
            active = nxt == tb
            idx = np.nonzero(active)[0].astype(np.int32)
            rp, vp = self._predict(tb, active, prev)
            a_new, _ = force(rp, self.m, self.eps, idx)
            h = (tb - self.t[idx]) * TICK
            # corrector (Section 2 leapfrog): the new position is the predicted one
            self.r[:, idx] = rp[:, idx]
            self.v[:, idx] = self.v[:, idx] + 0.5 * (self.a[:, idx] + a_new) * h
            self.a[:, idx] = a_new
            self.dtp[idx] = tb - self.t[idx]
            self.t[idx] = tb
            # criterion: corrected active particles, predicted others
            vc = vp.copy()
            vc[:, idx] = self.v[:, idx]
            dtc = self._criterion(rp, vc, idx)
            self.dtc[idx] = dtc
            hist.append(idx, tb, self.r[:, idx], self.v[:, idx], self.a[:, idx], dtc)
            for k, i in enumerate(idx):
                self.dt[i] = self._new_step(int(i), tb, float(dtc[k]), prev)
            if self._log is not None:
                self._log.append((tb * TICK, idx.copy(), self.dt[idx] * TICK))
            self.stats["block_steps"] += 1
            self.stats["force_calls"] += 1
            self.stats["interactions"] += int(idx.size) * self.n
        return hist.freeze(self.n)

    # ------------------------------------------------------------------ one era
    def _first_steps(self, T0: int, prev: History):
        """Later passes: the step of every particle at the era start chosen again by
        Algorithm 1, from the step that brought it there, with the previous pass's end
        values (particles that have not taken a step yet keep their initial step)."""
        for i in np.nonzero((self.t == T0) & (self.dtp > 0))[0]:
            self.dt[i] = self.dtp[i]
            self.dt[i] = self._new_step(int(i), T0, float(self.dtc[i]), prev)

    def era_step(self):
        T0 = self.time
        T1 = self._era_end(T0)
        names = ("r", "v", "a", "t", "dt", "dtc", "dtp")
        saved = [getattr(self, x).copy() for x in names]
        prev = None
        era_rec = None
        if self.schedule is not None:
            era_rec = {"passes": [], "dt_start": []}
            self.schedule["eras"].append(era_rec)
        for p in range(self.passes):
            if p > 0:
                for name, src in zip(names, saved):
                    getattr(self, name)[...] = src
                self._first_steps(T0, prev)
            if era_rec is not None:
                self._log = []
                era_rec["passes"].append(self._log)
                era_rec["dt_start"].append(self.dt * TICK)
            prev = self._pass(T1, prev)
        self._log = None
        self.last_history = prev
        self.time = T1
        self.stats["eras"] += 1
        key = repr((T1 - T0) * TICK)
        self.stats["era_sizes"][key] = self.stats["era_sizes"].get(key, 0) + 1
        return T1

    def run(self, t_end: float, energy_every: float | None = None):
        """Integrate to t_end; return [(t, E)] at era ends that are multiples of
        energy_every (default dt_max), where every particle is synchronised."""
        stop = ticks(t_end)
        every = self.dt_max if energy_every is None else ticks(energy_every)
        out = [(0.0, self.total_energy())]
        while self.time < stop:
            T1 = self.era_step()
            if T1 % every == 0:
                assert np.all(self.t == T1), "particles not synchronised at a dt_max multiple"
                out.append((T1 * TICK, self.total_energy()))
        return out

    def total_energy(self):
        k, w = energy(self.r, self.v, self.m, self.eps)
        return k + w

    def state(self):
        return {"r": self.r.copy(), "v": self.v.copy(), "a": self.a.copy(),
                "t": self.t.copy(), "dt": self.dt.copy(), "dtc": self.dtc.copy(),
                "dtp": self.dtp.copy(), "time": self.time}

    def load_state(self, s):
        for name in ("r", "v", "a", "t", "dt", "dtc", "dtp"):
            getattr(self, name)[...] = s[name]
        self.time = int(s["time"])
