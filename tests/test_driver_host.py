"""CPU checks of the product's host scheduler (paper_1205_2288_amd.driver).

The driver is run with a CPU stand-in context that evaluates every kernel call with the
oracle's arithmetic, so any difference from the oracle's own TSBTS scheduler comes from
the host logic alone (block selection, Eq. blockcondition, Algorithm 1, Algorithm 3,
era restarts, criterion history).  The two schedulers are independent implementations
of the same readings and must agree bit for bit.
"""
import numpy as np
import pytest

from fake_context import FakeContext
from oracle.tsbts import OracleTSBTS, level_from_criterion
from paper_1205_2288_amd.driver import TSBTS, admissible, CriterionHistory
from workloads import config, plummer


def test_admissible_matches_oracle_block_condition():
    rng = np.random.default_rng(0)
    b = 2.0 ** rng.uniform(-24, 2, 4000)
    e = b * 2.0 ** rng.uniform(-3, 3, 4000)
    b[:20] = 2.0 ** -np.arange(20)           # exact powers of two (ties)
    e[:20] = b[:20]
    got = admissible(b, e, 1, 1 << 14)
    ref = [level_from_criterion(x, y, 1, 1 << 14) for x, y in zip(b, e)]
    assert np.array_equal(got, ref)
    assert admissible(np.inf, np.inf, 1, 1 << 14) == 1 << 14


def test_criterion_history_lookup():
    h = CriterionHistory()
    t0 = np.array([0, 0], dtype=np.int64)
    c0 = np.array([1.0, 8.0])
    h.add([0, 1], t0, c0)
    t0[:] = 99   # the stored start values must not follow later in-place updates
    c0[:] = -1.0
    h.add([0], 4, [3.0])
    h.add([0, 1], 8, [5.0, 2.0])
    h.close(2)
    pid = np.array([0, 0, 0, 1, 1, 1])
    t = np.array([0, 2, 6, 4, 8, 9])
    got = h.value_at(pid, t, np.full(6, 7.0))
    assert np.allclose(got, [1.0, 2.0, 4.0, 5.0, 2.0, 7.0])


@pytest.mark.parametrize("name,eras", [("plummer256", 4), ("plummer4096", 4)])
def test_scheduler_matches_oracle_bitwise(name, eras):
    cfg = config(name)
    r, v, m = cfg.ic()
    kw = dict(eta=cfg.eta, passes=3, era=cfg.era, dt_max=cfg.dt_max, dt_min=cfg.dt_min)
    prod = TSBTS(r, v, m, cfg.eps, context=FakeContext(cfg.n, cfg.eps), **kw)
    ref = OracleTSBTS(r, v, m, cfg.eps, **kw)
    assert np.array_equal(prod.dt, ref.dt)
    for _ in range(eras):
        assert prod.era_step() == ref.era_step()
        st = prod.state()
        assert np.array_equal(st["t"], ref.t)
        assert np.array_equal(st["dt"], ref.dt)
        assert np.array_equal(st["r"], ref.r)
        assert np.array_equal(st["v"], ref.v)
    assert prod.stats["block_steps"] == ref.stats["block_steps"]


def test_era_start_steps_and_schedule_match_oracle():
    # era = dt_max with a large eta: every particle is at each era start and its first
    # step is chosen again in the later passes; same choices and recorded schedule
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    kw = dict(eta=0.5, passes=3, era=cfg.dt_max, dt_max=cfg.dt_max, dt_min=cfg.dt_min)
    prod = TSBTS(r, v, m, cfg.eps, context=FakeContext(cfg.n, cfg.eps),
                 record_schedule=True, **kw)
    ref = OracleTSBTS(r, v, m, cfg.eps, record_schedule=True, **kw)
    for _ in range(12):
        assert prod.era_step() == ref.era_step()
        st = prod.state()
        for key in ("t", "dt", "dtp", "r", "v"):
            assert np.array_equal(st[key], getattr(ref, key)), key
    changed = 0
    for ea, eb in zip(prod.schedule["eras"], ref.schedule["eras"]):
        for p in range(3):
            assert np.array_equal(ea["dt_start"][p], eb["dt_start"][p])
            for (ta, ia, da), (tb, ib, db) in zip(ea["passes"][p], eb["passes"][p]):
                assert ta == tb and np.array_equal(ia, ib) and np.array_equal(da, db)
        changed += int(np.count_nonzero(ea["dt_start"][2] != ea["dt_start"][0]))
    assert changed > 0


def test_one_pass_and_energy_series_match_oracle():
    r, v, m = plummer(64, 8)
    kw = dict(eta=0.2, passes=1, era=1 / 32, dt_max=1 / 64, dt_min=2.0 ** -20)
    prod = TSBTS(r, v, m, 1 / 64, context=FakeContext(64, 1 / 64), **kw)
    ref = OracleTSBTS(r, v, m, 1 / 64, **kw)
    assert prod.run(0.25) == ref.run(0.25)


# ------------------------------------------------------------------ native scheduler rules
def test_native_admissible_matches_oracle():
    from paper_1205_2288_amd import _lib as L
    rng = np.random.default_rng(1)
    b = 2.0 ** rng.uniform(-24, 2, 3000)
    e = b * 2.0 ** rng.uniform(-3, 3, 3000)
    b[:20] = 2.0 ** -np.arange(20)
    e[:20] = b[:20]
    for x, y in zip(b, e):
        assert L.tsbts_sched_admissible(x, y, 1, 1 << 14) == \
            level_from_criterion(x, y, 1, 1 << 14)
    assert L.tsbts_sched_admissible(np.inf, 1.0, 1, 1 << 14) == 1 << 14


def test_native_rule_matches_oracle_rules():
    from paper_1205_2288_amd import _lib as L
    from oracle.tsbts import History
    DT, DTMAX = 1 << 10, 1 << 14
    rng = np.random.default_rng(2)
    for trial in range(400):
        dt = DT >> int(rng.integers(0, 3))
        tb = dt * int(rng.integers(1, 16))
        begin = dt * 2.0 ** -20 * 2.0 ** rng.uniform(-2, 3)
        ends = {c: dt * 2.0 ** -20 * 2.0 ** rng.uniform(-2, 3) for c in (dt, 2 * dt)}
        # oracle: previous-pass history holding exactly these end values
        s = OracleTSBTS.__new__(OracleTSBTS)
        s.n, s.dt_max, s.dt_min = 1, DTMAX, 1
        s.dt = np.array([dt], dtype=np.int64)
        h = History()
        for t, c in ((0, begin), (tb + dt, ends[dt]), (tb + 2 * dt, ends[2 * dt])):
            h.append([0], t, np.zeros((3, 1)), np.zeros((3, 1)), np.zeros((3, 1)), [c])
        h.freeze(1)
        first = trial % 3 == 0
        ref = s._new_step(0, tb, begin, None if first else h)
        got = L.tsbts_sched_rule(first, dt, tb, begin, ends[dt], ends[2 * dt], 1, DTMAX)
        assert got == ref, (trial, dt, tb, begin, ends)


def _oracle_era_end(t, dt, t0, dt_max, era=None):
    s = OracleTSBTS.__new__(OracleTSBTS)
    s.t = np.asarray(t, dtype=np.int64)
    s.dt = np.asarray(dt, dtype=np.int64)
    s.dt_max, s.era = dt_max, era
    return s._era_end(t0)


def _era_start_table(rng, n, t0, dt_max, top):
    """Particles in an era-start state at t0: power-of-two steps up to `top`, each at the
    last multiple of its step at or before t0."""
    lv = rng.integers(0, 9, n)
    dt = np.maximum(top >> lv, 1).astype(np.int64)
    t = (t0 // dt) * dt
    return t, dt


def test_native_era_end_matches_oracle():
    from paper_1205_2288_amd import _lib as L
    DTMAX = 1 << 14
    rng = np.random.default_rng(3)
    seen = set()
    for trial in range(600):
        top = DTMAX >> int(rng.integers(0, 6))  # largest step in use, up to dt_max/32
        n = int(rng.integers(1, 40))
        t0 = int(rng.integers(0, 64)) * (DTMAX >> 5)
        t, dt = _era_start_table(rng, n, t0, DTMAX, top)
        got = L.tsbts_sched_era_end(t0, t, dt, DTMAX)
        ref = _oracle_era_end(t, dt, t0, DTMAX)
        assert got == ref, (trial, t0, t, dt)
        seen.add(ref - t0 if ref % (ref - t0) == 0 else None)
        # fixed era: t0 + era
        assert L.tsbts_sched_era_end(t0, t, dt, DTMAX, 2 * DTMAX) == \
            _oracle_era_end(t, dt, t0, DTMAX, 2 * DTMAX) == t0 + 2 * DTMAX
    # the random tables reach every era size from dt_max/8 to dt_max
    assert {DTMAX >> k for k in range(4)} <= seen


def test_era_end_rule_cases_from_algorithm_3():
    """Algorithm 3 read literally: the era is the last minus the first block time, kept
    between the lower limit (dt_max/8, Section 4's 2^-3 multiples) and dt_max."""
    from paper_1205_2288_amd import _lib as L
    D = 1 << 14
    cases = [
        # every particle on one level far below dt_max: the difference is zero -> the
        # lower limit dt_max/8 (an era longer than every step)
        (0, [0, 0, 0], [D // 64] * 3, D // 8),
        # first block at t0 + D/64, last at t0 + D/4: difference 15D/64 -> 2^k above it
        # (D/4), the largest step D/4 fits
        (0, [0, 0], [D // 64, D // 4], D // 4),
        # a particle on the top level: last - first = D - D/64 -> dt_max
        (D, [D, D], [D // 64, D], 2 * D),
        # first block at t0 + D/32, last (a D/2 particle) at D: the difference 3D/16
        # rounds up to D/4, below the largest step D/2 -> dt_max (Section 4: the D/2
        # particles would have no past to be symmetrized with); the era ends at the next
        # multiple of dt_max
        (3 * D // 4 + D // 32, [D // 2, 3 * D // 4 + D // 32], [D // 2, D // 32], D),
        # era ends keep alignment: the next multiple of the size after t0
        (D // 16 + D // 64, [D // 16 + D // 64], [D // 64], D // 8),
    ]
    for t0, t, dt, end in cases:
        assert _oracle_era_end(t, dt, t0, D) == end, (t0, t, dt)
        assert L.tsbts_sched_era_end(t0, t, dt, D) == end, (t0, t, dt)


def test_native_era_end_refuses_a_state_that_is_not_an_era_start():
    from paper_1205_2288_amd import _lib as L
    D = 1 << 14
    for t0, t, dt in [(D, [D - D // 4], [D // 8]),   # due before t0
                      (D, [D // 3], [D]),            # not aligned to its step
                      (D, [D], [3])]:                # not a power of two
        with pytest.raises(L.TsbtsError):
            L.tsbts_sched_era_end(t0, t, dt, D)
    with pytest.raises(L.TsbtsError):
        L.tsbts_sched_era_end(0, [0], [D // 2], D, D // 2)  # era not a multiple of dt_max


def test_scheduler_dynamic_era_follows_oracle_bitwise():
    # eta = 0.05, dt_max = 1/8 on the 256-body sphere: Algorithm 3 sets the era to 1/8
    # while a particle is on the top level and to 1/16 afterwards
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    kw = dict(eta=0.05, passes=3, era=None, dt_max=1 / 8, dt_min=cfg.dt_min)
    prod = TSBTS(r, v, m, cfg.eps, context=FakeContext(cfg.n, cfg.eps), **kw)
    ref = OracleTSBTS(r, v, m, cfg.eps, **kw)
    for _ in range(4):
        assert prod.era_step() == ref.era_step()
        st = prod.state()
        for key in ("t", "dt", "dtp", "r", "v"):
            assert np.array_equal(st[key], getattr(ref, key)), key
    assert prod.stats["era_sizes"] == ref.stats["era_sizes"] == {"0.125": 2, "0.0625": 2}


def test_run_log_and_nonfinite_energy():
    # the run loop's JSON metrics (one line per energy sample) and its stop on a
    # non-finite energy
    import io
    import json
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    kw = dict(eta=cfg.eta, passes=2, era=cfg.era, dt_max=cfg.dt_max, dt_min=cfg.dt_min)
    prod = TSBTS(r, v, m, cfg.eps, context=FakeContext(cfg.n, cfg.eps), **kw)
    buf = io.StringIO()
    series = prod.run(0.25, energy_every=0.125, log=buf)
    recs = [json.loads(x) for x in buf.getvalue().splitlines()]
    assert [x["t"] for x in recs] == [t for t, _ in series] == [0.0, 0.125, 0.25]
    assert [x["E"] for x in recs] == [e for _, e in series]
    assert recs[0]["rel_dE"] == 0.0 and recs[0]["block_steps"] == 0
    assert recs[-1]["block_steps"] == prod.stats["block_steps"]
    assert recs[-1]["eras"] == prod.stats["eras"] == 2
    for x in recs:
        assert sum(x["levels"].values()) == cfg.n and x["excluded"] == 0
        assert all(6 <= int(k) <= 20 for k in x["levels"])
    prod.energy = lambda: float("nan")
    with pytest.raises(FloatingPointError, match="not finite"):
        prod.run(0.5, energy_every=0.125)
