"""Pins of the oracle's force adjoint and of its gradient through a leapfrog run.

The force adjoint is checked against central finite differences of the oracle force
(a different code path: only the forward loops), and against two exact identities:
translation invariance (the gradient summed over particles vanishes) and Euler's theorem
(acceleration and potential are homogeneous of degree one in the masses).  The gradients
through runs (shared step, fixed block schedule, eras with several passes) are checked
against central finite differences of the oracle runs, and the multi-pass run itself
against the era driver of `oracle.tsbts` on the same fixed schedule."""
import numpy as np
import pytest

from workloads import plummer, active_subset, gaussian
from oracle import adjoint


def _loss(oracle, r, m, eps, idx, ga, gp):
    a, p = oracle.force(r, m, eps, idx)
    return float((a * ga).sum() + (p * gp).sum())


@pytest.mark.parametrize("n_act", [1, 5, 12])
def test_force_backward_vs_finite_differences(oracle, n_act):
    n, eps = 12, 0.05
    r, _, m = plummer(n, 21, masses="loguniform")
    idx = active_subset(n, n_act, 3 + n_act)
    ga = gaussian((3, n_act), 31)
    gp = gaussian(n_act, 32)
    gr, gm = oracle.force_backward(r, m, eps, idx, ga, gp)
    h = 1e-5
    for trial in range(6):
        dr = gaussian((3, n), 100 + trial)
        dm = gaussian(n, 200 + trial) * m
        fd_r = (_loss(oracle, r + h * dr, m, eps, idx, ga, gp)
                - _loss(oracle, r - h * dr, m, eps, idx, ga, gp)) / (2 * h)
        fd_m = (_loss(oracle, r, m + h * dm, eps, idx, ga, gp)
                - _loss(oracle, r, m - h * dm, eps, idx, ga, gp)) / (2 * h)
        assert (gr * dr).sum() == pytest.approx(fd_r, rel=1e-6, abs=1e-9)
        assert (gm * dm).sum() == pytest.approx(fd_m, rel=1e-6, abs=1e-9)


def test_force_backward_identities(oracle):
    n, eps = 200, 0.02
    r, _, m = plummer(n, 22, masses="loguniform")
    idx = active_subset(n, 50, 9)
    ga = gaussian((3, 50), 41)
    gp = gaussian(50, 42)
    gr, gm = oracle.force_backward(r, m, eps, idx, ga, gp)
    a, p = oracle.force(r, m, eps, idx)
    scale = np.abs(gr).sum()
    assert np.abs(gr.sum(axis=1)).max() <= 1e-12 * scale
    euler = (a * ga).sum() + (p * gp).sum()
    assert (m * gm).sum() == pytest.approx(euler, rel=1e-11)


def test_force_backward_accumulates(oracle):
    n = 20
    r, _, m = plummer(n, 23)
    idx = np.arange(n, dtype=np.int32)
    ga = gaussian((3, n), 5)
    gr, gm = oracle.force_backward(r, m, 0.1, idx, ga)
    gr2, gm2 = oracle.force_backward(r, m, 0.1, idx, 2.0 * ga)
    assert np.allclose(gr2, 2 * gr, rtol=1e-14, atol=0)
    assert np.allclose(gm2, 2 * gm, rtol=1e-14, atol=0)


def test_leapfrog_gradient_vs_finite_differences(oracle):
    n, eps, h, steps = 16, 1.0 / 16, 1.0 / 64, 8
    r0, v0, m = plummer(n, 24, masses="loguniform")
    target = adjoint.forward(r0, v0, m, eps, h, steps)[0] + 0.01 * gaussian((3, n), 6)
    L, gr, gv, gm = adjoint.gradient(r0, v0, m, eps, h, steps, target)
    assert L == pytest.approx(adjoint.loss(r0, v0, m, eps, h, steps, target), rel=1e-15)
    step = 1e-6
    for trial in range(4):
        dr = gaussian((3, n), 300 + trial)
        dv = gaussian((3, n), 400 + trial)
        dm = gaussian(n, 500 + trial) * m
        for (g, d, which) in ((gr, dr, "r"), (gv, dv, "v"), (gm, dm, "m")):
            def f(sgn):
                rr = r0 + sgn * step * d if which == "r" else r0
                vv = v0 + sgn * step * d if which == "v" else v0
                mm = m + sgn * step * d if which == "m" else m
                return adjoint.loss(rr, vv, mm, eps, h, steps, target)
            fd = (f(1) - f(-1)) / (2 * step)
            assert (g * d).sum() == pytest.approx(fd, rel=2e-6, abs=1e-10), which


def _levels_dt(n, h, seed, nlev=3):
    rng = np.random.default_rng(seed)
    return h * 2.0 ** rng.integers(0, nlev, size=n)


def test_block_forward_schedule_and_shared_limit(oracle):
    # the schedule: particle i is active exactly every dt_i; with one common step the
    # block run is the shared-step leapfrog
    n, eps, h = 12, 1.0 / 16, 1.0 / 64
    r0, v0, m = plummer(n, 31)
    dt = _levels_dt(n, h, 3)
    _, _, trace = adjoint.block_forward(r0, v0, m, eps, dt, 8 * h)
    assert [t for (t, *_rest) in trace] == [h * (s + 1) for s in range(8)]
    for (t_b, act, *_rest) in trace:
        expect = np.nonzero(np.mod(t_b, dt) == 0.0)[0]
        assert np.array_equal(act, expect)
    rb, vb, _ = adjoint.block_forward(r0, v0, m, eps, np.full(n, h), 8 * h)
    rs, states = adjoint.forward(r0, v0, m, eps, h, 8)
    assert np.array_equal(rb, rs) and np.array_equal(vb, states[-1][1])


def test_block_gradient_vs_finite_differences(oracle):
    n, eps, h = 14, 1.0 / 16, 1.0 / 64
    t_end = 8 * h
    r0, v0, m = plummer(n, 25, masses="loguniform")
    dt = _levels_dt(n, h, 4)
    rt, vt, _ = adjoint.block_forward(r0, v0, m, eps, dt, t_end)
    rt = rt + 0.01 * gaussian((3, n), 7)
    vt = vt + 0.01 * gaussian((3, n), 8)
    L, gr, gv, gm = adjoint.block_gradient(r0, v0, m, eps, dt, t_end, rt, vt)
    assert L == pytest.approx(adjoint.block_loss(r0, v0, m, eps, dt, t_end, rt, vt),
                              rel=1e-15)
    step = 1e-6
    for trial in range(3):
        dr = gaussian((3, n), 600 + trial)
        dv = gaussian((3, n), 700 + trial)
        dm = gaussian(n, 800 + trial) * m
        for (g, d, which) in ((gr, dr, "r"), (gv, dv, "v"), (gm, dm, "m")):
            def f(sgn):
                rr = r0 + sgn * step * d if which == "r" else r0
                vv = v0 + sgn * step * d if which == "v" else v0
                mm = m + sgn * step * d if which == "m" else m
                return adjoint.block_loss(rr, vv, mm, eps, dt, t_end, rt, vt)
            fd = (f(1) - f(-1)) / (2 * step)
            assert (g * d).sum() == pytest.approx(fd, rel=2e-6, abs=1e-10), which


def test_block_gradient_shared_limit(oracle):
    # one common step: the block gradient must equal the shared-step gradient plus the
    # velocity part of the loss (checked with a zero-weight velocity target)
    n, eps, h = 10, 1.0 / 16, 1.0 / 64
    r0, v0, m = plummer(n, 26)
    dt = np.full(n, h)
    rt = adjoint.forward(r0, v0, m, eps, h, 6)[0] + 0.01 * gaussian((3, n), 9)
    v_end = adjoint.block_forward(r0, v0, m, eps, dt, 6 * h)[1]
    Lb, gr_b, gv_b, gm_b = adjoint.block_gradient(r0, v0, m, eps, dt, 6 * h, rt, v_end)
    Ls, gr_s, gv_s, gm_s = adjoint.gradient(r0, v0, m, eps, h, 6, rt)
    assert Lb == pytest.approx(Ls, rel=1e-14)
    for a, b in ((gr_b, gr_s), (gv_b, gv_s), (gm_b, gm_s)):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * np.abs(b).max())


@pytest.mark.parametrize("n_act", [1, 40, 97])
def test_force_backward_rows_equal_full(oracle, n_act):
    # the row-restricted gradient is the full one's rows, element by element (the same
    # per-row loops; the full function is pinned by finite differences above)
    n, eps = 97, 1.0 / 32
    r, _, m = plummer(n, 33, masses="loguniform")
    idx = active_subset(n, n_act, 4)
    ga, gp = gaussian((3, n_act), 5), gaussian(n_act, 6)
    gr, gm = oracle.force_backward(r, m, eps, idx, ga, gp)
    rows = np.array([0, 5, 17, 96, 40, 41], dtype=np.int32)
    rr, rm = oracle.force_backward_rows(r, m, eps, idx, ga, rows, gp)
    assert np.array_equal(rr, gr[:, rows]) and np.array_equal(rm, gm[rows])


@pytest.mark.parametrize("n_act", [1, 40, 97])
def test_force_backward_scale_bounds_and_equality(oracle, n_act):
    # the rounding scale bounds the gradient component by component (triangle
    # inequality) and its row form is the full form's rows
    n, eps = 97, 1.0 / 32
    r, _, m = plummer(n, 34, masses="loguniform")
    m[3] = 0.0  # a massless particle: its position gradient and scale vanish
    idx = active_subset(n, n_act, 7)
    ga, gp = gaussian((3, n_act), 8), gaussian(n_act, 9)
    gr, gm = oracle.force_backward(r, m, eps, idx, ga, gp)
    sr, sm = oracle.force_backward_scale(r, m, eps, idx, ga, gp)
    assert (np.abs(gr) <= sr * (1 + 1e-12)).all() and (np.abs(gm) <= sm * (1 + 1e-12)).all()
    # every particle with a target other than itself has a nonzero mass-gradient scale
    others = np.setdiff1d(np.arange(n), idx) if n_act == 1 else np.arange(n)
    assert (sr > 0).sum() >= 3 * (n - 2) and sm[others].min() > 0
    if 3 not in idx:
        assert (sr[:, 3] == 0).all() and (gr[:, 3] == 0).all()
    rows = np.array([0, 3, 17, 96, 40], dtype=np.int32)
    srr, smr = oracle.force_backward_scale(r, m, eps, idx, ga, gp, rows=rows)
    assert np.array_equal(srr, sr[:, rows]) and np.array_equal(smr, sm[rows])


def test_force_backward_scale_single_term_equality(oracle):
    # two particles, one target: with the seed along x and the separation along y (no
    # d.g term), or a potential seed alone, every component of the source row is one
    # term, so the scale equals the gradient's magnitude exactly
    eps = 0.1
    r = np.array([[0.0, 0.0], [0.0, 0.7], [0.0, 0.0]])
    m = np.array([0.3, 0.9])
    idx = np.array([0], dtype=np.int32)
    for ga, gp in ((np.array([[2.0], [0.0], [0.0]]), np.zeros(1)),
                   (np.zeros((3, 1)), np.array([-1.5]))):
        gr, gm = oracle.force_backward(r, m, eps, idx, ga, gp)
        sr, sm = oracle.force_backward_scale(r, m, eps, idx, ga, gp)
        assert np.array_equal(sr[:, 1], np.abs(gr[:, 1]))
        assert sm[1] == abs(gm[1])


# ---------------------------------------------------------------- eras and passes
def test_era_forward_matches_the_era_driver(oracle):
    # the fixed-schedule multi-pass run is the era driver's run when the criterion hands
    # every particle its own fixed step (two independent codings of Section 2's passes)
    from oracle.tsbts import OracleTSBTS, TICK
    n, eps, h = 16, 1.0 / 16, 1.0 / 64
    r0, v0, m = plummer(n, 41)
    dt = _levels_dt(n, h, 5)
    for passes in (1, 3):
        r, v, _ = adjoint.era_forward(r0, v0, m, eps, dt, 16 * h, 8 * h, passes)
        sim = OracleTSBTS(r0, v0, m, eps, passes=passes, dt_max=4 * h, era=8 * h,
                          criterion=lambda rr, vv, idx: dt[idx])
        sim.run(16 * h)
        assert np.all(sim.dt * TICK == dt)
        assert np.allclose(r, sim.r, rtol=0, atol=1e-13)
        assert np.allclose(v, sim.v, rtol=0, atol=1e-12)


def test_era_forward_passes_change_the_run(oracle):
    # later passes interpolate the non-active particles, so the result moves (by the
    # interpolation error, small but far above rounding); one pass is the block run
    n, eps, h = 16, 1.0 / 16, 1.0 / 64
    r0, v0, m = plummer(n, 42)
    dt = _levels_dt(n, h, 6)
    r1, v1, _ = adjoint.era_forward(r0, v0, m, eps, dt, 16 * h, 8 * h, 1)
    rb, vb, _ = adjoint.block_forward(r0, v0, m, eps, dt, 16 * h)
    assert np.array_equal(r1, rb) and np.array_equal(v1, vb)
    r2, _, _ = adjoint.era_forward(r0, v0, m, eps, dt, 16 * h, 8 * h, 2)
    r3, _, _ = adjoint.era_forward(r0, v0, m, eps, dt, 16 * h, 8 * h, 3)
    assert 1e-10 < np.abs(r2 - r1).max() < 1e-4
    assert 1e-12 < np.abs(r3 - r2).max() < np.abs(r2 - r1).max()


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_era_gradient_vs_finite_differences(oracle, passes):
    n, eps, h = 10, 1.0 / 16, 1.0 / 64
    t_end, era = 16 * h, 8 * h
    r0, v0, m = plummer(n, 27, masses="loguniform")
    dt = _levels_dt(n, h, 7)
    rt, vt, _ = adjoint.era_forward(r0, v0, m, eps, dt, t_end, era, passes)
    rt = rt + 0.01 * gaussian((3, n), 17)
    vt = vt + 0.01 * gaussian((3, n), 18)
    L, gr, gv, gm = adjoint.era_gradient(r0, v0, m, eps, dt, t_end, era, passes, rt, vt)
    assert L == pytest.approx(
        adjoint.era_loss(r0, v0, m, eps, dt, t_end, era, passes, rt, vt), rel=1e-15)
    if passes == 1:
        ref = adjoint.block_gradient(r0, v0, m, eps, dt, t_end, rt, vt)
        for a, b in zip((L, gr, gv, gm), ref):
            assert np.array_equal(a, b)
    step = 1e-6
    for trial in range(2):
        dr = gaussian((3, n), 610 + trial)
        dv = gaussian((3, n), 710 + trial)
        dm = gaussian(n, 810 + trial) * m
        for (g, d, which) in ((gr, dr, "r"), (gv, dv, "v"), (gm, dm, "m")):
            def f(sgn):
                rr = r0 + sgn * step * d if which == "r" else r0
                vv = v0 + sgn * step * d if which == "v" else v0
                mm = m + sgn * step * d if which == "m" else m
                return adjoint.era_loss(rr, vv, mm, eps, dt, t_end, era, passes, rt, vt)
            fd = (f(1) - f(-1)) / (2 * step)
            assert (g * d).sum() == pytest.approx(fd, rel=2e-6, abs=1e-10), which


# ---------------------------------------------------------------- recorded schedules
def _recorded(n, seed, passes, era, t_end):
    from oracle.tsbts import OracleTSBTS
    r0, v0, m = plummer(n, seed)
    sim = OracleTSBTS(r0, v0, m, 1.0 / 64, passes=passes, dt_max=1.0 / 64, era=era,
                      record_schedule=True)
    sim.run(t_end)
    return r0, v0, m, sim


@pytest.mark.parametrize("passes,era", [(1, None), (3, None), (3, 1.0 / 32)])
def test_schedule_replay_matches_the_era_driver(oracle, passes, era):
    # the era driver's own steps (criterion, Algorithm 1, dynamic or fixed eras), replayed
    # by the schedule run, give the driver's end state
    r0, v0, m, sim = _recorded(20, 43, passes, era, 0.25)
    levels = {float(d) for e in sim.schedule["eras"] for p in e["passes"]
              for (_, _, dts) in p for d in dts}
    assert len(levels) >= 3     # a schedule with several step levels
    assert all(len(e["passes"]) == passes for e in sim.schedule["eras"])
    r, v, _ = adjoint.schedule_forward(r0, v0, m, 1.0 / 64, sim.schedule)
    assert np.array_equal(r, sim.r) and np.array_equal(v, sim.v)


def test_schedule_gradient_vs_finite_differences(oracle):
    r0, v0, m, sim = _recorded(10, 44, 3, None, 0.125)
    eps, sched = 1.0 / 64, sim.schedule
    rt = sim.r + 0.01 * gaussian((3, 10), 19)
    vt = sim.v + 0.01 * gaussian((3, 10), 20)
    L, gr, gv, gm = adjoint.schedule_gradient(r0, v0, m, eps, sched, rt, vt)
    step = 1e-6
    for trial in range(2):
        dr = gaussian((3, 10), 620 + trial)
        dv = gaussian((3, 10), 720 + trial)
        dm = gaussian(10, 820 + trial) * m
        for (g, d, which) in ((gr, dr, "r"), (gv, dv, "v"), (gm, dm, "m")):
            def f(sgn):
                rr = r0 + sgn * step * d if which == "r" else r0
                vv = v0 + sgn * step * d if which == "v" else v0
                mm = m + sgn * step * d if which == "m" else m
                return adjoint.schedule_loss(rr, vv, mm, eps, sched, rt, vt)
            fd = (f(1) - f(-1)) / (2 * step)
            assert (g * d).sum() == pytest.approx(fd, rel=2e-6, abs=1e-10), which
