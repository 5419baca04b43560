"""Host logic of the differentiated block-schedule run (no device needed).

``TsbtsBlockLeapfrog`` drives a CPU stand-in context whose entry points follow the C
header's definitions with the oracle's arithmetic; its schedule (block times, active
sets), checkpoint / recompute bookkeeping and reverse ordering must then reproduce the
oracle's reverse-mode gradient through the same fixed block schedule.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from workloads import plummer, gaussian
from fake_context import FakeContext
from paper_1205_2288_amd.autograd import (BlockSchedule, tsbts_block_leapfrog,
                                          tsbts_era_leapfrog, tsbts_schedule_leapfrog)


def _dt(n, h, seed, nlev=3):
    rng = np.random.default_rng(seed)
    return h * 2.0 ** rng.integers(0, nlev, size=n)


def test_block_schedule_matches_oracle_active_sets():
    n, h = 40, 1.0 / 64
    dt = _dt(n, h, 1, nlev=4)
    r0, v0, m = plummer(n, 3)
    sched = BlockSchedule(FakeContext(n, 0.1), dt, 16 * h)
    _, _, trace = oadj.block_forward(r0, v0, m, 0.1, dt, 16 * h)
    assert sched.K == len(trace)
    for s, (t_b, act, *_rest) in enumerate(trace):
        assert sched.time(s) == t_b
        assert np.array_equal(np.sort(sched.active(s).numpy()), act)


@pytest.mark.parametrize("bad", ["ratio", "t_end"])
def test_block_schedule_rejects_bad_steps(bad):
    n, h = 6, 1.0 / 64
    dt = np.full(n, h)
    t_end = 4 * h
    if bad == "ratio":
        dt[2] = 3 * h
    else:
        t_end = 4.5 * h
    with pytest.raises(ValueError):
        BlockSchedule(FakeContext(n, 0.1), dt, t_end)


@pytest.mark.parametrize("era", [1, 3, 16])
def test_block_leapfrog_gradient_matches_oracle(era):
    n, eps, h = 14, 1.0 / 16, 1.0 / 64
    t_end = 8 * h
    r0, v0, m = plummer(n, 27, masses="loguniform")
    dt = _dt(n, h, 5)
    rt, vt, _ = oadj.block_forward(r0, v0, m, eps, dt, t_end)
    rt = rt + 0.01 * gaussian((3, n), 11)
    vt = vt + 0.01 * gaussian((3, n), 12)
    L, gr, gv, gm = oadj.block_gradient(r0, v0, m, eps, dt, t_end, rt, vt)
    ctx = FakeContext(n, eps)
    r = torch.tensor(r0, requires_grad=True)
    v = torch.tensor(v0, requires_grad=True)
    mm = torch.tensor(m, requires_grad=True)
    r_end, v_end = tsbts_block_leapfrog(r, v, mm, ctx, dt, t_end, era)
    loss = ((r_end - torch.tensor(rt)) ** 2).sum() + ((v_end - torch.tensor(vt)) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(L, rel=1e-13)
    for got, ref in ((r.grad, gr), (v.grad, gv), (mm.grad, gm)):
        assert np.allclose(got.numpy(), ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_era_leapfrog_gradient_matches_oracle(passes):
    # eras with several passes: the reverse sweep's bookkeeping (rebuilt interpolation
    # sources, record adjoints handed from pass to pass, era-start sums) against the
    # oracle's reverse-mode gradient through the same schedule
    n, eps, h = 12, 1.0 / 16, 1.0 / 64
    t_end, era = 16 * h, 8 * h
    r0, v0, m = plummer(n, 28, masses="loguniform")
    dt = _dt(n, h, 6)
    rt, vt, _ = oadj.era_forward(r0, v0, m, eps, dt, t_end, era, passes)
    rt = rt + 0.01 * gaussian((3, n), 13)
    vt = vt + 0.01 * gaussian((3, n), 14)
    L, gr, gv, gm = oadj.era_gradient(r0, v0, m, eps, dt, t_end, era, passes, rt, vt)
    ctx = FakeContext(n, eps)
    r = torch.tensor(r0, requires_grad=True)
    v = torch.tensor(v0, requires_grad=True)
    mm = torch.tensor(m, requires_grad=True)
    r_end, v_end = tsbts_era_leapfrog(r, v, mm, ctx, dt, t_end, era, passes)
    loss = ((r_end - torch.tensor(rt)) ** 2).sum() + ((v_end - torch.tensor(vt)) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(L, rel=1e-13)
    for got, ref in ((r.grad, gr), (v.grad, gv), (mm.grad, gm)):
        assert np.allclose(got.numpy(), ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("era", [3.0 / 64, 4.0 / 64 + 1.0 / 128])
def test_era_leapfrog_rejects_bad_eras(era):
    n, h = 6, 1.0 / 64
    dt = np.full(n, h)
    dt[0] = 4 * h
    r0, v0, m = plummer(n, 3)
    with pytest.raises(ValueError):
        tsbts_era_leapfrog(torch.tensor(r0), torch.tensor(v0), torch.tensor(m),
                           FakeContext(n, 0.1), dt, 16 * h, era, 2)


@pytest.mark.parametrize("passes,era", [(1, None), (3, None), (2, 1.0 / 32)])
def test_recorded_schedule_gradient_matches_oracle(passes, era):
    # a schedule chosen by the criterion (the oracle's era driver, dynamic or fixed eras),
    # replayed: end state and gradient against the oracle's replay of the same schedule
    from oracle.tsbts import OracleTSBTS
    n, eps = 12, 1.0 / 64
    r0, v0, m = plummer(n, 45, masses="loguniform")
    sim = OracleTSBTS(r0, v0, m, eps, passes=passes, dt_max=1.0 / 64, era=era,
                      record_schedule=True)
    sim.run(0.125)
    sched = sim.schedule
    rt = sim.r + 0.01 * gaussian((3, n), 15)
    vt = sim.v + 0.01 * gaussian((3, n), 16)
    L, gr, gv, gm = oadj.schedule_gradient(r0, v0, m, eps, sched, rt, vt)
    ctx = FakeContext(n, eps)
    r = torch.tensor(r0, requires_grad=True)
    v = torch.tensor(v0, requires_grad=True)
    mm = torch.tensor(m, requires_grad=True)
    r_end, v_end = tsbts_schedule_leapfrog(r, v, mm, ctx, sched)
    assert np.array_equal(r_end.detach().numpy(), sim.r)
    loss = ((r_end - torch.tensor(rt)) ** 2).sum() + ((v_end - torch.tensor(vt)) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(L, rel=1e-13)
    for got, ref in ((r.grad, gr), (v.grad, gv), (mm.grad, gm)):
        assert np.allclose(got.numpy(), ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
