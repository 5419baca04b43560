"""Split calls of large partial active sets (the pairs among the targets once for both
particles by the symmetric kernels on a compact copy of the targets, the pairs with the
other particles by the gather kernels on a compact copy of those): the criterion must
equal the one-part gather bit for bit (maxima and minima do not depend on order), the
force and potential must agree with the gather kernels up to the rounding of the partial
sums and with the oracle within the usual bars.  Sizes span one and several symmetric
work items and gather tiles, ragged counts on both sides, unsorted lists, one inactive
particle, and the benchmark size."""
import time

import numpy as np
import pytest
import torch

import oracle
from workloads import plummer, config
from gpu_util import rel_err, rel_err_vec, summary, make_ctx

pytestmark = pytest.mark.gpu

CASES = [("fp64", "hilo"), ("mixed", "hilo"), ("mixed", "f64")]
# (particles, active): the smallest split call, ragged counts, one inactive particle
SHAPES = [(20000, 8192), (20000, 12345), (20000, 19999), (40961, 30001)]


def _subset(n, k, seed):
    return np.random.default_rng(seed).permutation(n)[:k].astype(np.int32)


def _ctx(n, eps, prec, sep, seed):
    r, v, m = plummer(n, seed, masses="loguniform")
    ctx = make_ctx(n, eps, prec, sep)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    return ctx, r, v, m


@pytest.mark.parametrize("prec,sep", CASES)
@pytest.mark.parametrize("n,k", SHAPES)
def test_split_criterion_equals_gather(prec, sep, n, k):
    eps, eta = 1 / 256, 0.1
    ctx, r, v, m = _ctx(n, eps, prec, sep, 4100 + k)
    idx = _subset(n, k, k)
    ctx.tune(split=0)
    ref = ctx.timestep(idx, eta).cpu().numpy()
    ctx.tune(split=1)
    got = ctx.timestep(idx, eta).cpu().numpy()
    assert np.array_equal(got, ref), (np.flatnonzero(got != ref)[:10], got[got != ref][:5])
    sample = np.arange(0, k, max(1, k // 64))
    e = rel_err(got[sample], oracle.timestep(r, v, m, eps, eta, idx[sample]))
    assert e.max() <= (1e-12 if prec == "fp64" else 2e-6), summary(e)
    ctx.close()


@pytest.mark.parametrize("prec,sep", CASES)
@pytest.mark.parametrize("n,k", SHAPES)
def test_split_force_matches_gather_and_oracle(prec, sep, n, k):
    eps = 1 / 256
    ctx, r, v, m = _ctx(n, eps, prec, sep, 4200 + k)
    idx = _subset(n, k, k + 1)
    ctx.tune(split=0)
    a0, p0 = (x.cpu().numpy() for x in ctx.force(idx, 0.0))
    ctx.tune(split=1)
    a1, p1 = (x.cpu().numpy() for x in ctx.force(idx, 0.0))
    a2, p2 = (x.cpu().numpy() for x in ctx.force(idx, 0.0))
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)  # fixed order
    # without the potential (the symmetric part groups its column sums differently, so
    # the accelerations agree up to rounding)
    a3 = ctx.force(idx, 0.0, with_pot=False)[0].cpu().numpy()
    d3 = rel_err_vec(a3, a1)
    sample = np.arange(0, k, max(1, k // 128))
    ra, rp = oracle.force(r, m, eps, idx[sample])
    e = rel_err_vec(a1[:, sample], ra)
    ep = rel_err(p1[sample], rp)
    d = rel_err_vec(a1, a0)
    if prec == "fp64":
        assert e.max() <= 1e-12, summary(e)
        assert ep.max() <= 1e-12, summary(ep)
        assert d.max() <= 1e-12 and d3.max() <= 1e-12, (summary(d), summary(d3))
        assert rel_err(p1, p0).max() <= 1e-12
    else:
        assert np.median(e) <= 1e-6 and e.max() <= 1e-5, summary(e)
        assert ep.max() <= 1e-5, summary(ep)
        # the gather kernels' sums up to float32 rounding of the partial sums
        assert np.median(d) <= 1e-6 and d.max() <= 1e-5, summary(d)
        assert np.median(d3) <= 1e-6 and d3.max() <= 1e-5, summary(d3)
    ctx.close()


def test_split_not_used_below_its_sizes():
    # below 8192 targets, and with every particle a target, a forced split changes nothing
    n, eps, eta = 20000, 1 / 256, 0.1
    ctx, r, v, m = _ctx(n, eps, "mixed", "f64", 4300)
    for k in (8191, n):
        idx = _subset(n, k, 7)
        out = []
        for split in (0, 1):
            ctx.tune(split=split)
            out.append((ctx.force(idx, 0.0)[0].cpu().numpy(),
                        ctx.timestep(idx, eta).cpu().numpy()))
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    ctx.close()


@pytest.mark.parametrize("case", ["newton", "chunk"])
def test_split_not_used_for_newton_or_tuned_chunk(case):
    # the Newton-step form (no symmetric kernel) and a tuned j-unit keep the gather
    # kernels: a forced split changes nothing
    n, k, eps, eta = 20000, 12000, 1 / 256, 0.1
    r, v, m = plummer(n, 4310, masses="loguniform")
    ctx = make_ctx(n, eps, "mixed", "f64", newton=(case == "newton"))
    if case == "chunk":
        ctx.tune(chunk=256)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _subset(n, k, 8)
    out = []
    for split in (0, 1):
        ctx.tune(split=split)
        out.append((ctx.force(idx, 0.0)[0].cpu().numpy(), ctx.timestep(idx, eta).cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_split_after_corrector(prec):
    # the corrector from split forces, then the criterion (the targets' velocities are
    # rewritten, so the copies are taken again): the corrected velocities differ from the
    # gather run's by the force differences times h/2, the criterion by about as much
    n, eps, eta, h = 20000, 1 / 256, 0.1, 1 / 1024
    r, v, m = plummer(n, 4400, masses="loguniform")
    idx = _subset(n, 10000, 9)
    out = []
    for split in (0, 1):
        ctx = make_ctx(n, eps, prec)
        ctx.tune(split=split)
        ctx.bind(r, v, m, dt=np.full(n, h))
        ctx.predict(h)
        acc = ctx.force(idx, h, with_pot=False)[0]
        ctx.correct(idx, h, acc)
        out.append((acc.cpu().numpy(), ctx.v.cpu().numpy().copy(),
                    ctx.timestep(idx, eta).cpu().numpy()))
        ctx.close()
    (a0, v0, d0), (a1, v1, d1) = out
    dv = np.abs(v1[:, idx] - v0[:, idx])
    assert np.all(dv <= h * np.abs(a1 - a0) + 1e-15 * (np.abs(v0[:, idx]) + h * np.abs(a0)))
    rest = np.setdiff1d(np.arange(n), idx)
    assert np.array_equal(v1[:, rest], v0[:, rest])
    assert rel_err(d1, d0).max() <= (1e-12 if prec == "fp64" else 1e-5)


def test_split_in_native_runs():
    # whole runs of the native scheduler (force with the corrector in its finishing step,
    # criterion) with and without split calls: the criterion is the same function of the
    # state and the forces differ only by rounding, so schedules and energy errors agree
    from paper_1205_2288_amd.driver import NativeTSBTS
    # (a largest step of 1/16 spreads the particles over several levels: the block steps
    # between era ends have thousands of active particles, many of them at least 8192)
    n, eps = 16384, 1 / 256
    r, v, m = plummer(n, 4500)
    runs = []
    for split in (0, 1):
        sim = NativeTSBTS(r, v, m, eps, passes=3, era=1 / 16, dt_max=1 / 16,
                          tune={"split": split})
        series = sim.run(1 / 8)
        e0 = series[0][1]
        runs.append((sim.stats["block_steps"], abs(series[-1][1] - e0) / abs(e0),
                     sim.ctx.r.cpu().numpy().copy()))
        # the block steps at odd multiples of a step size s have every particle with a step
        # of at most s active: some of those counts lie in [8192, n), so split calls ran
        dt = np.asarray(sim.dt)
        active = [int((dt <= s).sum()) for s in np.unique(dt)[:-1]]
        assert any(8192 <= a < n for a in active), active
        sim.close()
    print(f"native runs N={n}: gather {runs[0][0]} block steps, drift {runs[0][1]:.3e}; "
          f"split {runs[1][0]} block steps, drift {runs[1][1]:.3e}")
    assert abs(runs[0][0] - runs[1][0]) <= 0.01 * runs[0][0]
    assert abs(runs[0][1] - runs[1][1]) <= 0.05 * runs[0][1] + 1e-9
    assert np.abs(runs[0][2] - runs[1][2]).max() <= 1e-5


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_plummer131k_half_active_split(prec):
    # the benchmark workload with half the particles active: force and criterion with and
    # without split calls (prints both times), sampled rows against the oracle
    cfg = config("plummer131k")
    n, eps, eta = cfg.n, cfg.eps, 0.1
    r, v, m = cfg.ic()
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    k = n // 2
    idx = _subset(n, k, 11)
    acc = torch.empty((3, k), dtype=torch.float64, device="cuda")
    out, ms = {}, {}
    for split in (0, 1):
        ctx.tune(split=split)
        ctx.force(idx, 0.0, with_pot=False, acc=acc)
        d = ctx.timestep(idx, eta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ctx.force(idx, 0.0, with_pot=False, acc=acc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(3):
            d = ctx.timestep(idx, eta)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ms[split] = ((t1 - t0) / 3 * 1e3, (t2 - t1) / 3 * 1e3)
        out[split] = (acc.cpu().numpy().copy(), d.cpu().numpy())
    print(f"plummer131k {prec}, {k} targets: force gather {ms[0][0]:.2f} ms, split "
          f"{ms[1][0]:.2f} ms; criterion gather {ms[0][1]:.2f} ms, split {ms[1][1]:.2f} ms")
    assert np.array_equal(out[0][1], out[1][1])
    sample = np.arange(0, k, k // 256)
    ra, _ = oracle.force(r, m, eps, idx[sample])
    e = rel_err_vec(out[1][0][:, sample], ra)
    if prec == "fp64":
        assert e.max() <= 1e-12, summary(e)
    else:
        assert np.median(e) <= 1e-6 and e.max() <= 1e-5, summary(e)
        assert np.median(rel_err_vec(out[1][0], out[0][0])) <= 1e-6
    ctx.close()
