"""Symmetric all-targets kernels (every particle a target, each unordered pair evaluated
once for both particles): the criterion must equal the gather kernels bit for bit (its
maxima and minima do not depend on order) and the oracle within the usual bars, at sizes
below, at and above one work item, with ragged tails, any order of the active list, and
at the full benchmark size."""
import time

import numpy as np
import pytest
import torch

import oracle
from workloads import plummer, gaussian, config
from gpu_util import rel_err, summary, make_ctx, check_adjoint

pytestmark = pytest.mark.gpu

CASES = [("fp64", "hilo"), ("mixed", "hilo"), ("mixed", "f64")]


def _perm(n, seed):
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


def _state(n, seed):
    r, v, m = plummer(n, seed, masses="loguniform")
    return r, v, m


@pytest.mark.parametrize("prec,sep", CASES)
@pytest.mark.parametrize("n", [3, 300, 512, 700, 1100, 5000])
def test_symmetric_criterion_equals_gather(prec, sep, n):
    eps, eta = 1 / 256, 0.1
    r, v, m = _state(n, 3100 + n)
    ctx = make_ctx(n, eps, prec, sep)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, n)
    ctx.tune(symmetric=0)
    ref = ctx.timestep(idx, eta).cpu().numpy()
    ctx.tune(symmetric=1)
    got = ctx.timestep(idx, eta).cpu().numpy()
    assert np.array_equal(got, ref), (np.flatnonzero(got != ref)[:10], got[got != ref][:5])
    e = rel_err(got, oracle.timestep(r, v, m, eps, eta, idx))
    assert e.max() <= (1e-12 if prec == "fp64" else 2e-6), summary(e)
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_symmetric_criterion_after_corrector_and_zero_velocities(prec):
    # after a corrector (the planes the criterion reads are rewritten) and with explicit
    # positions (zero velocities: the collision term vanishes for every pair)
    n, eps, eta, h = 2000, 1 / 256, 0.1, 1 / 1024
    r, v, m = _state(n, 3200)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m, dt=np.full(n, h))
    every = np.arange(n, dtype=np.int32)
    ctx.predict(h)
    acc = ctx.force(every, h, with_pot=False)[0]
    ctx.correct(every, h, acc)
    outs = []
    for sym in (0, 1):
        ctx.tune(symmetric=sym)
        outs.append(ctx.timestep(every, eta).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    ctx.load_positions(r, m, 0.0)
    outs = []
    for sym in (0, 1):
        ctx.tune(symmetric=sym)
        outs.append(ctx.timestep(every, eta).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    ctx.close()


def test_symmetric_criterion_not_used_for_subsets():
    # a proper subset takes the gather kernels even when forced (same answer either way)
    n, eps, eta = 3000, 1 / 256, 0.1
    r, v, m = _state(n, 3300)
    ctx = make_ctx(n, eps, "mixed")
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, 5)[:2999]
    ctx.tune(symmetric=1)
    a = ctx.timestep(idx, eta).cpu().numpy()
    ctx.tune(symmetric=0)
    b = ctx.timestep(idx, eta).cpu().numpy()
    assert np.array_equal(a, b)
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_plummer131k_symmetric_criterion(prec):
    # the benchmark workload, all particles: bitwise against the gather kernel, sampled
    # against the oracle; prints both kernels' times
    cfg = config("plummer131k")
    n, eps, eta = cfg.n, cfg.eps, 0.1
    r, v, m = cfg.ic()
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, 7)
    out, ms = {}, {}
    for sym in (0, 1):
        ctx.tune(symmetric=sym)
        ctx.timestep(idx, eta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            d = ctx.timestep(idx, eta)
        torch.cuda.synchronize()
        ms[sym] = (time.perf_counter() - t0) / 3 * 1e3
        out[sym] = d.cpu().numpy()
    print(f"plummer131k {prec} criterion, all targets: gather {ms[0]:.2f} ms, "
          f"symmetric {ms[1]:.2f} ms")
    assert np.array_equal(out[0], out[1])
    sample = idx[:: n // 256]
    e = rel_err(out[1][np.argsort(idx)][sample], oracle.timestep(r, v, m, eps, eta, sample))
    assert e.max() <= (1e-12 if prec == "fp64" else 2e-6), summary(e)
    ctx.close()


# ---------------------------------------------------------------- force and potential
from gpu_util import rel_err_vec  # noqa: E402


@pytest.mark.parametrize("prec,sep", CASES)
@pytest.mark.parametrize("n", [3, 300, 700, 1100, 5000])
def test_symmetric_force_matches_gather_and_oracle(prec, sep, n):
    eps = 1 / 256
    r, v, m = _state(n, 3400 + n)
    ctx = make_ctx(n, eps, prec, sep)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, n + 1)
    ctx.tune(symmetric=0)
    a0, p0 = (x.cpu().numpy() for x in ctx.force(idx, 0.0))
    ctx.tune(symmetric=1)
    a1, p1 = (x.cpu().numpy() for x in ctx.force(idx, 0.0))
    a2, p2 = (x.cpu().numpy() for x in ctx.force(idx, 0.0))
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)   # fixed order
    ra, rp = oracle.force(r, m, eps, idx)
    e = rel_err_vec(a1, ra)
    if prec == "fp64":
        assert e.max() <= 1e-12, summary(e)
        assert rel_err(p1, rp).max() <= 1e-12
        assert rel_err_vec(a1, a0).max() <= 1e-12
    else:
        assert np.median(e) <= 1e-6 and e.max() <= 1e-4, summary(e)
        assert rel_err(p1, rp).max() <= 1e-5
        # same sums as the gather kernel up to float32 rounding of the partial sums
        assert np.median(rel_err_vec(a1, a0)) <= 1e-6
    ctx.close()


def test_symmetric_kernels_in_native_runs():
    # whole runs of the native scheduler (all-particle block steps at every era end use
    # the symmetric force with the corrector in its reduction, and the symmetric
    # criterion) against the same runs on the gather kernels: the criterion is the same
    # function of the state and the forces differ only by rounding, so the schedules and
    # the energy errors agree
    from paper_1205_2288_amd.driver import NativeTSBTS
    n, eps = 2048, 1 / 256
    r, v, m = plummer(n, 3500)
    runs = []
    for sym in (0, 1):
        sim = NativeTSBTS(r, v, m, eps, passes=3, era=1 / 64, dt_max=1 / 64,
                          tune={"symmetric": sym})
        series = sim.run(0.25)
        e0 = series[0][1]
        runs.append((sim.stats["block_steps"], abs(series[-1][1] - e0) / abs(e0),
                     sim.ctx.r.cpu().numpy().copy()))
        sim.close()
    print(f"native runs N={n}: gather {runs[0][0]} block steps, drift {runs[0][1]:.3e}; "
          f"symmetric {runs[1][0]} block steps, drift {runs[1][1]:.3e}")
    assert abs(runs[0][0] - runs[1][0]) <= 0.01 * runs[0][0]
    assert abs(runs[0][1] - runs[1][1]) <= 0.05 * runs[0][1] + 1e-9
    assert np.abs(runs[0][2] - runs[1][2]).max() <= 1e-5


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_plummer131k_symmetric_force(prec):
    cfg = config("plummer131k")
    n, eps = cfg.n, cfg.eps
    r, v, m = cfg.ic()
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, 9)
    acc = torch.empty((3, n), dtype=torch.float64, device="cuda")
    out, ms = {}, {}
    for sym in (0, 1):
        ctx.tune(symmetric=sym)
        ctx.force(idx, 0.0, with_pot=False, acc=acc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            ctx.force(idx, 0.0, with_pot=False, acc=acc)
        torch.cuda.synchronize()
        ms[sym] = (time.perf_counter() - t0) / 3 * 1e3
        out[sym] = acc.cpu().numpy().copy()
    print(f"plummer131k {prec} force, all targets: gather {ms[0]:.2f} ms, "
          f"symmetric {ms[1]:.2f} ms")
    order = np.argsort(idx)
    sample = np.arange(0, n, n // 256)
    ra, _ = oracle.force(r, m, eps, sample.astype(np.int32))
    e = rel_err_vec(out[1][:, order][:, sample], ra)
    if prec == "fp64":
        assert e.max() <= 1e-12, summary(e)
    else:
        assert np.median(e) <= 1e-6 and e.max() <= 1e-4, summary(e)
        assert np.median(rel_err_vec(out[1], out[0])) <= 1e-6
    ctx.close()


# ---------------------------------------------------------------- force adjoint
@pytest.mark.parametrize("prec,sep", CASES)
@pytest.mark.parametrize("n", [3, 300, 700, 5000])
@pytest.mark.parametrize("with_gp", [False, True])
def test_symmetric_adjoint_matches_gather_and_oracle(prec, sep, n, with_gp):
    eps = 1 / 256
    r, v, m = _state(n, 3600 + n)
    ctx = make_ctx(n, eps, prec, sep)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, n + 2)
    g = gaussian((3, n), 11)
    gp = gaussian(n, 12) if with_gp else None
    out = {}
    for sym in (0, 1, 1):
        ctx.tune(symmetric=sym)
        gr = torch.zeros((3, n), dtype=torch.float64, device="cuda")   # accumulates
        gm = torch.zeros((n,), dtype=torch.float64, device="cuda")
        ctx.force_backward(idx, 0.0, g, gp, gr, gm)
        res = (gr.cpu().numpy(), gm.cpu().numpy())
        if sym in out:
            assert all(np.array_equal(a, b) for a, b in zip(res, out[sym]))   # fixed order
        out[sym] = res
    rr, rm = oracle.force_backward(r, m, eps, idx, g, gp)
    sr, sm = oracle.force_backward_scale(r, m, eps, idx, g, gp)
    for sym in (1, 0):
        check_adjoint(out[sym][0], out[sym][1], rr, rm, sr, sm, prec,
                      f"n={n} symmetric={sym} gp={with_gp}")
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_plummer131k_symmetric_adjoint(prec):
    cfg = config("plummer131k")
    n, eps = cfg.n, cfg.eps
    r, v, m = cfg.ic()
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, 13)
    g = torch.tensor(gaussian((3, n), 14), dtype=torch.float64, device="cuda")
    out, ms = {}, {}
    for sym in (0, 1):
        ctx.tune(symmetric=sym)
        gr = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        gm = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.force_backward(idx, 0.0, g, None, gr, gm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            ctx.force_backward(idx, 0.0, g, None, gr, gm)
        torch.cuda.synchronize()
        ms[sym] = (time.perf_counter() - t0) / 2 * 1e3
        out[sym] = (gr.cpu().numpy() / 3, gm.cpu().numpy() / 3)
    print(f"plummer131k {prec} adjoint, all targets: gather {ms[0]:.2f} ms, "
          f"symmetric {ms[1]:.2f} ms")
    # sampled rows against the oracle, both kernels
    rows = np.arange(0, n, n // 128).astype(np.int32)
    gh = g.cpu().numpy()
    rr, rm = oracle.force_backward_rows(r, m, eps, idx, gh, rows)
    sr, sm = oracle.force_backward_scale(r, m, eps, idx, gh, rows=rows)
    for sym in (1, 0):
        check_adjoint(out[sym][0][:, rows], out[sym][1][rows], rr, rm, sr, sm, prec,
                      f"plummer131k symmetric={sym} sampled rows")
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_large_ragged_n_symmetric_paths(prec):
    # twice the benchmark size and not a multiple of the padding (262147 particles):
    # criterion bitwise and force / adjoint close to the gather kernels, sampled rows
    # against the oracle
    n, eps, eta = 262147, 1 / 4096, 0.1
    r, v, m = _state(n, 4242)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = _perm(n, 17)
    order = np.argsort(idx)
    g = torch.tensor(gaussian((3, n), 18), dtype=torch.float64, device="cuda")
    out = {}
    for sym in (0, 1):
        ctx.tune(symmetric=sym)
        dtc = ctx.timestep(idx, eta).cpu().numpy()
        acc, _ = ctx.force(idx, 0.0, with_pot=False)
        gr = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        gm = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.force_backward(idx, 0.0, g, None, gr, gm)
        out[sym] = (dtc, acc.cpu().numpy(), gr.cpu().numpy(), gm.cpu().numpy())
    assert np.array_equal(out[0][0], out[1][0])
    sample = idx[:: n // 64]
    # adjoint: sampled rows of both kernels against the oracle
    gh = g.cpu().numpy()
    rows = np.sort(sample).astype(np.int32)
    rr, rm = oracle.force_backward_rows(r, m, eps, idx, gh, rows)
    sr, sm = oracle.force_backward_scale(r, m, eps, idx, gh, rows=rows)
    for sym in (1, 0):
        check_adjoint(out[sym][2][:, rows], out[sym][3][rows], rr, rm, sr, sm, prec,
                      f"n=262147 symmetric={sym} sampled rows")
    # force: symmetric against gather, every particle, at the force bars
    e = rel_err_vec(out[1][1], out[0][1])
    assert np.median(e) <= (1e-13 if prec == "fp64" else 1e-6) and \
        e.max() <= (1e-11 if prec == "fp64" else 1e-5), summary(e)
    e = rel_err(out[1][0][order][sample], oracle.timestep(r, v, m, eps, eta, sample))
    assert e.max() <= (1e-12 if prec == "fp64" else 2e-6), summary(e)
    ra, _ = oracle.force(r, m, eps, sample.astype(np.int32))
    e = rel_err_vec(out[1][1][:, order][:, sample], ra)
    if prec == "fp64":
        assert e.max() <= 1e-12, summary(e)
    else:
        assert np.median(e) <= 1e-6 and e.max() <= 1e-4, summary(e)
    ctx.close()
