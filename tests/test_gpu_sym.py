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
from gpu_util import rel_err, summary, make_ctx

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
