"""The fused force + criterion variant (tsbts_force_criterion; the criterion taken before
the corrector, with the predicted velocities of the active particles).

* against the oracle: force and potential on the predicted positions, criterion on the
  predicted positions and velocities (Taylor prediction of every particle);
* against the separate kernels on the same predicted state: the force bitwise (same
  pair arithmetic, same split), the criterion bitwise (same pair terms; max and min are
  exact);
* whole runs with the native scheduler in this order: energy drift within twice the
  oracle's (paper's-order) drift, and a comparable amount of schedule work.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from workloads import plummer, active_subset, config
from gpu_util import rel_err_vec, rel_err, summary, make_ctx, TOL

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _state(n, seed, eps):
    r, v, m = plummer(n, seed, masses="loguniform")
    a, _ = oracle.force(r, m, eps)
    rng = np.random.default_rng(seed)
    h0 = 2.0 ** -9
    t_last = rng.integers(0, 4, n) * h0
    dt = 4 * h0 - t_last      # every particle's next time is 4 h0
    return r, v, m, a, t_last, dt, 4 * h0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,n_act", [(700, 1), (700, 33), (4099, 500), (4099, 4099)])
def test_fused_matches_oracle(prec, n, n_act):
    eps, eta = 1 / 64, 0.1
    r, v, m, a, t_last, dt, tb = _state(n, 90 + n_act, eps)
    idx = active_subset(n, n_act, 3)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m, a=a, t_last=t_last, dt=dt)
    ctx.predict(tb)
    acc, pot, dtc = ctx.force_criterion(idx, tb, eta)
    rp, vp = oracle.taylor(r, v, a, tb - t_last)
    a_ref, p_ref = oracle.force(rp, m, eps, idx)
    ea = summary(rel_err_vec(acc.cpu().numpy(), a_ref))
    assert ea["median"] <= TOL[prec]["median"] and ea["max"] <= TOL[prec]["max"], ea
    assert rel_err(pot.cpu().numpy(), p_ref).max() <= TOL[prec]["max"]
    d_ref = oracle.timestep(rp, vp, m, eps, eta, idx)
    assert rel_err(dtc.cpu().numpy(), d_ref).max() <= (1e-12 if prec == "fp64" else 2e-6)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,n_act", [(5000, 40), (5000, 1700), (20000, 20000)])
def test_fused_equals_separate_kernels(prec, n, n_act):
    eps, eta = 1 / 256, 0.1
    r, v, m = plummer(n, 91)
    idx = active_subset(n, n_act, 4)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    acc, pot, dtc = ctx.force_criterion(idx, 0.0, eta)
    acc2, pot2 = ctx.force(idx, 0.0)
    dtc2 = ctx.timestep(idx, eta)
    assert torch.equal(acc, acc2) and torch.equal(pot, pot2)
    assert torch.equal(dtc, dtc2)
    ctx.close()


def test_fused_bad_arguments():
    from paper_1205_2288_amd._lib import TsbtsError, TSBTS_EINVAL, TSBTS_ESTATE
    n = 100
    r, v, m = plummer(n, 92)
    ctx = make_ctx(n, 0.01, "mixed")
    ctx.bind(r, v, m)
    idx = np.arange(n, dtype=np.int32)
    with pytest.raises(TsbtsError) as e:
        ctx.force_criterion(idx, 0.0, 0.1)      # nothing predicted yet
    assert e.value.status == TSBTS_ESTATE
    ctx.predict(0.0)
    with pytest.raises(TsbtsError) as e:
        ctx.force_criterion(idx, 0.0, 0.0)      # eta must be positive
    assert e.value.status == TSBTS_EINVAL
    from paper_1205_2288_amd import _lib as L
    with pytest.raises(TsbtsError) as e:       # no scheduler yet
        L.tsbts_sched_option(ctx.ctx, L.TSBTS_SCHED_CRITERION_BEFORE_CORRECTOR, 1)
    assert e.value.status == TSBTS_ESTATE
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["plummer256", "plummer4096_t1"])
def test_native_run_criterion_before_corrector(prec, name):
    from paper_1205_2288_amd.driver import NativeTSBTS
    with open(os.path.join(GOLDEN, f"tsbts_{name}.json")) as f:
        g = json.load(f)
    cfg = config(g["workload"])
    r, v, m = cfg.ic()
    sim = NativeTSBTS(r, v, m, cfg.eps, eta=cfg.eta, passes=g["passes"], era=cfg.era,
                      dt_max=cfg.dt_max, dt_min=cfg.dt_min, precision=prec,
                      criterion="before")
    series = sim.run(g["t_end"])
    e0 = series[0][1]
    d = max(abs(e - e0) / abs(e0) for _, e in series)
    steps = sim.stats["block_steps"]
    print(f"{name} {prec} criterion before corrector: drift {d:.3e} (oracle, paper's "
          f"order {g['max_rel_energy_error']:.3e}), block steps {steps} vs "
          f"{g['stats']['block_steps']}, {sim.stats['wall_s']:.2f} s")
    assert len(series) == len(g["times"])
    assert d <= 2.0 * g["max_rel_energy_error"]
    assert 0.9 <= steps / g["stats"]["block_steps"] <= 1.1
    sim.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["plummer256", "plummer4096_t1"])
def test_native_run_predict_on_load(prec, name):
    # small active sets predicting their sources inside the force kernel: the same run,
    # bit for bit, with one launch less per small block step
    from paper_1205_2288_amd.driver import NativeTSBTS
    with open(os.path.join(GOLDEN, f"tsbts_{name}.json")) as f:
        g = json.load(f)
    cfg = config(g["workload"])
    r, v, m = cfg.ic()
    out = {}
    for pol in (False, True):
        sim = NativeTSBTS(r, v, m, cfg.eps, eta=cfg.eta, passes=g["passes"], era=cfg.era,
                          dt_max=cfg.dt_max, dt_min=cfg.dt_min, precision=prec,
                          predict_on_load=pol)
        series = sim.run(g["t_end"])
        out[pol] = (sim.stats["block_steps"], sim.stats["wall_s"], series,
                    sim.ctx.r.cpu().numpy().copy(), sim.ctx.v.cpu().numpy().copy())
        sim.close()
    print(f"{name} {prec}: {out[False][0]} block steps; separate predictor "
          f"{out[False][1] / out[False][0] * 1e6:.1f} us/step, predicted on load "
          f"{out[True][1] / out[True][0] * 1e6:.1f} us/step")
    assert out[True][0] == out[False][0]
    assert out[True][2] == out[False][2]
    assert np.array_equal(out[True][3], out[False][3])
    assert np.array_equal(out[True][4], out[False][4])
