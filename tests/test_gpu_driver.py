"""GPU TSBTS integrations (host scheduler + HIP kernels) against the oracle.

* One shared level (huge eta): the scheme reduces to the shared-step leapfrog of
  Section 2, for any number of passes.
* The N=256 fixed-era workload in float64: same schedule and trajectory as the oracle
  over t = 0..1 (differences only from rounding order).
* Energy drift of the GPU runs (float64 and mixed force) within a factor 2 of the
  oracle's drift over the same run (stored references written by
  tests/golden/make_golden.py, which calls only the oracle).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle.tsbts import OracleTSBTS
from workloads import plummer, config

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, f"tsbts_{name}.json")) as f:
        return json.load(f)


def _drift(series):
    e = np.array([x[1] for x in series])
    return np.abs((e - e[0]) / e[0]).max()


@pytest.mark.parametrize("native", [False, True])
@pytest.mark.parametrize("passes", [1, 3])
def test_shared_level_reduces_to_leapfrog(passes, native):
    from paper_1205_2288_amd.driver import TSBTS, NativeTSBTS
    r, v, m = plummer(64, 17)
    eps = 1 / 64
    cls = NativeTSBTS if native else TSBTS
    sim = cls(r, v, m, eps, eta=1e9, passes=passes, era=1 / 8, precision="fp64")
    assert np.all(sim.dt == 1 << 14)
    sim.run(0.25)
    st = sim.state()
    r_ref, v_ref, _ = oracle.leapfrog_shared(r, v, m, eps, 1 / 64, 16)
    assert np.abs(st["r"] - r_ref).max() <= 1e-12
    assert np.abs(st["v"] - v_ref).max() <= 1e-12
    sim.close()


def test_plummer256_fp64_follows_oracle():
    from paper_1205_2288_amd.driver import TSBTS
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    kw = dict(eta=cfg.eta, passes=3, era=cfg.era, dt_max=cfg.dt_max, dt_min=cfg.dt_min)
    gpu = TSBTS(r, v, m, cfg.eps, precision="fp64", **kw)
    ref = OracleTSBTS(r, v, m, cfg.eps, **kw)
    assert np.array_equal(gpu.dt, ref.dt)
    for _ in range(4):  # four eras of 1/8: t = 0..1/2, compared era by era
        gpu.era_step()
        ref.era_step()
        st = gpu.state()
        assert np.array_equal(st["t"], ref.t)
        assert np.array_equal(st["dt"], ref.dt), "schedules diverged"
        assert np.abs(st["r"] - ref.r).max() <= 1e-9
        assert np.abs(st["v"] - ref.v).max() <= 1e-8
    gpu.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name,eras", [("plummer256", 4), ("plummer4096", 3)])
def test_native_scheduler_matches_python_scheduler(prec, name, eras):
    from paper_1205_2288_amd.driver import TSBTS, NativeTSBTS
    cfg = config(name)
    r, v, m = cfg.ic()
    kw = dict(eta=cfg.eta, passes=3, era=cfg.era, dt_max=cfg.dt_max, dt_min=cfg.dt_min,
              precision=prec)
    py = TSBTS(r, v, m, cfg.eps, **kw)
    nat = NativeTSBTS(r, v, m, cfg.eps, **kw)
    assert np.array_equal(py.dt, nat.dt) and np.array_equal(py.dtc, nat.dtc)
    for _ in range(eras):
        assert py.era_step() == nat.era_step()
        a, b = py.state(), nat.state()
        for key in ("t", "dt", "dtc", "r", "v", "a"):
            assert np.array_equal(a[key], b[key]), key
    assert py.stats["block_steps"] == nat.stats["block_steps"]
    assert py.stats["interactions"] == nat.stats["interactions"]
    py.close()
    nat.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_era_of_one_max_step_first_steps(prec):
    # era = dt_max: every particle is at the era start each era and its first step is
    # chosen again in every later pass; the native scheduler, the Python one and (float64)
    # the oracle make the same choices
    from paper_1205_2288_amd.driver import TSBTS, NativeTSBTS
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    kw = dict(eta=0.5, passes=3, era=cfg.dt_max, dt_max=cfg.dt_max, dt_min=cfg.dt_min)
    py = TSBTS(r, v, m, cfg.eps, precision=prec, record_schedule=True, **kw)
    nat = NativeTSBTS(r, v, m, cfg.eps, precision=prec, **kw)
    ref = OracleTSBTS(r, v, m, cfg.eps, **kw) if prec == "fp64" else None
    for _ in range(16):
        py.era_step()
        nat.era_step()
        a, b = py.state(), nat.state()
        for key in ("t", "dt", "dtc", "r", "v", "a"):
            assert np.array_equal(a[key], b[key]), key
        if ref is not None:
            ref.era_step()
            assert np.array_equal(b["dt"], ref.dt), "schedules diverged"
            assert np.abs(b["r"] - ref.r).max() <= 1e-9
    # some particles took a first step other than the one chosen when they arrived
    changed = sum(int(np.count_nonzero(e["dt_start"][-1] != e["dt_start"][0]))
                  for e in py.schedule["eras"])
    assert changed > 0
    py.close()
    nat.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["plummer256", "plummer256_1pass", "plummer4096_t1",
                                  "plummer256_dyn"])
def test_energy_drift_within_twice_oracle(prec, name):
    from paper_1205_2288_amd.driver import NativeTSBTS
    g = _golden(name)
    cfg = config(g["workload"])
    r, v, m = cfg.ic()
    sim = NativeTSBTS(r, v, m, cfg.eps, eta=g["eta"], passes=g["passes"], era=g["era"],
                      dt_max=g["dt_max"], dt_min=g["dt_min"], precision=prec)
    series = sim.run(g["t_end"])
    d = _drift(series)
    print(f"{name} {prec}: GPU drift {d:.3e}, oracle {g['max_rel_energy_error']:.3e}, "
          f"steps {sim.stats['block_steps']} vs {g['stats']['block_steps']}, "
          f"eras {sim.stats['era_sizes']} vs {g['stats'].get('era_sizes')}, "
          f"{sim.stats['wall_s']:.1f} s")
    assert len(series) == len(g["times"])
    assert d <= 2.0 * g["max_rel_energy_error"]
    # the schedule work is comparable (chaotic divergence allowed)
    assert 0.5 <= sim.stats["block_steps"] / g["stats"]["block_steps"] <= 2.0
    if prec == "fp64" and "era_sizes" in g["stats"]:
        # t <= 1 is short enough for float64 runs to keep the oracle's schedule
        assert sim.stats["era_sizes"] == g["stats"]["era_sizes"]
    sim.close()


@pytest.mark.parametrize("native", [False, True])
def test_plummer256_dynamic_era_follows_oracle(native):
    """eta = 0.05, dt_max = 1/8, dynamic era: Algorithm 3 sets eras of 1/8 and then 1/16.
    In float64 both schedulers take the oracle's era ends, times and steps era by era."""
    from paper_1205_2288_amd.driver import TSBTS, NativeTSBTS
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    kw = dict(eta=0.05, passes=3, era=None, dt_max=1 / 8, dt_min=cfg.dt_min)
    gpu = (NativeTSBTS if native else TSBTS)(r, v, m, cfg.eps, precision="fp64", **kw)
    ref = OracleTSBTS(r, v, m, cfg.eps, **kw)
    assert np.array_equal(gpu.dt, ref.dt)
    ends = []
    while ref.time * 2.0 ** -20 < 0.5:
        T1 = ref.era_step()
        assert gpu.era_step() == T1, "era ends differ"
        ends.append(T1)
        st = gpu.state()
        assert np.array_equal(st["t"], ref.t)
        assert np.array_equal(st["dt"], ref.dt), "schedules diverged"
        assert np.abs(st["r"] - ref.r).max() <= 1e-9
        assert np.abs(st["v"] - ref.v).max() <= 1e-8
    sizes = np.diff([0] + ends)
    dt_max = 1 << 17
    assert (sizes == dt_max).any() and (sizes < dt_max).any(), sizes
    assert gpu.stats["era_sizes"] == ref.stats["era_sizes"]
    gpu.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plummer4096_dynamic_era_t10_drift(prec):
    path = os.path.join(GOLDEN, "tsbts_plummer4096.json")
    if not os.path.exists(path):
        pytest.skip("oracle reference for the t=10 run not generated")
    from paper_1205_2288_amd.driver import NativeTSBTS
    g = _golden("plummer4096")
    cfg = config("plummer4096")
    r, v, m = cfg.ic()
    sim = NativeTSBTS(r, v, m, cfg.eps, eta=cfg.eta, passes=3, era=None, dt_max=cfg.dt_max,
                      dt_min=cfg.dt_min, precision=prec)
    series = sim.run(cfg.t_end)
    d = _drift(series)
    print(f"plummer4096 t=10 {prec}: GPU drift {d:.3e}, oracle "
          f"{g['max_rel_energy_error']:.3e}, {sim.stats['block_steps']} block steps, "
          f"{sim.stats['wall_s']:.1f} s")
    assert d <= 2.0 * g["max_rel_energy_error"]
    sim.close()


def test_experiments_module_small():
    # the era-size / dynamic-era study drivers on a tiny sphere: structure, finiteness,
    # and block steps proportional to the pass count
    import io
    import json
    from paper_1205_2288_amd import experiments as ex
    buf = io.StringIO()
    rows, summary = ex.era_study(n=32, seeds=1, t_end=0.5, eras=(1 / 64, 1 / 16),
                                 passes=(1, 3), every=0.25, out=buf)
    assert len(rows) == 4 and len(summary) == 4
    lines = [json.loads(x) for x in buf.getvalue().splitlines()]
    assert lines[-1]["study"] == "era"
    for r in rows:
        assert np.isfinite(r["max_err"]) and 0.0 <= r["final_err"] <= r["max_err"]
    by = {(r["passes"], r["era"]): r["block_steps"] for r in rows}
    for era in (1 / 64, 1 / 16):
        assert 2.5 <= by[(3, era)] / by[(1, era)] <= 3.5
    rows, summary = ex.dynamic_era_study(n=32, seeds=2, t_end=0.5, every=0.25, out=buf)
    assert 0.0 <= summary["dynamic_smaller_final_err_fraction"] <= 1.0
    # the same runs in two child processes: identical results (the runs are deterministic)
    rows2, summary2 = ex.dynamic_era_study(n=32, seeds=2, t_end=0.5, every=0.25, out=buf,
                                           workers=2)
    for key in ("dynamic_smaller_final_err_fraction", "median_final_err_fixed",
                "median_final_err_dynamic"):
        assert summary2[key] == summary[key]
    for a, b in zip(rows, rows2):
        for kind in ("fixed", "dynamic"):
            assert a[kind]["series_err"] == b[kind]["series_err"]
            assert a[kind]["block_steps"] == b[kind]["block_steps"]


def test_era_study_matches_oracle():
    # the era-size / iteration study driver (64 bodies, two spheres, eras 1/64 and 1/8,
    # 1 and 3 passes, float64, t = 0..2) against the oracle's integrations of the same
    # spheres with the same parameters, run by run: the same number of block steps and
    # the same energy-error series up to rounding, hence the same drift
    import io
    from paper_1205_2288_amd import experiments as ex
    rows, summary = ex.era_study(n=64, seeds=2, t_end=2.0, eras=(1 / 64, 1 / 8),
                                 passes=(1, 3), every=1.0, seed0=1205, out=io.StringIO())
    assert len(rows) == 8 and len(summary) == 4
    for row in rows:
        r, v, m = plummer(64, row["seed"])
        ref = OracleTSBTS(r, v, m, row["eps"], eta=row["eta"], passes=row["passes"],
                          era=row["era"], dt_max=row["dt_max"])
        series = ref.run(row["t_end"], energy_every=1.0)
        e0 = series[0][1]
        err = np.array([abs(e - e0) / abs(e0) for _, e in series])
        print(f"seed {row['seed']} passes {row['passes']} era {row['era']}: block steps "
              f"{row['block_steps']} (oracle {ref.stats['block_steps']}), max error "
              f"{row['max_err']:.4e} (oracle {err.max():.4e})")
        assert row["series_t"] == [t for t, _ in series]
        assert row["block_steps"] == ref.stats["block_steps"]
        assert np.abs(np.array(row["series_err"]) - err).max() <= 1e-10 * max(1.0, err.max())
        assert row["max_err"] <= 2.0 * err.max() + 1e-14


def test_experiment_run_resumes_across_sessions(tmp_path):
    # a study run stopped at its deadline after its first segment and continued from its
    # saved era-end checkpoint by a later call equals the uninterrupted run bit for bit
    from paper_1205_2288_amd import experiments as ex
    kw = dict(n=64, seed=1205, eps=0.01, eta=0.1, passes=3, era=1 / 16, dt_max=1 / 64,
              t_end=2.0, every=0.25, segment=0.5)
    full = ex.energy_error_run(**kw)
    assert full["complete"] and full["t_reached"] == 2.0
    part = ex.energy_error_run(**kw, state_dir=str(tmp_path), deadline=0.0)
    assert not part["complete"] and part["t_reached"] == 0.5
    assert part["series_err"] == full["series_err"][:len(part["series_err"])]
    rest = ex.energy_error_run(**kw, state_dir=str(tmp_path))
    assert rest["complete"]
    assert rest["series_t"] == full["series_t"]
    assert rest["series_err"] == full["series_err"]
    assert rest["block_steps"] == full["block_steps"]
    assert rest["growth"] == full["growth"]
    assert rest["era_sizes"] == full["era_sizes"] and sum(full["era_sizes"].values()) == 32


@pytest.mark.parametrize("prec,era", [("fp64", 1.0 / 8), ("mixed", None)])
def test_native_checkpoint_resume_bitwise(prec, era):
    # an era-end checkpoint, saved through numpy's npz format and restored into a fresh
    # scheduler, continues the run bit for bit (fixed and dynamic eras)
    import io
    from paper_1205_2288_amd._lib import TsbtsError
    from paper_1205_2288_amd.driver import NativeTSBTS
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    kw = dict(eta=cfg.eta, passes=3, era=era, dt_max=cfg.dt_max, dt_min=cfg.dt_min,
              precision=prec)
    full = NativeTSBTS(r, v, m, cfg.eps, **kw)
    e_full = full.run(0.5, energy_every=1.0 / 8)
    first = NativeTSBTS(r, v, m, cfg.eps, **kw)
    first.run(0.25, energy_every=1.0 / 8)
    ck = first.checkpoint()
    first.close()
    buf = io.BytesIO()
    np.savez(buf, **ck)
    buf.seek(0)
    with np.load(buf) as z:
        ck = {k: z[k] for k in z.files}
    second = NativeTSBTS(r, v, m, cfg.eps, **kw)
    before = second.checkpoint()
    bad = dict(ck, t=ck["t"] + 1)  # no longer aligned to the steps: refused
    with pytest.raises(TsbtsError):
        second.restore(bad)
    bad = dict(ck, dt=np.where(np.arange(cfg.n) == 7, 3, ck["dt"]))  # not a power of two
    with pytest.raises(TsbtsError, match="particle 7"):
        second.restore(bad)
    with pytest.raises(ValueError):
        second.restore(dict(ck, r=ck["r"][:, :-1]))
    after = second.checkpoint()  # the refusals changed nothing
    for key in ("r", "v", "a", "t", "dt", "dtp", "dtc", "stats"):
        assert np.array_equal(before[key], after[key]), key
    second.restore(ck)
    e_second = second.run(0.5, energy_every=1.0 / 8)
    a, b = full.checkpoint(), second.checkpoint()
    for key in ("r", "v", "a", "t", "dt", "dtp", "dtc", "stats"):
        assert np.array_equal(a[key], b[key]), key
    assert a["time"] == b["time"]
    assert e_second == [x for x in e_full if x[0] >= 0.25]
    full.close()
    second.close()


def test_native_step_timing_accounts_for_every_block_step():
    # tsbts_sched_timing: the class counts add up to the scheduler's block steps and
    # interactions, and the phases of each class fit inside its whole-step time
    from paper_1205_2288_amd.driver import NativeTSBTS
    cfg = config("plummer256")
    r, v, m = cfg.ic()
    sim = NativeTSBTS(r, v, m, cfg.eps, eta=cfg.eta, passes=3, era=cfg.era, dt_max=cfg.dt_max,
                      dt_min=cfg.dt_min)
    for _ in range(2):
        sim.era_step()
    sec, cnt = sim._L.tsbts_sched_timing(sim.ctx.ctx)
    st = sim.stats
    assert int(cnt[:, 0].sum()) == st["block_steps"]
    assert int(cnt[:, 1].sum()) * sim.n == st["interactions"]
    assert (sec >= 0).all()
    for c in range(4):
        assert sec[c, :3].sum() <= sec[c, 3] * (1 + 1e-9) + 1e-6
    t = sim.step_timing()
    assert sum(x["block_steps"] for x in t.values()) == st["block_steps"]
    sim.close()


def test_threaded_step_rule_equals_serial():
    # block steps with at least 8192 active particles (here every era's all-particle
    # steps and the larger partial ones) share the step rule among host threads; each
    # particle's rule reads and writes its own state only, so the run is the same bit for
    # bit with the calling thread alone
    from paper_1205_2288_amd.driver import NativeTSBTS
    n, eps = 16384, 1 / 256
    r, v, m = plummer(n, 4600)
    out = []
    for threads in (1, 4):
        sim = NativeTSBTS(r, v, m, eps, passes=3, era=1 / 16, dt_max=1 / 16,
                          rule_threads=threads)
        series = sim.run(1 / 8)
        out.append((series, sim.state(), sim.stats["block_steps"]))
        sim.close()
    assert out[0][0] == out[1][0]
    for key in ("t", "dt", "dtc", "r", "v", "a"):
        assert np.array_equal(out[0][1][key], out[1][1][key]), key
    assert out[0][2] == out[1][2]
