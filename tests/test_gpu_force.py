"""GPU parity of the force / potential kernels against the FP64 oracle.

Element by element on seeded Plummer spheres spanning several 256-particle tiles with a
ragged tail, random active subsets (including a single particle and the full set),
eps > 0 and eps = 0 (masked self pair), every precision variant; and, at the full
N=32768 and N=131072 sizes in the launch configuration the benchmark uses, on sampled
targets the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import plummer, active_subset, config
from gpu_util import rel_err_vec, rel_err, summary, make_ctx, VARIANTS, TOL

pytestmark = pytest.mark.gpu


def _run(ctx, r, v, m, idx, t=0.0):
    ctx.bind(r, v, m)
    ctx.predict(t)
    acc, pot = ctx.force(idx, t)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), pot.cpu().numpy()


@pytest.mark.parametrize("prec,sep,newton", VARIANTS)
@pytest.mark.parametrize("n,eps,n_act", [
    (2, 0.0, 2), (3, 0.01, 1), (16, 1 / 64, 16), (257, 1 / 64, 100), (1000, 0.0, 999),
    (4099, 1 / 256, 4099), (4099, 1 / 256, 1), (4099, 1 / 256, 37), (1536, 1 / 1024, 1536),
])
def test_force_matches_oracle(prec, sep, newton, n, eps, n_act):
    r, v, m = plummer(n, 1000 + n, masses="loguniform")
    idx = active_subset(n, n_act, 7 + n_act)
    ctx = make_ctx(n, eps, prec, sep, newton)
    acc, pot = _run(ctx, r, v, m, idx)
    a_ref, p_ref = oracle.force(r, m, eps, idx)
    ea = summary(rel_err_vec(acc, a_ref))
    ep = summary(rel_err(pot, p_ref))
    tol = TOL[prec]
    assert ea["median"] <= tol["median"], ea
    assert ea["max"] <= tol["max"], ea
    assert ep["median"] <= tol["median"], ep
    assert ep["max"] <= tol["max"], ep
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_force_bitwise_reproducible_and_third_law(prec):
    n = 3000
    r, v, m = plummer(n, 5, masses="loguniform")
    ctx = make_ctx(n, 1 / 256, prec)
    idx = np.arange(n, dtype=np.int32)
    a1, p1 = _run(ctx, r, v, m, idx)
    a2, p2 = _run(ctx, r, v, m, idx)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
    # Newton's third law: sum m a = 0 up to rounding of the pair sums
    tot = np.abs((a1 * m).sum(axis=1)).max()
    scale = (np.abs(a1) * m).sum()
    assert tot <= (1e-13 if prec == "fp64" else 1e-6) * scale
    ctx.close()


def test_force_subset_rows_match_full():
    n = 2048
    r, v, m = plummer(n, 6)
    ctx = make_ctx(n, 1 / 128, "fp64")
    full, fp = _run(ctx, r, v, m, np.arange(n, dtype=np.int32))
    idx = active_subset(n, 33, 2)
    sub, sp = _run(ctx, r, v, m, idx)
    assert np.allclose(sub, full[:, idx], rtol=1e-13, atol=0)
    assert np.allclose(sp, fp[idx], rtol=1e-13, atol=0)
    ctx.close()


@pytest.mark.parametrize("name", ["sweep32768", "plummer131k"])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_force_full_size_sampled(name, prec):
    cfg = config(name)
    r, v, m = cfg.ic()
    n = cfg.n
    ctx = make_ctx(n, cfg.eps, prec)
    sizes = [n, n // 8, 64, 1] if name == "plummer131k" else [1, 8, 64, 512, 4096, 32768]
    for k, n_act in enumerate(sizes):
        idx = active_subset(n, n_act, cfg.seed + 1000 * k)
        acc, pot = _run(ctx, r, v, m, idx)
        take = np.sort(np.random.default_rng(k).choice(n_act, size=min(n_act, 256),
                                                       replace=False))
        a_ref, p_ref = oracle.force(r, m, cfg.eps, idx[take])
        ea = summary(rel_err_vec(acc[:, take], a_ref))
        ep = summary(rel_err(pot[take], p_ref))
        assert ea["median"] <= TOL[prec]["median"], (n_act, ea)
        assert ea["max"] <= TOL[prec]["max"], (n_act, ea)
        assert ep["max"] <= TOL[prec]["max"], (n_act, ep)
    ctx.close()


def test_sweep32768_error_histograms():
    # one prediction + force call per active-set size, mixed and float64, 512 sampled
    # targets against the oracle; histogram of log10 per-particle relative error in bins
    # of 0.25 over [-12, -2] (printed), medians checked against the 1e-6 bar
    cfg = config("sweep32768")
    r, v, m = cfg.ic()
    n = cfg.n
    edges = np.arange(-12.0, -1.99, 0.25)
    for prec in ("mixed", "fp64"):
        ctx = make_ctx(n, cfg.eps, prec)
        for k, n_act in enumerate([1, 8, 64, 512, 4096, 32768]):
            idx = active_subset(n, n_act, cfg.seed + 1000 * k)
            acc, _ = _run(ctx, r, v, m, idx)
            take = np.sort(np.random.default_rng(k).choice(n_act, size=min(n_act, 512),
                                                           replace=False))
            a_ref, _ = oracle.force(r, m, cfg.eps, idx[take])
            e = rel_err_vec(acc[:, take], a_ref)
            h, _ = np.histogram(np.log10(np.maximum(e, 1e-300)), bins=edges)
            print(f"hist {prec} n_act={n_act} median={np.median(e):.2e} max={e.max():.2e} "
                  f"below={int((e < 1e-12).sum())} counts={h.tolist()}")
            assert np.median(e) <= TOL[prec]["median"]
        ctx.close()


def test_force_out_of_order_and_bad_arguments():
    from paper_1205_2288_amd._lib import TsbtsError, TSBTS_ESTATE, TSBTS_EINVAL
    n = 100
    r, v, m = plummer(n, 3)
    ctx = make_ctx(n, 0.01, "mixed")
    ctx.bind(r, v, m)
    with pytest.raises(TsbtsError) as e:
        ctx.force(np.arange(n, dtype=np.int32), 0.0)  # nothing predicted yet
    assert e.value.status == TSBTS_ESTATE
    ctx.predict(0.25)
    with pytest.raises(TsbtsError) as e:
        ctx.force(np.arange(n, dtype=np.int32), 0.5)  # not the predicted time
    assert e.value.status == TSBTS_ESTATE
    with pytest.raises(TsbtsError) as e:
        ctx.force(np.arange(n + 1, dtype=np.int32) % n, 0.25)  # more targets than particles
    assert e.value.status == TSBTS_EINVAL
    ctx.close()


SHAPES = [(8192, 0, 0), (64, 0, 0), (65536, 0, 0), (8192, 0, 64), (8192, 0, 256),
          (64, 0, 64), (8192, 1, 0), (8192, 2, 0), (8192, 4, 0), (512, 2, 0), (65536, 4, 0)]


@pytest.mark.parametrize("prec,sep", [("mixed", "f64"), ("mixed", "hilo"), ("fp64", "f64")])
def test_launch_shapes_agree(prec, sep):
    # every launch shape (scalar-load kernel with 64..65536 workgroups, LDS kernels with
    # 1, 2, 4 targets per lane) against the oracle, and against the default shape up to
    # the order of the float64 tile sums
    n = 9000
    r, v, m = plummer(n, 71, masses="loguniform")
    ctx = make_ctx(n, 1 / 256, prec, sep)
    sets = [np.arange(n, dtype=np.int32), active_subset(n, 8500, 1), active_subset(n, 300, 2),
            active_subset(n, 33, 3)]
    base = [_run(ctx, r, v, m, idx) for idx in sets]
    refs = [oracle.force(r, m, 1 / 256, idx) for idx in sets]
    for blocks, ipl, chunk in SHAPES:
        ctx.tune(blocks=blocks, ipl=ipl, chunk=chunk)
        for idx, (a0, p0), (ar, pr) in zip(sets, base, refs):
            acc, pot = _run(ctx, r, v, m, idx)
            ea = summary(rel_err_vec(acc, ar))
            assert ea["median"] <= TOL[prec]["median"] and ea["max"] <= TOL[prec]["max"], \
                (blocks, ipl, chunk, idx.size, ea)
            ep = summary(rel_err(pot, pr))
            assert ep["max"] <= TOL[prec]["max"], (blocks, ipl, chunk, idx.size, ep)
            # float32 sums run over j-units of 64 or 256: a unit size other than the
            # default changes their rounding (bounded by ~256 float32 roundings), any
            # other shape only the order of the float64 sums
            same = 1e-12 if prec == "fp64" else (1e-6 if chunk == 0 else 2e-5)
            assert rel_err_vec(acc, a0).max() <= same, (blocks, ipl, chunk, idx.size)
    ctx.close()


def test_tune_rejects_bad_values():
    from paper_1205_2288_amd._lib import TsbtsError, TSBTS_EINVAL
    ctx = make_ctx(100, 0.01, "mixed")
    for kw in ({"blocks": 63}, {"blocks": 65537}, {"ipl": 3}, {"ipl": -1}, {"ipl": 8},
               {"chunk": 32}, {"chunk": 128}, {"chunk": -64}, {"symmetric": 3},
               {"symmetric": -1}):
        with pytest.raises(TsbtsError) as e:
            ctx.tune(**kw)
        assert e.value.status == TSBTS_EINVAL
    ctx.close()
