"""GPU parity of the criterion, energy, adjoint, predictor / Hermite and corrector kernels
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from workloads import plummer, active_subset, gaussian, config
from gpu_util import rel_err_vec, rel_err, summary, make_ctx, VARIANTS, check_adjoint

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ criterion (Eq. nbdt)
@pytest.mark.parametrize("prec,sep", [("fp64", "hilo"), ("mixed", "hilo"), ("mixed", "f64")])
@pytest.mark.parametrize("n,n_act", [(3, 3), (257, 57), (4099, 4099), (4099, 1)])
def test_timestep_matches_oracle(prec, sep, n, n_act):
    eps, eta = 1 / 256, 0.1
    r, v, m = plummer(n, 2000 + n, masses="loguniform")
    idx = active_subset(n, n_act, 3)
    ctx = make_ctx(n, eps, prec, sep)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    dtc = ctx.timestep(idx, eta).cpu().numpy()
    ref = oracle.timestep(r, v, m, eps, eta, idx)
    e = rel_err(dtc, ref)
    assert e.max() <= (1e-12 if prec == "fp64" else 2e-6), summary(e)
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_timestep_and_adjoint_launch_shapes(prec):
    # criterion and force adjoint under every launch shape against the oracle
    n, eps, eta = 9000, 1 / 256, 0.1
    r, v, m = plummer(n, 72, masses="loguniform")
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    sets = [np.arange(n, dtype=np.int32), active_subset(n, 8500, 4), active_subset(n, 300, 5)]
    refs = []
    for idx in sets:
        g = gaussian((3, idx.size), 9)
        refs.append((g, oracle.timestep(r, v, m, eps, eta, idx),
                     oracle.force_backward(r, m, eps, idx, g),
                     oracle.force_backward_scale(r, m, eps, idx, g)))
    for blocks, ipl, chunk in [(8192, 0, 0), (64, 0, 0), (65536, 0, 0), (8192, 0, 64),
                               (8192, 0, 256), (8192, 1, 0), (8192, 2, 0), (8192, 4, 0)]:
        ctx.tune(blocks=blocks, ipl=ipl, chunk=chunk)
        for idx, (g, dref, (rr, rm), (sr, sm)) in zip(sets, refs):
            dtc = ctx.timestep(idx, eta).cpu().numpy()
            e = rel_err(dtc, dref)
            assert e.max() <= (1e-12 if prec == "fp64" else 2e-6), (blocks, ipl, chunk,
                                                                    idx.size)
            gr, gm = ctx.force_backward(idx, 0.0, g)
            check_adjoint(gr.cpu().numpy(), gm.cpu().numpy(), rr, rm, sr, sm, prec,
                          f"launch shape {(blocks, ipl, chunk)} n_act={idx.size}")
    ctx.close()


def test_timestep_three_body_by_hand():
    # particle 0 at rest, 1 at (1,0,0) moving (-2,0,0) with mass 1/4, 2 at (0,3,0), mass 1
    r = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 3.0], [0.0, 0.0, 0.0]])
    v = np.array([[0.0, -2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    m = np.array([0.5, 0.25, 1.0])
    ctx = make_ctx(3, 0.0, "fp64")
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    dtc = ctx.timestep(np.arange(3, dtype=np.int32), 0.1).cpu().numpy()
    assert np.allclose(dtc, [0.05, 0.05, 0.1 * np.sqrt(10.0) / 2], rtol=1e-14)
    ctx.close()


# ------------------------------------------------------------------ energy
@pytest.mark.parametrize("n,eps", [(2, 0.0), (255, 1 / 64), (257, 1 / 64), (4099, 1 / 256),
                                   (1024, 0.0)])
def test_energy_matches_oracle(n, eps):
    r, v, m = plummer(n, 3000 + n, masses="loguniform")
    ctx = make_ctx(n, eps, "mixed")
    ctx.bind(r, v, m)
    kw = ctx.energy().cpu().numpy()
    k, w = oracle.energy(r, v, m, eps)
    assert kw[0] == pytest.approx(k, rel=1e-13)
    assert kw[1] == pytest.approx(w, rel=1e-12)
    kw2 = ctx.energy().cpu().numpy()
    assert np.array_equal(kw, kw2)  # fixed-order reduction
    ctx.close()


def test_energy_two_body_closed_form():
    r = np.array([[0.0, 3.0], [0.0, 4.0], [0.0, 0.0]])
    v = np.array([[1.0, 0.0], [0.0, -2.0], [0.0, 0.5]])
    m = np.array([0.5, 0.25])
    ctx = make_ctx(2, 12.0, "fp64")
    ctx.bind(r, v, m)
    kw = ctx.energy().cpu().numpy()
    assert kw[0] == pytest.approx(0.25 + 0.125 * 4.25, rel=1e-15)
    assert kw[1] == pytest.approx(-0.125 / 13.0, rel=1e-14)
    ctx.close()


def test_energy_full_size_potential_identity():
    # W = 1/2 sum m_i phi_i with phi from the float64 force kernel, sampled rows checked
    # against the oracle; holds at the full N=131072 size
    cfg = config("plummer131k")
    r, v, m = cfg.ic()
    n = cfg.n
    ctx = make_ctx(n, cfg.eps, "fp64")
    ctx.bind(r, v, m)
    kw = ctx.energy().cpu().numpy()
    ctx.predict(0.0)
    _, pot = ctx.force(np.arange(n, dtype=np.int32), 0.0)
    pot = pot.cpu().numpy()
    assert kw[1] == pytest.approx(0.5 * (m * pot).sum(), rel=1e-12)
    assert kw[0] == pytest.approx(0.5 * (m * (v ** 2).sum(axis=0)).sum(), rel=1e-13)
    take = np.arange(0, n, 997, dtype=np.int32)
    _, p_ref = oracle.force(r, m, cfg.eps, take)
    assert np.allclose(pot[take], p_ref, rtol=1e-12)
    ctx.close()


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("prec,sep", [("fp64", "hilo"), ("mixed", "hilo"), ("mixed", "f64")])
@pytest.mark.parametrize("n,n_act,eps,with_gp", [(5, 5, 0.0, True), (300, 17, 1 / 64, True),
                                                 (1100, 1100, 1 / 128, False),
                                                 (2600, 1, 1 / 256, True),
                                                 (3001, 700, 1 / 256, True)])
def test_backward_matches_oracle(prec, sep, n, n_act, eps, with_gp):
    r, v, m = plummer(n, 4000 + n, masses="loguniform")
    idx = active_subset(n, n_act, 11)
    if n >= 300:
        # massless particles: one active and one not (their position gradients have no
        # source terms; a massless target still feels the others)
        m[idx[0]] = 0.0
        rest = np.setdiff1d(np.arange(n), idx)
        if rest.size:
            m[rest[-1]] = 0.0
    ga = gaussian((3, n_act), 12)
    gp = gaussian(n_act, 13) if with_gp else None
    ctx = make_ctx(n, eps, prec, sep)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    gr, gm = ctx.force_backward(idx, 0.0, ga, gp)
    gr, gm = gr.cpu().numpy(), gm.cpu().numpy()
    rr, rm = oracle.force_backward(r, m, eps, idx, ga, gp)
    sr, sm = oracle.force_backward_scale(r, m, eps, idx, ga, gp)
    check_adjoint(gr, gm, rr, rm, sr, sm, prec, f"n={n} n_act={n_act} sep={sep}")
    # the kernels add into their outputs: into 0.5 / -0.25 the results move by the same
    # gradient, up to the rounding of one or two additions to the offset
    gr0 = torch.full((3, n), 0.5, dtype=torch.float64, device="cuda")
    gm0 = torch.full((n,), -0.25, dtype=torch.float64, device="cuda")
    ctx.force_backward(idx, 0.0, ga, gp, gr0, gm0)
    ulp = 2.0 ** -52
    assert (np.abs(gr0.cpu().numpy() - 0.5 - gr) <= 2 * ulp * (0.5 + np.abs(gr))).all()
    assert (np.abs(gm0.cpu().numpy() + 0.25 - gm) <= 2 * ulp * (0.25 + np.abs(gm))).all()
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_backward_full_size_identities_and_sampled_rows(prec):
    # the N=131072 workload in the launch configuration the benchmark times (every
    # particle active: the fused kernel; half of them: the source / target kernels)
    cfg = config("plummer131k")
    r, v, m = cfg.ic()
    n = cfg.n
    ctx = make_ctx(n, cfg.eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    rows = np.sort(np.random.default_rng(8).choice(n, 96, replace=False)).astype(np.int32)
    for idx in (np.arange(n, dtype=np.int32), active_subset(n, n // 2, cfg.seed + 11)):
        ga = gaussian((3, idx.size), 21)
        acc, pot = ctx.force(idx, 0.0)
        gr, gm = ctx.force_backward(idx, 0.0, ga)
        gr, gm = gr.cpu().numpy(), gm.cpu().numpy()
        # translation invariance: sum over particles of dL/dr vanishes
        assert np.abs(gr.sum(axis=1)).max() <= 1e-5 * np.abs(gr).sum()
        # Euler: sum m dL/dm = sum g . a (acceleration homogeneous of degree one in m)
        euler = (acc.cpu().numpy() * ga).sum()
        assert (m * gm).sum() == pytest.approx(euler, rel=1e-5)
        # sampled rows against the oracle's row-restricted gradient
        rr, rm = oracle.force_backward_rows(r, m, cfg.eps, idx, ga, rows)
        sr, sm = oracle.force_backward_scale(r, m, cfg.eps, idx, ga, rows=rows)
        check_adjoint(gr[:, rows], gm[rows], rr, rm, sr, sm, prec,
                      f"plummer131k n_act={idx.size} sampled rows")
    ctx.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_timestep_full_size_sampled(prec):
    # the criterion at N=131072 in the benchmark's launch configuration, full and half
    # active sets, sampled targets against the oracle
    cfg = config("plummer131k")
    r, v, m = cfg.ic()
    n = cfg.n
    ctx = make_ctx(n, cfg.eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    for idx in (np.arange(n, dtype=np.int32), active_subset(n, n // 2, cfg.seed + 11)):
        dtc = ctx.timestep(idx, cfg.eta).cpu().numpy()
        take = np.sort(np.random.default_rng(9).choice(idx.size, 256, replace=False))
        ref = oracle.timestep(r, v, m, cfg.eps, cfg.eta, idx[take])
        e = rel_err(dtc[take], ref)
        assert e.max() <= (1e-12 if prec == "fp64" else 2e-6), summary(e)
    ctx.close()


# ------------------------------------------------------------------ predictor, corrector, Hermite
def test_taylor_predict_and_corrector_match_oracle():
    n, eps = 700, 1 / 64
    r, v, m = plummer(n, 51)
    a0, _ = oracle.force(r, m, eps)
    rng = np.random.default_rng(1)
    t_last = rng.integers(0, 8, n) * 2.0 ** -10
    dt = 2.0 ** -10 * (8 - t_last / 2.0 ** -10)     # everyone lands on 8 * 2^-10
    ctx = make_ctx(n, eps, "fp64")
    ctx.bind(r, v, m, a=a0, t_last=t_last, dt=dt)
    tb = 8 * 2.0 ** -10
    ctx.predict(tb)
    idx = active_subset(n, 91, 4)
    acc, pot = ctx.force(idx, tb)
    rp, vp = oracle.taylor(r, v, a0, tb - t_last)
    a_ref, p_ref = oracle.force(rp, m, eps, idx)
    assert summary(rel_err_vec(acc.cpu().numpy(), a_ref))["max"] <= 1e-11
    # corrector on the active set
    ctx.correct(idx, tb, acc)
    torch.cuda.synchronize()
    h = (tb - t_last[idx])
    v_ref = v[:, idx] + 0.5 * (a0[:, idx] + a_ref) * h
    assert np.allclose(ctx.r.cpu().numpy()[:, idx], rp[:, idx], rtol=0, atol=1e-14)
    assert np.allclose(ctx.v.cpu().numpy()[:, idx], v_ref, rtol=1e-12, atol=1e-14)
    assert np.array_equal(ctx.t_last.cpu().numpy()[idx], np.full(idx.size, tb))
    others = np.setdiff1d(np.arange(n), idx)
    assert np.array_equal(ctx.r.cpu().numpy()[:, others], r[:, others])
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_history_hermite_prediction_and_snapshot(prec):
    n, eps, h = 600, 1 / 64, 2.0 ** -7
    r, v, m = plummer(n, 52, masses="loguniform")
    a0, _ = oracle.force(r, m, eps)
    everyone = np.arange(n, dtype=np.int32)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m, a=a0, t_last=np.zeros(n), dt=np.full(n, h))
    # pass 0: one shared step of size h, recorded
    ctx.history_begin()
    ctx.predict(h)
    acc, _ = ctx.force(everyone, h)
    ctx.correct(everyone, h, acc)
    ctx.history_end()
    torch.cuda.synchronize()
    r1, v1, a1 = (x.cpu().numpy().copy() for x in (ctx.r, ctx.v, ctx.a))
    # snapshot inside the step: cubic Hermite between the records at 0 and h
    rs, vs = ctx.snapshot(h / 3)
    r_ref, v_ref = oracle.hermite(0.0, r, v, a0, h, r1, v1, a1, h / 3)
    assert np.allclose(rs.cpu().numpy(), r_ref, rtol=0, atol=1e-14)
    assert np.allclose(vs.cpu().numpy(), v_ref, rtol=0, atol=1e-14)
    # pass 1 from the same start: a subset steps h/2, the others are interpolated
    sub = active_subset(n, 50, 9)
    dt = np.full(n, h)
    dt[sub] = h / 2
    ctx.bind(r, v, m, a=a0, t_last=np.zeros(n), dt=dt)
    ctx.predict(h / 2, use_history=True)
    acc2, _ = ctx.force(sub, h / 2)
    rp = oracle.hermite(0.0, r, v, a0, h, r1, v1, a1, h / 2)[0]
    rp[:, sub] = oracle.taylor(r, v, a0, h / 2)[0][:, sub]
    a_ref, _ = oracle.force(rp, m, eps, sub)
    e = summary(rel_err_vec(acc2.cpu().numpy(), a_ref))
    assert e["max"] <= (1e-11 if prec == "fp64" else 1e-4), e
    assert e["median"] <= (1e-13 if prec == "fp64" else 1e-6), e
    ctx.close()


def test_history_multi_tile_records():
    # N spans several 8192-particle scan tiles; three block levels give 1, 2 or 4 records
    # per particle after the era-start record; snapshots inside the era must equal the
    # oracle's Hermite interpolation of the recorded states
    n, eps, h = 20000, 1 / 64, 2.0 ** -8
    r, v, m = plummer(n, 53)
    a0, _ = oracle.force(r, m, eps)
    lev = np.random.default_rng(3).integers(0, 3, n)
    dt = h / 2.0 ** lev
    ctx = make_ctx(n, eps, "fp64")
    ctx.bind(r, v, m, a=a0, t_last=np.zeros(n), dt=dt)
    rec = {j: [(0.0, r[:, j].copy(), v[:, j].copy(), a0[:, j].copy())] for j in range(n)}
    ctx.history_begin()
    t_last = np.zeros(n)
    for tb in (h / 4, h / 2, 3 * h / 4, h):
        act = np.flatnonzero(t_last + dt == tb).astype(np.int32)
        ctx.predict(tb)
        acc, _ = ctx.force(act, tb)
        ctx.correct(act, tb, acc)
        torch.cuda.synchronize()
        rr, vv, aa = (x.cpu().numpy() for x in (ctx.r, ctx.v, ctx.a))
        for j in act:
            rec[j].append((tb, rr[:, j].copy(), vv[:, j].copy(), aa[:, j].copy()))
        t_last[act] = tb
    ctx.history_end()
    assert all(len(rec[j]) == 1 + (1 << lev[j]) for j in range(n))
    for T in (h / 8, 3 * h / 8, h / 2, 7 * h / 8):
        rs, vs = ctx.snapshot(T)
        rs, vs = rs.cpu().numpy(), vs.cpu().numpy()
        for j in range(0, n, 97):
            ts = [x[0] for x in rec[j]]
            k = int(np.searchsorted(ts, T, side="right")) - 1
            if ts[k] == T:
                r_ref, v_ref = rec[j][k][1], rec[j][k][2]
            else:
                p0, p1 = rec[j][k], rec[j][k + 1]
                r_ref, v_ref = oracle.hermite(p0[0], p0[1], p0[2], p0[3], p1[0], p1[1],
                                              p1[2], p1[3], T)
            assert np.allclose(rs[:, j], r_ref, rtol=0, atol=1e-14), (T, j)
            assert np.allclose(vs[:, j], v_ref, rtol=0, atol=1e-13), (T, j)
    ctx.close()


def test_leapfrog_adjoint_elementwise():
    n, h = 300, 0.01
    ctx = make_ctx(n, 0.0, "fp64")
    rbar = torch.tensor(gaussian((3, n), 1), device="cuda")
    vbar = torch.tensor(gaussian((3, n), 2), device="cuda")
    abar = torch.tensor(gaussian((3, n), 3), device="cuda")
    g = torch.empty_like(abar)
    v0, a0 = vbar.clone(), abar.clone()
    ctx.leapfrog_adjoint(0, h, rbar, vbar, abar, g)
    ctx.leapfrog_adjoint(1, h, rbar, vbar, abar, g)
    torch.cuda.synchronize()
    assert torch.allclose(g, a0 + 0.5 * h * v0, rtol=1e-15, atol=1e-15)
    assert torch.allclose(abar, 0.5 * h * v0 + 0.5 * h * h * rbar, rtol=1e-15, atol=1e-15)
    assert torch.allclose(vbar, v0 + h * rbar, rtol=1e-15, atol=1e-15)
    ctx.close()
