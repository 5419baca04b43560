"""GPU gradients through torch.autograd against the oracle and finite differences.

* TsbtsForce: torch backward of (acc, pot) equals the oracle's vector-Jacobian product.
* TsbtsLeapfrog (shared-step leapfrog with era checkpoints): gradients of
  L = sum |r_S - r_target|^2 with respect to r0, v0 and m agree with the oracle's
  reverse-mode gradient (small sphere), and, at the N=8192 / 64 steps / 16-step era
  workload, with central finite differences of the float64 GPU forward along random
  directions to 1e-5 relative.
* TsbtsBlockLeapfrog / TsbtsEraLeapfrog (fixed block schedule; eras with several passes
  and time-symmetric interpolation): the same two checks, plus the history adjoint
  kernels against their definitions and the predictor's history cursor run backwards.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint as oadj
from workloads import plummer, active_subset, gaussian, config
from gpu_util import check_adjoint, check_run_gradient, check_fd

pytestmark = pytest.mark.gpu


def _t(x, grad=False):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda",
                        requires_grad=grad)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_force_function_backward_matches_oracle(prec):
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_force
    n, eps = 700, 1 / 64
    r, _, m = plummer(n, 61, masses="loguniform")
    idx_np = active_subset(n, 123, 3)
    ga, gp = gaussian((3, 123), 1), gaussian(123, 2)
    ctx = Context(n, eps, precision=prec)
    rt, mt = _t(r, True), _t(m, True)
    acc, pot = tsbts_force(rt, mt, ctx.idx(idx_np), ctx)
    ((acc * _t(ga)).sum() + (pot * _t(gp)).sum()).backward()
    rr, rm = oracle.force_backward(r, m, eps, idx_np, ga, gp)
    sr, sm = oracle.force_backward_scale(r, m, eps, idx_np, ga, gp)
    check_adjoint(rt.grad.cpu().numpy(), mt.grad.cpu().numpy(), rr, rm, sr, sm, prec,
                  "autograd force function")
    ctx.close()


def _leapfrog_grads(prec, r0, v0, m, eps, h, steps, era, target):
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_leapfrog
    ctx = Context(m.size, eps, precision=prec)
    rt, vt, mt = _t(r0, True), _t(v0, True), _t(m, True)
    r_end, _ = tsbts_leapfrog(rt, vt, mt, ctx, h, steps, era)
    loss = ((r_end - _t(target)) ** 2).sum()
    loss.backward()
    out = (float(loss), rt.grad.cpu().numpy(), vt.grad.cpu().numpy(), mt.grad.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("era", [3, 8])
def test_leapfrog_gradient_matches_oracle(prec, era):
    n, eps, h, steps = 300, 1 / 64, 1 / 128, 8
    r0, v0, m = plummer(n, 62, masses="loguniform")
    target = oadj.forward(r0, v0, m, eps, h, steps)[0] + 0.01 * gaussian((3, n), 7)
    L, gr, gv, gm = _leapfrog_grads(prec, r0, v0, m, eps, h, steps, era, target)
    Lr, rr, rv, rm = oadj.gradient(r0, v0, m, eps, h, steps, target)
    assert L == pytest.approx(Lr, rel=1e-9 if prec == "fp64" else 1e-5)
    for name, got, ref in (("r", gr, rr), ("v", gv, rv), ("m", gm, rm)):
        check_run_gradient(got, ref, prec, f"dL/d{name}")


def _loss_fp64(ctx, r0, v0, m, h, steps, target):
    from paper_1205_2288_amd.autograd import tsbts_leapfrog
    with torch.no_grad():
        r_end, _ = tsbts_leapfrog(_t(r0), _t(v0), _t(m), ctx, h, steps, steps)
        return float(((r_end - _t(target)) ** 2).sum())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint8192_gradients_vs_finite_differences(prec):
    from paper_1205_2288_amd import Context
    cfg = config("adjoint8192")
    n, eps, h, steps, era = cfg.n, cfg.eps, 1 / 256, 64, 16
    r0, v0, m = cfg.ic()
    ref_ctx = Context(n, eps, precision="fp64")
    r_fin = None
    from paper_1205_2288_amd.autograd import tsbts_leapfrog
    with torch.no_grad():
        r_fin, _ = tsbts_leapfrog(_t(r0), _t(v0), _t(m), ref_ctx, h, steps, era)
    target = r_fin.cpu().numpy() + 0.01 * gaussian((3, n), cfg.seed + 7)
    L, gr, gv, gm = _leapfrog_grads(prec, r0, v0, m, eps, h, steps, era, target)
    step = 1e-6
    rows = []
    for trial in range(8):
        for which, g in (("r", gr), ("v", gv), ("m", gm)):
            d = gaussian((3, n) if which != "m" else n, 900 + 10 * trial + len(which))
            if which == "m":
                d = d * m
            def f(sgn):
                rr = r0 + sgn * step * d if which == "r" else r0
                vv = v0 + sgn * step * d if which == "v" else v0
                mm = m + sgn * step * d if which == "m" else m
                return _loss_fp64(ref_ctx, rr, vv, mm, h, steps, target)
            fd = (f(1) - f(-1)) / (2 * step)
            rows.append((which, (g * d).sum(), fd))
            print(f"{prec} {which}: adjoint {(g * d).sum():.10e} fd {fd:.10e}")
    check_fd(rows, prec, "adjoint8192 shared steps")
    ref_ctx.close()


# ---------------------------------------------------------------- fixed block schedule
def _levels(n, h, seed, nlev=3):
    rng = np.random.default_rng(seed)
    return h * 2.0 ** rng.integers(0, nlev, size=n)


def _block_grads(prec, r0, v0, m, eps, dt, t_end, era, rt, vt):
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_block_leapfrog
    ctx = Context(m.size, eps, precision=prec)
    r, v, mm = _t(r0, True), _t(v0, True), _t(m, True)
    r_end, v_end = tsbts_block_leapfrog(r, v, mm, ctx, dt, t_end, era)
    loss = ((r_end - _t(rt)) ** 2).sum() + ((v_end - _t(vt)) ** 2).sum()
    loss.backward()
    out = (float(loss.detach()), r.grad.cpu().numpy(), v.grad.cpu().numpy(),
           mm.grad.cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("era", [5, 64])
def test_block_leapfrog_gradient_matches_oracle(prec, era):
    # 600 particles (two full 256-tiles and a ragged one), steps h, 2h, 4h, 16 block steps
    n, eps, h = 600, 1 / 64, 1 / 128
    t_end = 16 * h
    r0, v0, m = plummer(n, 63, masses="loguniform")
    dt = _levels(n, h, 8)
    rt, vt, _ = oadj.block_forward(r0, v0, m, eps, dt, t_end)
    rt = rt + 0.01 * gaussian((3, n), 21)
    vt = vt + 0.01 * gaussian((3, n), 22)
    Lr, rr, rv, rm = oadj.block_gradient(r0, v0, m, eps, dt, t_end, rt, vt)
    L, gr, gv, gm = _block_grads(prec, r0, v0, m, eps, dt, t_end, era, rt, vt)
    assert L == pytest.approx(Lr, rel=1e-9 if prec == "fp64" else 1e-5)
    for name, got, ref in (("r", gr, rr), ("v", gv, rv), ("m", gm, rm)):
        check_run_gradient(got, ref, prec, f"dL/d{name}")


def test_block_adjoint_phases_elementwise():
    # the two element-wise phases against their definitions, on random adjoints
    from paper_1205_2288_amd import Context
    n, tb = 777, 0.75
    r, v, m = plummer(n, 64)
    rng = np.random.default_rng(3)
    dt = 2.0 ** -rng.integers(2, 5, size=n)
    t_last = tb - dt * rng.integers(0, 2, size=n) - dt * (rng.random(n) < 0.5) * 0.5
    idx_np = np.sort(rng.choice(n, 123, replace=False)).astype(np.int32)
    ctx = Context(n, 0.01, precision="fp64")
    ctx.bind(r, v, m, t_last=t_last, dt=dt)
    rb, vb, ab = (gaussian((3, n), 40 + k) for k in range(3))
    R, V, A = _t(rb), _t(vb), _t(ab)
    P = _t(gaussian((3, n), 50))          # garbage: phase 0 must clear it
    S = torch.empty((3, idx_np.size), dtype=torch.float64, device="cuda")
    ctx.block_adjoint(0, idx_np, tb, R, V, A, P, S)
    torch.cuda.synchronize()
    i = idx_np.astype(np.int64)
    half = 0.5 * dt[i]
    p_ref = np.zeros((3, n))
    p_ref[:, i] = rb[:, i]
    a_ref, r_ref = ab.copy(), rb.copy()
    a_ref[:, i] = half * vb[:, i]
    r_ref[:, i] = 0.0
    assert np.allclose(S.cpu().numpy(), ab[:, i] + half * vb[:, i], rtol=0, atol=1e-15)
    assert np.array_equal(P.cpu().numpy(), p_ref)
    assert np.array_equal(A.cpu().numpy(), a_ref)
    assert np.array_equal(R.cpu().numpy(), r_ref)
    assert np.array_equal(V.cpu().numpy(), vb)
    pb = gaussian((3, n), 60)
    P.copy_(_t(pb))
    ctx.block_adjoint(1, None, tb, R, V, A, P, None)
    torch.cuda.synchronize()
    hh = tb - t_last
    assert np.array_equal(R.cpu().numpy(), r_ref + pb)
    assert np.allclose(V.cpu().numpy(), vb + hh * pb, rtol=0, atol=1e-15)
    assert np.allclose(A.cpu().numpy(), a_ref + 0.5 * hh * hh * pb, rtol=0, atol=1e-15)
    ctx.close()


def test_block_adjoint_bad_arguments():
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd._lib import TsbtsError, TSBTS_EINVAL
    n = 50
    r, v, m = plummer(n, 65)
    ctx = Context(n, 0.01, precision="fp64")
    ctx.bind(r, v, m, dt=np.full(n, 0.25))
    z = lambda: torch.zeros((3, n), dtype=torch.float64, device="cuda")  # noqa: E731
    R, V, A, P = z(), z(), z(), z()
    with pytest.raises(TsbtsError) as e:
        ctx.block_adjoint(2, None, 0.25, R, V, A, P, None)
    assert e.value.status == TSBTS_EINVAL
    with pytest.raises(TsbtsError) as e:
        ctx.block_adjoint(0, None, 0.25, R, V, A, P, None)   # phase 0 needs the active set
    assert e.value.status == TSBTS_EINVAL
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint8192_block_schedule_vs_finite_differences(prec):
    # the N=8192 workload on a three-level block schedule (h, 2h, 4h with h = 2^-8, 32
    # block steps, checkpoints every 8): adjoint directional derivatives against central
    # differences of the float64 GPU forward
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_block_leapfrog
    cfg = config("adjoint8192")
    n, eps, h = cfg.n, cfg.eps, 1 / 256
    t_end, era = 32 * h, 8
    r0, v0, m = cfg.ic()
    dt = _levels(n, h, cfg.seed + 3)
    ref = Context(n, eps, precision="fp64")

    def fwd(rr, vv, mm):
        with torch.no_grad():
            return tsbts_block_leapfrog(_t(rr), _t(vv), _t(mm), ref, dt, t_end, 1 << 30)

    r_fin, v_fin = fwd(r0, v0, m)
    rt = r_fin.cpu().numpy() + 0.01 * gaussian((3, n), cfg.seed + 8)
    vt = v_fin.cpu().numpy() + 0.01 * gaussian((3, n), cfg.seed + 9)

    def loss(rr, vv, mm):
        r_e, v_e = fwd(rr, vv, mm)
        return float(((r_e - _t(rt)) ** 2).sum() + ((v_e - _t(vt)) ** 2).sum())

    L, gr, gv, gm = _block_grads(prec, r0, v0, m, eps, dt, t_end, era, rt, vt)
    step = 1e-6
    rows = []
    for trial in range(8):
        for which, g in (("r", gr), ("v", gv), ("m", gm)):
            d = gaussian((3, n) if which != "m" else n, 950 + 10 * trial + len(which))
            if which == "m":
                d = d * m
            def f(sgn):
                return loss(r0 + sgn * step * d if which == "r" else r0,
                            v0 + sgn * step * d if which == "v" else v0,
                            m + sgn * step * d if which == "m" else m)
            fd = (f(1) - f(-1)) / (2 * step)
            rows.append((which, (g * d).sum(), fd))
            print(f"block {prec} {which}: adjoint {(g * d).sum():.10e} fd {fd:.10e}")
    check_fd(rows, prec, "adjoint8192 block")
    ref.close()


# ---------------------------------------------------------------- eras with several passes
def _era_grads(prec, r0, v0, m, eps, dt, t_end, era, passes, rt, vt):
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_era_leapfrog
    ctx = Context(m.size, eps, precision=prec)
    r, v, mm = _t(r0, True), _t(v0, True), _t(m, True)
    r_end, v_end = tsbts_era_leapfrog(r, v, mm, ctx, dt, t_end, era, passes)
    loss = ((r_end - _t(rt)) ** 2).sum() + ((v_end - _t(vt)) ** 2).sum()
    loss.backward()
    out = (float(loss.detach()), r.grad.cpu().numpy(), v.grad.cpu().numpy(),
           mm.grad.cpu().numpy(), r_end.detach().cpu().numpy(), v_end.detach().cpu().numpy())
    ctx.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("passes", [2, 3])
def test_era_leapfrog_gradient_matches_oracle(prec, passes):
    # 300 particles (a full 256-tile and a ragged one), steps h, 2h, 4h, two eras of 8h
    n, eps, h = 300, 1 / 64, 1 / 128
    t_end, era = 16 * h, 8 * h
    r0, v0, m = plummer(n, 66, masses="loguniform")
    dt = _levels(n, h, 9)
    r_ref, v_ref, _ = oadj.era_forward(r0, v0, m, eps, dt, t_end, era, passes)
    rt = r_ref + 0.01 * gaussian((3, n), 23)
    vt = v_ref + 0.01 * gaussian((3, n), 24)
    Lr, rr, rv, rm = oadj.era_gradient(r0, v0, m, eps, dt, t_end, era, passes, rt, vt)
    L, gr, gv, gm, r_end, v_end = _era_grads(prec, r0, v0, m, eps, dt, t_end, era, passes,
                                             rt, vt)
    fwd_tol = 1e-12 if prec == "fp64" else 1e-6
    assert np.abs(r_end - r_ref).max() <= fwd_tol * np.abs(r_ref).max()
    assert np.abs(v_end - v_ref).max() <= fwd_tol * np.abs(v_ref).max() * 10
    assert L == pytest.approx(Lr, rel=1e-9 if prec == "fp64" else 1e-5)
    for name, got, ref in (("r", gr, rr), ("v", gv, rv), ("m", gm, rm)):
        check_run_gradient(got, ref, prec, f"dL/d{name}")


def _history_pass(ctx, dt, h, steps):
    """Record one pass of `steps` block steps of size h from the bound state."""
    ctx.history_begin()
    for s in range(1, steps + 1):
        tb = s * h
        act = np.flatnonzero(np.mod(tb, dt) == 0.0).astype(np.int32)
        ctx.predict(tb)
        acc = ctx.force(act, tb, with_pot=False)[0]
        ctx.correct(act, tb, acc)
    ctx.history_end()


def test_interp_and_record_adjoint_elementwise():
    # the two history adjoint kernels against their definitions (oracle Hermite weights)
    from paper_1205_2288_amd import Context
    n, eps, h = 777, 1 / 64, 1 / 64
    r0, v0, m = plummer(n, 67)
    dt = _levels(n, h, 10)
    ctx = Context(n, eps, precision="fp64")
    ctx.bind(r0, v0, m, dt=dt)
    _history_pass(ctx, dt, h, 8)
    n_rec, off_t, t_t = ctx.history_layout()
    off, t = off_t.cpu().numpy(), t_t.cpu().numpy()
    counts = np.diff(off)
    assert n_rec == off[-1] == int((1 + 8 * h / dt).sum())
    assert np.array_equal(counts, (1 + 8 * h / dt).astype(np.int64))
    for j in (0, 1, n - 1):
        assert np.array_equal(t[off[j]:off[j + 1]], dt[j] * np.arange(counts[j]))
    # back at the era start: at t_b the particles with dt == t_b are active; the others
    # are interpolated (exact at stored times, Hermite otherwise)
    ctx.bind(r0, v0, m, dt=dt)
    for tb in (h, 2 * h, 3 * h, 6 * h):
        pb = gaussian((3, n), 70 + int(tb / h))
        P = _t(pb)
        hb0 = gaussian((6, n_rec), 80 + int(tb / h))
        Hb = _t(hb0)
        ctx.interp_adjoint(tb, P, Hb)
        torch.cuda.synchronize()
        hb_ref, pb_ref = hb0.copy(), pb.copy()
        for j in range(n):
            if dt[j] == tb:
                continue
            lo, hi = off[j], off[j + 1]
            k = lo + int(np.searchsorted(t[lo:hi], tb, side="right")) - 1
            if t[k] == tb:
                hb_ref[0:3, k] += pb[:, j]
            else:
                w = oadj.hermite_weights(t[k], t[k + 1], tb)
                hb_ref[0:3, k] += w[0] * pb[:, j]
                hb_ref[3:6, k] += w[1] * pb[:, j]
                hb_ref[0:3, k + 1] += w[2] * pb[:, j]
                hb_ref[3:6, k + 1] += w[3] * pb[:, j]
            pb_ref[:, j] = 0.0
        assert np.array_equal(P.cpu().numpy(), pb_ref)
        assert np.allclose(Hb.cpu().numpy(), hb_ref, rtol=1e-15, atol=1e-15)
    # record injection at a stored time of a random subset
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(n, 200, replace=False)).astype(np.int32)
    hb = gaussian((6, n_rec), 90)
    rb, vb = gaussian((3, n), 91), gaussian((3, n), 92)
    R, V = _t(rb), _t(vb)
    for tb in (4 * h, 0.0):
        ctx.record_adjoint(idx, tb, (n_rec, off_t, t_t), _t(hb), R, V)
        for i in idx:
            ks = np.flatnonzero(t[off[i]:off[i + 1]] == tb)
            if ks.size:
                k = off[i] + ks[0]
                rb[:, i] += hb[0:3, k]
                vb[:, i] += hb[3:6, k]
    torch.cuda.synchronize()
    assert np.array_equal(R.cpu().numpy(), rb)
    assert np.array_equal(V.cpu().numpy(), vb)
    ctx.close()


def test_predict_history_cursor_both_directions():
    # predictions from the history at decreasing block times (a reverse sweep) equal the
    # ones made going forward, bit for bit
    from paper_1205_2288_amd import Context
    n, eps, h = 500, 1 / 64, 1 / 64
    r0, v0, m = plummer(n, 68)
    dt = _levels(n, h, 11)
    ctx = Context(n, eps, precision="mixed")
    ctx.bind(r0, v0, m, dt=dt)
    _history_pass(ctx, dt, h, 8)
    ctx.bind(r0, v0, m, dt=dt)
    every = np.arange(n, dtype=np.int32)
    fwd = {}
    for s in range(1, 8):
        ctx.predict(s * h, True)
        fwd[s] = ctx.force(every, s * h)[0].cpu().numpy()
    for s in (7, 5, 2, 1, 6, 3):
        ctx.predict(s * h, True)
        assert np.array_equal(ctx.force(every, s * h)[0].cpu().numpy(), fwd[s]), s
    ctx.close()


def test_history_adjoint_bad_arguments():
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd._lib import TsbtsError, TSBTS_EINVAL, TSBTS_ESTATE
    n, h = 64, 1 / 64
    r, v, m = plummer(n, 69)
    dt = np.full(n, h)
    ctx = Context(n, 0.01, precision="fp64")
    ctx.bind(r, v, m, dt=dt)
    P = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    with pytest.raises(TsbtsError) as e:
        ctx.history_layout()
    assert e.value.status == TSBTS_ESTATE
    with pytest.raises(TsbtsError) as e:
        ctx.interp_adjoint(h, P, torch.zeros((6, 1), dtype=torch.float64, device="cuda"))
    assert e.value.status == TSBTS_ESTATE
    _history_pass(ctx, dt, h, 2)
    n_rec = ctx.history_layout()[0]
    assert n_rec == 3 * n
    with pytest.raises(TsbtsError) as e:   # record adjoint sized for another history
        ctx.interp_adjoint(h, P, torch.zeros((6, n_rec - 1), dtype=torch.float64,
                                             device="cuda"))
    assert e.value.status == TSBTS_EINVAL
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint8192_era_passes_vs_finite_differences(prec):
    # the N=8192 workload on the three-level schedule cut into eras of 8h with three
    # passes each (4 eras, 96 block-step evaluations per forward run): adjoint
    # directional derivatives against central differences of the float64 GPU forward
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_era_leapfrog
    cfg = config("adjoint8192")
    n, eps, h = cfg.n, cfg.eps, 1 / 256
    t_end, era, passes = 32 * h, 8 * h, 3
    r0, v0, m = cfg.ic()
    dt = _levels(n, h, cfg.seed + 3)
    ref = Context(n, eps, precision="fp64")

    def fwd(rr, vv, mm):
        with torch.no_grad():
            return tsbts_era_leapfrog(_t(rr), _t(vv), _t(mm), ref, dt, t_end, era, passes)

    r_fin, v_fin = fwd(r0, v0, m)
    rt = r_fin.cpu().numpy() + 0.01 * gaussian((3, n), cfg.seed + 18)
    vt = v_fin.cpu().numpy() + 0.01 * gaussian((3, n), cfg.seed + 19)

    def loss(rr, vv, mm):
        r_e, v_e = fwd(rr, vv, mm)
        return float(((r_e - _t(rt)) ** 2).sum() + ((v_e - _t(vt)) ** 2).sum())

    L, gr, gv, gm, _, _ = _era_grads(prec, r0, v0, m, eps, dt, t_end, era, passes, rt, vt)
    step = 1e-6
    rows = []
    for trial in range(8):
        for which, g in (("r", gr), ("v", gv), ("m", gm)):
            d = gaussian((3, n) if which != "m" else n, 960 + 10 * trial + len(which))
            if which == "m":
                d = d * m
            def f(sgn):
                return loss(r0 + sgn * step * d if which == "r" else r0,
                            v0 + sgn * step * d if which == "v" else v0,
                            m + sgn * step * d if which == "m" else m)
            fd = (f(1) - f(-1)) / (2 * step)
            rows.append((which, (g * d).sum(), fd))
            print(f"era passes {prec} {which}: adjoint {(g * d).sum():.10e} fd {fd:.10e}")
    check_fd(rows, prec, "adjoint8192 era passes")
    ref.close()


# ---------------------------------------------------------------- recorded schedules
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_recorded_schedule_gradient_matches_oracle(prec):
    # a schedule chosen by the criterion in the oracle's era driver (dynamic eras, three
    # passes), replayed on the GPU: end state and gradient against the oracle's replay
    from oracle.tsbts import OracleTSBTS
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_schedule_leapfrog
    n, eps = 100, 1 / 64
    r0, v0, m = plummer(n, 70, masses="loguniform")
    sim = OracleTSBTS(r0, v0, m, eps, passes=3, dt_max=1 / 64, record_schedule=True)
    sim.run(1 / 32)
    sched = sim.schedule
    rt = sim.r + 0.01 * gaussian((3, n), 25)
    vt = sim.v + 0.01 * gaussian((3, n), 26)
    Lr, rr, rv, rm = oadj.schedule_gradient(r0, v0, m, eps, sched, rt, vt)
    ctx = Context(n, eps, precision=prec)
    r, v, mm = _t(r0, True), _t(v0, True), _t(m, True)
    r_end, v_end = tsbts_schedule_leapfrog(r, v, mm, ctx, sched)
    fwd_tol = 1e-12 if prec == "fp64" else 1e-6
    assert np.abs(r_end.detach().cpu().numpy() - sim.r).max() <= fwd_tol
    loss = ((r_end - _t(rt)) ** 2).sum() + ((v_end - _t(vt)) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(Lr, rel=1e-9 if prec == "fp64" else 1e-5)
    for name, got, ref in (("r", r.grad, rr), ("v", v.grad, rv), ("m", mm.grad, rm)):
        check_run_gradient(got.cpu().numpy(), ref, prec, f"recorded schedule dL/d{name}")
    ctx.close()


def test_driver_schedule_replay_and_finite_differences():
    # the GPU driver records the schedule it chose (N = 2048, three passes, dynamic eras);
    # replaying it reproduces the run bit for bit, and the replay's gradient matches
    # central differences of the replayed float64 forward
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.driver import TSBTS
    from paper_1205_2288_amd.autograd import tsbts_schedule_leapfrog
    n, eps = 2048, 1 / 256
    r0, v0, m = plummer(n, 71)
    drv = TSBTS(r0, v0, m, eps, passes=3, dt_max=1 / 64, precision="fp64",
                record_schedule=True)
    drv.run(1 / 64)
    sched = drv.schedule
    steps = sum(len(p) for e in sched["eras"] for p in e["passes"])
    st = drv.state()
    drv.close()
    ctx = Context(n, eps, precision="fp64")

    def fwd(rr, vv, mm):
        with torch.no_grad():
            return tsbts_schedule_leapfrog(_t(rr), _t(vv), _t(mm), ctx, sched)

    r_e, v_e = fwd(r0, v0, m)
    assert np.array_equal(r_e.cpu().numpy(), st["r"])
    assert np.array_equal(v_e.cpu().numpy(), st["v"])
    rt = st["r"] + 0.01 * gaussian((3, n), 27)
    vt = st["v"] + 0.01 * gaussian((3, n), 28)

    def loss(rr, vv, mm):
        a, b = fwd(rr, vv, mm)
        return float(((a - _t(rt)) ** 2).sum() + ((b - _t(vt)) ** 2).sum())

    r, v, mm = _t(r0, True), _t(v0, True), _t(m, True)
    a, b = tsbts_schedule_leapfrog(r, v, mm, ctx, sched)
    ((a - _t(rt)) ** 2).sum().add(((b - _t(vt)) ** 2).sum()).backward()
    grads = {"r": r.grad.cpu().numpy(), "v": v.grad.cpu().numpy(), "m": mm.grad.cpu().numpy()}
    step = 1e-6
    rows = []
    for trial, which in [(k, w) for k in range(3) for w in ("r", "v", "m")]:
        d = gaussian((3, n) if which != "m" else n, 990 + 10 * trial + len(which))
        if which == "m":
            d = d * m
        fd = (loss(r0 + step * d if which == "r" else r0, v0 + step * d if which == "v" else v0,
                   m + step * d if which == "m" else m)
              - loss(r0 - step * d if which == "r" else r0,
                     v0 - step * d if which == "v" else v0,
                     m - step * d if which == "m" else m)) / (2 * step)
        g = (grads[which] * d).sum()
        rows.append((which, g, fd))
        print(f"driver schedule ({steps} block steps, {len(sched['eras'])} eras) {which}: "
              f"adjoint {g:.10e} fd {fd:.10e}")
    check_fd(rows, "fp64", "driver schedule replay")
    ctx.close()
