"""Degenerate inputs through the C ABI against the oracle and the definitions.

* one particle: no pair at all — zero acceleration and potential, an infinite criterion
  (no collision or free-fall time), kinetic energy only, zero adjoint;
* massless particles: they feel forces but exert none, and never set a free-fall time;
* coincident particles with eps > 0: finite softened pull, zero separation;
* widely separated scales (a tight pair inside a sphere) in both precisions.
"""
import numpy as np
import pytest
import torch

import oracle
from workloads import plummer, gaussian
from gpu_util import rel_err_vec, make_ctx

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_single_particle(prec):
    r = np.array([[0.3], [-0.2], [0.1]])
    v = np.array([[1.0], [0.0], [0.5]])
    m = np.array([0.7])
    ctx = make_ctx(1, 0.01, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    idx = np.zeros(1, dtype=np.int32)
    acc, pot = ctx.force(idx, 0.0)
    assert np.array_equal(acc.cpu().numpy(), np.zeros((3, 1)))
    assert np.array_equal(pot.cpu().numpy(), np.zeros(1))
    dtc = ctx.timestep(idx, 0.1).cpu().numpy()
    assert np.isinf(dtc[0]) and np.isinf(oracle.timestep(r, v, m, 0.01, 0.1, idx)[0])
    kw = ctx.energy().cpu().numpy()
    assert kw[0] == pytest.approx(0.5 * 0.7 * 1.25, rel=1e-15) and kw[1] == 0.0
    gr, gm = ctx.force_backward(idx, 0.0, gaussian((3, 1), 1))
    assert np.array_equal(gr.cpu().numpy(), np.zeros((3, 1)))
    assert np.array_equal(gm.cpu().numpy(), np.zeros(1))
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n_act", [5, 600])
def test_massless_particles(prec, n_act):
    n, eps = 600, 1 / 64
    r, v, m = plummer(n, 81)
    m = m.copy()
    m[::3] = 0.0
    idx = np.sort(np.random.default_rng(2).choice(n, n_act, replace=False)).astype(np.int32)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    acc, pot = ctx.force(idx, 0.0)
    a_ref, p_ref = oracle.force(r, m, eps, idx)
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert rel_err_vec(acc.cpu().numpy(), a_ref).max() <= tol
    dtc = ctx.timestep(idx, 0.1).cpu().numpy()
    ref = oracle.timestep(r, v, m, eps, 0.1, idx)
    assert np.all(np.isfinite(dtc))
    assert np.allclose(dtc, ref, rtol=1e-12 if prec == "fp64" else 2e-6)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_coincident_particles_softened(prec):
    # two particles at the same point among others: their mutual pull vanishes
    # (zero separation), the potential keeps the softened -m/eps term
    n, eps = 300, 1 / 32
    r, v, m = plummer(n, 82)
    r = r.copy()
    r[:, 1] = r[:, 0]
    idx = np.arange(n, dtype=np.int32)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    acc, pot = ctx.force(idx, 0.0)
    a_ref, p_ref = oracle.force(r, m, eps, idx)
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert rel_err_vec(acc.cpu().numpy(), a_ref).max() <= tol
    assert np.allclose(pot.cpu().numpy(), p_ref, rtol=tol)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tight_binary_inside_sphere(prec):
    # a pair at separation 1e-5 (eps = 1e-6) at radius ~1: the float64 separation keeps
    # the pair's pull accurate although both positions are O(1)
    n, eps = 1000, 1e-6
    r, v, m = plummer(n, 83)
    r = r.copy()
    r[:, 1] = r[:, 0] + np.array([1e-5, 0.0, 0.0])
    idx = np.array([0, 1, 2], dtype=np.int32)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    acc, _ = ctx.force(idx, 0.0)
    a_ref, _ = oracle.force(r, m, eps, idx)
    e = rel_err_vec(acc.cpu().numpy(), a_ref)
    assert e.max() <= (1e-12 if prec == "fp64" else 1e-5), e
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,n_act", [(300, 300), (300, 7), (9000, 9000)])
def test_criterion_bulk_motion(prec, n, n_act):
    # every particle moves with the same velocity: no collision time anywhere, the
    # criterion is the free-fall term alone (padding particles must not contribute)
    eps, eta = 1 / 64, 0.1
    r, _, m = plummer(n, 84, masses="loguniform")
    v = np.tile(np.array([[0.3], [-0.7], [0.2]]), (1, n))
    idx = np.sort(np.random.default_rng(5).choice(n, n_act, replace=False)).astype(np.int32)
    ctx = make_ctx(n, eps, prec)
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    dtc = ctx.timestep(idx, eta).cpu().numpy()
    ref = oracle.timestep(r, v, m, eps, eta, idx)
    vz = np.zeros_like(v)
    assert np.array_equal(ref, oracle.timestep(r, vz, m, eps, eta, idx))  # velocity-free
    assert np.allclose(dtc, ref, rtol=1e-12 if prec == "fp64" else 2e-6)
    ctx.close()


def test_index_check_mode():
    # TSBTS_TUNE_CHECK_INDICES: a device active set with an index outside [0, n) is refused
    # before any kernel uses it; valid sets give the same results as without the check.
    # The bad index is n itself, which lies in the arrays' padding, so nothing could be
    # touched outside them even without the check.
    from paper_1205_2288_amd._lib import TsbtsError
    n = 1000
    r, v, m = plummer(n, 3)
    ctx = make_ctx(n, 0.01, "mixed")
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    good = ctx.idx(np.arange(0, n, 3, dtype=np.int32))
    acc_ref, _ = ctx.force(good, 0.0)
    dtc_ref = ctx.timestep(good, 0.1)
    ctx.tune(check_indices=1)
    acc, _ = ctx.force(good, 0.0)
    assert torch.equal(acc, acc_ref)
    assert torch.equal(ctx.timestep(good, 0.1), dtc_ref)
    bad = torch.tensor([0, 5, n], dtype=torch.int32, device=ctx.device)
    with pytest.raises(TsbtsError, match="outside"):
        ctx.force(bad, 0.0)
    with pytest.raises(TsbtsError, match="outside"):
        ctx.timestep(bad, 0.1)
    acc, _ = ctx.force(good, 0.0)  # still usable after a refusal
    assert torch.equal(acc, acc_ref)
    rep = torch.tensor([0, 5, 9, 5], dtype=torch.int32, device=ctx.device)
    with pytest.raises(TsbtsError, match="repeats"):
        ctx.force(rep, 0.0)
    with pytest.raises(TsbtsError, match="repeats"):
        ctx.force_backward(rep, 0.0, np.ones((3, 4)))
    acc, _ = ctx.force(good, 0.0)
    assert torch.equal(acc, acc_ref)
    with pytest.raises(TsbtsError):
        ctx.tune(check_indices=2)
    ctx.tune(check_indices=0)
    ctx.close()


def test_index_check_mode_full_set_permutation():
    # every particle a target at N = 32768 (the symmetric kernels, which write their rows
    # through the inverse of the active list): a list with a repeated index is refused in
    # check mode; a permutation gives the same results as without the check
    from paper_1205_2288_amd._lib import TsbtsError
    n = 32768
    r, v, m = plummer(n, 4)
    ctx = make_ctx(n, 1 / 1024, "mixed")
    ctx.bind(r, v, m)
    ctx.predict(0.0)
    perm = np.random.default_rng(2).permutation(n).astype(np.int32)
    good = ctx.idx(perm)
    acc_ref, _ = ctx.force(good, 0.0)
    ctx.tune(check_indices=1)
    acc, _ = ctx.force(good, 0.0)
    assert torch.equal(acc, acc_ref)
    dup = perm.copy()
    dup[100] = dup[2000]
    with pytest.raises(TsbtsError, match="repeats"):
        ctx.force(ctx.idx(dup), 0.0)
    with pytest.raises(TsbtsError, match="repeats"):
        ctx.timestep(ctx.idx(dup), 0.1)
    ctx.close()
