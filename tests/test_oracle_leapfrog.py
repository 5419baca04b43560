"""Pins of the oracle's predictor, Hermite interpolant and leapfrog (Section 2).

Closed forms: Kepler two-body orbits (period, energy error O(h^2), eccentric orbit from
Kepler's equation), polynomial trajectories, and exact time reversibility."""
import math

import numpy as np
import pytest

from workloads import plummer, gaussian


def _kepler_pair(e, a_semi=1.0, mtot=1.0):
    # relative orbit starting at pericentre, centre of mass at rest
    m = np.array([0.6, 0.4]) * mtot
    rp = a_semi * (1 - e)
    vp = math.sqrt(mtot * (1 + e) / rp)
    rel_r = np.array([rp, 0.0, 0.0])
    rel_v = np.array([0.0, vp, 0.0])
    r = np.stack([-m[1] / mtot * rel_r, m[0] / mtot * rel_r], axis=1)
    v = np.stack([-m[1] / mtot * rel_v, m[0] / mtot * rel_v], axis=1)
    return r, v, m


def test_taylor_exact_on_quadratic(oracle):
    r0 = gaussian((3, 5), 1)
    v0 = gaussian((3, 5), 2)
    a0 = gaussian((3, 5), 3)
    h = np.array([0.25, 0.5, 0.125, 1.0, 0.0])
    rp, vp = oracle.taylor(r0, v0, a0, h)
    assert np.allclose(rp, r0 + v0 * h + a0 * h * h / 2, rtol=0, atol=1e-15)
    assert np.allclose(vp, v0 + a0 * h, rtol=0, atol=1e-15)


def test_hermite_reproduces_cubics(oracle):
    c = gaussian((4, 3), 7)  # r(t) = c0 + c1 t + c2 t^2 + c3 t^3
    r = lambda t: c[0] + c[1] * t + c[2] * t * t + c[3] * t ** 3
    v = lambda t: c[1] + 2 * c[2] * t + 3 * c[3] * t * t
    a = lambda t: 2 * c[2] + 6 * c[3] * t
    t0, t1 = 0.375, 0.875
    for t in (t0, 0.4, 0.5, 0.7, t1):
        rr, vv = oracle.hermite(t0, r(t0), v(t0), a(t0), t1, r(t1), v(t1), a(t1), t)
        assert np.allclose(rr, r(t), rtol=0, atol=1e-14)
        # velocity interpolant is the cubic Hermite of (v, a): exact for quadratic v
        assert np.allclose(vv, v(t), rtol=0, atol=1e-14)
    # endpoints are reproduced exactly
    rr, _ = oracle.hermite(t0, r(t0), v(t0), a(t0), t1, r(t1), v(t1), a(t1), t0)
    assert np.array_equal(rr, r(t0))


def test_hermite_time_reversal_symmetry(oracle):
    p = gaussian((6, 3), 8)
    t0, t1, t = 0.0, 0.5, 0.125
    r_f, v_f = oracle.hermite(t0, p[0], p[1], p[2], t1, p[3], p[4], p[5], t)
    # swap the ends and reverse time: t -> -t, v -> -v, a -> a
    r_b, v_b = oracle.hermite(-t1, p[3], -p[4], p[5], -t0, p[0], -p[1], p[2], -t)
    assert np.allclose(r_b, r_f, atol=1e-15)
    assert np.allclose(v_b, -v_f, atol=1e-15)


def test_circular_kepler_period_and_second_order(oracle):
    r, v, m = _kepler_pair(0.0)
    period = 2 * math.pi
    errs = []
    for steps in (256, 512):
        h = period / steps
        r1, v1, _ = oracle.leapfrog_shared(r, v, m, 0.0, h, steps)
        errs.append(np.abs(r1 - r).max())
    assert errs[1] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0  # second order


def test_eccentric_orbit_vs_kepler_equation(oracle):
    e = 0.5
    r, v, m = _kepler_pair(e)
    t_end = 1.7
    steps = 4000
    r1, v1, _ = oracle.leapfrog_shared(r, v, m, 0.0, t_end / steps, steps)
    M = t_end  # mean anomaly, n = sqrt(M/a^3) = 1
    E = M
    for _ in range(50):
        E = E - (E - e * math.sin(E) - M) / (1 - e * math.cos(E))
    rel = np.array([math.cos(E) - e, math.sqrt(1 - e * e) * math.sin(E), 0.0])
    got = r1[:, 1] - r1[:, 0]
    assert np.abs(got - rel).max() < 1e-5


def test_energy_error_second_order_and_momentum(oracle):
    r, v, m = _kepler_pair(0.3)
    k0, w0 = oracle.energy(r, v, m, 0.0)
    errs = []
    for steps in (400, 800):
        h = 3.0 / steps
        r1, v1, _ = oracle.leapfrog_shared(r, v, m, 0.0, h, steps)
        k1, w1 = oracle.energy(r1, v1, m, 0.0)
        errs.append(abs((k1 + w1) - (k0 + w0)))
        p = (v1 * m).sum(axis=1)
        assert np.abs(p).max() < 1e-15
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_time_reversibility(oracle):
    r, v, m = plummer(64, 5)
    h, steps, eps = 1.0 / 256, 32, 1.0 / 64
    r1, v1, _ = oracle.leapfrog_shared(r, v, m, eps, h, steps)
    r2, v2, _ = oracle.leapfrog_shared(r1, -v1, m, eps, h, steps)
    assert np.abs(r2 - r).max() < 1e-12
    assert np.abs(v2 + v).max() < 1e-12
