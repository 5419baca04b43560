"""Pins of the oracle's force and potential (Section 2 force step, Section 3 softening).

Checks against closed forms, a 50-digit brute force, Newton's third law and the exact
symmetries of the definition; none of them re-uses the oracle's own loops."""
import math

import mpmath
import numpy as np
import pytest

from workloads import plummer, active_subset


def test_two_body_closed_form(oracle):
    # particle 1 sits at (3, 4, 0) relative to particle 0: |d| = 5
    r = np.array([[1.0, 4.0], [-2.0, 2.0], [0.5, 0.5]])
    m = np.array([0.75, 0.25])
    acc, pot = oracle.force(r, m, 0.0)
    # a_0 = m_1 d / |d|^3 = 0.25 (3, 4, 0) / 125 ; phi_0 = -0.25 / 5
    assert np.allclose(acc[:, 0], [0.25 * 3 / 125, 0.25 * 4 / 125, 0.0], rtol=1e-15, atol=0)
    assert np.allclose(acc[:, 1], [-0.75 * 3 / 125, -0.75 * 4 / 125, 0.0], rtol=1e-15, atol=0)
    assert pot[0] == pytest.approx(-0.05, rel=1e-15)
    assert pot[1] == pytest.approx(-0.15, rel=1e-15)


def test_two_body_softened(oracle):
    # |d| = 1, eps = 0.75  ->  s = 1.5625 = 1.25^2, s^(3/2) = 1.953125
    r = np.array([[0.0, 0.0], [0.0, 0.0], [0.0, 1.0]])
    m = np.array([0.5, 2.0])
    acc, pot = oracle.force(r, m, 0.75)
    assert acc[2, 0] == pytest.approx(2.0 / 1.953125, rel=1e-15)
    assert acc[2, 1] == pytest.approx(-0.5 / 1.953125, rel=1e-15)
    assert pot[0] == pytest.approx(-2.0 / 1.25, rel=1e-15)
    assert pot[1] == pytest.approx(-0.5 / 1.25, rel=1e-15)


def _brute_50(r, m, eps, i):
    mpmath.mp.dps = 50
    n = r.shape[1]
    ax = ay = az = ph = mpmath.mpf(0)
    e2 = mpmath.mpf(eps) ** 2
    for j in range(n):
        if j == i:
            continue
        dx = mpmath.mpf(r[0, j]) - mpmath.mpf(r[0, i])
        dy = mpmath.mpf(r[1, j]) - mpmath.mpf(r[1, i])
        dz = mpmath.mpf(r[2, j]) - mpmath.mpf(r[2, i])
        s = dx * dx + dy * dy + dz * dz + e2
        w = mpmath.mpf(m[j]) / mpmath.sqrt(s)
        ax += w * dx / s
        ay += w * dy / s
        az += w * dz / s
        ph -= w
    return np.array([float(ax), float(ay), float(az)]), float(ph)


@pytest.mark.parametrize("eps", [0.0, 1.0 / 64])
def test_brute_force_50_digits(oracle, eps):
    r, _, m = plummer(13, 7, masses="loguniform")
    acc, pot = oracle.force(r, m, eps)
    for i in range(13):
        a_ref, p_ref = _brute_50(r, m, eps, i)
        scale = np.abs(a_ref).max()
        assert np.abs(acc[:, i] - a_ref).max() <= 1e-14 * scale
        assert abs(pot[i] - p_ref) <= 1e-14 * abs(p_ref)


def test_newton_third_law(oracle):
    r, _, m = plummer(512, 11, masses="loguniform")
    acc, _ = oracle.force(r, m, 1.0 / 256)
    tot = (acc * m).sum(axis=1)
    scale = (np.abs(acc) * m).sum()
    assert np.abs(tot).max() <= 1e-14 * scale


def test_translation_and_mass_scaling(oracle):
    r, _, m = plummer(200, 12)
    a0, p0 = oracle.force(r, m, 0.01)
    a1, p1 = oracle.force(r + np.array([[0.5], [-0.25], [0.125]]), m, 0.01)
    assert np.allclose(a1, a0, rtol=1e-9, atol=1e-12 * np.abs(a0).max())
    assert np.allclose(p1, p0, rtol=1e-12)
    a2, p2 = oracle.force(r, 4.0 * m, 0.01)  # powers of two scale exactly
    assert np.array_equal(a2, 4.0 * a0)
    assert np.array_equal(p2, 4.0 * p0)


def test_active_subset_rows(oracle):
    r, _, m = plummer(300, 13)
    full_a, full_p = oracle.force(r, m, 0.02)
    idx = active_subset(300, 37, 5)
    a, p = oracle.force(r, m, 0.02, idx)
    assert np.array_equal(a, full_a[:, idx])
    assert np.array_equal(p, full_p[idx])


def test_symmetric_shell_cancels(oracle):
    # a particle at the centre of a regular octahedron of equal masses feels no force
    pts = [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
    r = np.array(pts, dtype=float).T
    m = np.full(7, 1.0 / 7)
    acc, pot = oracle.force(r, m, 0.1)
    assert np.abs(acc[:, 0]).max() == 0.0
    assert pot[0] == pytest.approx(-6.0 / 7.0 / math.sqrt(1.01), rel=1e-15)
