"""Pins of the oracle's O(N^2) energy (Section 3 energy-error diagnostic)."""
import math

import mpmath
import numpy as np
import pytest

from workloads import plummer


def test_two_body_closed_form(oracle):
    r = np.array([[0.0, 3.0], [0.0, 4.0], [0.0, 0.0]])
    v = np.array([[1.0, 0.0], [0.0, -2.0], [0.0, 0.5]])
    m = np.array([0.5, 0.25])
    k, w = oracle.energy(r, v, m, 0.0)
    assert k == pytest.approx(0.5 * 0.5 * 1.0 + 0.5 * 0.25 * 4.25, rel=1e-15)
    assert w == pytest.approx(-0.5 * 0.25 / 5.0, rel=1e-15)
    # softened: |d| = 5, eps = 12 -> sqrt(169) = 13
    _, w2 = oracle.energy(r, v, m, 12.0)
    assert w2 == pytest.approx(-0.125 / 13.0, rel=1e-15)


def test_brute_force_50_digits(oracle):
    r, v, m = plummer(11, 3, masses="loguniform")
    eps = 1.0 / 32
    k, w = oracle.energy(r, v, m, eps)
    mpmath.mp.dps = 50
    kk = sum(mpmath.mpf(m[i]) * sum(mpmath.mpf(v[c, i]) ** 2 for c in range(3)) / 2
             for i in range(11))
    ww = mpmath.mpf(0)
    for i in range(11):
        for j in range(i + 1, 11):
            s = sum((mpmath.mpf(r[c, i]) - mpmath.mpf(r[c, j])) ** 2 for c in range(3))
            ww -= mpmath.mpf(m[i]) * mpmath.mpf(m[j]) / mpmath.sqrt(s + mpmath.mpf(eps) ** 2)
    assert k == pytest.approx(float(kk), rel=1e-15)
    assert w == pytest.approx(float(ww), rel=1e-14)


def test_plummer_virial_and_units(oracle):
    # Henon units: E = -1/4, virial ratio 2K/|W| = 1 (sampling noise ~ 1/sqrt(N))
    n = 4096
    r, v, m = plummer(n, 99)
    k, w = oracle.energy(r, v, m, 0.0)
    tol = 4.0 / math.sqrt(n)
    assert abs(2 * k / abs(w) - 1.0) < tol
    assert abs((k + w) + 0.25) < 0.25 * tol
    # potential consistency: W = 1/2 sum m_i phi_i (unsoftened)
    _, pot = oracle.force(r, m, 0.0)
    assert w == pytest.approx(0.5 * (m * pot).sum(), rel=1e-12)
