"""Pins of the oracle's time-step criterion, Eq. (nbdt) of Section 2.

Values below are worked out by hand from the equation (collision time |r|/|v|,
free-fall time sqrt(|r|/|a|) with |a| = m_j |r| / s^(3/2))."""
import math

import numpy as np
import pytest

from workloads import plummer


def _three_body():
    # 0 at the origin at rest; 1 at (1,0,0) moving at (-2,0,0), mass 1/4;
    # 2 at (0,3,0) at rest, mass 1
    r = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 3.0], [0.0, 0.0, 0.0]])
    v = np.array([[0.0, -2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    m = np.array([0.5, 0.25, 1.0])
    return r, v, m


def test_three_body_by_hand(oracle):
    r, v, m = _three_body()
    eta = 0.1
    dt = oracle.timestep(r, v, m, 0.0, eta)
    # i=0: j=1 -> collision 1/2, free fall sqrt(1/0.25)=2 ; j=2 -> inf, sqrt(27)
    assert dt[0] == pytest.approx(eta * 0.5, rel=1e-15)
    # i=1: j=0 -> collision 1/2, free fall sqrt(1/0.5); j=2 -> |r|=sqrt10, |v|=2
    assert dt[1] == pytest.approx(eta * 0.5, rel=1e-15)
    # i=2: j=0 -> inf, sqrt(27/0.5); j=1 -> sqrt(10)/2 = 1.58, sqrt(10^1.5/0.25)
    assert dt[2] == pytest.approx(eta * math.sqrt(10.0) / 2.0, rel=1e-15)


def test_free_fall_branch_and_softening(oracle):
    # two particles at rest: only the free-fall term, softened
    r = np.array([[0.0, 0.6], [0.0, 0.8], [0.0, 0.0]])  # |d| = 1
    v = np.zeros((3, 2))
    m = np.array([1.0, 0.25])
    eps = 0.75  # s = 1.5625, s^(3/2) = 1.953125
    dt = oracle.timestep(r, v, m, eps, 1.0)
    assert dt[0] == pytest.approx(math.sqrt(1.953125 / 0.25), rel=1e-15)
    assert dt[1] == pytest.approx(math.sqrt(1.953125 / 1.0), rel=1e-15)


def test_galilean_and_translation_invariance(oracle):
    r, v, m = plummer(128, 4)
    d0 = oracle.timestep(r, v, m, 0.01, 0.1)
    d1 = oracle.timestep(r + 0.375, v - 0.25, m, 0.01, 0.1)
    assert np.allclose(d1, d0, rtol=1e-9)
    # eta scales the result exactly (power of two)
    d2 = oracle.timestep(r, v, m, 0.01, 0.2)
    assert np.array_equal(d2, 2.0 * d0)


def test_subset_and_self_exclusion(oracle):
    r, v, m = _three_body()
    dt = oracle.timestep(r, v, m, 0.0, 1.0, np.array([2], dtype=np.int32))
    assert dt.shape == (1,) and dt[0] == pytest.approx(math.sqrt(10.0) / 2.0, rel=1e-15)
