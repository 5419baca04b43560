"""FP64 CPU oracle for the TSBTS hot path (Kaplan & Saygin, arXiv 1205.2288).

TEST INFRASTRUCTURE ONLY: this package exists to check the HIP path.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it; the product path
never calls it, and it imports nothing from the product package.

Contents
--------
* ``force``, ``energy``, ``timestep``, ``force_backward``, ``force_backward_rows``,
  ``force_backward_scale``: ctypes wrappers around the plain C double loops in
  ``oracle.c`` (definitions cited there).
* ``taylor``: the predictor of Section 2 (second-order positions, first-order
  velocities).
* ``hermite``: the cubic Hermite interpolant used as the time-symmetric interpolation of
  stored era data (Section 2, second pass onwards).
* ``leapfrog_shared``: the self-starting leapfrog of Section 2 with one shared step.
* ``tsbts``: the era / pass / block-step driver (Algorithms 1-3).
* ``adjoint``: reverse-mode gradients through a shared-step leapfrog run and through a
  run on a fixed block schedule.

Parity status of each function is recorded in its docstring; every one is pinned by the
CPU-only tests under ``tests/`` (closed forms, invariants, brute force, finite
differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        dbl = ctypes.c_double
        lib.oracle_force.argtypes = [i64, _d, _d, _d, _d, dbl, _i, i64, _d, _d, _d, _d]
        lib.oracle_energy.argtypes = [i64, _d, _d, _d, _d, _d, _d, _d, dbl, _d, _d]
        lib.oracle_timestep.argtypes = [i64, _d, _d, _d, _d, _d, _d, _d, dbl, dbl, _i, i64, _d]
        lib.oracle_force_backward.argtypes = [i64, _d, _d, _d, _d, dbl, _i, i64,
                                              _d, _d, _d, _d, _d, _d, _d, _d]
        lib.oracle_force_backward_rows.argtypes = [i64, _d, _d, _d, _d, dbl, _i, i64,
                                                   _d, _d, _d, _d, _i, i64, _d, _d]
        lib.oracle_force_backward_scale.argtypes = [i64, _d, _d, _d, _d, dbl, _i, i64,
                                                    _d, _d, _d, _d, _i, i64, _d, _d, _d, _d]
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_d)


def _pi(a):
    return a.ctypes.data_as(_i)


def _soa(a, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != 3:
        raise ValueError(f"{name} must have shape (3, N)")
    return a


def _idx(idx, n):
    if idx is None:
        return np.arange(n, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise ValueError("active index out of range")
    return idx


def threads() -> int:
    return int(_load().oracle_threads())


def force(r, m, eps, idx=None):
    """Softened acceleration [3, n_act] and potential [n_act] on the listed particles.

    Plain definition (Section 2, Algorithm 2 force step; Plummer softening of
    Section 3).  Pinned by two-body closed forms, brute force at 50 digits, Newton's
    third law and translation / mass scaling (tests/test_oracle_force.py)."""
    lib = _load()
    r = _soa(r, "r")
    n = r.shape[1]
    m = np.ascontiguousarray(m, dtype=np.float64)
    idx = _idx(idx, n)
    k = idx.size
    acc = np.zeros((3, k))
    pot = np.zeros(k)
    lib.oracle_force(n, _p(r[0]), _p(r[1]), _p(r[2]), _p(m), float(eps), _pi(idx), k,
                     _p(acc[0]), _p(acc[1]), _p(acc[2]), _p(pot))
    return acc, pot


def energy(r, v, m, eps):
    """(K, W) with the softened pair potential (Section 3 energy diagnostic).

    Pinned by the two-body closed form and the Plummer virial ratio."""
    lib = _load()
    r = _soa(r, "r")
    v = _soa(v, "v")
    m = np.ascontiguousarray(m, dtype=np.float64)
    n = r.shape[1]
    kin = ctypes.c_double()
    pot = ctypes.c_double()
    lib.oracle_energy(n, _p(r[0]), _p(r[1]), _p(r[2]), _p(v[0]), _p(v[1]), _p(v[2]),
                      _p(m), float(eps), ctypes.byref(kin), ctypes.byref(pot))
    return kin.value, pot.value


def timestep(r, v, m, eps, eta, idx=None):
    """Eq. (nbdt): eta * min over j != i of the collision and free-fall times.

    Pinned by two- and three-body closed forms (tests/test_oracle_timestep.py)."""
    lib = _load()
    r = _soa(r, "r")
    v = _soa(v, "v")
    m = np.ascontiguousarray(m, dtype=np.float64)
    n = r.shape[1]
    idx = _idx(idx, n)
    out = np.zeros(idx.size)
    lib.oracle_timestep(n, _p(r[0]), _p(r[1]), _p(r[2]), _p(v[0]), _p(v[1]), _p(v[2]),
                        _p(m), float(eps), float(eta), _pi(idx), idx.size, _p(out))
    return out


def force_backward_rows(r, m, eps, idx, g_acc, rows, g_pot=None):
    """``force_backward`` evaluated for the listed rows only: (dL/dr [3, len(rows)],
    dL/dm [len(rows)]), at O(len(rows) N) cost.  Same per-row loops as the full function
    (pinned to it element by element, tests/test_oracle_adjoint.py)."""
    lib = _load()
    r = _soa(r, "r")
    n = r.shape[1]
    m = np.ascontiguousarray(m, dtype=np.float64)
    idx = _idx(idx, n)
    rows = _idx(rows, n)
    g_acc = _soa(g_acc, "g_acc")
    if g_acc.shape[1] != idx.size:
        raise ValueError("g_acc must have shape (3, n_act)")
    gp = None
    if g_pot is not None:
        gp = np.ascontiguousarray(g_pot, dtype=np.float64)
    out_r = np.zeros((3, rows.size))
    out_m = np.zeros(rows.size)
    lib.oracle_force_backward_rows(n, _p(r[0]), _p(r[1]), _p(r[2]), _p(m), float(eps),
                                   _pi(idx), idx.size, _p(g_acc[0]), _p(g_acc[1]),
                                   _p(g_acc[2]),
                                   _p(gp) if gp is not None else ctypes.cast(None, _d),
                                   _pi(rows), rows.size, _p(out_r), _p(out_m))
    return out_r, out_m


def force_backward(r, m, eps, idx, g_acc, g_pot=None):
    """(dL/dr [3, N], dL/dm [N]) from dL/da [3, n_act] and optionally dL/dphi [n_act].

    Pinned by central finite differences of ``force`` and by the translation and
    mass-homogeneity identities (tests/test_oracle_adjoint.py)."""
    lib = _load()
    r = _soa(r, "r")
    n = r.shape[1]
    m = np.ascontiguousarray(m, dtype=np.float64)
    idx = _idx(idx, n)
    g_acc = _soa(g_acc, "g_acc")
    if g_acc.shape[1] != idx.size:
        raise ValueError("g_acc must have shape (3, n_act)")
    gp = None
    if g_pot is not None:
        gp = np.ascontiguousarray(g_pot, dtype=np.float64)
    gr = np.zeros((3, n))
    gm = np.zeros(n)
    lib.oracle_force_backward(n, _p(r[0]), _p(r[1]), _p(r[2]), _p(m), float(eps),
                              _pi(idx), idx.size, _p(g_acc[0]), _p(g_acc[1]), _p(g_acc[2]),
                              _p(gp) if gp is not None else ctypes.cast(None, _d),
                              _p(gr[0]), _p(gr[1]), _p(gr[2]), _p(gm))
    return gr, gm


def force_backward_scale(r, m, eps, idx, g_acc, g_pot=None, rows=None):
    """Rounding scale of ``force_backward``: (S_r [3, K], S_m [K]) for all N particles
    (K = N) or the listed rows, the same sums with every term replaced by its magnitude
    (definition in oracle.c).  |dL/dr| <= S_r and |dL/dm| <= S_m component by component
    (triangle inequality), with equality when one term of one sign enters; an element
    whose terms are each evaluated with relative error u is off by at most about u S.

    Pinned by those two properties (tests/test_oracle_adjoint.py)."""
    lib = _load()
    r = _soa(r, "r")
    n = r.shape[1]
    m = np.ascontiguousarray(m, dtype=np.float64)
    idx = _idx(idx, n)
    g_acc = _soa(g_acc, "g_acc")
    if g_acc.shape[1] != idx.size:
        raise ValueError("g_acc must have shape (3, n_act)")
    gp = None
    if g_pot is not None:
        gp = np.ascontiguousarray(g_pot, dtype=np.float64)
    if rows is not None:
        rows = _idx(rows, n)
    k = n if rows is None else rows.size
    sr = np.zeros((3, k))
    sm = np.zeros(k)
    lib.oracle_force_backward_scale(n, _p(r[0]), _p(r[1]), _p(r[2]), _p(m), float(eps),
                                    _pi(idx), idx.size, _p(g_acc[0]), _p(g_acc[1]),
                                    _p(g_acc[2]),
                                    _p(gp) if gp is not None else ctypes.cast(None, _d),
                                    _pi(rows) if rows is not None else ctypes.cast(None, _i),
                                    k, _p(sr[0]), _p(sr[1]), _p(sr[2]), _p(sm))
    return sr, sm


def taylor(r, v, a, h):
    """Predictor of Section 2: r + v h + a h^2 / 2 and v + a h (h broadcast per particle).

    Pinned: exact on quadratic trajectories; equals the leapfrog position update."""
    h = np.asarray(h, dtype=np.float64)
    rp = r + v * h + 0.5 * a * h * h
    vp = v + a * h
    return rp, vp


def hermite(t0, r0, v0, a0, t1, r1, v1, a1, t):
    """Cubic Hermite interpolation between two stored points (time-symmetric
    interpolation of Section 2 for passes after the first).

    Positions use (r, v) at both ends, velocities use (v, a) at both ends; with
    tau = (t - t0) / h and h = t1 - t0:
      H00 = 2 tau^3 - 3 tau^2 + 1, H10 = tau^3 - 2 tau^2 + tau,
      H01 = -2 tau^3 + 3 tau^2,    H11 = tau^3 - tau^2.
    Pinned: reproduces any cubic exactly, endpoint values, swap-ends symmetry."""
    h = np.asarray(t1, dtype=np.float64) - np.asarray(t0, dtype=np.float64)
    tau = (np.asarray(t, dtype=np.float64) - t0) / h
    tau2 = tau * tau
    tau3 = tau2 * tau
    h00 = 2.0 * tau3 - 3.0 * tau2 + 1.0
    h10 = tau3 - 2.0 * tau2 + tau
    h01 = -2.0 * tau3 + 3.0 * tau2
    h11 = tau3 - tau2
    r = h00 * r0 + h10 * h * v0 + h01 * r1 + h11 * h * v1
    v = h00 * v0 + h10 * h * a0 + h01 * v1 + h11 * h * a1
    return r, v


def leapfrog_shared(r, v, m, eps, h, nsteps, a=None):
    """Self-starting leapfrog of Section 2 with one shared step h for all particles.

    Returns (r, v, a) after nsteps.  Pinned by Kepler orbits, momentum conservation,
    second-order energy error and time reversibility (tests/test_oracle_leapfrog.py)."""
    r = np.array(r, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    if a is None:
        a, _ = force(r, m, eps)
    a = np.array(a, dtype=np.float64)
    for _ in range(nsteps):
        r = r + v * h + 0.5 * a * h * h
        a_new, _ = force(r, m, eps)
        v = v + 0.5 * (a + a_new) * h
        a = a_new
    return r, v, a
