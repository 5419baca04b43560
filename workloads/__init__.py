"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out; it performs none of the
integrator's arithmetic (no forces, no prediction, no scheduling), so both the
independent CPU oracle and the HIP path may take their inputs from here.

Initial conditions follow the paper's test problems (Section 3 and Section 6): Plummer
spheres in standard N-body (Henon) units, G = 1, total mass M = 1, total energy close
to -1/4.  Positions and speeds are drawn with the Aarseth-Henon-Wielen recipe:

* radius from the cumulative mass fraction X:  r = (X^(-2/3) - 1)^(-1/2), redrawn
  when r >= 10 (Plummer scale length a = 1);
* isotropic direction for the position;
* speed q * v_esc(r) with v_esc = sqrt(2) (1 + r^2)^(-1/4) and q drawn by von Neumann
  rejection from g(q) = q^2 (1 - q^2)^(7/2) with envelope 0.1;
* isotropic direction for the velocity;
* scaling r *= 3 pi / 16 and v *= sqrt(16 / (3 pi)) to reach E = -1/4;
* the centre of mass position and velocity are removed.

Masses are 1/N each, or, for the log-uniform variant, 10**U[0,1) normalised to sum 1
(assigned independently of the phase-space draw).

All draws come from numpy's Generator(PCG64(seed)).  Arrays are float64 structure of
arrays: r and v have shape (3, N).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "plummer",
    "active_subset",
    "Config",
    "CONFIGS",
    "config",
    "TICK",
    "SEED_BASE",
]

# Block times are handled in integer ticks of 2^-20 (the smallest block level used by
# the workloads below).
TICK = 2.0 ** -20
SEED_BASE = 12052288


def _isotropic(rng: np.random.Generator, mag: np.ndarray) -> np.ndarray:
    n = mag.shape[0]
    u = rng.random(n)
    w = rng.random(n)
    z = (1.0 - 2.0 * u) * mag
    rxy = np.sqrt(np.maximum(mag * mag - z * z, 0.0))
    phi = 2.0 * math.pi * w
    return np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z])


def plummer(n: int, seed: int, masses: str = "equal", rmax: float = 10.0):
    """Return (r[3,N], v[3,N], m[N]) float64 arrays of a seeded Plummer sphere.

    masses: "equal" (1/N each) or "loguniform" (10**U[0,1), normalised to total 1).
    """
    if n <= 0:
        raise ValueError("n must be positive")
    rng = np.random.Generator(np.random.PCG64(seed))
    # radii: redraw every rejected entry until all are below rmax
    rad = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x = rng.random(todo.size)
        with np.errstate(divide="ignore", invalid="ignore"):
            rr = 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
        ok = np.isfinite(rr) & (rr < rmax) & (x > 0.0)
        rad[todo[ok]] = rr[ok]
        todo = todo[~ok]
    pos = _isotropic(rng, rad)
    # speed fraction q by rejection from q^2 (1-q^2)^3.5 under the envelope 0.1
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x4 = rng.random(todo.size)
        x5 = rng.random(todo.size)
        ok = 0.1 * x5 < x4 * x4 * (1.0 - x4 * x4) ** 3.5
        q[todo[ok]] = x4[ok]
        todo = todo[~ok]
    vesc = math.sqrt(2.0) * (1.0 + rad * rad) ** -0.25
    vel = _isotropic(rng, q * vesc)
    pos *= 3.0 * math.pi / 16.0
    vel *= math.sqrt(16.0 / (3.0 * math.pi))
    if masses == "equal":
        m = np.full(n, 1.0 / n)
    elif masses == "loguniform":
        m = 10.0 ** rng.random(n)
        m /= m.sum()
    else:
        raise ValueError(f"unknown mass spectrum {masses!r}")
    mtot = m.sum()
    pos -= (pos * m).sum(axis=1, keepdims=True) / mtot
    vel -= (vel * m).sum(axis=1, keepdims=True) / mtot
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), m


def active_subset(n: int, n_active: int, seed: int) -> np.ndarray:
    """Sorted int32 indices of a random subset of size n_active (without replacement)."""
    if not 0 <= n_active <= n:
        raise ValueError("n_active out of range")
    rng = np.random.Generator(np.random.PCG64(seed))
    if n_active == n:
        return np.arange(n, dtype=np.int32)
    idx = rng.choice(n, size=n_active, replace=False)
    return np.sort(idx).astype(np.int32)


def gaussian(shape, seed: int) -> np.ndarray:
    """Standard normal float64 array (seeded), e.g. for adjoint seeds or perturbations."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape)


def uniform_levels(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Integers drawn uniformly from lo..hi inclusive (e.g. block levels)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=n)


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload: particle count, softening, mass spectrum and integration setup."""

    name: str
    n: int
    eps: float
    masses: str = "equal"
    seed: int = SEED_BASE
    eta: float = 0.1
    passes: int = 3
    dt_max: float = 1.0 / 64.0
    dt_min: float = 2.0 ** -20
    era: float | None = None  # None: dynamic era size
    t_end: float = 1.0
    note: str = ""

    def ic(self):
        return plummer(self.n, self.seed, self.masses)


CONFIGS = {
    # fixed-era TSBTS integration of a small Plummer sphere
    "plummer256": Config("plummer256", 256, 1.0 / 64.0, seed=SEED_BASE + 1,
                         era=1.0 / 8.0, t_end=1.0,
                         note="N=256, eps=1/64, fixed era 1/8, dt_max=1/64, t=0..1"),
    # dynamic-era integration; force in FP64 and in mixed precision
    "plummer4096": Config("plummer4096", 4096, 1.0 / 256.0, seed=SEED_BASE + 2,
                          era=None, t_end=10.0, dt_max=2.0 ** -6, dt_min=2.0 ** -20,
                          note="N=4096, eps=1/256, dynamic era, levels 2^-6..2^-20, t=0..10"),
    # force sweep over active-set sizes
    "sweep32768": Config("sweep32768", 32768, 1.0 / 1024.0, seed=SEED_BASE + 3,
                         note="N=32768, eps=1/1024, n_act = 1, 8, ..., 32768"),
    # adjoint through a shared-step leapfrog
    "adjoint8192": Config("adjoint8192", 8192, 1.0 / 256.0, seed=SEED_BASE + 4,
                          note="N=8192, eps=1/256, 64 shared steps dt=1/256, 16-step eras"),
    # large log-uniform-mass sphere: force, adjoint, energy throughput
    "plummer131k": Config("plummer131k", 131072, 1.0 / 4096.0, masses="loguniform",
                          seed=SEED_BASE + 5,
                          note="N=131072, eps=1/4096, log-uniform masses"),
}


def config(name: str) -> Config:
    return CONFIGS[name]
