"""Helpers shared by the GPU tests (error metrics, context construction)."""
import numpy as np


def rel_err_vec(got, ref):
    """Per-particle |got - ref| / |ref| for [3, k] arrays."""
    num = np.sqrt(((got - ref) ** 2).sum(axis=0))
    den = np.sqrt((ref ** 2).sum(axis=0))
    return num / np.maximum(den, np.finfo(float).tiny)


def rel_err(got, ref):
    return np.abs(got - ref) / np.maximum(np.abs(ref), np.finfo(float).tiny)


def summary(e):
    e = np.asarray(e)
    return {"median": float(np.median(e)), "p90": float(np.quantile(e, 0.9)),
            "p99": float(np.quantile(e, 0.99)), "max": float(e.max())}


def make_ctx(n, eps, precision="mixed", separation="f64", newton=False):
    from paper_1205_2288_amd import Context
    return Context(n, eps, precision=precision, separation=separation, newton=newton)


VARIANTS = [
    ("fp64", "hilo", True),
    ("mixed", "hilo", True),
    ("mixed", "hilo", False),
    ("mixed", "f64", True),
    ("mixed", "f64", False),
]

# bars: float64 and mixed precision (median relative error per particle)
TOL = {
    "fp64": {"median": 1e-13, "max": 1e-9},
    "mixed": {"median": 1e-6, "max": 1e-5},
}

# Force adjoint against the oracle: the median over particles of the per-particle relative
# error (vector norm for dL/dr_k), and every element's error in units of its rounding
# scale S (the oracle's sum of the magnitudes of the terms that enter the element).  An
# implementation whose terms each carry a relative error u is off by at most about u S:
# u ~ 1e-16 with float64 pair arithmetic, a few float32 units (6e-8) in mixed precision.
# Measured worst cases over the suite: float64 median 2e-15, 1.4e-14 units; mixed median
# 3.7e-7, 1.4e-6 units.
ADJ_TOL = {
    "fp64": {"median": 1e-12, "unit": 1e-12},
    "mixed": {"median": 1e-5, "unit": 1e-5},
}

# Gradients through whole runs against the oracle's reverse mode: median per-particle
# relative error, and every particle's error in units of the root-mean-square particle
# magnitude of the reference gradient.
# Measured worst cases: float64 median 4.4e-15, 1.3e-13 rms units; mixed median 7.6e-7,
# 1.0e-5 rms units (mass gradients through 16 block steps).
RUN_GRAD_TOL = {
    "fp64": {"median": 1e-12, "rms_units": 1e-11},
    "mixed": {"median": 1e-5, "rms_units": 1e-4},
}

# Directional derivatives of run gradients against central finite differences of the
# float64 forward (step 1e-6): the error of each direction relative to the root-mean-
# square finite difference of its input group (r, v or m) over the directions drawn, at
# most 1e-5; float64 gradients also per direction relative to that direction's own finite
# difference.  A random direction can make g.d cancel to a small fraction of its typical
# size, where the mixed-precision gradient's error (relative to |g||d|) shows up enlarged.
FD_TOL = 1e-5


def _per_particle(x):
    x = np.asarray(x)
    return np.sqrt((x ** 2).sum(axis=0)) if x.ndim == 2 else np.abs(x)


def check_adjoint(got_r, got_m, ref_r, ref_m, scale_r, scale_m, prec, label=""):
    """Element-wise check of a force adjoint (dL/dr [3, K], dL/dm [K]) against the oracle's
    and its rounding scale (oracle.force_backward_scale); returns the statistics."""
    tol = ADJ_TOL[prec]
    tiny = np.finfo(float).tiny
    stats = {}
    for name, got, ref, sc in (("r", got_r, ref_r, scale_r), ("m", got_m, ref_m, scale_m)):
        got, ref, sc = np.asarray(got), np.asarray(ref), np.asarray(sc)
        e = _per_particle(got - ref) / np.maximum(_per_particle(ref), tiny)
        diff = np.abs(got - ref)
        # an element with no terms (massless source, no target) must be exactly zero
        assert (diff[sc == 0] == 0).all(), f"{label} dL/d{name}: nonzero element with no terms"
        u = diff[sc > 0] / sc[sc > 0]
        stats[name] = {"median_rel": float(np.median(e)), "max_rel": float(e.max()),
                       "max_units": float(u.max()) if u.size else 0.0}
    print(f"adjoint {label} {prec}: {stats}")
    for name in ("r", "m"):
        assert stats[name]["median_rel"] <= tol["median"], (label, name, stats)
        assert stats[name]["max_units"] <= tol["unit"], (label, name, stats)
    return stats


def check_run_gradient(got, ref, prec, label=""):
    """Per-particle check of a gradient through a run ([3, n] or [n]) against the oracle's
    reverse-mode gradient; returns the statistics."""
    tol = RUN_GRAD_TOL[prec]
    pe = _per_particle(np.asarray(got) - np.asarray(ref))
    pr = _per_particle(ref)
    rel = pe / np.maximum(pr, np.finfo(float).tiny)
    units = pe / np.sqrt((pr ** 2).mean())
    stats = {"median_rel": float(np.median(rel)), "max_rel": float(rel.max()),
             "max_rms_units": float(units.max())}
    print(f"gradient {label} {prec}: {stats}")
    assert stats["median_rel"] <= tol["median"], (label, stats)
    assert stats["max_rms_units"] <= tol["rms_units"], (label, stats)
    return stats


def check_fd(rows, prec, label=""):
    """rows: (group, adjoint directional derivative, finite difference) per direction."""
    rows = [(w, float(g), float(f)) for w, g, f in rows]
    worst_rms = worst_own = 0.0
    for w in sorted({x[0] for x in rows}):
        sel = [x for x in rows if x[0] == w]
        rms = np.sqrt(np.mean([f * f for _, _, f in sel]))
        for _, g, f in sel:
            worst_rms = max(worst_rms, abs(g - f) / rms)
            worst_own = max(worst_own, abs(g - f) / abs(f))
    print(f"finite differences {label} {prec}: {len(rows)} directions, worst error "
          f"{worst_rms:.2e} of the group rms, {worst_own:.2e} of its own value")
    assert worst_rms <= FD_TOL, (label, worst_rms)
    if prec == "fp64":
        assert worst_own <= FD_TOL, (label, worst_own)
    return worst_rms, worst_own
