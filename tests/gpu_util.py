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
    "mixed": {"median": 1e-6, "max": 1e-3},
}
