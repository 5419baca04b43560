"""ctypes binding of libtsbts.so: one Python function per C entry point, same names.

Argument marshalling only.  Device arrays are torch tensors on the HIP device (float64 or
int32, contiguous); the stream is torch's current stream unless one is given.  Every
status other than TSBTS_OK raises TsbtsError with the library's message.  There is no
fallback: if the shared library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsbts.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "tsbts.h")

TSBTS_OK = 0
TSBTS_EINVAL = -1
TSBTS_ENOMEM = -2
TSBTS_EHIP = -3
TSBTS_ESTATE = -4
TSBTS_FP64 = 0
TSBTS_MIXED = 1
TSBTS_FLAG_HILO_SEPARATION = 1
TSBTS_FLAG_NEWTON = 2


class TsbtsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "python paper_1205_2288_amd/build.py")

lib = ctypes.CDLL(LIB_PATH)

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double
_int = ctypes.c_int

_SIGS = {
    "tsbts_version": ([], _int),
    "tsbts_strerror": ([_int], ctypes.c_char_p),
    "tsbts_last_error": ([_p], ctypes.c_char_p),
    "tsbts_create": ([ctypes.POINTER(_p), _i64, _d, _int, _int], _int),
    "tsbts_destroy": ([_p], _int),
    "tsbts_tune": ([_p, _int, _int], _int),
    "tsbts_bind_state": ([_p, _p, _p, _p, _p, _p, _p], _int),
    "tsbts_predict": ([_p, _d, _int, _p], _int),
    "tsbts_load_positions": ([_p, _p, _p, _d, _p], _int),
    "tsbts_force": ([_p, _p, _i32, _d, _p, _p, _p], _int),
    "tsbts_force_noalloc": ([_p, _p, _i32, _d, _p, _p, _p], _int),
    "tsbts_force_criterion": ([_p, _p, _i32, _d, _d, _p, _p, _p, _p], _int),
    "tsbts_sched_option": ([_p, _int, _int], _int),
    "tsbts_force_backward": ([_p, _p, _i32, _d, _p, _p, _p, _p, _p], _int),
    "tsbts_correct": ([_p, _p, _i32, _d, _p, _p], _int),
    "tsbts_timestep": ([_p, _p, _i32, _d, _p, _p], _int),
    "tsbts_set_dt": ([_p, _p, _i32, _p, _p], _int),
    "tsbts_history_begin": ([_p, _p], _int),
    "tsbts_history_end": ([_p, _p], _int),
    "tsbts_history_clear": ([_p], _int),
    "tsbts_snapshot": ([_p, _d, _p, _p, _p], _int),
    "tsbts_energy": ([_p, _p, _p, _p, _p, _p], _int),
    "tsbts_leapfrog_adjoint": ([_p, _int, _d, _p, _p, _p, _p, _p], _int),
    "tsbts_block_adjoint": ([_p, _int, _p, _int, _d, _p, _p, _p, _p, _p, _p], _int),
    "tsbts_history_layout": ([_p, ctypes.POINTER(_i64), _p, _p, _p], _int),
    "tsbts_interp_adjoint": ([_p, _d, _p, _p, _i64, _p], _int),
    "tsbts_record_adjoint": ([_p, _p, _i32, _d, _p, _p, _i64, _p, _p, _p, _p], _int),
    "tsbts_adjoint_accumulate": ([_p, _p, _p, _p, _p, _p, _p, _p], _int),
    "tsbts_sched_admissible": ([_d, _d, _i64, _i64, ctypes.POINTER(_i64)], _int),
    "tsbts_sched_rule": ([_int, _i64, _i64, _d, _d, _d, _i64, _i64, ctypes.POINTER(_i64)],
                         _int),
    "tsbts_sched_era_end": ([_i64, _p, _p, _i64, _i64, _i64, ctypes.POINTER(_i64)], _int),
    "tsbts_sched_init": ([_p, _d, _int, _d, _d, _d, _p], _int),
    "tsbts_sched_era": ([_p, ctypes.POINTER(_d), _p], _int),
    "tsbts_sched_state": ([_p, _p, _p, _p, _p, ctypes.POINTER(_d)], _int),
    "tsbts_sched_prev_steps": ([_p, _p], _int),
    "tsbts_sched_timing": ([_p, _p, _p], _int),
    "tsbts_sched_restore": ([_p, _p, _p, _p, _p, _p, _d, _p], _int),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def header_symbols() -> list[str]:
    """Names of the functions declared in include/tsbts.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"\b(tsbts_[a-z_]+)\s*\(", text)))


def _check(ctx, status: int):
    if status != TSBTS_OK:
        msg = lib.tsbts_last_error(ctx).decode() if ctx else ""
        if not msg:
            msg = lib.tsbts_strerror(status).decode()
        raise TsbtsError(status, msg)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, shape=None, name="array"):
    """Device pointer of a contiguous tensor (None -> NULL), with light validation."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, shape=None, name="array"):
    return _ptr(t, torch.float64, shape, name)


def _i32p(t, name="active_idx"):
    return _ptr(t, torch.int32, None, name)


# ------------------------------------------------------------------ entry points

def tsbts_version() -> int:
    return lib.tsbts_version()


def tsbts_strerror(status: int) -> str:
    return lib.tsbts_strerror(status).decode()


def tsbts_last_error(ctx) -> str:
    return lib.tsbts_last_error(ctx).decode()


def tsbts_create(n: int, eps: float, precision: int, flags: int = 0):
    out = ctypes.c_void_p()
    st = lib.tsbts_create(ctypes.byref(out), int(n), float(eps), int(precision), int(flags))
    if st != TSBTS_OK:
        raise TsbtsError(st, f"tsbts_create: {tsbts_strerror(st)}")
    return out


def tsbts_destroy(ctx):
    _check(None, lib.tsbts_destroy(ctx))


TSBTS_TUNE_BLOCKS = 1
TSBTS_TUNE_IPL = 2
TSBTS_TUNE_CHUNK = 3
TSBTS_TUNE_SYMMETRIC = 4
TSBTS_TUNE_CHECK_INDICES = 5
TSBTS_TUNE_SPLIT = 6
TSBTS_SCHED_CRITERION_BEFORE_CORRECTOR = 1
TSBTS_SCHED_PREDICT_ON_LOAD = 2
TSBTS_SCHED_RULE_THREADS = 3


def tsbts_tune(ctx, param: int, value: int):
    _check(ctx, lib.tsbts_tune(ctx, int(param), int(value)))


def tsbts_bind_state(ctx, n, r, v, a, m, t_last, dt):
    _check(ctx, lib.tsbts_bind_state(ctx, _f64(r, (3, n), "r"), _f64(v, (3, n), "v"),
                                     _f64(a, (3, n), "a"), _f64(m, (n,), "m"),
                                     _f64(t_last, (n,), "t_last"), _f64(dt, (n,), "dt")))


def tsbts_predict(ctx, t_block, use_history=False, stream=None):
    _check(ctx, lib.tsbts_predict(ctx, float(t_block), int(bool(use_history)), _stream(stream)))


def tsbts_load_positions(ctx, n, r, m, t_label=0.0, stream=None):
    _check(ctx, lib.tsbts_load_positions(ctx, _f64(r, (3, n), "r"), _f64(m, (n,), "m"),
                                         float(t_label), _stream(stream)))


def tsbts_force_criterion(ctx, active_idx, t_block, eta, acc, pot, dtc, stream=None):
    k = active_idx.numel()
    _check(ctx, lib.tsbts_force_criterion(ctx, _i32p(active_idx), k, float(t_block),
                                          float(eta), _f64(acc, (3, k), "acc"),
                                          _f64(pot, (k,), "pot"), _f64(dtc, (k,), "dtc"),
                                          _stream(stream)))


def tsbts_force(ctx, active_idx, t_block, acc, pot=None, stream=None):
    k = active_idx.numel()
    _check(ctx, lib.tsbts_force(ctx, _i32p(active_idx), k, float(t_block),
                                _f64(acc, (3, k), "acc"), _f64(pot, (k,), "pot"),
                                _stream(stream)))


TSBTS_NOALLOC_PARTIALS = 1 << 23


def tsbts_force_noalloc(ctx, active_idx, t_block, acc, pot=None, stream=None):
    k = active_idx.numel()
    _check(ctx, lib.tsbts_force_noalloc(ctx, _i32p(active_idx), k, float(t_block),
                                        _f64(acc, (3, k), "acc"), _f64(pot, (k,), "pot"),
                                        _stream(stream)))


def tsbts_force_backward(ctx, n, active_idx, t_block, grad_acc, grad_pot, grad_r, grad_m,
                         stream=None):
    k = active_idx.numel()
    _check(ctx, lib.tsbts_force_backward(
        ctx, _i32p(active_idx), k, float(t_block), _f64(grad_acc, (3, k), "grad_acc"),
        _f64(grad_pot, (k,), "grad_pot"), _f64(grad_r, (3, n), "grad_r"),
        _f64(grad_m, (n,), "grad_m"), _stream(stream)))


def tsbts_correct(ctx, active_idx, t_block, acc_new, stream=None):
    k = active_idx.numel()
    _check(ctx, lib.tsbts_correct(ctx, _i32p(active_idx), k, float(t_block),
                                  _f64(acc_new, (3, k), "acc_new"), _stream(stream)))


def tsbts_timestep(ctx, active_idx, eta, dtc, stream=None):
    k = active_idx.numel()
    _check(ctx, lib.tsbts_timestep(ctx, _i32p(active_idx), k, float(eta),
                                   _f64(dtc, (k,), "dtc"), _stream(stream)))


def tsbts_set_dt(ctx, active_idx, dt_new, stream=None):
    k = active_idx.numel()
    _check(ctx, lib.tsbts_set_dt(ctx, _i32p(active_idx), k, _f64(dt_new, (k,), "dt_new"),
                                 _stream(stream)))


def tsbts_history_begin(ctx, stream=None):
    _check(ctx, lib.tsbts_history_begin(ctx, _stream(stream)))


def tsbts_history_end(ctx, stream=None):
    _check(ctx, lib.tsbts_history_end(ctx, _stream(stream)))


def tsbts_history_clear(ctx):
    _check(ctx, lib.tsbts_history_clear(ctx))


def tsbts_snapshot(ctx, n, T, r_out, v_out, stream=None):
    _check(ctx, lib.tsbts_snapshot(ctx, float(T), _f64(r_out, (3, n), "r_out"),
                                   _f64(v_out, (3, n), "v_out"), _stream(stream)))


def tsbts_energy(ctx, n, r, v, m, out_kw, stream=None):
    _check(ctx, lib.tsbts_energy(ctx, _f64(r, (3, n), "r"), _f64(v, (3, n), "v"),
                                 _f64(m, (n,), "m"), _f64(out_kw, (2,), "out_KW"),
                                 _stream(stream)))


def tsbts_leapfrog_adjoint(ctx, n, phase, h, rbar, vbar, abar, g_out, stream=None):
    _check(ctx, lib.tsbts_leapfrog_adjoint(
        ctx, int(phase), float(h), _f64(rbar, (3, n), "rbar"), _f64(vbar, (3, n), "vbar"),
        _f64(abar, (3, n), "abar"), _f64(g_out, (3, n), "g_out"), _stream(stream)))


def tsbts_block_adjoint(ctx, n, phase, active_idx, t_block, rbar, vbar, abar, pbar, seeds,
                        stream=None):
    k = 0 if active_idx is None else active_idx.numel()
    _check(ctx, lib.tsbts_block_adjoint(
        ctx, int(phase), _i32p(active_idx), k, float(t_block), _f64(rbar, (3, n), "rbar"),
        _f64(vbar, (3, n), "vbar"), _f64(abar, (3, n), "abar"), _f64(pbar, (3, n), "pbar"),
        _f64(seeds, None if seeds is None else (3, k), "seeds"), _stream(stream)))


def tsbts_history_layout(ctx, n, off=None, t=None, stream=None) -> int:
    """Number of records of the finished history; copies its offsets / times when given
    (off int32 [n+1], t float64 [n_records])."""
    count = ctypes.c_int64()
    _check(ctx, lib.tsbts_history_layout(ctx, ctypes.byref(count), None, None, None))
    n_rec = count.value
    if off is not None or t is not None:
        _check(ctx, lib.tsbts_history_layout(
            ctx, ctypes.byref(count), _ptr(off, torch.int32, (n + 1,), "off"),
            _f64(t, (n_rec,), "t"), _stream(stream)))
    return n_rec


def tsbts_interp_adjoint(ctx, n, n_records, t_block, pbar, hbar, stream=None):
    _check(ctx, lib.tsbts_interp_adjoint(ctx, float(t_block), _f64(pbar, (3, n), "pbar"),
                                         _f64(hbar, (6, n_records), "hbar"), int(n_records),
                                         _stream(stream)))


def tsbts_record_adjoint(ctx, n, active_idx, t_block, off, t, hbar, rbar, vbar,
                         stream=None):
    n_rec = t.numel()
    _check(ctx, lib.tsbts_record_adjoint(
        ctx, _i32p(active_idx), active_idx.numel(), float(t_block),
        _ptr(off, torch.int32, (n + 1,), "off"), _f64(t, (n_rec,), "t"), n_rec,
        _f64(hbar, (6, n_rec), "hbar"), _f64(rbar, (3, n), "rbar"),
        _f64(vbar, (3, n), "vbar"), _stream(stream)))


def tsbts_adjoint_accumulate(ctx, n, rbar, vbar, abar, rbar_acc, vbar_acc, abar_acc,
                             stream=None):
    _check(ctx, lib.tsbts_adjoint_accumulate(
        ctx, _f64(rbar, (3, n), "rbar"), _f64(vbar, (3, n), "vbar"),
        _f64(abar, (3, n), "abar"), _f64(rbar_acc, (3, n), "rbar_acc"),
        _f64(vbar_acc, (3, n), "vbar_acc"), _f64(abar_acc, (3, n), "abar_acc"),
        _stream(stream)))


# ------------------------------------------------------------------ native scheduler

def tsbts_sched_admissible(begin: float, end: float, dt_min: int, dt_max: int) -> int:
    out = ctypes.c_int64()
    _check(None, lib.tsbts_sched_admissible(float(begin), float(end), int(dt_min),
                                            int(dt_max), ctypes.byref(out)))
    return out.value


def tsbts_sched_rule(first_pass: bool, dt: int, t_block: int, begin: float, end_dt: float,
                     end_2dt: float, dt_min: int, dt_max: int) -> int:
    out = ctypes.c_int64()
    _check(None, lib.tsbts_sched_rule(int(bool(first_pass)), int(dt), int(t_block),
                                      float(begin), float(end_dt), float(end_2dt),
                                      int(dt_min), int(dt_max), ctypes.byref(out)))
    return out.value


def tsbts_sched_era_end(t0: int, t, dt, dt_max: int, era: int = 0) -> int:
    """End of the era starting at t0 (all in ticks; t, dt host int64 arrays)."""
    import numpy as np
    t = np.ascontiguousarray(t, dtype=np.int64)
    dt = np.ascontiguousarray(dt, dtype=np.int64)
    if t.shape != dt.shape or t.ndim != 1:
        raise ValueError("t and dt must be 1-d arrays of one length")
    out = ctypes.c_int64()
    _check(None, lib.tsbts_sched_era_end(int(t0), ctypes.c_void_p(t.ctypes.data),
                                         ctypes.c_void_p(dt.ctypes.data), t.size, int(dt_max),
                                         int(era), ctypes.byref(out)))
    return out.value


def tsbts_sched_option(ctx, option, value):
    _check(ctx, lib.tsbts_sched_option(ctx, int(option), int(value)))


def tsbts_sched_init(ctx, eta, passes, dt_min, dt_max, era, stream=None):
    _check(ctx, lib.tsbts_sched_init(ctx, float(eta), int(passes), float(dt_min),
                                     float(dt_max), float(era), _stream(stream)))


def tsbts_sched_era(ctx, stream=None) -> float:
    end = ctypes.c_double()
    _check(ctx, lib.tsbts_sched_era(ctx, ctypes.byref(end), _stream(stream)))
    return end.value


def tsbts_sched_state(ctx, n):
    """Host copies: (t_ticks int64[n], dt_ticks int64[n], dtc float64[n], stats int64[4],
    time)."""
    import numpy as np
    t = np.empty(n, dtype=np.int64)
    dt = np.empty(n, dtype=np.int64)
    dtc = np.empty(n, dtype=np.float64)
    stats = np.empty(4, dtype=np.int64)
    time = ctypes.c_double()
    _check(ctx, lib.tsbts_sched_state(ctx, ctypes.c_void_p(t.ctypes.data),
                                      ctypes.c_void_p(dt.ctypes.data),
                                      ctypes.c_void_p(dtc.ctypes.data),
                                      ctypes.c_void_p(stats.ctypes.data), ctypes.byref(time)))
    return t, dt, dtc, stats, time.value


def tsbts_sched_timing(ctx):
    """Wall-clock breakdown of the block steps: (seconds float64[4, 4] by active-set class
    (k <= 32, <= 256, <= 1024, larger) and phase (issue, wait, rule, whole step), counts
    int64[4, 2] (block steps, summed active-set sizes))."""
    import numpy as np
    sec = np.empty((4, 4), dtype=np.float64)
    cnt = np.empty((4, 2), dtype=np.int64)
    _check(ctx, lib.tsbts_sched_timing(ctx, ctypes.c_void_p(sec.ctypes.data),
                                       ctypes.c_void_p(cnt.ctypes.data)))
    return sec, cnt


def tsbts_sched_prev_steps(ctx, n):
    """Host copy of each particle's previous step (ticks, int64[n])."""
    import numpy as np
    dtp = np.empty(n, dtype=np.int64)
    _check(ctx, lib.tsbts_sched_prev_steps(ctx, ctypes.c_void_p(dtp.ctypes.data)))
    return dtp


def tsbts_sched_restore(ctx, n, t, dt, dtp, dtc, stats, time, stream=None):
    """Resume the scheduler from an era-end checkpoint (host arrays of n particles, ticks;
    time in time units); the bound r, v, a must already hold the checkpoint's values."""
    import numpy as np
    arrs = [np.ascontiguousarray(x, dtype=dt_) for x, dt_ in
            ((t, np.int64), (dt, np.int64), (dtp, np.int64), (dtc, np.float64))]
    if any(a.shape != (n,) for a in arrs):
        raise ValueError(f"checkpoint arrays must have shape ({n},)")
    st = None if stats is None else np.ascontiguousarray(stats, dtype=np.int64)
    if st is not None and st.size != 4:
        raise ValueError("stats must have 4 entries")
    _check(ctx, lib.tsbts_sched_restore(
        ctx, *(ctypes.c_void_p(a.ctypes.data) for a in arrs),
        None if st is None else ctypes.c_void_p(st.ctypes.data), float(time),
        _stream(stream)))
