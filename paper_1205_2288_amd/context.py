"""Context: a libtsbts context plus the device tensors of one particle state.

Thin convenience layer over the C ABI (paper_1205_2288_amd._lib): it allocates the
caller-owned state tensors (float64 structure of arrays on the HIP device), binds them,
and wraps the entry points so that callers pass index tensors and get result tensors.
All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L

PRECISIONS = {"fp64": L.TSBTS_FP64, "mixed": L.TSBTS_MIXED}


def _dev(x, dtype=torch.float64, device="cuda"):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


class Context:
    """Device-resident particle state and a libtsbts context.

    precision: "mixed" (float32 pair arithmetic, float64 sums) or "fp64".
    separation: "f64" (float64 separation rounded to float32, the default) or "hilo"
    (float32 hi/lo position pairs); newton: refine the float32 1/sqrt by one Newton step
    (mixed precision only; off by default).
    """

    def __init__(self, n: int, eps: float, precision: str = "mixed", separation: str = "f64",
                 newton: bool = False, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("libtsbts needs a HIP device")
        self.n = int(n)
        self.eps = float(eps)
        self.precision = precision
        self.device = torch.device(device)
        flags = 0
        if separation == "hilo":
            flags |= L.TSBTS_FLAG_HILO_SEPARATION
        elif separation != "f64":
            raise ValueError("separation must be 'hilo' or 'f64'")
        if newton:
            flags |= L.TSBTS_FLAG_NEWTON
        self.flags = flags
        self.ctx = L.tsbts_create(self.n, self.eps, PRECISIONS[precision], flags)
        self.r = self.v = self.a = self.m = self.t_last = self.dt = None

    # ---------------------------------------------------------------- state
    def bind(self, r, v, m, a=None, t_last=None, dt=None):
        n = self.n
        self.r = _dev(r, device=self.device).reshape(3, n).contiguous()
        self.v = _dev(v, device=self.device).reshape(3, n).contiguous()
        self.m = _dev(m, device=self.device).reshape(n).contiguous()
        self.a = (torch.zeros((3, n), dtype=torch.float64, device=self.device) if a is None
                  else _dev(a, device=self.device).reshape(3, n).contiguous())
        self.t_last = (torch.zeros(n, dtype=torch.float64, device=self.device) if t_last is None
                       else _dev(t_last, device=self.device).reshape(n).contiguous())
        self.dt = (torch.zeros(n, dtype=torch.float64, device=self.device) if dt is None
                   else _dev(dt, device=self.device).reshape(n).contiguous())
        L.tsbts_bind_state(self.ctx, n, self.r, self.v, self.a, self.m, self.t_last, self.dt)
        return self

    def tune(self, blocks=None, ipl=None, chunk=None, symmetric=None, check_indices=None,
             split=None):
        """Launch-shape tuning (see tsbts_tune): workgroups per split launch, kernel form
        (0 = scalar-load kernels, 1/2/4 = LDS kernels with that many targets per lane), j
        per split unit of the scalar-load kernels (0 = automatic, 64, 256), symmetric
        all-targets kernels (0 = never, 1 = always, 2 = automatic), split calls of large
        partial active sets (0 = never, 1 = from 8192 targets, 2 = automatic);
        check_indices = 1: every call checks its device active set against [0, n) first
        (debugging aid)."""
        if check_indices is not None:
            L.tsbts_tune(self.ctx, L.TSBTS_TUNE_CHECK_INDICES, int(check_indices))
        if symmetric is not None:
            L.tsbts_tune(self.ctx, L.TSBTS_TUNE_SYMMETRIC, symmetric)
        if split is not None:
            L.tsbts_tune(self.ctx, L.TSBTS_TUNE_SPLIT, split)
        if blocks is not None:
            L.tsbts_tune(self.ctx, L.TSBTS_TUNE_BLOCKS, blocks)
        if ipl is not None:
            L.tsbts_tune(self.ctx, L.TSBTS_TUNE_IPL, ipl)
        if chunk is not None:
            L.tsbts_tune(self.ctx, L.TSBTS_TUNE_CHUNK, chunk)
        return self

    def host_buffer(self, n, dtype):
        """Page-locked host staging buffer (for asynchronous copies)."""
        return torch.empty(n, dtype=dtype, pin_memory=True)

    def synchronize(self, stream=None):
        (stream or torch.cuda.current_stream()).synchronize()

    def idx(self, active):
        """Active-set index tensor; host arrays are range-checked here (the kernels index
        particle arrays with these values directly)."""
        if not isinstance(active, torch.Tensor):
            a = np.asarray(active)
            if a.size and (a.min() < 0 or a.max() >= self.n):
                raise IndexError("active index outside [0, n)")
        elif active.device.type == "cpu" and active.numel():
            if int(active.min()) < 0 or int(active.max()) >= self.n:
                raise IndexError("active index outside [0, n)")
        return _dev(active, dtype=torch.int32, device=self.device).reshape(-1).contiguous()

    # ---------------------------------------------------------------- entry points
    def predict(self, t_block, use_history=False, stream=None):
        L.tsbts_predict(self.ctx, t_block, use_history, stream)

    def load_positions(self, r, m=None, t_label=0.0, stream=None):
        r = _dev(r, device=self.device).reshape(3, self.n).contiguous()
        m = self.m if m is None else _dev(m, device=self.device).reshape(self.n).contiguous()
        self._loaded = (r, m)  # keep the buffers alive until the kernels have run
        L.tsbts_load_positions(self.ctx, self.n, r, m, t_label, stream)

    def force(self, active, t_block, with_pot=True, acc=None, pot=None, stream=None):
        idx = active if isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
            and active.device.type == "cuda" else self.idx(active)
        k = idx.numel()
        if acc is None:
            acc = torch.empty((3, k), dtype=torch.float64, device=self.device)
        if with_pot and pot is None:
            pot = torch.empty(k, dtype=torch.float64, device=self.device)
        L.tsbts_force(self.ctx, idx, t_block, acc, pot if with_pot else None, stream)
        return acc, pot

    def force_criterion(self, active, t_block, eta, with_pot=True, acc=None, pot=None,
                        dtc=None, stream=None):
        """Force, potential and criterion in one pass, the criterion with the predicted
        velocities (tsbts_force_criterion).  Returns (acc, pot, dtc)."""
        idx = active if isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
            and active.device.type == "cuda" else self.idx(active)
        k = idx.numel()
        if acc is None:
            acc = torch.empty((3, k), dtype=torch.float64, device=self.device)
        if with_pot and pot is None:
            pot = torch.empty(k, dtype=torch.float64, device=self.device)
        if dtc is None:
            dtc = torch.empty(k, dtype=torch.float64, device=self.device)
        L.tsbts_force_criterion(self.ctx, idx, t_block, eta, acc, pot if with_pot else None,
                                dtc, stream)
        return acc, (pot if with_pot else None), dtc

    def force_backward(self, active, t_block, grad_acc, grad_pot=None, grad_r=None,
                       grad_m=None, stream=None):
        idx = active if isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
            and active.device.type == "cuda" else self.idx(active)
        if grad_r is None:
            grad_r = torch.zeros((3, self.n), dtype=torch.float64, device=self.device)
        if grad_m is None:
            grad_m = torch.zeros(self.n, dtype=torch.float64, device=self.device)
        ga = _dev(grad_acc, device=self.device).contiguous()
        gp = None if grad_pot is None else _dev(grad_pot, device=self.device).contiguous()
        L.tsbts_force_backward(self.ctx, self.n, idx, t_block, ga, gp, grad_r, grad_m, stream)
        return grad_r, grad_m

    def correct(self, active, t_block, acc_new, stream=None):
        idx = active if isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
            and active.device.type == "cuda" else self.idx(active)
        L.tsbts_correct(self.ctx, idx, t_block, acc_new, stream)

    def timestep(self, active, eta, dtc=None, stream=None):
        idx = active if isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
            and active.device.type == "cuda" else self.idx(active)
        if dtc is None:
            dtc = torch.empty(idx.numel(), dtype=torch.float64, device=self.device)
        L.tsbts_timestep(self.ctx, idx, eta, dtc, stream)
        return dtc

    def set_dt(self, active, dt_new, stream=None):
        idx = active if isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
            and active.device.type == "cuda" else self.idx(active)
        L.tsbts_set_dt(self.ctx, idx, _dev(dt_new, device=self.device), stream)

    def history_begin(self, stream=None):
        L.tsbts_history_begin(self.ctx, stream)

    def history_end(self, stream=None):
        L.tsbts_history_end(self.ctx, stream)

    def history_clear(self):
        L.tsbts_history_clear(self.ctx)

    def history_layout(self, stream=None):
        """(n_records, off int32 [n+1], t float64 [n_records]) of the finished history,
        copied to new device tensors."""
        n_rec = L.tsbts_history_layout(self.ctx, self.n)
        off = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        t = torch.empty(n_rec, dtype=torch.float64, device=self.device)
        L.tsbts_history_layout(self.ctx, self.n, off, t, stream)
        return n_rec, off, t

    def interp_adjoint(self, t_block, pbar, hbar, stream=None):
        """Move the adjoint of interpolated predicted positions into the record adjoint
        hbar [6][n_records] of the finished history (tsbts_interp_adjoint)."""
        L.tsbts_interp_adjoint(self.ctx, self.n, hbar.shape[1], t_block, pbar, hbar, stream)

    def record_adjoint(self, active, t_block, layout, hbar, rbar, vbar, stream=None):
        """Add the adjoints of the records written at t_block (history `layout` as
        returned by history_layout) into rbar, vbar (tsbts_record_adjoint)."""
        idx = active if isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
            and active.device.type == "cuda" else self.idx(active)
        _, off, t = layout
        L.tsbts_record_adjoint(self.ctx, self.n, idx, t_block, off, t, hbar, rbar, vbar,
                               stream)

    def adjoint_accumulate(self, rbar, vbar, abar, rbar_acc, vbar_acc, abar_acc, stream=None):
        L.tsbts_adjoint_accumulate(self.ctx, self.n, rbar, vbar, abar, rbar_acc, vbar_acc,
                                   abar_acc, stream)

    def snapshot(self, T, stream=None):
        r = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        v = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        L.tsbts_snapshot(self.ctx, self.n, T, r, v, stream)
        return r, v

    def energy(self, r=None, v=None, m=None, out=None, stream=None):
        r = self.r if r is None else _dev(r, device=self.device)
        v = self.v if v is None else _dev(v, device=self.device)
        m = self.m if m is None else _dev(m, device=self.device)
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=self.device)
        L.tsbts_energy(self.ctx, self.n, r, v, m, out, stream)
        return out

    def leapfrog_adjoint(self, phase, h, rbar, vbar, abar, g_out=None, stream=None):
        L.tsbts_leapfrog_adjoint(self.ctx, self.n, phase, h, rbar, vbar, abar, g_out, stream)

    def block_adjoint(self, phase, active, t_block, rbar, vbar, abar, pbar, seeds,
                      stream=None):
        """Reverse of one block step of a fixed schedule (tsbts_block_adjoint); phase 1
        needs neither the active set nor the seeds (pass None)."""
        if active is None:
            idx = None
        elif isinstance(active, torch.Tensor) and active.dtype == torch.int32 \
                and active.device.type == "cuda":
            idx = active
        else:
            idx = self.idx(active)
        L.tsbts_block_adjoint(self.ctx, self.n, phase, idx, t_block, rbar, vbar, abar, pbar,
                              seeds, stream)

    # ---------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "ctx", None) is not None:
            L.tsbts_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
