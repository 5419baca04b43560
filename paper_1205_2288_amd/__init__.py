"""MI355X (gfx950) hot path of the dynamic-era time-symmetric block time-step (TSBTS)
N-body method of Kaplan & Saygin (arXiv 1205.2288).

* ``libtsbts.so`` (C ABI, include/tsbts.h): prediction and time-symmetric interpolation,
  softened direct-summation force and potential of an active set (mixed precision or
  float64), the time-step criterion, the leapfrog corrector with era-history recording,
  the O(N^2) float64 energy and the force adjoint - all hand-written HIP kernels.
* ``_lib``: ctypes binding with the C names.
* ``Context``: device-resident state and convenience wrappers.
* ``driver.TSBTS``: host-side era / pass / block-step scheduler (Algorithms 1-3) in
  Python; ``driver.NativeTSBTS``: the same loop in the library (tsbts_sched_*).
* ``autograd``: torch.autograd Functions over the force adjoint, a checkpointed
  shared-step leapfrog and a run on a fixed block schedule.
* ``experiments``: era-size / iteration and fixed / dynamic era energy-error studies.
"""
from .context import Context  # noqa: F401

__all__ = ["Context"]
