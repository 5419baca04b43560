"""Benchmark of the TSBTS hot path on one MI355X.

Workload: seeded Plummer sphere, N = 131072, eps = 1/4096, log-uniform masses (1 decade,
total mass 1), Henon units.  Particles sit on two block levels (half at step h, half at
h/2, h = 2^-10), and one benchmark step is one era [0, h] of the method with two passes:

  for each pass: restore the era-start state, start recording history,
      block step at h/2: predict all (pass 2: Hermite interpolation of the non-active
          half from pass 1's records), force on the active half, corrector, criterion;
      block step at h:   predict all, force on all, corrector, criterion;
      finish the history (group records by particle);
  then the float64 energy of the synchronised state and the force adjoint for all
  particles at time h (dL/dacc drawn from a seeded normal distribution).

So each step issues 3 N^2 force interactions (mixed precision) and N^2 adjoint
interactions; `value` is (force + adjoint interactions) per second over the timed steps
(inputs resident in HBM).  The library chooses its kernels as for any caller: the
symmetric all-targets kernels for the calls with every particle active, split calls
(symmetric kernels on the pairs among the active half, gather kernels on its pairs with
the other half) for the half-active ones.  The same step is timed with the float64 force as the
comparison, plus a sweep of single force calls at active fractions 2^-k.

Prints one JSON line.  `--gpus` above 1 is not supported (one-GPU build).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from workloads import config, active_subset, gaussian  # noqa: E402

METRIC = "force interactions/s (mixed vs FP64, same accuracy) + adjoint interactions/s"
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic work per unit of the method (FMA = 2 flops), independent of how a kernel
# issues it: force 20 flop per interaction (n_act x N interactions per call, the masked
# self pair counted), force adjoint 52 per interaction when every particle is active (34
# when the particle is not a target), time-step criterion 15 per pair, energy 12 per
# unordered pair.
FLOPS_FORCE = 20.0
FLOPS_ADJOINT_ALL = 52.0
FLOPS_CRITERION = 15.0
FLOPS_ENERGY_PAIR = 12.0
# The same kernels counted by what they evaluate: the gather criterion 20 flop per pair
# (separation 3, r^2 3 FMA, velocity difference 3 and v^2 3 FMA, v^2/r^2 2, free-fall
# term 2, max and min 2); the symmetric all-targets kernels per unordered pair, each
# evaluated once for both particles: criterion 26 (separation 3, r^2 5, velocity
# difference 3, v^2 5, v^2/r^2 2, two free-fall terms 4, two maxima and two minima 4),
# force 26 (separation 3, s 6, 1/sqrt(s) 1, y^3 2, two mass factors 2, row and column
# sums 12), adjoint 64 (both rows' tidal-tensor products and mass terms from one pair).
FLOPS_CRITERION_GATHER = 20.0
FLOPS_CRITERION_SYM = 26.0
FLOPS_FORCE_SYM = 26.0
FLOPS_ADJOINT_SYM = 64.0
FLOPS_ADJOINT_GATHER = 73.0  # fused all-active gather kernel: source 38 + target 35

# HBM bytes per launch in the default (mixed) era step, from two rocprofv3 --pmc passes
# over this workload: FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch, averaged over the
# dispatches of one step (the same half / full mix the timing averages over), scaled by
# what the same counters read for a 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x
# 1.0).  Each entry names the sources the kernel is built from and their SHA-256 (first
# 16 hex digits) when the counters were taken; if they differ now, traffic is null.
COUNTER_SCALE = {"fetch": 2.0, "write": 1.0}
TRAFFIC_KIB = {
    "k_timestep_sym": (200805.3, 132102.7,
        ("timestep_sym.hip", "sym.hpp", "criterion.hpp", "pair.hpp", "internal.hpp"),
        "0ea120b43c4f421b"),
    "k_force_sym": (134479.5, 363360.7,
        ("force_sym.hip", "sym.hpp", "force_pair.hpp", "pair.hpp", "internal.hpp",
         "correct.hpp"),
        "9cb14d1bc07128f4"),
    "k_bwd_sym": (237130.6, 396422.7,
        ("backward_sym.hip", "sym.hpp", "pair.hpp", "internal.hpp"),
        "b631e093cddd99c9"),
    "k_energy_pairs": (18756.6, 256.0,
        ("energy.hip", "internal.hpp"),
        "999bec6dbfe71a46"),
}


def traffic_bytes(kernel: str):
    """Counter-measured HBM bytes per launch, or None if the kernel's sources changed."""
    import hashlib
    if kernel not in TRAFFIC_KIB:
        return None
    fetch, write, files, digest = TRAFFIC_KIB[kernel]
    csrc = os.path.join(ROOT, "paper_1205_2288_amd", "csrc")
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != digest:
        return None
    return (fetch * COUNTER_SCALE["fetch"] + write * COUNTER_SCALE["write"]) * 1024.0


class Timer:
    """HIP-event timing of calls on torch's current stream (the stream the library
    launches on)."""

    def __init__(self):
        self.events = {}

    def __call__(self, name, fn, *a, **k):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        out = fn(*a, **k)
        e.record()
        self.events.setdefault(name, []).append((s, e))
        return out

    def ms(self):
        torch.cuda.synchronize()
        return {k: [s.elapsed_time(e) for s, e in v] for k, v in self.events.items()}


class EraBench:
    """fused=True: the variant that takes the criterion before the corrector, in the same
    pass over the pairs as the force (tsbts_force_criterion)."""

    def __init__(self, cfg, r, v, m, precision, h=2.0 ** -10, seed=0, fused=False,
                 symmetric=2, split=2):
        from paper_1205_2288_amd import Context
        n = cfg.n
        self.n, self.h = n, h
        self.fused = fused
        self.ctx = c = Context(n, cfg.eps, precision=precision)
        c.tune(symmetric=symmetric, split=split)
        fine = active_subset(n, n // 2, cfg.seed + 11)
        dt = np.full(n, h)
        dt[fine] = h / 2
        c.bind(r, v, m, t_last=np.zeros(n), dt=dt)
        self.idx_all = c.idx(np.arange(n, dtype=np.int32))
        self.idx_fine = c.idx(fine)
        c.predict(0.0)
        acc, _ = c.force(self.idx_all, 0.0, with_pot=False)
        c.a.copy_(acc)
        self.s0 = [x.clone() for x in (c.r, c.v, c.a, c.t_last, c.dt)]
        dev = c.device
        self.acc_all = torch.empty((3, n), dtype=torch.float64, device=dev)
        self.acc_fine = torch.empty((3, fine.size), dtype=torch.float64, device=dev)
        self.dtc_all = torch.empty(n, dtype=torch.float64, device=dev)
        self.dtc_fine = torch.empty(fine.size, dtype=torch.float64, device=dev)
        self.kw = torch.empty(2, dtype=torch.float64, device=dev)
        self.g = torch.tensor(gaussian((3, n), cfg.seed + 7), device=dev)
        self.gr = torch.zeros((3, n), dtype=torch.float64, device=dev)
        self.gm = torch.zeros(n, dtype=torch.float64, device=dev)
        self.eta = cfg.eta
        self.interactions = 3 * n * n + n * n  # force (2 passes x 1.5 N^2) + adjoint
        torch.cuda.synchronize()

    def step(self, T: Timer | None = None):
        c, h = self.ctx, self.h
        t = T if T is not None else (lambda name, fn, *a, **k: fn(*a, **k))
        for p in range(2):
            for dst, src in zip((c.r, c.v, c.a, c.t_last, c.dt), self.s0):
                dst.copy_(src)
            c.history_begin()
            for tb, idx, acc, dtc in ((h / 2, self.idx_fine, self.acc_fine, self.dtc_fine),
                                      (h, self.idx_all, self.acc_all, self.dtc_all)):
                t("predict", c.predict, tb, use_history=p > 0)
                if self.fused:
                    t("force_criterion_full" if idx is self.idx_all else
                      "force_criterion_half", c.force_criterion, idx, tb, self.eta,
                      with_pot=False, acc=acc, dtc=dtc)
                    t("correct", c.correct, idx, tb, acc)
                    continue
                t("force_full" if idx is self.idx_all else "force_half", c.force, idx, tb,
                  with_pot=False, acc=acc)
                t("correct", c.correct, idx, tb, acc)
                t("timestep_full" if idx is self.idx_all else "timestep_half", c.timestep,
                  idx, self.eta, dtc=dtc)
            t("history_end", c.history_end)
        t("energy", c.energy, out=self.kw)
        self.gr.zero_()
        self.gm.zero_()
        t("backward", c.force_backward, self.idx_all, h, self.g, None, self.gr, self.gm)

    def close(self):
        self.ctx.close()


def time_steps(b: EraBench, steps: int, warmup: int):
    for _ in range(warmup):
        b.step()
    torch.cuda.synchronize()
    T = Timer()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.step(T)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, T.ms()


def sweep(cfg, r, v, m, precision, reps=5):
    """Single force calls at active fractions 2^-k (k = 0..17), median of reps.  Each entry
    also gives the call's algorithmic HBM bytes (every source record read once: float64
    x, y, z and a float32 mass in mixed precision, 28 B; x, y, z, m in float64, 32 B; plus
    each target's record and its acceleration and potential, 32 B) over its time: the
    bandwidth view that matters at small active sets, where the pair work is tiny."""
    from paper_1205_2288_amd import Context
    n = cfg.n
    jb = 28 if precision == "mixed" else 32
    out = []
    with Context(n, cfg.eps, precision=precision) as c:
        c.bind(r, v, m)
        c.predict(0.0)
        for k in range(18):
            n_act = max(1, n >> k)
            idx = c.idx(active_subset(n, n_act, cfg.seed + 1000 * k))
            acc = torch.empty((3, n_act), dtype=torch.float64, device=c.device)
            pot = torch.empty(n_act, dtype=torch.float64, device=c.device)
            for _ in range(2):
                c.force(idx, 0.0, acc=acc, pot=pot)
            T = Timer()
            for _ in range(reps):
                T("force", c.force, idx, 0.0, acc=acc, pot=pot)
            ms = float(np.median(T.ms()["force"]))
            nbytes = n * jb + n_act * (jb + 32)
            out.append({"n_active": n_act, "us": round(ms * 1e3, 2),
                        "interactions_per_s": n_act * n / (ms * 1e-3),
                        "algorithmic_bytes": nbytes,
                        "hbm_gbs": round(nbytes / (ms * 1e-3) / 1e9, 1)})
    return out


def sweep_c3(reps=20):
    """Force sweep at N = 32768 (eps = 1/1024, equal masses): the state at t_block = 1/64
    with t_last = t_block - 2^-(6+l), l drawn uniformly from 0..8 per particle, and the
    accelerations of the float64 force at the initial positions; active sets of 1, 8, 64,
    512, 4096 and 32768 random particles.  Each timed call is one prediction of all
    particles to t_block and one force call (median and minimum over `reps` calls after
    5 untimed ones), mixed precision against float64."""
    from paper_1205_2288_amd import Context
    cfg = config("sweep32768")
    n = cfg.n
    r, v, m = cfg.ic()
    tb = 1.0 / 64
    lev = np.random.default_rng(cfg.seed + 5).integers(0, 9, n)
    dt = 2.0 ** -(6 + lev)
    t_last = tb - dt
    with Context(n, cfg.eps, precision="fp64") as c:
        c.bind(r, v, m)
        c.predict(0.0)
        a0, _ = c.force(np.arange(n, dtype=np.int32), 0.0, with_pot=False)
        a0 = a0.cpu().numpy()
    res = {}
    for prec in ("mixed", "fp64"):
        rows = []
        with Context(n, cfg.eps, precision=prec) as c:
            c.bind(r, v, m, a=a0, t_last=t_last, dt=dt)
            for n_act in (1, 8, 64, 512, 4096, 32768):
                idx = c.idx(active_subset(n, n_act, cfg.seed + 1000 * int(np.log2(n_act))))
                acc = torch.empty((3, n_act), dtype=torch.float64, device=c.device)
                pot = torch.empty(n_act, dtype=torch.float64, device=c.device)

                def call():
                    c.predict(tb)
                    c.force(idx, tb, acc=acc, pot=pot)

                for _ in range(5):
                    call()
                T = Timer()
                for _ in range(reps):
                    T("call", call)
                t = np.array(T.ms()["call"])
                rows.append({"n_active": n_act, "median_us": round(float(np.median(t)) * 1e3, 2),
                             "min_us": round(float(t.min()) * 1e3, 2),
                             "interactions_per_s": n_act * n / (float(np.median(t)) * 1e-3)})
        res[prec] = rows
    for a, b in zip(res["mixed"], res["fp64"]):
        a["fp64_over_mixed"] = b["median_us"] / a["median_us"]
    return {"workload": "sweep32768: Plummer N=32768, eps=1/1024, equal masses; "
                        "one predict + one force per call",
            "mixed": res["mixed"], "fp64": res["fp64"]}


def adjoint_c4(reps=3):
    """The N = 8192 gradient workload: 64 shared leapfrog steps of 1/256 with era-start
    checkpoints every 16 steps, L = sum |r_final - r_target|^2 (r_target = the float64 run's
    end positions plus 0.01 N(0, 1)).  Times the forward run alone (no graph), the forward
    run that keeps the checkpoints, and the backward pass (per-era recompute of the
    forward plus the reverse sweep with the force adjoint at every step); adjoint
    interactions/s = 64 N^2 over the backward time."""
    from paper_1205_2288_amd import Context
    from paper_1205_2288_amd.autograd import tsbts_leapfrog
    cfg = config("adjoint8192")
    n, h, steps, era = cfg.n, 1.0 / 256, 64, 16
    r0, v0, m = cfg.ic()
    dev = torch.device("cuda")

    def t_(x, grad=False):
        return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev,
                            requires_grad=grad)

    with Context(n, cfg.eps, precision="fp64") as c:
        with torch.no_grad():
            r_fin, _ = tsbts_leapfrog(t_(r0), t_(v0), t_(m), c, h, steps, era)
    target = t_(r_fin.cpu().numpy() + 0.01 * gaussian((3, n), cfg.seed + 7))
    out = {}
    for prec in ("mixed", "fp64"):
        with Context(n, cfg.eps, precision=prec) as c:
            tf, tg, tb = [], [], []
            for k in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                with torch.no_grad():
                    tsbts_leapfrog(t_(r0), t_(v0), t_(m), c, h, steps, era)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                rt, vt, mt = t_(r0, True), t_(v0, True), t_(m, True)
                r_end, _ = tsbts_leapfrog(rt, vt, mt, c, h, steps, era)
                loss = ((r_end - target) ** 2).sum()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                loss.backward()
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                if k > 0:  # the first run is a warm-up
                    tf.append(t1 - t0)
                    tg.append(t2 - t1)
                    tb.append(t3 - t2)
            b = float(np.median(tb))
            out[prec] = {"forward_s": float(np.median(tf)),
                         "forward_with_checkpoints_s": float(np.median(tg)),
                         "backward_s": b,
                         "adjoint_interactions_per_s": steps * float(n) * n / b,
                         "force_interactions_per_s_forward":
                             steps * float(n) * n / float(np.median(tf))}
    return {"workload": "adjoint8192: Plummer N=8192, eps=1/256, 64 shared steps of 1/256, "
                        "checkpoints every 16 steps", **out}


def cpu_baseline(cfg, r, v, m, gpu_force_rows, target_s=12.0):
    """The oracle (plain FP64 C loops, OpenMP) on a bounded sample of the same step's
    work: force plus adjoint for a sample of targets against all N particles."""
    import oracle
    n = cfg.n
    g = gaussian((3, n), cfg.seed + 7)
    # a probe large enough that thread start-up does not dominate its time
    probe = np.arange(0, n, max(1, n // 1024), dtype=np.int32)[:1024]
    t0 = time.perf_counter()
    oracle.force(r, m, cfg.eps, probe)
    oracle.force_backward(r, m, cfg.eps, probe, g[:, probe])
    dt_probe = time.perf_counter() - t0
    per_target = dt_probe / probe.size
    s = int(np.clip(target_s / max(per_target, 1e-9), 64, n))
    sample = np.sort(np.random.default_rng(cfg.seed).choice(n, size=s, replace=False)
                     ).astype(np.int32)
    t0 = time.perf_counter()
    a_ref, _ = oracle.force(r, m, cfg.eps, sample)
    t_force = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.force_backward(r, m, cfg.eps, sample, g[:, sample])
    t_bwd = time.perf_counter() - t0
    rate = 2.0 * s * n / (t_force + t_bwd)
    # accuracy of the GPU force on the same sample (same arrays, time 0)
    acc = {}
    for prec, rows in gpu_force_rows.items():
        got = rows[:, sample]
        err = np.sqrt(((got - a_ref) ** 2).sum(0) / (a_ref ** 2).sum(0))
        acc[prec] = {"median_rel_err": float(np.median(err)),
                     "p99_rel_err": float(np.quantile(err, 0.99)),
                     "max_rel_err": float(err.max())}
    return {"value": rate, "unit": "interactions/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"force + adjoint of {s} random targets against all {n} particles "
                      f"(plain FP64 C, {oracle.threads()} OpenMP threads); "
                      f"force {t_force:.2f} s, adjoint {t_bwd:.2f} s",
            "force_accuracy_vs_oracle": acc}


def gpu_force_rows(cfg, r, v, m):
    from paper_1205_2288_amd import Context
    out = {}
    for prec in ("mixed", "fp64"):
        with Context(cfg.n, cfg.eps, precision=prec) as c:
            c.bind(r, v, m)
            c.predict(0.0)
            acc, _ = c.force(np.arange(cfg.n, dtype=np.int32), 0.0, with_pot=False)
            out[prec] = acc.cpu().numpy()
    return out


def rooflines(ms, n, precision="mixed", symmetric=True, split=True):
    """Roofline entries per kernel from HIP-event times of their calls in the timed steps.

    `achieved` = algorithmic TFLOP/s: the per-unit work of the method (force 20 flop per
    interaction, all-active adjoint 52 per interaction, criterion 15 per pair, energy 12
    per unordered pair) x the units one call processes (n_act x N interactions or pairs;
    N(N-1)/2 for the energy), over the mean call time.  `as_evaluated` gives the same
    time counted by what the kernel evaluates: the symmetric all-targets kernels take
    each unordered pair once for both particles (N(N-1)/2 pairs at 26, 26 and 64 flop),
    the gather criterion 20 flop per pair.  The events enclose each call's reduction
    kernels too.  With split, the half-active calls are split calls (the symmetric kernels
    on the pairs among the targets, the gather kernels on their pairs with the others:
    several kernels, so no counter traffic); their `as_evaluated` counts those two parts'
    pairs."""
    peak32 = PEAK_FP32_TFLOPS if precision == "mixed" else PEAK_FP64_TFLOPS
    out = {}
    pairs = n * (n - 1) / 2

    def entry(kernel, flop_per_unit, units_per_call, unit, ms_list, peak, evaluated=None):
        t = float(np.sum(ms_list)) * 1e-3
        calls = len(ms_list)
        achieved = flop_per_unit * units_per_call * calls / t / 1e12
        traffic = traffic_bytes(kernel) if precision == "mixed" else None
        e = {"kernel": kernel, "bound": "alu", "achieved": achieved, "peak": peak,
             "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
             "flop_per_unit": flop_per_unit, "work_unit": unit,
             "units_per_launch": units_per_call,
             "avg_launch_us": t / calls * 1e6, "calls": calls, "total_ms": t * 1e3}
        if evaluated is not None:
            f, u, name = evaluated
            a = f * u * calls / t / 1e12
            e["as_evaluated"] = {"flop_per_unit": f, "work_unit": name,
                                 "units_per_launch": u, "achieved": a, "frac": a / peak}
        return e

    nn, nh = float(n) * n, float(n) * (n // 2)
    if split:
        k = n // 2
        within, across = k * (k - 1) / 2.0, float(k) * (n - k)
        out["split_force"] = entry(
            "split_force", FLOPS_FORCE, nh, "interaction", ms["force_half"], peak32,
            (FLOPS_FORCE_SYM * within + FLOPS_FORCE * across, 1.0, "call"))
        out["split_timestep"] = entry(
            "split_timestep", FLOPS_CRITERION, nh, "pair", ms["timestep_half"], peak32,
            (FLOPS_CRITERION_SYM * within + FLOPS_CRITERION_GATHER * across, 1.0, "call"))
    else:
        out["k_force_scalar"] = entry("k_force_scalar", FLOPS_FORCE, nh, "interaction",
                                      ms["force_half"], peak32)
        out["k_timestep_scalar"] = entry("k_timestep_scalar", FLOPS_CRITERION, nh, "pair",
                                         ms["timestep_half"], peak32,
                                         (FLOPS_CRITERION_GATHER, nh, "pair"))
    if symmetric:
        out["k_force_sym"] = entry("k_force_sym", FLOPS_FORCE, nn, "interaction",
                                   ms["force_full"], peak32,
                                   (FLOPS_FORCE_SYM, pairs, "unordered pair"))
        out["k_timestep_sym"] = entry("k_timestep_sym", FLOPS_CRITERION, nn, "pair",
                                      ms["timestep_full"], peak32,
                                      (FLOPS_CRITERION_SYM, pairs, "unordered pair"))
        out["k_bwd_sym"] = entry("k_bwd_sym", FLOPS_ADJOINT_ALL, nn, "interaction",
                                 ms["backward"], peak32,
                                 (FLOPS_ADJOINT_SYM, pairs, "unordered pair"))
    else:
        out["k_force_scalar"] = entry(
            "k_force_scalar", FLOPS_FORCE, (nn * len(ms["force_full"]) +
                                            nh * len(ms["force_half"])) /
            (len(ms["force_full"]) + len(ms["force_half"])), "interaction",
            ms["force_full"] + ms["force_half"], peak32)
        u_c = (nn * len(ms["timestep_full"]) + nh * len(ms["timestep_half"])) / \
            (len(ms["timestep_full"]) + len(ms["timestep_half"]))
        out["k_timestep_scalar"] = entry("k_timestep_scalar", FLOPS_CRITERION, u_c, "pair",
                                         ms["timestep_full"] + ms["timestep_half"], peak32,
                                         (FLOPS_CRITERION_GATHER, u_c, "pair"))
        out["k_bwd_all"] = entry("k_bwd_all", FLOPS_ADJOINT_ALL, nn, "interaction",
                                 ms["backward"], peak32,
                                 (FLOPS_ADJOINT_GATHER, nn, "interaction"))
    out["k_energy_pairs"] = entry("k_energy_pairs", FLOPS_ENERGY_PAIR, pairs,
                                  "unordered pair", ms["energy"], PEAK_FP64_TFLOPS)
    return out


def force_variants(cfg, r, v, m, reps=5):
    """Full-active force time and accuracy (vs the float64 kernel) of each mixed variant,
    all on the gather kernels (symmetric kernels off) so that the pair-arithmetic variants
    compare on one kernel form."""
    from paper_1205_2288_amd import Context
    n = cfg.n
    res = {}
    ref = None
    for prec, sep, newton in (("fp64", "f64", False), ("mixed", "f64", False),
                              ("mixed", "f64", True), ("mixed", "hilo", False),
                              ("mixed", "hilo", True)):
        with Context(n, cfg.eps, precision=prec, separation=sep, newton=newton) as c:
            c.tune(symmetric=0)
            c.bind(r, v, m)
            c.predict(0.0)
            idx = c.idx(np.arange(n, dtype=np.int32))
            acc = torch.empty((3, n), dtype=torch.float64, device=c.device)
            for _ in range(2):
                c.force(idx, 0.0, with_pot=False, acc=acc)
            T = Timer()
            for _ in range(reps):
                T("f", c.force, idx, 0.0, with_pot=False, acc=acc)
            ms = float(np.median(T.ms()["f"]))
            a = acc.cpu().numpy()
        if ref is None:
            ref = a
        err = np.sqrt(((a - ref) ** 2).sum(0) / (ref ** 2).sum(0))
        name = "fp64" if prec == "fp64" else f"mixed-{sep}-{'newton' if newton else 'rsq'}"
        res[name] = {"ms": ms, "interactions_per_s": n * n / (ms * 1e-3),
                     "median_rel_err_vs_fp64_kernel": float(np.median(err)),
                     "max_rel_err_vs_fp64_kernel": float(err.max())}
    return res


def pass_cost(t_end=1.0):
    """Wall-clock of the same integration with one pass (the plain block-step scheme) and
    with three time-symmetrization passes, native scheduler, mixed precision: the GPU
    counterpart of the paper's iteration-cost comparison (Section 6)."""
    from paper_1205_2288_amd.driver import NativeTSBTS
    out = {}
    for name in ("plummer256", "plummer4096"):
        cfg = config(name)
        r, v, m = cfg.ic()
        res = {}
        for passes in (1, 3):
            sim = NativeTSBTS(r, v, m, cfg.eps, eta=cfg.eta, passes=passes, era=cfg.era,
                              dt_max=cfg.dt_max, dt_min=cfg.dt_min)
            series = sim.run(t_end)
            st = sim.stats
            e0 = series[0][1]
            res[passes] = {"wall_s": st["wall_s"], "block_steps": st["block_steps"],
                           "interactions": st["interactions"], "eras": st["eras"],
                           "drift": max(abs(e - e0) / abs(e0) for _, e in series),
                           "us_per_block_step": st["wall_s"] / st["block_steps"] * 1e6}
            sim.close()
        out[name] = {"t_end": t_end, "one_pass": res[1], "three_passes": res[3],
                     "wall_ratio": res[3]["wall_s"] / res[1]["wall_s"],
                     "block_step_ratio": res[3]["block_steps"] / res[1]["block_steps"]}
    return out


def force_calls(sizes, precision, reps=5):
    """predict + force + criterion (on the predicted state) at each active-set size on the
    N = 131072 workload (the sweep's subsets), mean call times over `reps` calls after 2
    untimed ones."""
    from paper_1205_2288_amd import Context
    cfg = config("plummer131k")
    n = cfg.n
    r, v, m = cfg.ic()
    out = []
    with Context(n, cfg.eps, precision=precision) as c:
        c.bind(r, v, m)
        for n_act in sizes:
            k = int(np.log2(n // n_act)) if n_act < n else 0
            idx = c.idx(active_subset(n, n_act, cfg.seed + 1000 * k))
            acc = torch.empty((3, n_act), dtype=torch.float64, device=c.device)
            pot = torch.empty(n_act, dtype=torch.float64, device=c.device)
            for _ in range(2):
                c.predict(0.0)
                c.force(idx, 0.0, acc=acc, pot=pot)
            dtc = torch.empty(n_act, dtype=torch.float64, device=c.device)
            for _ in range(2):
                c.timestep(idx, cfg.eta, dtc=dtc)
            T = Timer()
            for _ in range(reps):
                c.predict(0.0)
                T("force", c.force, idx, 0.0, acc=acc, pot=pot)
                T("criterion", c.timestep, idx, cfg.eta, dtc=dtc)
            ms = T.ms()
            out.append({"n_active": n_act, "force_us": float(np.mean(ms["force"])) * 1e3,
                        "criterion_us": float(np.mean(ms["criterion"])) * 1e3})
    return {"workload": "plummer131k", "precision": precision, "calls": out}


def native_run(name, t_end, precision, predict_on_load=None, split=None):
    """One whole integration of a workload with the native scheduler (its own era, step
    bounds and eta): wall time, block steps and the mean wall time per block step.
    ``split`` sets the split calls of large partial active sets (0 off, 1 from 8192
    targets, 2 the library's automatic choice; None leaves the default)."""
    from paper_1205_2288_amd.driver import NativeTSBTS
    cfg = config(name)
    r, v, m = cfg.ic()
    kw = {} if predict_on_load is None else {"predict_on_load": bool(predict_on_load)}
    if split is not None:
        kw["tune"] = {"split": int(split)}
    sim = NativeTSBTS(r, v, m, cfg.eps, eta=cfg.eta, passes=3, era=cfg.era,
                      dt_max=cfg.dt_max, dt_min=cfg.dt_min, precision=precision, **kw)
    series = sim.run(t_end)
    st = sim.stats
    e0 = series[0][1]
    out = {"workload": name, "precision": precision, "t_end": t_end,
           "predict_on_load": predict_on_load, "split": split,
           "wall_s": st["wall_s"], "block_steps": st["block_steps"],
           "us_per_block_step": st["wall_s"] / st["block_steps"] * 1e6,
           "interactions": st["interactions"], "eras": st["eras"],
           "era_sizes": st["era_sizes"],
           "drift": max(abs(e - e0) / abs(e0) for _, e in series),
           "phases": sim.step_timing()}
    sim.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-pass-cost", action="store_true")
    ap.add_argument("--native-run", default=None, metavar="WORKLOAD",
                    help="only integrate WORKLOAD (plummer256, plummer4096, plummer131k) with the native "
                         "scheduler to --t-end and print its block-step statistics (for "
                         "kernel traces of whole runs)")
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--force-calls", default=None, metavar="N_ACT[,N_ACT...]",
                    help="only time predict + force + criterion calls on the N=131072 "
                         "workload at these active-set sizes (5 each after 2 untimed; for "
                         "counter runs)")
    ap.add_argument("--precision", default="mixed", choices=("mixed", "fp64"))
    ap.add_argument("--predict-on-load", type=int, default=None, choices=(0, 1),
                    help="native run: small active sets predicted inside the force kernel "
                         "(default: the scheduler's choice)")
    ap.add_argument("--split", type=int, default=None, choices=(0, 1, 2),
                    help="native run: split calls of large partial active sets (0 off, "
                         "1 from 8192 targets, 2 automatic; default: the library's)")
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB "
                         "(reference kernel for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.calibration_copy_mb > 0:
        nbytes = args.calibration_copy_mb << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.native_run:
        print(json.dumps(native_run(args.native_run, args.t_end, args.precision,
                                    args.predict_on_load, args.split)))
        return
    if args.force_calls:
        sizes = [int(x) for x in args.force_calls.split(",")]
        print(json.dumps(force_calls(sizes, args.precision)))
        return
    cfg = config("plummer131k")
    n = cfg.n
    r, v, m = cfg.ic()

    b = EraBench(cfg, r, v, m, "mixed")
    wall, ms = time_steps(b, args.steps, args.warmup)
    per_call = {k: {"calls_per_step": len(x) / args.steps, "mean_us": float(np.mean(x)) * 1e3}
                for k, x in ms.items()}
    value = b.interactions * args.steps / wall
    roofs = rooflines(ms, n)
    dominant = max(roofs, key=lambda k: roofs[k]["total_ms"])
    roof = roofs[dominant]
    b.close()

    fp64 = None
    if not args.no_fp64:
        b64 = EraBench(cfg, r, v, m, "fp64")
        steps64 = max(2, args.steps // 2)
        wall64, ms64 = time_steps(b64, steps64, 1)
        fp64 = {"ms_per_step": wall64 / steps64 * 1e3,
                "value": b64.interactions * steps64 / wall64,
                "force_full_us": float(np.mean(ms64["force_full"])) * 1e3,
                "force_interactions_per_s": n * n / (np.mean(ms64["force_full"]) * 1e-3),
                "backward_us": float(np.mean(ms64["backward"])) * 1e3}
        b64.close()

    out = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 pair arithmetic (separation formed in f64, rounded once to f32), "
                 "f64 sums", "data": "synthetic",
        "config": {"workload": "plummer131k: Plummer N=131072, eps=1/4096, log-uniform "
                               "masses; one two-level two-pass era per step",
                   "n": n, "eps": cfg.eps, "seed": cfg.seed, "precision": "mixed",
                   "interactions_per_step": b.interactions,
                   "potential": "not computed in the timed block steps (the integrator "
                                "does not use it); the sweeps time force + potential",
                   "kernels": "library defaults: symmetric all-targets kernels when every "
                              "particle is active, split calls for the half-active block "
                              "steps; gather_kernels_only times the same step without "
                              "either"},
        "roofline": roof,
        "rooflines": roofs,
        "force_interactions_per_s": n * n / (np.mean(ms["force_full"]) * 1e-3),
        "adjoint_interactions_per_s": n * n / (np.mean(ms["backward"]) * 1e-3),
        "energy_pairs_per_s": n * (n - 1) / 2 / (np.mean(ms["energy"]) * 1e-3),
        "breakdown_us": per_call,
        "fp64_mode": fp64,
    }
    if not args.no_sweep:
        out["force_variants"] = force_variants(cfg, r, v, m)
        out["sweep_mixed"] = sweep(cfg, r, v, m, "mixed")
        out["sweep_fp64"] = sweep(cfg, r, v, m, "fp64")
    if not args.no_pass_cost:
        out["pass_cost"] = pass_cost()
    if not args.no_sweep:
        out["sweep32768"] = sweep_c3()
        out["adjoint8192"] = adjoint_c4()
    if not args.no_sweep:
        bf = EraBench(cfg, r, v, m, "mixed", fused=True)
        stepsf = max(2, args.steps // 2)
        wallf, msf = time_steps(bf, stepsf, 1)
        out["criterion_before_corrector"] = {
            "ms_per_step": wallf / stepsf * 1e3,
            "value": bf.interactions * stepsf / wallf,
            "speedup_vs_paper_order": (wall / args.steps) / (wallf / stepsf),
            "breakdown_us": {k: float(np.mean(x)) * 1e3 for k, x in msf.items()}}
        bf.close()
        # the same era step on the gather kernels only (symmetric all-targets kernels off)
        bg = EraBench(cfg, r, v, m, "mixed", symmetric=0, split=0)
        wallg, msg = time_steps(bg, stepsf, 1)
        out["gather_kernels_only"] = {
            "ms_per_step": wallg / stepsf * 1e3,
            "value": bg.interactions * stepsf / wallg,
            "speedup_of_symmetric": (wallg / stepsf) / (wall / args.steps),
            "rooflines": rooflines(msg, n, symmetric=False, split=False),
            "breakdown_us": {k: float(np.mean(x)) * 1e3 for k, x in msg.items()}}
        bg.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, r, v, m, gpu_force_rows(cfg, r, v, m))
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
