"""Era-size and iteration studies of the method at GPU speed (the paper's Section 3 tests
of era size and iteration count, and Section 4's fixed versus dynamic era), on seeded
Plummer spheres with the native scheduler.

Each run integrates one sphere and samples the relative energy error
|E(t) - E(0)| / |E(0)| (float64 O(N^2) energy) at a fixed interval.  A run is summarised
by its largest error, its final error and the growth ratio err(t_end) / err(t_end / 2),
taken on the running maximum of the error: about 2 for a linearly growing error, about
sqrt(2) for a random walk, about 1 once the error has saturated.

The paper's own initial conditions and curves are not published, and its runs last
1000 time units; these studies use fresh seeded spheres and shorter runs, so only the
trends compare (larger eras with too few passes drift linearly; more passes or smaller
eras keep the error in a random walk; dynamic eras perform like the best fixed era).

    python -m paper_1205_2288_amd.experiments era --n 100 --t-end 100 --seeds 3
    python -m paper_1205_2288_amd.experiments dynamic --n 100 --t-end 100 --seeds 10
    python -m paper_1205_2288_amd.experiments era --n 500 --eta 0.5 --workers 12 ...

Long runs can span several sessions: with --state-dir DIR each run saves an era-end
checkpoint of the scheduler (bit-exact continuation) and its energy series after every
segment, and a later invocation with the same DIR continues each run from its checkpoint;
with --deadline SECONDS every run stops after the first segment that ends that long after
the study started and reports itself incomplete (a summary counts complete runs only).

Each finished run prints one JSON line (progress and result); the last line is a summary.
With --workers K > 1 the runs go to K child processes at a time (each its own GPU context;
a run at N of a few hundred is bound by launch latency, not by the GPU's throughput, so
concurrent runs share one GPU almost for free).  The parent process never touches the GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor, as_completed

import numpy as np


def _plummer(n: int, seed: int):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from workloads import plummer
    return plummer(n, seed)


def _state_path(state_dir: str, n, seed, eps, eta, passes, era, dt_max, every, precision):
    key = (f"n{n}_seed{seed}_eps{eps:g}_eta{eta:g}_p{passes}_era"
           f"{'dyn' if era is None else format(era, 'g')}_dtmax{dt_max:g}_every{every:g}_"
           f"{precision}")
    return os.path.join(state_dir, key + ".npz")


def energy_error_run(n: int, seed: int, eps: float, eta: float, passes: int,
                     era: float | None, dt_max: float, t_end: float, every: float,
                     precision: str = "fp64", state_dir: str | None = None,
                     deadline: float | None = None, segment: float = 25.0) -> dict:
    """One integration; era=None selects the dynamic era (Algorithm 3).  The run goes in
    segments of `segment` time units (at least `every`).  state_dir: keep (and continue
    from) an era-end checkpoint and the energy series there after every segment;
    deadline: a wall-clock time (time.time() seconds) after which the run stops at the end
    of its current segment and reports complete = False."""
    from .driver import NativeTSBTS
    r, v, m = _plummer(n, seed)
    sim = NativeTSBTS(r, v, m, eps, eta=eta, passes=passes, era=era, dt_max=dt_max,
                      precision=precision)
    path = None if state_dir is None else _state_path(state_dir, n, seed, eps, eta, passes,
                                                      era, dt_max, every, precision)
    series, wall_before, t_mark = [], 0.0, 0.0
    eras_before = {}  # eras of each size in earlier sessions of this run

    def era_sizes():
        out = dict(eras_before)
        for k, c in sim.era_sizes.items():
            out[k] = out.get(k, 0) + c
        return out

    if path is not None and os.path.exists(path):
        with np.load(path) as z:  # arrays only (no pickles)
            ck = {k: z[k] for k in z.files}
        sim.restore(ck)
        series = list(zip(ck["series_t"].tolist(), ck["series_e"].tolist()))
        wall_before = float(ck["wall_s"])
        t_mark = series[-1][0]
        if "era_keys" in ck:
            eras_before = dict(zip(ck["era_keys"].tolist(), ck["era_counts"].tolist()))
    t0 = time.perf_counter()
    complete = True
    while t_mark < t_end:
        # integrate segment by segment, reporting progress on stderr
        t_mark = min(t_end, t_mark + max(every, segment))
        seg = sim.run(t_mark, energy_every=every)
        series.extend(seg if not series else seg[1:])
        wall = wall_before + time.perf_counter() - t0
        print(f"n={n} seed={seed} passes={passes} era={era} t={t_mark:g} "
              f"steps={sim.stats['block_steps']} wall={wall:.1f}s",
              file=sys.stderr, flush=True)
        if path is not None:
            ck = sim.checkpoint()
            ck["series_t"] = np.array([p[0] for p in series])
            ck["series_e"] = np.array([p[1] for p in series])
            ck["wall_s"] = np.array(wall)
            sizes = era_sizes()
            ck["era_keys"] = np.array(list(sizes.keys()), dtype=str)
            ck["era_counts"] = np.array(list(sizes.values()), dtype=np.int64)
            tmp = path + ".tmp.npz"
            np.savez(tmp, **ck)
            os.replace(tmp, path)
        if deadline is not None and t_mark < t_end and time.time() > deadline:
            complete = False
            break
    wall = wall_before + time.perf_counter() - t0
    st = sim.stats
    sizes = era_sizes()
    sim.close()
    e0 = series[0][1]
    t = np.array([p[0] for p in series])
    err = np.array([abs(p[1] - e0) / abs(e0) for p in series])
    run_max = np.maximum.accumulate(err)
    growth = math.nan
    if complete:
        half = run_max[np.searchsorted(t, 0.5 * t_end)]
        growth = float(run_max[-1] / half) if half > 0 else math.nan
    return {"n": n, "seed": seed, "passes": passes, "era": era if era else "dynamic",
            "eta": eta, "eps": eps, "dt_max": dt_max, "t_end": t_end,
            "complete": complete, "t_reached": float(t[-1]),
            "max_err": float(err.max()), "final_err": float(err[-1]), "growth": growth,
            "block_steps": st["block_steps"], "eras": st["eras"], "era_sizes": sizes,
            "wall_s": wall,
            "series_t": t.tolist(), "series_err": err.tolist()}


def _run_child(spec: dict) -> dict:
    """One energy_error_run in a child process (its own GPU context); returns its result."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cmd = [sys.executable, "-m", "paper_1205_2288_amd.experiments", "run",
           "--spec", json.dumps(spec)]
    # progress lines of the child go to this process's stderr as they come
    proc = subprocess.run(cmd, cwd=root, stdout=subprocess.PIPE, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"run {spec} failed with exit status {proc.returncode}")
    return json.loads(proc.stdout.strip().splitlines()[-1])


def run_many(specs: list, workers: int = 1, out=sys.stdout) -> list:
    """energy_error_run over a list of keyword dicts, in this process (workers <= 1) or in
    up to `workers` child processes at a time; results returned in the order of `specs`,
    each one emitted (without its series) as soon as it finishes."""
    def emit(res):
        _emit(out, {key: val for key, val in res.items() if not key.startswith("series")})
        return res

    if workers <= 1:
        return [emit(energy_error_run(**s)) for s in specs]
    if workers > 15:
        raise ValueError("at most 15 child processes (each holds a GPU context)")
    with ThreadPoolExecutor(max_workers=workers) as pool:
        futs = [pool.submit(_run_child, s) for s in specs]
        for f in as_completed(futs):  # each result is emitted as soon as it is known
            emit(f.result())
        return [f.result() for f in futs]


def era_study(n=100, seeds=3, t_end=100.0, eta=0.1, eps=0.01, dt_max=1.0 / 64,
              eras=(1 / 64, 1 / 32, 1 / 16, 1 / 8, 1 / 4), passes=(3, 5), every=1.0,
              seed0=1205, out=sys.stdout, workers=1, state_dir=None, deadline=None):
    """Fixed era sizes x pass counts x initial conditions (Section 3, fixed-era tests)."""
    specs = [dict(n=n, seed=seed0 + k, eps=eps, eta=eta, passes=p, era=era, dt_max=dt_max,
                  t_end=t_end, every=every, state_dir=state_dir, deadline=deadline)
             for k in range(seeds) for p in passes for era in eras]
    rows = run_many(specs, workers, out)
    summary = {}
    for p in passes:
        for era in eras:
            sel = [r for r in rows if r["passes"] == p and r["era"] == era and r["complete"]]
            summary[f"passes={p} era={era:g}"] = {
                "complete_runs": len(sel),
                "median_max_err": float(np.median([r["max_err"] for r in sel])) if sel else None,
                "median_growth": float(np.median([r["growth"] for r in sel])) if sel else None,
                "median_block_steps":
                    float(np.median([r["block_steps"] for r in sel])) if sel else None}
    _emit(out, {"study": "era", "n": n, "t_end": t_end, "seeds": seeds, "summary": summary})
    return rows, summary


def dynamic_era_study(n=100, seeds=10, t_end=100.0, eta=0.1, eps=0.01, dt_max=1.0 / 64,
                      passes=3, every=1.0, seed0=2205, out=sys.stdout, workers=1,
                      state_dir=None, deadline=None):
    """Fixed era (= dt_max) against the dynamic era (Section 4), same initial conditions."""
    specs = [dict(n=n, seed=seed0 + k, eps=eps, eta=eta, passes=passes, era=era,
                  dt_max=dt_max, t_end=t_end, every=every, state_dir=state_dir,
                  deadline=deadline)
             for k in range(seeds) for era in (dt_max, None)]
    res = run_many(specs, workers, out)
    rows = [{"fixed": res[2 * k], "dynamic": res[2 * k + 1]} for k in range(seeds)
            if res[2 * k]["complete"] and res[2 * k + 1]["complete"]]
    if not rows:
        _emit(out, {"study": "dynamic", "n": n, "t_end": t_end, "seeds": seeds,
                    "summary": {"complete_pairs": 0}})
        return rows, {}
    better = sum(1 for p in rows if p["dynamic"]["final_err"] < p["fixed"]["final_err"])
    summary = {
        "complete_pairs": len(rows),
        "dynamic_smaller_final_err_fraction": better / len(rows),
        "median_final_err_fixed": float(np.median([p["fixed"]["final_err"] for p in rows])),
        "median_final_err_dynamic": float(np.median([p["dynamic"]["final_err"] for p in rows])),
        "wall_ratio_dynamic_to_fixed": float(sum(p["dynamic"]["wall_s"] for p in rows)
                                             / sum(p["fixed"]["wall_s"] for p in rows))}
    _emit(out, {"study": "dynamic", "n": n, "t_end": t_end, "seeds": seeds,
                "summary": summary})
    return rows, summary


def _emit(out, obj):
    out.write(json.dumps(obj) + "\n")
    out.flush()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("study", choices=["era", "dynamic", "run"])
    ap.add_argument("--spec", default=None, help="run: energy_error_run keywords as JSON")
    ap.add_argument("--workers", type=int, default=1,
                    help="child processes running at a time (each its own GPU context)")
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--t-end", type=float, default=100.0)
    ap.add_argument("--eta", type=float, default=0.1)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--dt-max", type=float, default=1.0 / 64,
                    help="largest step, and the fixed era of the dynamic study's fixed runs")
    ap.add_argument("--passes", type=int, nargs="+", default=None)
    ap.add_argument("--eras", type=float, nargs="+", default=None,
                    help="fixed era sizes of the era study (default 1/64 ... 1/4)")
    ap.add_argument("--seed0", type=int, default=None, help="first sphere's seed")
    ap.add_argument("--every", type=float, default=1.0, help="energy sampling interval")
    ap.add_argument("--state-dir", default=None,
                    help="keep each run's era-end checkpoint and energy series here and "
                         "continue runs found there")
    ap.add_argument("--deadline", type=float, default=None,
                    help="seconds after the start of the study at which every run stops at "
                         "the end of its current 25-unit segment (reported as incomplete)")
    args = ap.parse_args(argv)
    if args.state_dir is not None:
        os.makedirs(args.state_dir, exist_ok=True)
        args.state_dir = os.path.abspath(args.state_dir)
    resume = {"state_dir": args.state_dir,
              "deadline": None if args.deadline is None else time.time() + args.deadline}
    if args.study == "run":
        _emit(sys.stdout, energy_error_run(**json.loads(args.spec)))
        return
    if not 1 <= args.workers <= 15:
        ap.error("--workers must be between 1 and 15")
    if args.study == "era":
        kw = {} if args.eras is None else {"eras": tuple(args.eras)}
        if args.seed0 is not None:
            kw["seed0"] = args.seed0
        era_study(n=args.n, seeds=args.seeds, t_end=args.t_end, eta=args.eta, eps=args.eps,
                  dt_max=args.dt_max, passes=tuple(args.passes or (3, 5)), every=args.every,
                  workers=args.workers, **kw, **resume)
    else:
        kw = {} if args.seed0 is None else {"seed0": args.seed0}
        dynamic_era_study(n=args.n, seeds=args.seeds, t_end=args.t_end, eta=args.eta,
                          eps=args.eps, dt_max=args.dt_max, passes=(args.passes or [3])[0],
                          every=args.every, workers=args.workers, **kw, **resume)


if __name__ == "__main__":
    main()
