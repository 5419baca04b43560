"""Write the oracle's whole-integration references used by the GPU driver tests.

Calls only the oracle (and the seeded input generators).  For each workload it runs the
oracle's TSBTS integration and stores the energy series at every dt_max multiple, the
schedule statistics and the final state digest:

    python tests/golden/make_golden.py plummer256 plummer4096

Each reference also lists the era ends and the number of eras of each size.

Output: tests/golden/tsbts_<workload>.json
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle.tsbts import OracleTSBTS, TICK  # noqa: E402
from workloads import config  # noqa: E402

RUNS = {
    # name: (workload, passes, t_end, overrides of the workload's parameters)
    "plummer256": ("plummer256", 3, None, {}),
    "plummer256_1pass": ("plummer256", 1, None, {}),
    "plummer4096": ("plummer4096", 3, None, {}),
    "plummer4096_t1": ("plummer4096", 3, 1.0, {}),
    # dynamic era on the 256-body sphere with dt_max = 1/8 and eta = 0.05: Algorithm 3
    # sets the era to 1/8 while a particle is on the top level, to 1/16 afterwards
    "plummer256_dyn": ("plummer256", 3, 1.0, {"eta": 0.05, "dt_max": 0.125, "era": None}),
}


def run(name: str):
    wl, passes, t_end, over = RUNS[name]
    cfg = config(wl)
    r, v, m = cfg.ic()
    t_end = cfg.t_end if t_end is None else t_end
    par = {"eta": cfg.eta, "era": cfg.era, "dt_max": cfg.dt_max, "dt_min": cfg.dt_min}
    par.update(over)
    sim = OracleTSBTS(r, v, m, cfg.eps, passes=passes, **par)
    ends = []
    era_step = sim.era_step

    def step():
        T1 = era_step()
        ends.append(T1 * TICK)
        return T1

    sim.era_step = step
    t0 = time.time()
    series = sim.run(t_end)
    wall = time.time() - t0
    e = np.array([x[1] for x in series])
    rel = (e - e[0]) / abs(e[0])
    out = {
        "workload": wl, "passes": passes, "t_end": t_end, "eps": cfg.eps, "eta": par["eta"],
        "dt_max": par["dt_max"], "dt_min": par["dt_min"], "era": par["era"], "seed": cfg.seed,
        "era_ends": ends,
        "times": [x[0] for x in series], "energy": e.tolist(),
        "max_rel_energy_error": float(np.abs(rel).max()),
        "final_rel_energy_error": float(rel[-1]),
        "stats": sim.stats, "oracle_wall_s": wall, "oracle_threads": oracle.threads(),
        "final_r_rms": float(np.sqrt((sim.r ** 2).mean())),
        "level_histogram": np.bincount(np.log2(sim.dt).astype(int), minlength=21).tolist(),
    }
    path = os.path.join(HERE, f"tsbts_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: max |dE/E| = {out['max_rel_energy_error']:.3e}, "
          f"{sim.stats['block_steps']} block steps, {wall:.1f} s -> {path}")


if __name__ == "__main__":
    for name in sys.argv[1:] or list(RUNS):
        run(name)
