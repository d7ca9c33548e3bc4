"""Write the oracle's seed-ensemble profiles of the small discharge.

Calls only ``oracle/`` (and the seeded configuration of the small workload):
for each gather (EC, MC) and seeds 0..S-1 it runs the 128-cell, 2.5 cm, 200 V,
50 mTorr argon discharge (12 800 + 12 800 particles, dt = T_RF/400, FP64) for
2000 steps, averaging n_e, n_i and phi over the last two RF cycles (every
step from step 1200) and sampling the central EEDF every T_RF/10.  The mean
over seeds and the standard deviation across seeds of every profile value are
stored as JSON next to this script.

    python tests/golden/make_ensemble.py [--seeds 32] [--jobs 8]
"""
import argparse
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

STEPS = 2000
AVG_START = 1200
EEDF_EVERY = 40


def ensemble_config(gather, seed, precision=0):
    import inputs
    from oracle import physics as ph
    n_g = ph.gas_density(50.0 * inputs.MTORR, 300.0)
    return inputs.small_discharge(gather=gather, seed=seed, precision=precision, gamma_see=0.1,
                                  nu_max_e=ph.nu_max_electron(n_g),
                                  nu_max_i=ph.nu_max_ion(n_g, 200.0, 300.0),
                                  avg_start=AVG_START, avg_every=1, eedf_every=EEDF_EVERY,
                                  k_stop=STEPS, sort_interval=20)


def run_one(args):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    gather, seed = args
    from oracle.sim import Sim
    sim = Sim(ensemble_config(gather, seed))
    sim.run(STEPS)
    p = sim.profiles()
    return dict(ne=list(map(float, p["ne"])), ni=list(map(float, p["ni"])),
                phi=list(map(float, p["phi"])), eedf=list(map(int, p["eedf"])))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=32)
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--out", default=HERE)
    a = ap.parse_args()
    jobs = [(g, s) for g in (0, 1) for s in range(a.seeds)]
    with Pool(a.jobs) as pool:
        res = pool.map(run_one, jobs)
    import numpy as np
    for g, name in ((0, "ec"), (1, "mc")):
        runs = [r for (gg, _), r in zip(jobs, res) if gg == g]
        stats = {}
        for key in ("ne", "ni", "phi", "eedf"):
            arr = np.array([r[key] for r in runs], dtype=np.float64)
            stats[key] = dict(mean=[float(f"{v:.10g}") for v in arr.mean(axis=0)],
                              std=[float(f"{v:.4g}") for v in arr.std(axis=0, ddof=1)])
        out = dict(description=("oracle seed ensemble, small argon discharge (128 cells, 2.5 cm, 200 V, "
                                "50 mTorr, 12800 + 12800 particles, dt = T_RF/400, FP64), "
                                f"{'EC' if g == 0 else 'MC'} gather, {STEPS} steps, profiles averaged "
                                f"from step {AVG_START}, EEDF every {EEDF_EVERY} steps"),
                   gather=g, seeds=list(range(a.seeds)), steps=STEPS, avg_start=AVG_START,
                   eedf_every=EEDF_EVERY, profiles=stats)
        with open(os.path.join(a.out, f"ensemble_small_{name}.json"), "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    main()
