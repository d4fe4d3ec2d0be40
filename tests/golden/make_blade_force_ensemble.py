"""Writes blade_force_ensemble.json: the FP64 oracle's blade force on the
4,800-sphere jammed bed with a blade cutting at 1 m/s (150 sweeps, dt 1/60 s)
from an ensemble of starts one FP32 ulp apart (scenegen.ulp_nudge, seeds
1..K): per run the mean force over 1 s (60 steps).

The cut is chaotic: the force difference between two runs grows about tenfold
every two steps, so after 1 s single trajectories of the same bed differ by
several per cent even in the oracle alone.  The ensemble mean and spread are
what a second implementation can be held to.  Calls only the oracle and the
seeded input generator:  python tests/golden/make_blade_force_ensemble.py
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "oracle"))

import pyoracle as O  # noqa: E402
from paper_2011_00459_amd import scenegen as SG  # noqa: E402

K = 16
STEPS = 60
BED = dict(seed=23, nx=30, ny=16, nz=10, r0=0.03, sweeps=150, blade=True)


def run(seed):
    spec = SG.jammed_bed(**BED)
    spec = dict(spec, x=SG.ulp_nudge(spec["x"], seed))
    o = O.OracleScene(spec)
    f = [o.step()["body_ft"][1][:3].tolist() for _ in range(STEPS)]
    return seed, f


def main():
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        runs = sorted(pool.map(run, range(1, K + 1)))
    forces = np.array([f for _, f in runs])           # K x STEPS x 3
    mean60 = forces.mean(axis=1)
    out = dict(bed=BED, steps=STEPS, seeds=[s for s, _ in runs],
               mean_1s=mean60.tolist(), ensemble_mean_1s=mean60.mean(axis=0).tolist(),
               ensemble_std_1s=mean60.std(axis=0, ddof=1).tolist())
    with open(os.path.join(HERE, "blade_force_ensemble.json"), "w") as fh:
        json.dump(out, fh)
    print("ensemble mean", out["ensemble_mean_1s"], "std", out["ensemble_std_1s"])


if __name__ == "__main__":
    main()
