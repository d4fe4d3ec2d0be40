"""Sweeps of the oracle's Gauss-Seidel to R_k <= 1e-4 against the error of
the start (FP64, CPU): the previous-step impulses, the cold start, and the
step's own converged impulses with random per-contact or uniform relative
errors of given sizes.  Prints one JSON line per scene.

    python tests/studies/warm_start_error.py column   # 1,000-sphere column, settled
    python tests/studies/warm_start_error.py bed      # bed 205 of the 256-bed batch, tool held still

Not a test: it measures how the sweep count depends on the size and the
shape of the start's error, which sets what a learned start would have to
reach to save sweeps.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path[:0] = [os.path.dirname(os.path.dirname(HERE)), os.path.join(os.path.dirname(os.path.dirname(HERE)), "oracle"),
                os.path.dirname(HERE)]

import pyoracle as O  # noqa: E402
from helpers import with_  # noqa: E402
from paper_2011_00459_amd import scenegen as SG  # noqa: E402


def settle(spec, steps=60):
    o = O.OracleScene(with_(spec, warm_start="prev", tol=1e-4, max_sweeps=4000))
    for _ in range(steps):
        o.step()
    return with_(spec, x=SG.fp32(o.x), v=SG.fp32(o.v), w=SG.fp32(o.w))


def study(spec, steps_before=3, seed=0):
    spec = with_(spec, warm_start="prev", tol=1e-4, max_sweeps=20000)
    o = O.OracleScene(spec)
    for _ in range(steps_before):
        o.step()
    x, v, w = o.x.copy(), o.v.copy(), o.w.copy()
    pk, pl = o.prev_keys.copy(), o.prev_lam.copy()
    # the step's solution, from the previous-step start, converged to R_k <= 1e-9
    ref = O.OracleScene(with_(spec, x=x, v=v, w=w, tol=1e-9, max_sweeps=100000))
    ref.prev_keys, ref.prev_lam = pk, pl
    rr = ref.step()
    keys, lstar = rr["keys"], rr["lam"]

    def sweeps_from(start):
        t = O.OracleScene(with_(spec, x=x, v=v, w=w))
        t.prev_keys, t.prev_lam = keys.copy(), start
        return int(t.step()["sweeps"])

    def err(l0):
        return float(np.linalg.norm(l0 - lstar) / np.linalg.norm(lstar))

    res = {"contacts": int(len(keys)), "reference_sweeps": int(rr["sweeps"])}
    prev = np.zeros_like(lstar)
    at = {int(k): i for i, k in enumerate(pk)}
    for i, k in enumerate(keys):
        j = at.get(int(k))
        if j is not None:
            prev[i] = pl[j]
    res["previous_step"] = dict(err=err(prev), sweeps=sweeps_from(prev))
    res["cold"] = dict(err=1.0, sweeps=sweeps_from(np.zeros_like(lstar)))
    rng = np.random.default_rng(seed)
    res["random_per_contact"] = []
    for e in (1e-5, 1e-4, 1e-3, 3e-3, 1e-2, 3e-2, 0.1, 0.3):
        sw = []
        for _ in range(3):
            d = rng.normal(0, 1, lstar.shape) * np.abs(lstar).max(axis=1, keepdims=True)
            d *= e * np.linalg.norm(lstar) / np.linalg.norm(d)
            sw.append(sweeps_from(lstar + d))
        res["random_per_contact"].append(dict(err=e, sweeps=sw))
    res["uniform_scale"] = [dict(err=err(lstar * (1 + e)), sweeps=sweeps_from(lstar * (1 + e)))
                            for e in (1e-3, 1e-2, 0.1)]
    return res


def main(which):
    if which == "column":
        spec = settle(SG.column_scene(seed=900, n=1000, sweeps=100))
    else:
        bed = SG.batch_spec(3000, 205, sweeps=100)
        still = [dict(b, linvel=(0.0, 0.0, 0.0)) for b in bed["bodies"]]
        spec = settle(with_(bed, bodies=still))
    print(json.dumps({which: study(spec)}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "column")
