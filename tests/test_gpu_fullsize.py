"""Parity at the workloads' full sizes, in the launch configuration bench.py times.

  - 50,400-sphere jammed bed with a blade (the bulldozing bed's size, 150 sweeps,
    grouped schedule): one step against the FP64 oracle — contact lists bit-exact,
    velocities to the one-step bar;
  - 500,000-sphere jammed bed (the excavation bed's size and radius): the contact
    list of a step bit-exact against the oracle's detection, and the momentum
    balance of the step (pair impulses cancel: the change of total momentum is
    the gravity impulse plus the boundary impulses the library reports);
  - blade force on a jammed bed with a moving blade: the first five steps in
    every component to 1 %, and the 1 s mean force of an ensemble of starts one
    FP32 ulp apart against the oracle's ensemble (the cut is chaotic).
"""
import numpy as np
import pytest

import pyoracle as O
from helpers import jammed_bed, vel_tol, with_

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")


def test_bed50k_one_step_matches_oracle():
    spec = jammed_bed(seed=21, nx=60, ny=30, nz=28, r0=0.03, sweeps=150)
    n = len(spec["x"])
    assert n == 50400
    g = T.scene_from_specs(spec, cap_contacts=16 * n)
    assert g.get_solver_config()["mode"] == "grouped"
    st = g.step(1)[0]
    o = O.OracleScene(spec)
    oo = o.step()
    keys, lam = g.get_contacts(0)
    assert st["contacts"] == oo["contacts"] > 100000
    assert np.array_equal(keys, oo["keys"])
    assert st["colours"] == oo["colours"] and st["sweeps"] == oo["sweeps"] == 150
    assert np.array_equal(g.get_colours(0), oo["colour"])
    p = g.get_particles(0)
    assert np.max(np.abs(p["v"] - o.v)) <= vel_tol(o.v)
    lt = 1e-3 * np.max(np.abs(oo["lam"]))
    assert np.max(np.abs(lam - oo["lam"])) <= lt


def test_bed500k_contacts_bit_exact_and_momentum_balance():
    spec = jammed_bed(seed=5, nx=100, ny=50, nz=100, r0=0.02, sweeps=200, blade=True)
    n = len(spec["x"])
    assert n == 500000
    g = T.scene_from_specs(spec, cap_contacts=8 * n)
    before = g.get_particles(0)
    st = g.step(1)[0]
    keys, _ = g.get_contacts(0)
    # the oracle's detection on the same FP32 start state
    okeys, _ = O.detect(spec, O.CELLS)
    assert st["contacts"] == len(okeys) > 1_000_000
    assert np.array_equal(keys, okeys)
    # pair impulses cancel, so the change of total momentum is the gravity
    # impulse minus the impulses the kinematic bodies received (FP64 sums)
    after = g.get_particles(0)
    r = before["r"].astype(np.float64)
    m = spec["material"]["rho"] * (4.0 / 3.0) * np.pi * r ** 3
    dp = np.sum(m[:, None] * (after["v"] - before["v"]), axis=0)
    grav = np.sum(m) * np.asarray(spec["gravity"], dtype=np.float64) * spec["dt"]
    fb = sum(np.asarray(g.get_contact_forces(0, b)[0]) for b in range(len(spec["bodies"])))
    resid = dp - (grav - spec["dt"] * fb)
    assert np.linalg.norm(resid) <= 1e-3 * np.linalg.norm(grav), (dp, grav, spec["dt"] * fb)


def test_blade_force_first_steps_and_one_second_ensemble_match_oracle():
    # The cut is chaotic: the oracle's own mean force over 1 s moves by several
    # per cent when its start moves by one FP32 ulp (the per-step difference
    # grows about tenfold every two steps).  So (a) the first five steps from
    # the identical start agree in every component to 1 % of |F|, before the
    # trajectories separate; (b) the 1 s mean force averaged over 16 starts one
    # ulp apart agrees with the oracle's average over the same 16 starts
    # (tests/golden/blade_force_ensemble.json, written by the script beside it)
    # to four standard errors of the difference, in every component.
    import json
    import os
    from paper_2011_00459_amd import scenegen as SG
    path = os.path.join(os.path.dirname(__file__), "golden", "blade_force_ensemble.json")
    with open(path) as fh:
        ens = json.load(fh)
    spec = jammed_bed(**ens["bed"])
    g = T.scene_from_specs(spec)
    o = O.OracleScene(spec)
    for k in range(5):
        g.step(1, stats=False)
        fo = o.step()["body_ft"][1][:3]
        f, _ = g.get_contact_forces(0, 1)
        assert np.linalg.norm(f - fo) <= 1e-2 * np.linalg.norm(fo), (k, f, fo)
    g.close()
    means = []
    for seed in ens["seeds"]:
        g = T.scene_from_specs(dict(spec, x=SG.ulp_nudge(spec["x"], seed)))
        f = []
        for _ in range(ens["steps"]):
            g.step(1, stats=False)
            f.append(g.get_contact_forces(0, 1)[0])
        means.append(np.mean(f, axis=0))
        g.close()
    means = np.asarray(means)
    k = len(means)
    mg, sg = means.mean(axis=0), means.std(axis=0, ddof=1)
    mo, so = np.asarray(ens["ensemble_mean_1s"]), np.asarray(ens["ensemble_std_1s"])
    se = np.sqrt(sg ** 2 / k + so ** 2 / k)
    print(f"1 s mean blade force over {k} starts: GPU {mg} +- {sg}, oracle {mo} +- {so}")
    assert mo[0] < -100.0  # the bed resists the blade moving along +x
    assert np.all(np.abs(mg - mo) <= 4.0 * se), (mg, mo, se)
