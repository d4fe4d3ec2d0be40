"""Rolling resistance (Eq. signCoul3) on the HIP path against the FP64 oracle.

With mu_r > 0 each contact carries a rolling row after its tangential rows:
the relative angular velocity of the two bodies is driven towards zero by an
impulse bounded by r mu_r |lambda_n| (r the smaller radius).  Bars as for the
other parity tests: bit-exact contact lists and colours, velocities and spins
to the one-step bound, contact and rolling impulses to the impulse bound; the
closed forms of one sphere (rolling deceleration, spin stop) at FP32 accuracy.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from helpers import jammed_bed, settled_column, vel_tol, with_
from paper_2011_00459_amd import scenegen as SG

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")

G = 9.81
DT = 1.0 / 60.0


def rolling(spec, mu_r, **kw):
    mat = dict(spec["material"])
    mat["mu_r"] = mu_r
    return with_(spec, material=mat, **kw)


def compare(spec, steps, g=None, env=0, rel=1e-4):
    g = g or T.scene_from_specs(spec)
    o = O.OracleScene(spec)
    for k in range(steps):
        st = g.step(1)[env]
        oo = o.step()
        keys, lam = g.get_contacts(env)
        assert np.array_equal(keys, oo["keys"]), k
        assert st["colours"] == oo["colours"] and st["sweeps"] == oo["sweeps"]
        assert np.array_equal(g.get_colours(env), oo["colour"]), k
        p = g.get_particles(env)
        tol = vel_tol(o.v, rel=rel) * (1 + 4 * k)
        assert np.max(np.abs(p["v"] - o.v)) <= tol, (k, np.max(np.abs(p["v"] - o.v)), tol)
        wtol = tol / max(float(np.min(spec["r"])), 1e-3)
        assert np.max(np.abs(p["w"] - o.w)) <= wtol, (k, np.max(np.abs(p["w"] - o.w)), wtol)
        lt = 10 * rel * max(np.max(np.abs(oo["lam"])), 1e-12) * (1 + 4 * k)
        assert np.max(np.abs(lam - oo["lam"])) <= lt
        lr = g.get_rolling_impulses(env)
        assert lr.shape == oo["lr"].shape
        assert np.max(np.abs(lr - oo["lr"])) <= lt, (k, np.max(np.abs(lr - oo["lr"])), lt)
        # the rolling bound holds on the GPU side too (FP32 slack)
        rmin = rolling_radius(spec, keys)
        bound = rmin * spec["material"]["mu_r"] * np.abs(lam[:, 0])
        assert np.all(np.linalg.norm(lr.astype(np.float64), axis=1) <= bound * (1 + 1e-5) + 1e-12)
        assert np.any(np.linalg.norm(oo["lr"], axis=1) > 0.0)
    return g, o


def rolling_radius(spec, keys):
    """Smaller radius of each contact.  A pair key is a<<32 | b (the two
    particle ids); a boundary key is id<<32 | 0x80000000 | shape."""
    r = np.asarray(spec["r"], dtype=np.float64)
    ids = np.asarray(spec.get("id", np.arange(len(r))), dtype=np.int64)
    order = np.argsort(ids)
    keys = np.asarray(keys, dtype=np.uint64)
    a = (keys >> np.uint64(32)).astype(np.int64)
    lo = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    boundary = (lo & 0x80000000) != 0
    ra = r[order[np.searchsorted(ids[order], a)]]
    b = np.where(boundary, a, lo)
    rb = r[order[np.searchsorted(ids[order], b)]]
    return np.minimum(ra, rb)


def test_column_rolling_one_step_cold():
    spec = rolling(settled_column(seed=3, n=800, footprint=0.8), 0.1, max_sweeps=60)
    compare(spec, 2)


def test_column_rolling_prev_warm_start():
    # the rolling impulses are cached with the contact impulses and matched by key
    spec = rolling(settled_column(seed=4, n=600, footprint=0.7), 0.2, max_sweeps=40, warm_start="prev")
    compare(spec, 4)


def test_bed_with_moving_blade_rolling():
    # boundary contacts take the kinematic body's spin in the rolling row
    spec = jammed_bed(seed=31, nx=16, ny=10, nz=8, r0=0.03, sweeps=60, blade=True)
    spec = rolling(spec, 0.15)
    b = dict(spec["bodies"][1])
    b["angvel"] = (0.0, 0.4, 0.0)
    spec = with_(spec, bodies=[spec["bodies"][0], b])
    compare(spec, 2)


def test_rolling_impulses_zero_without_rolling_resistance():
    spec = with_(settled_column(seed=5, n=300, footprint=0.5), max_sweeps=20)
    g = T.scene_from_specs(spec)
    g.step(1)
    keys, _ = g.get_contacts(0)
    lr = g.get_rolling_impulses(0)
    assert lr.shape == (len(keys), 3) and not np.any(lr)


def one_sphere(r, mu_t, mu_r, v, w, sweeps):
    m = 2000.0 * 4.0 / 3.0 * math.pi * r ** 3
    estar = 1e9 / (2.0 * (1.0 - 0.15 ** 2))
    kn = estar * math.sqrt(2 * r) / 3.0
    d0 = (m * G / kn) ** (2.0 / 3.0)
    floor = dict(pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), linvel=(0.0, 0.0, 0.0), angvel=(0.0, 0.0, 0.0),
                 shapes=[dict(type="plane", n=(0.0, 0.0, 1.0), d=0.0)])
    spec = dict(x=SG.fp32([[0.0, 0.0, r - d0]]), r=SG.fp32([r]), v=SG.fp32([v]), w=SG.fp32([w]), id=np.arange(1),
                bodies=[floor], material=SG.material(mu_t, 0.0, mu_r=mu_r), dt=DT, gravity=(0.0, 0.0, -G),
                max_sweeps=sweeps, tol=0.0, warm_start="cold", grid_lo=(-1.0, -1.0, -1.0), grid_hi=(3.0, 1.0, 1.0),
                r_ref=0.05)
    return spec, m, d0


def test_single_sphere_rolling_deceleration_closed_form():
    r, mu_r, v0 = 0.05, 0.1, 1.5
    spec, m, d0 = one_sphere(r, 0.5, mu_r, [v0, 0.0, 0.0], [0.0, 0.0, 0.0], 400)
    # rolling without slip about the contact point at lever r - d0/2
    spec["w"] = SG.fp32([[0.0, float(spec["v"][0, 0]) / (r - d0 / 2), 0.0]])
    I = 0.4 * m * r * r
    l = r - d0 / 2
    expect = -l * r * mu_r * m * G * DT / (I + m * l * l)
    g = T.scene_from_specs(spec)
    vprev = float(spec["v"][0, 0])
    for k in range(20):
        g.step(1)
        v = g.get_particles(0)["v"][0, 0]
        assert v - vprev == pytest.approx(expect, rel=2e-3, abs=1e-5), k
        lr = g.get_rolling_impulses(0)
        assert np.linalg.norm(lr[0]) == pytest.approx(r * mu_r * m * G * DT, rel=1e-4)
        vprev = v


def test_single_sphere_spin_stops_closed_form():
    r, mu_r, w0 = 0.05, 0.2, 30.0
    spec, m, _ = one_sphere(r, 0.5, mu_r, [0.0, 0.0, 0.0], [0.0, 0.0, w0], 5)
    dw = 2.5 * mu_r * G * DT / r
    g = T.scene_from_specs(spec)
    wprev = w0
    for k in range(int(w0 / dw) + 3):
        g.step(1)
        wz = g.get_particles(0)["w"][0, 2]
        assert wz == pytest.approx(max(wprev - dw, 0.0), rel=1e-5, abs=1e-4), k
        wprev = max(wprev - dw, 0.0)
    assert abs(g.get_particles(0)["w"][0, 2]) < 1e-4


SCHEDULES = {
    "grouped": dict(mode="grouped", blocks_per_xcd=4, dataflow=0),
    "grouped_flow": dict(mode="grouped", blocks_per_xcd=4, dataflow=1),
    "per_env_lds": dict(mode="per_env", lds_particles=100000, cluster_particles=0),
    "per_env_global": dict(mode="per_env", lds_particles=0, cluster_particles=0),
    "per_env_solo": dict(mode="per_env", lds_particles=350, cluster_particles=-1),
    "per_env_clusters": dict(mode="per_env", lds_particles=350, cluster_particles=150, dataflow=0),
}


def rolling_batch():
    specs = [settled_column(seed=40, n=300, footprint=0.5), jammed_bed(seed=41, nx=12, ny=8, nz=6),
             settled_column(seed=42, n=500, footprint=0.6)]
    mat = dict(specs[0]["material"])
    mat["mu_r"] = 0.15
    return [with_(s, material=mat, max_sweeps=30, warm_start="prev") for s in specs]


def test_rolling_schedules_bitwise_identical_and_match_oracle():
    specs = rolling_batch()
    cap = max(len(s["x"]) for s in specs)
    states = {}
    for sched, cfg in SCHEDULES.items():
        g = T.scene_from_specs(specs, cap_particles=cap)
        g.set_solver_config(**cfg)
        g.step(2)
        states[sched] = [(g.get_particles(e)["w"].copy(), g.get_rolling_impulses(e).copy())
                         for e in range(len(specs))]
        if sched == "per_env_lds":
            for e, s in enumerate(specs):
                o = O.OracleScene(with_(s, id=e * cap + np.arange(len(s["x"]))))
                o.step()
                oo = o.step()
                assert np.array_equal(g.get_contacts(e)[0], oo["keys"])
                lt = 50e-4 * max(np.max(np.abs(oo["lam"])), 1e-12)
                assert np.max(np.abs(g.get_rolling_impulses(e) - oo["lr"])) <= lt, e
                tol = vel_tol(o.v) * 5
                assert np.max(np.abs(g.get_particles(e)["v"] - o.v)) <= tol, e
        g.close()
    ref = states["grouped"]
    for sched, st in states.items():
        for e in range(len(specs)):
            for a, b in zip(ref[e], st[e]):
                assert np.array_equal(a, b), (sched, e)


def test_rolling_save_load_resumes_exactly():
    specs = rolling_batch()
    cap = max(len(s["x"]) for s in specs)
    g = T.scene_from_specs(specs, cap_particles=cap)
    g.step(2)
    snap = g.save_state()
    g.step(2)
    ref = [(g.get_particles(e)["w"].copy(), g.get_rolling_impulses(e).copy()) for e in range(len(specs))]
    g.load_state(snap)
    g.step(2)
    for e in range(len(specs)):
        assert np.array_equal(g.get_particles(e)["w"], ref[e][0])
        assert np.array_equal(g.get_rolling_impulses(e), ref[e][1])
