"""Impact stage on the HIP path against the FP64 oracle and collision closed forms.

With v_imp > 0 a contact whose start-of-step normal velocity approaches faster
than v_imp gets the Newton law G_n v+ = -e G_n v- in a stage solved before the
main solve, every other contact of its env G v+ = 0; envs without impacts are
left as they are.  Bars: the closed forms of one or two spheres at FP32
accuracy; against the oracle bit-exact contact lists, the same impact count and
sweeps, velocities to the one-step bound, body forces to 1e-3.
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


def sphere_mass(r, rho=2000.0):
    return rho * 4.0 / 3.0 * math.pi * r ** 3


def impacting(spec, e, v_imp, **kw):
    return with_(spec, material=dict(spec["material"], restitution=e, v_imp=v_imp), **kw)


def free_spec(x, r, v, w=None, bodies=(), g=(0.0, 0.0, -G), mu=0.5, e=0.5, v_imp=1.0, sweeps=20):
    n = len(x)
    return dict(x=SG.fp32(x), r=SG.fp32(r), v=SG.fp32(v), w=SG.fp32(np.zeros((n, 3)) if w is None else w),
                id=np.arange(n), bodies=list(bodies), material=SG.material(mu, 0.0, restitution=e, v_imp=v_imp),
                dt=DT, gravity=g, max_sweeps=sweeps, tol=0.0, warm_start="cold", grid_lo=(-1.0, -1.0, -1.0),
                grid_hi=(1.0, 1.0, 1.0), r_ref=0.05)


def floor():
    return dict(id=0, pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), linvel=(0.0, 0.0, 0.0),
                angvel=(0.0, 0.0, 0.0), shapes=[dict(type="plane", n=(0.0, 0.0, 1.0), d=0.0)])


@pytest.mark.parametrize("e", [0.25, 1.0])
def test_bounce_closed_form(e):
    r, v0 = 0.05, 3.0
    m = sphere_mass(r)
    spec = free_spec([[0.0, 0.0, r - 1e-5]], [r], [[0.0, 0.0, -v0]], bodies=[floor()], e=e)
    g = T.scene_from_specs(spec)
    st = g.step(1)[0]
    assert st["impacts"] == 1 and st["impact_sweeps"] == 20
    vz = g.get_particles(0)["v"][0, 2]
    assert vz == pytest.approx(e * v0 - G * DT, rel=1e-5)
    f, _ = g.get_contact_forces(0, 0)
    assert f[2] == pytest.approx(-m * (1.0 + e) * v0 / DT, rel=1e-4)


def test_head_on_pair_closed_form():
    r1, r2, U1, U2, e = 0.05, 0.04, 1.5, 0.7, 0.3
    m1, m2 = sphere_mass(r1), sphere_mass(r2)
    spec = free_spec([[0.0, 0.0, 0.0], [r1 + r2 - 1e-5, 0.0, 0.0]], [r1, r2], [[U1, 0, 0], [-U2, 0, 0]],
                     g=(0.0, 0.0, 0.0), e=e, v_imp=0.5, sweeps=10)
    g = T.scene_from_specs(spec)
    assert g.step(1)[0]["impacts"] == 1
    v = g.get_particles(0)["v"]
    P = (1.0 + e) * (U1 + U2) / (1.0 / m1 + 1.0 / m2)
    assert v[0, 0] == pytest.approx(U1 - P / m1, rel=1e-5)
    assert v[1, 0] == pytest.approx(-U2 + P / m2, rel=1e-5)
    assert m1 * v[0, 0] + m2 * v[1, 0] == pytest.approx(m1 * U1 - m2 * U2, rel=1e-5)


@pytest.mark.parametrize("vx,mu,sticks", [(0.4, 0.5, True), (4.0, 0.2, False)])
def test_oblique_impact_stick_and_slip(vx, mu, sticks):
    r, v0, e, d0 = 0.05, 2.0, 0.4, 1e-5
    m = sphere_mass(r)
    I = 0.4 * m * r * r
    l = r - d0 / 2
    spec = free_spec([[0.0, 0.0, r - d0]], [r], [[vx, 0.0, -v0]], bodies=[floor()], mu=mu, e=e)
    g = T.scene_from_specs(spec)
    g.step(1)
    p = g.get_particles(0)
    Pn = m * (1.0 + e) * v0
    Pstick = vx / (1.0 / m + l * l / I)
    assert (Pstick <= mu * Pn) == sticks
    Pt = Pstick if sticks else mu * Pn
    assert p["v"][0, 0] == pytest.approx(vx - Pt / m, rel=2e-5)
    assert p["w"][0, 1] == pytest.approx(l * Pt / I, rel=2e-5)
    assert p["v"][0, 2] == pytest.approx(e * v0 - G * DT, rel=2e-5)


def compare(spec, steps, g=None, env=0, rel=1e-4, forces=False):
    g = g or T.scene_from_specs(spec)
    o = O.OracleScene(spec)
    impacts = []
    for k in range(steps):
        st = g.step(1)[env]
        oo = o.step()
        keys, lam = g.get_contacts(env)
        assert np.array_equal(keys, oo["keys"]), k
        assert st["impacts"] == oo["impacts"], (k, st["impacts"], oo["impacts"])
        assert st["impact_sweeps"] == oo["impact_sweeps"] and st["sweeps"] == oo["sweeps"]
        impacts.append(st["impacts"])
        p = g.get_particles(env)
        tol = vel_tol(o.v, rel=rel) * (1 + 4 * k)
        assert np.max(np.abs(p["v"] - o.v)) <= tol, (k, np.max(np.abs(p["v"] - o.v)), tol)
        wtol = tol / max(float(np.min(spec["r"])), 1e-3)
        assert np.max(np.abs(p["w"] - o.w)) <= wtol, (k, np.max(np.abs(p["w"] - o.w)), wtol)
        lt = 10 * rel * max(np.max(np.abs(oo["lam"])), 1e-12) * (1 + 4 * k)
        assert np.max(np.abs(lam - oo["lam"])) <= lt
        if forces and k == 0:
            for bi in range(len(spec["bodies"])):
                f, _ = g.get_contact_forces(env, bi)
                fo = oo["body_ft"][bi][:3]
                assert np.linalg.norm(f - fo) <= 1e-3 * max(np.linalg.norm(fo), 1.0), (bi, f, fo)
    return impacts


def test_column_hit_from_above_matches_oracle():
    # a settled column whose upper half is thrown down onto the lower half
    spec = settled_column(seed=6, n=600, footprint=0.6, c=0.0, mu=0.5)
    rng = np.random.default_rng(8)
    v = np.array(spec["v"])
    top = spec["x"][:, 2] > np.median(spec["x"][:, 2])
    v[top, 2] -= rng.uniform(0.5, 3.0, int(top.sum()))
    spec = impacting(with_(spec, v=SG.fp32(v), max_sweeps=40), e=0.3, v_imp=1.0)
    impacts = compare(spec, 2, forces=True)
    assert impacts[0] > 50


def test_bed_with_fast_blade_and_rolling_matches_oracle():
    # a blade pushed into the bed at 3 m/s: its contacts are impacts
    spec = jammed_bed(seed=33, nx=16, ny=10, nz=8, r0=0.03, sweeps=50, blade=True)
    blade = dict(spec["bodies"][1])
    blade["linvel"] = (3.0, 0.0, 0.0)
    spec = with_(spec, bodies=[spec["bodies"][0], blade])
    spec = impacting(with_(spec, material=dict(spec["material"], mu_r=0.1)), e=0.2, v_imp=1.0)
    impacts = compare(spec, 2, forces=True)
    assert impacts[0] >= 5  # the spheres the blade face meets


SCHEDULES = {
    "grouped": dict(mode="grouped", blocks_per_xcd=4, dataflow=0),
    "per_env_lds": dict(mode="per_env", lds_particles=100000, cluster_particles=0),
    "per_env_global": dict(mode="per_env", lds_particles=0, cluster_particles=0),
    "per_env_solo": dict(mode="per_env", lds_particles=350, cluster_particles=-1),
    "per_env_clusters": dict(mode="per_env", lds_particles=350, cluster_particles=150, dataflow=0),
    "per_env_clusters_flow": dict(mode="per_env", lds_particles=350, cluster_particles=150, dataflow=1),
}


def mixed_batch():
    # env 0 and 2 with impacts, env 1 without (settled, slow)
    a = settled_column(seed=40, n=300, footprint=0.5, c=0.0, mu=0.5)
    b = settled_column(seed=41, n=400, footprint=0.5, c=0.0, mu=0.5)
    c = settled_column(seed=42, n=500, footprint=0.6, c=0.0, mu=0.5)
    rng = np.random.default_rng(3)
    out = []
    for k, s in enumerate((a, b, c)):
        v = np.array(s["v"])
        if k != 1:
            top = s["x"][:, 2] > np.median(s["x"][:, 2])
            v[top, 2] -= rng.uniform(1.0, 3.0, int(top.sum()))
        out.append(impacting(with_(s, v=SG.fp32(v), max_sweeps=25, material=a["material"]), e=0.4, v_imp=1.0))
    return out


def test_schedules_bitwise_equal_and_envs_as_if_alone():
    specs = mixed_batch()
    cap = max(len(s["x"]) for s in specs)
    states = {}
    for sched, cfg in SCHEDULES.items():
        g = T.scene_from_specs(specs, cap_particles=cap)
        g.set_solver_config(**cfg)
        st = g.step(1)
        assert st[0]["impacts"] > 0 and st[1]["impacts"] == 0 and st[2]["impacts"] > 0
        states[sched] = [g.get_particles(e)["v"].copy() for e in range(len(specs))]
        if sched == "per_env_lds":
            for e, s in enumerate(specs):
                o = O.OracleScene(with_(s, id=e * cap + np.arange(len(s["x"]))))
                oo = o.step()
                assert st[e]["impacts"] == oo["impacts"]
                assert np.max(np.abs(states[sched][e] - o.v)) <= vel_tol(o.v), e
        g.close()
    for sched, st in states.items():
        for e in range(len(specs)):
            assert np.array_equal(states["grouped"][e], st[e]), (sched, e)
