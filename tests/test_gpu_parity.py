"""Parity of the HIP path (through the C-ABI) against the FP64 oracle.

Both sides start from the same seeded FP32-representable state; nothing the
GPU produces is fed to the oracle.  Bars:
  - contact lists: bit-exact sorted keys; colours identical per key;
  - one-step velocities: |v_gpu - v_orc|_inf <= 1e-4 max(|v_orc|_inf, g dt)
    (FP32 PGS against FP64, same schedule);
  - impulses: same bound scaled by the largest impulse;
  - FP64 aggregate reductions: 1e-12 relative on identical states.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from helpers import jammed_bed, settled_column, vel_tol, with_
from paper_2011_00459_amd import scenegen as SG

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")


def gpu_scene(specs, **kw):
    return T.scene_from_specs(specs, **kw)


def compare_step(spec, gpu_steps=1, rel=1e-4, check_lam=True, env=0, sc=None):
    """Run gpu_steps on both sides from spec; compare after each step."""
    g = sc or gpu_scene(spec)
    o = O.OracleScene(spec)
    for k in range(gpu_steps):
        st = g.step(1)[env]
        oo = o.step()
        keys, lam = g.get_contacts(env)
        assert st["overflow"] == 0
        assert np.array_equal(keys, oo["keys"]), f"step {k}: contact keys differ"
        assert st["contacts"] == oo["contacts"]
        assert st["pair_contacts"] == oo["pair_contacts"]
        assert st["colours"] == oo["colours"]
        assert np.array_equal(g.get_colours(env), oo["colour"]), f"step {k}: colours differ"
        assert st["sweeps"] == oo["sweeps"]
        p = g.get_particles(env)
        tol = vel_tol(o.v, rel=rel) * (1 + 4 * k)
        assert np.max(np.abs(p["v"] - o.v)) <= tol, (k, np.max(np.abs(p["v"] - o.v)), tol)
        wtol = tol / max(float(np.min(spec["r"])), 1e-3)
        assert np.max(np.abs(p["w"] - o.w)) <= wtol
        assert np.max(np.abs(p["x"] - o.x)) <= spec["dt"] * tol + 2e-7 * (1 + np.max(np.abs(o.x)))
        if check_lam and len(keys):
            lref = oo["lam"]
            lt = rel * max(np.max(np.abs(lref)), 1e-12) * (1 + 4 * k) * 10
            assert np.max(np.abs(lam - lref)) <= lt, (k, np.max(np.abs(lam - lref)), lt)
        assert st["residual"] == pytest.approx(oo["residual"], rel=2e-2, abs=1e-6)
    return g, o


def test_library_loads_and_scene_roundtrip():
    spec = settled_column(n=200, footprint=0.5)
    g = gpu_scene(spec)
    p = g.get_particles(0)
    assert np.array_equal(p["x"], spec["x"])
    assert np.array_equal(p["r"], spec["r"])
    assert np.array_equal(p["v"], spec["v"])


def test_column_contacts_bit_exact_and_one_step_parity():
    spec = settled_column()
    compare_step(spec, 1)


def test_column_prev_warm_start_three_steps():
    spec = with_(settled_column(), warm_start="prev", max_sweeps=60)
    compare_step(spec, 3)


def test_column_cold_fixed_sweeps_cohesionless():
    spec = settled_column(seed=2, n=600, footprint=0.8, c=0.0, mu=0.4)
    compare_step(with_(spec, max_sweeps=40), 2)


def test_jammed_bed_with_blade_one_step():
    spec = jammed_bed(nx=30, ny=16, nz=10)
    g, o = compare_step(spec, 1)
    f, t = g.get_contact_forces(0, 1)
    ft = o.last["body_ft"][1]
    scale = max(np.max(np.abs(ft[:3])), 1.0)
    assert np.max(np.abs(f - ft[:3])) <= 1e-3 * scale
    tscale = max(np.max(np.abs(ft[3:])), 1.0)
    assert np.max(np.abs(t - ft[3:])) <= 1e-3 * tscale


def test_blade_pushing_into_column_forces_and_aggregate():
    base = settled_column(seed=3, n=800, footprint=1.0)
    blade = SG.box_blade(-0.55, 0.02, width=0.9, height=0.5, vx=1.0,
                         zone_planes=[[-1.0, 0.0, 0.0, -0.02], [1.0, 0.0, 0.0, 0.6], [0.0, 0.0, 1.0, 0.8]])
    bodies = list(base["bodies"]) + [blade]
    spec = with_(base, bodies=bodies, max_sweeps=80)
    g, o = compare_step(spec, 4)
    f, _ = g.get_contact_forces(0, 1)
    ft = o.last["body_ft"][1]
    assert np.linalg.norm(ft[:3]) > 0.0
    assert np.max(np.abs(f - ft[:3])) <= 2e-3 * max(np.max(np.abs(ft[:3])), 1.0)
    ag = g.get_aggregates(0)
    oa = o.last["aggregates"]
    assert len(ag) == len(oa) == 1
    assert ag[0]["n_particles"] == oa[0]["n_particles"] > 0
    assert ag[0]["M"] == pytest.approx(oa[0]["M"], rel=1e-12)
    assert np.allclose(ag[0]["x"], oa[0]["x"], rtol=0, atol=1e-6)
    assert np.allclose(ag[0]["v"], oa[0]["v"], rtol=0, atol=1e-3 * max(1.0, np.max(np.abs(oa[0]["v"]))))


def test_boundary_shapes_bit_exact():
    # tilted heightfield floor, rotated box and planes, dense random spheres
    rng = np.random.default_rng(31)
    n = 3000
    r = SG.fp32(0.04 * rng.uniform(0.9, 1.1, n))
    x = SG.fp32(np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-0.2, 0.6, n)], axis=1))
    l0, nn = 0.125, 17
    xs = -1.0 + l0 * np.arange(nn)
    hh = (0.1 * np.sin(3 * xs)[None, :] + 0.05 * np.cos(2 * xs)[:, None]).astype(np.float32)
    hf = dict(pos=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0),
              shapes=[dict(type="hfield", nx=nn, ny=nn, ox=-1.0, oy=-1.0, l0=l0, h=hh.ravel())])
    ang = 0.3
    box = dict(pos=(0.1, -0.2, 0.3), quat=(math.cos(ang / 2), 0.2 * math.sin(ang / 2), 0.0,
                                         math.sqrt(1 - 0.04) * math.sin(ang / 2)),
               linvel=(0.5, 0.0, 0.0), angvel=(0.0, 0.0, 0.4),
               shapes=[dict(type="box", half=(0.3, 0.05, 0.2), off=(0.05, 0.0, 0.0)),
                       dict(type="box", half=(0.1, 0.4, 0.02), off=(0.0, 0.1, -0.2))])
    walls = SG.walls_body(2.0, 2.0, -0.5, True)
    spec = SG._spec(x, r, [hf, box, walls], SG.material(0.5, 1500.0), 1.0 / 60.0, 30,
                    ((-1.2, -1.2, -0.7), (1.2, 1.2, 0.9)), 0.04)
    keys_o, _ = O.detect(spec)
    g = gpu_scene(spec)
    g.step(1)
    keys_g, _ = g.get_contacts(0)
    assert len(keys_o) > n
    nb = np.sum((keys_o & np.uint64(0x80000000)) > 0)
    assert nb > 200
    assert np.array_equal(keys_g, keys_o)


def test_fp64_aggregate_reduction_exact_state():
    # no contacts, no gravity, dyadic dt and velocities: x + dt v is exact in
    # FP32, so both sides aggregate the same state
    rng = np.random.default_rng(8)
    n = 5000
    gridpts = np.stack(np.meshgrid(np.arange(20), np.arange(25), np.arange(10), indexing="ij"), -1).reshape(-1, 3)
    x = (gridpts[:n] * 0.25 - np.array([2.5, 3.0, 1.0])).astype(np.float64)
    v = np.round(rng.uniform(-1, 1, (n, 3)) * 64) / 64
    w = SG.fp32(rng.normal(0, 2.0, (n, 3)))
    r = SG.fp32(0.05 * rng.uniform(0.9, 1.1, n))
    zone = [[1.0, 0.0, 0.0, 1.0], [-1.0, 0.0, 0.0, 2.0], [0.0, 0.0, 1.0, 0.75], [0.2, 0.9, 0.0, 1.5]]
    body = dict(pos=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0), zone_planes=zone, shapes=[])
    spec = SG._spec(x, r, [body], SG.material(0.5, 0.0), 1.0 / 64.0, 5, ((-3, -3.5, -1.5), (3, 3.5, 1.5)), 0.05)
    spec = with_(spec, v=v, w=w, gravity=(0.0, 0.0, 0.0))
    g = gpu_scene(spec)
    st = g.step(1)[0]
    assert st["contacts"] == 0
    o = O.OracleScene(spec)
    o.step()
    p = g.get_particles(0)
    assert np.array_equal(p["x"], o.x) and np.array_equal(p["v"], o.v)
    ag, oa = g.get_aggregates(0)[0], o.last["aggregates"][0]
    assert ag["n_particles"] == oa["n_particles"] > 100
    assert ag["M"] == pytest.approx(oa["M"], rel=1e-13)
    for k in ("x", "v", "I", "w"):
        scale = max(np.max(np.abs(oa[k])), 1e-12)
        assert np.max(np.abs(ag[k] - oa[k])) <= 1e-12 * scale, k


def test_batched_envs_match_single_env_oracle():
    specs = [settled_column(seed=4, n=300, footprint=0.5), settled_column(seed=5, n=500, footprint=0.6),
             jammed_bed(seed=6, nx=12, ny=8, nz=6)]
    sweeps = 50
    specs = [with_(s, max_sweeps=sweeps, material=specs[0]["material"]) for s in specs]
    cap = max(len(s["x"]) for s in specs)
    g = gpu_scene(specs, cap_particles=cap)
    st = g.step(1)
    for e, s in enumerate(specs):
        # env e owns ids [e cap, (e + 1) cap): the oracle gets the same ids
        o = O.OracleScene(with_(s, id=e * cap + np.arange(len(s["x"]))))
        oo = o.step()
        keys, lam = g.get_contacts(e)
        assert np.array_equal(keys, oo["keys"])
        assert np.array_equal(g.get_colours(e), oo["colour"])
        assert st[e]["contacts"] == oo["contacts"]
        p = g.get_particles(e)
        # colours are shared across envs: the schedule of each env is its own
        # JP colouring, so per-env velocities match the single-env oracle
        assert np.max(np.abs(p["v"] - o.v)) <= vel_tol(o.v)


def test_runs_are_bitwise_deterministic():
    spec = with_(settled_column(seed=7, n=700, footprint=0.8), warm_start="prev", max_sweeps=40)
    outs = []
    for _ in range(2):
        g = gpu_scene(spec)
        g.step(3)
        p = g.get_particles(0)
        k, lam = g.get_contacts(0)
        outs.append((p["x"].copy(), p["v"].copy(), p["w"].copy(), k.copy(), lam.copy()))
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_contact_capacity_overflow_leaves_state_unchanged():
    spec = settled_column(n=400, footprint=0.6)
    g = gpu_scene(spec, cap_contacts=64)
    before = g.get_particles(0)
    with pytest.raises(T.TerrainError) as ei:
        g.step(1)
    assert ei.value.code == T.TR_E_CAPACITY
    after = g.get_particles(0)
    for k in ("x", "v", "w"):
        assert np.array_equal(before[k], after[k])


def test_capacity_failure_is_reported_by_every_step_call():
    # the failure flags of every step of a call are read back whether or not
    # stats are asked for, and reported once
    spec = settled_column(n=400, footprint=0.6)
    g = gpu_scene(spec, cap_contacts=64)
    before = g.get_particles(0)
    for stats in (False, True):
        with pytest.raises(T.TerrainError) as ei:
            g.step(3, stats=stats)
        assert ei.value.code == T.TR_E_CAPACITY
    after = g.get_particles(0)
    for k in ("x", "v", "w"):
        assert np.array_equal(before[k], after[k])
    # with few enough spheres left the steps succeed: no stale flag survives
    g.remove_particles(0, np.arange(5, len(spec["x"])))
    g.step(2, stats=False)
    st = g.step(1)[0]
    assert st["overflow"] == 0 and 0 < st["contacts"] <= 64


def test_tolerance_stopping_matches_oracle():
    spec = with_(settled_column(seed=9, n=500, footprint=0.7), tol=5e-3, max_sweeps=500)
    g = gpu_scene(spec)
    st = g.step(1)[0]
    o = O.OracleScene(spec)
    oo = o.step()
    assert 1 < oo["sweeps"] < 500
    assert abs(st["sweeps"] - oo["sweeps"]) <= 1
    assert st["residual"] <= 5e-3
    assert np.max(np.abs(g.get_particles(0)["v"] - o.v)) <= vel_tol(o.v, rel=3e-3)


def test_empty_env_and_no_contacts():
    spec = SG._spec(np.array([[0.0, 0.0, 1.0]]), np.array([0.05]), [SG.walls_body(1, 1)],
                    SG.material(0.5, 0.0), 1.0 / 60.0, 10, ((-1, -1, -0.2), (1, 1, 2)), 0.05)
    g = gpu_scene(spec)
    st = g.step(2)[0]
    assert st["contacts"] == 0 and st["overflow"] == 0
    p = g.get_particles(0)
    assert p["v"][0, 2] == pytest.approx(-2 * 9.81 / 60.0, rel=1e-6)


def test_particle_capacity_limit():
    # the solver addresses each particle's 32 B velocity record with a 31-bit
    # byte offset: at most 2^26 particle slots over all envs
    with pytest.raises(T.TerrainError) as ei:
        T.Scene(n_envs=2, cap_particles=(1 << 25) + 1, cap_contacts=16, env_bounds=[(0, 0, 0, 1, 1, 1)] * 2)
    assert ei.value.code == T.TR_E_CAPACITY
