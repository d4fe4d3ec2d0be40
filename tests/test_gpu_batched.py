"""Batched scenes under every PGS schedule, against the single-env FP64 oracle.

A schedule only spreads the solve over the GPU differently (grouped XCD
barriers, one block per env with LDS or global bodies, multi-block clusters);
the contacts of one colour touch disjoint particles, so with a fixed sweep
count every schedule must give bitwise the same state.  Each env is also
compared with the oracle stepping that env alone: bit-exact contact keys and
colour counts, velocities to the one-step bar, and, with a residual
tolerance, the env's own stopping sweep.
"""
import numpy as np
import pytest

import pyoracle as O
from helpers import jammed_bed, settled_column, vel_tol, with_

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")

SCHEDULES = {
    "grouped": dict(mode="grouped", blocks_per_xcd=4, dataflow=0),
    "grouped_flow": dict(mode="grouped", blocks_per_xcd=4, dataflow=1),
    "per_env_lds": dict(mode="per_env", lds_particles=100000, cluster_particles=0),
    "per_env_global": dict(mode="per_env", lds_particles=0, cluster_particles=0),
    "per_env_solo": dict(mode="per_env", lds_particles=350, cluster_particles=-1),
    "per_env_clusters": dict(mode="per_env", lds_particles=350, cluster_particles=150, dataflow=0),
    "per_env_clusters_flow": dict(mode="per_env", lds_particles=350, cluster_particles=150, dataflow=1),
    # every env solved by one block, those that do not fit the 350 LDS slots
    # with their first slots in LDS and the rest in global memory
    "per_env_partial_lds": dict(mode="per_env", lds_particles=350, cluster_particles=600, dataflow=0),
    # the cost-model plan with a small LDS: sets and clusters
    "per_env_auto_small_lds": dict(mode="per_env", lds_particles=350, cluster_particles=0, dataflow=0),
}


def batch(seed0=40, **kw):
    """Four uneven envs: two settled columns, a jammed bed with a blade, a small column."""
    specs = [settled_column(seed=seed0, n=300, footprint=0.5), jammed_bed(seed=seed0 + 1, nx=12, ny=8, nz=6),
             settled_column(seed=seed0 + 2, n=500, footprint=0.6), settled_column(seed=seed0 + 3, n=120, footprint=0.3)]
    mat = specs[0]["material"]
    return [with_(s, material=mat, **kw) for s in specs]


def oracle_env(spec, e, cap, mlp=None):
    # env e owns ids [e cap, (e + 1) cap): the oracle gets the same ids
    return O.OracleScene(with_(spec, id=e * cap + np.arange(len(spec["x"]))), mlp=mlp)


def scene(specs, sched):
    cap = max(len(s["x"]) for s in specs)
    g = T.scene_from_specs(specs, cap_particles=cap)
    g.set_solver_config(**SCHEDULES[sched])
    return g, cap


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_schedule_matches_single_env_oracle(sched):
    specs = batch(max_sweeps=40)
    g, cap = scene(specs, sched)
    orcs = [oracle_env(s, e, cap) for e, s in enumerate(specs)]
    for k in range(2):
        st = g.step(1)
        for e, o in enumerate(orcs):
            oo = o.step()
            keys, _ = g.get_contacts(e)
            assert np.array_equal(keys, oo["keys"]), (sched, k, e)
            assert st[e]["contacts"] == oo["contacts"]
            assert st[e]["colours"] == oo["colours"], (sched, e, st[e]["colours"], oo["colours"])
            assert np.array_equal(g.get_colours(e), oo["colour"]), (sched, k, e)
            assert st[e]["sweeps"] == oo["sweeps"]
            p = g.get_particles(e)
            assert np.max(np.abs(p["v"] - o.v)) <= vel_tol(o.v) * (1 + 4 * k), (sched, k, e)


def test_schedules_give_bitwise_identical_states():
    specs = batch(max_sweeps=30, warm_start="prev")
    states = {}
    for sched in SCHEDULES:
        g, _ = scene(specs, sched)
        g.step(2)
        states[sched] = [(g.get_particles(e)["v"].copy(), g.get_particles(e)["w"].copy(), g.get_contacts(e)[1].copy())
                         for e in range(len(specs))]
        g.close()
    ref = states["grouped"]
    for sched, st in states.items():
        for e in range(len(specs)):
            for a, b in zip(ref[e], st[e]):
                assert np.array_equal(a, b), (sched, e)


@pytest.mark.parametrize("sched", ["per_env_lds", "per_env_clusters", "per_env_clusters_flow"])
def test_per_env_tolerance_stops_each_env_on_its_own_residual(sched):
    specs = batch(seed0=50, tol=5e-3, max_sweeps=400)
    g, cap = scene(specs, sched)
    st = g.step(1)
    sweeps = []
    for e, s in enumerate(specs):
        o = oracle_env(s, e, cap)
        oo = o.step()
        assert 1 < oo["sweeps"] < 400
        assert abs(st[e]["sweeps"] - oo["sweeps"]) <= 1, (e, st[e]["sweeps"], oo["sweeps"])
        assert st[e]["residual"] <= 5e-3
        assert np.max(np.abs(g.get_particles(e)["v"] - o.v)) <= vel_tol(o.v, rel=3e-3)
        sweeps.append(st[e]["sweeps"])
    assert len(set(sweeps)) > 1  # the envs really stopped at different sweeps


def test_many_small_envs_per_env_mode():
    # more envs than blocks per XCD lane: several plan rows, padded lanes
    specs = [settled_column(seed=60 + e, n=int(60 + 37 * e), footprint=0.3 + 0.01 * e) for e in range(21)]
    mat = specs[0]["material"]
    specs = [with_(s, material=mat, max_sweeps=25) for s in specs]
    g, cap = scene(specs, "per_env_lds")
    assert g.get_solver_config()["mode"] == "per_env"
    st = g.step(1)
    for e in (0, 7, 13, 20):
        o = oracle_env(specs[e], e, cap)
        oo = o.step()
        keys, _ = g.get_contacts(e)
        assert np.array_equal(keys, oo["keys"])
        assert st[e]["colours"] == oo["colours"]
        assert np.array_equal(g.get_colours(e), oo["colour"])
        assert np.max(np.abs(g.get_particles(e)["v"] - o.v)) <= vel_tol(o.v)


def test_solver_config_validation():
    specs = batch(max_sweeps=5)
    g, _ = scene(specs, "grouped")
    with pytest.raises(T.TerrainError):
        g.set_solver_config(blocks_per_xcd=0)
    with pytest.raises(T.TerrainError):
        g.set_solver_config(lds_particles=-1)
    with pytest.raises(T.TerrainError):
        g.set_solver_config(dataflow=2)
    g.set_solver_config(mode="per_env", lds_particles=10 ** 9)
    c = g.get_solver_config()
    assert c["mode"] == "per_env" and 0 < c["lds_particles"] < 10 ** 9  # clamped to what LDS holds


@pytest.mark.parametrize("sched,warm", [("per_env_lds", "prev"), ("grouped", "cold")])
def test_graph_replay_matches_eager_steps(sched, warm):
    # every replay is checked against eagerly launched steps, with host reads
    # (synchronising copies) between the replays
    specs = batch(seed0=70, max_sweeps=20, warm_start=warm)
    ga, _ = scene(specs, sched)
    gb, _ = scene(specs, sched)
    gb.set_step_graphs(False)
    for k in range(5):
        sa, sb = ga.step(1), gb.step(1)
        for e in range(len(specs)):
            assert sa[e]["sweeps"] == sb[e]["sweeps"] and sa[e]["contacts"] == sb[e]["contacts"]
            pa, pb = ga.get_particles(e), gb.get_particles(e)
            for q in ("x", "v", "w"):
                assert np.array_equal(pa[q], pb[q]), (k, e, q)
            assert np.array_equal(ga.get_contacts(e)[1], gb.get_contacts(e)[1])
    # several steps in one call (replays back to back), then a schedule change
    ga.step(3, stats=False)
    gb.step(3, stats=False)
    ga.set_solver_config(mode="per_env" if sched == "grouped" else "grouped")
    ga.step(2)
    gb.step(2)
    for e in range(len(specs)):
        assert np.array_equal(ga.get_particles(e)["v"], gb.get_particles(e)["v"])


def test_phase_times_eager_and_replayed_steps():
    # an eager step times each phase; a step-graph replay only as a whole
    specs = batch(seed0=75, max_sweeps=10)
    g, _ = scene(specs, "grouped")
    g.set_step_graphs(False)
    g.step(2)
    ph = g.get_phase_times()
    assert all(np.isfinite(v) and v >= 0.0 for v in ph.values()), ph
    assert ph["pgs"] > 0.0 and ph["step"] >= ph["pgs"]
    g.set_step_graphs(True)
    for _ in range(2):
        g.step(1)
        ph = g.get_phase_times()
        assert all(np.isnan(ph[k]) for k in ("detect", "rows", "pgs", "finish")), ph
        assert np.isfinite(ph["step"]) and ph["step"] > 0.0
    g.set_step_graphs(False)
    g.step(1)
    assert np.isfinite(g.get_phase_times()["pgs"])


def test_save_load_state_resumes_exactly():
    specs = batch(seed0=80, max_sweeps=20, warm_start="prev")
    g, _ = scene(specs, "per_env_lds")
    g.step(3)
    snap = g.save_state()
    g.step(2)
    ref = [g.get_particles(e)["v"].copy() for e in range(len(specs))]
    g.load_state(snap)
    g.step(2)
    for e in range(len(specs)):
        assert np.array_equal(g.get_particles(e)["v"], ref[e])
    # a fresh scene of the same layout (another schedule) resumes the same way
    g2, _ = scene(specs, "grouped")
    g2.load_state(snap)
    g2.step(2)
    for e in range(len(specs)):
        assert np.array_equal(g2.get_particles(e)["v"], ref[e])
    # a scene with other envs refuses the snapshot
    g3, _ = scene(specs[:3], "grouped")
    with pytest.raises(T.TerrainError) as ei:
        g3.load_state(snap)
    assert ei.value.code == T.TR_E_STATE


def test_autotune_keeps_state_caches_and_changes_nothing(tmp_path):
    specs = batch(seed0=90, max_sweeps=20, warm_start="prev")
    cache = tmp_path / "tune.jsonl"
    g, _ = scene(specs, "grouped")
    g.step(2)
    before = [g.get_particles(e)["v"].copy() for e in range(len(specs))]
    cfg, ms = g.autotune(steps=2, cache_path=cache)
    assert ms > 0.0 and cache.exists()
    for e in range(len(specs)):  # the scene is left as it was
        assert np.array_equal(g.get_particles(e)["v"], before[e])
    g2, _ = scene(specs, "per_env_lds")
    g2.step(2)
    cfg2, ms2 = g2.autotune(steps=2, cache_path=cache)
    assert ms2 == -1.0 and cfg2 == cfg  # taken from the cache
    # a tuned schedule gives the same states as any other
    g.step(2)
    g3, _ = scene(specs, "grouped")
    g3.step(4)
    for e in range(len(specs)):
        assert np.array_equal(g.get_particles(e)["v"], g3.get_particles(e)["v"])


def test_two_contacts_per_thread_colours_are_bitwise_identical():
    # one block per XCD group: a colour of more than 512 contacts gives each
    # thread two (gathered together); the per-env schedule takes them one at
    # a time: the states must agree bit for bit, and with the oracle
    spec = jammed_bed(seed=61, nx=24, ny=16, nz=8)
    spec = with_(spec, max_sweeps=20, warm_start="prev")
    states = {}
    for name, cfg in (("grouped_1", dict(mode="grouped", blocks_per_xcd=1)), ("per_env", SCHEDULES["per_env_global"])):
        g = T.scene_from_specs(spec)
        g.set_solver_config(**cfg)
        st = g.step(2)
        states[name] = (g.get_particles(0), st[0])
    a, b = states["grouped_1"], states["per_env"]
    assert a[1]["contacts"] > 16 * 512  # colours of several hundred contacts
    for q in ("x", "v", "w"):
        assert np.array_equal(a[0][q], b[0][q]), q
    o = O.OracleScene(spec)
    o.step()
    o.step()
    assert np.max(np.abs(a[0]["v"] - o.v)) <= vel_tol(o.v) * 5
