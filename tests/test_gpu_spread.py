"""The spread schedule: one env's contacts on all eight XCDs (its sorted
spheres in eighths, the groups meeting after every colour, every body store
written through).  Within a colour no two contacts share a sphere, so the
schedule changes where the updates run, not their order: states are bitwise
those of the grouped schedule, and match the FP64 oracle to the usual bars."""
import numpy as np
import pytest

import pyoracle as O
from helpers import jammed_bed, settled_column, vel_tol, with_

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")

SPREAD = dict(mode="spread", blocks_per_xcd=32, lds_particles=0, cluster_particles=0, dataflow=0)
GROUPED = dict(mode="grouped", blocks_per_xcd=32, lds_particles=0, cluster_particles=0, dataflow=0)


def cases():
    col = with_(settled_column(seed=31, n=1000, footprint=1.0), max_sweeps=40, warm_start="prev")
    bed = jammed_bed(seed=32, nx=30, ny=16, nz=10, r0=0.03, sweeps=60)
    mat = dict(bed["material"], mu_r=0.1)
    return {
        "column_prev": col,
        "bed_blade": bed,
        "bed_rolling": with_(bed, material=mat),
        "bed_impact": with_(bed, material=dict(bed["material"], v_imp=0.05, restitution=0.3),
                            v=np.tile([0.0, 0.0, -0.4], (len(bed["x"]), 1))),
    }


@pytest.mark.parametrize("name", ["column_prev", "bed_blade", "bed_rolling", "bed_impact"])
def test_spread_is_bitwise_the_grouped_schedule(name):
    spec = cases()[name]
    out = {}
    for label, cfg in (("grouped", GROUPED), ("spread", SPREAD)):
        g = T.scene_from_specs(spec)
        g.set_solver_config(**cfg)
        assert g.get_solver_config()["mode"] == label
        st = g.step(3)[0]
        p = g.get_particles(0)
        keys, lam = g.get_contacts(0)
        out[label] = (st, p["x"].copy(), p["v"].copy(), p["w"].copy(), keys.copy(), lam.copy(),
                      g.get_rolling_impulses(0).copy(), g.get_contact_forces(0, len(spec["bodies"]) - 1)[0])
        g.close()
    a, b = out["grouped"], out["spread"]
    assert a[0]["sweeps"] == b[0]["sweeps"] and a[0]["colours"] == b[0]["colours"]
    assert a[0]["contacts"] == b[0]["contacts"] > 0
    for u, v in zip(a[1:], b[1:]):
        assert np.array_equal(u, v), name


def test_spread_bed50k_one_step_matches_oracle():
    spec = jammed_bed(seed=21, nx=60, ny=30, nz=28, r0=0.03, sweeps=150)
    n = len(spec["x"])
    g = T.scene_from_specs(spec, cap_contacts=16 * n)
    g.set_solver_config(**SPREAD)
    st = g.step(1)[0]
    o = O.OracleScene(spec)
    oo = o.step()
    keys, lam = g.get_contacts(0)
    assert np.array_equal(keys, oo["keys"])
    assert np.array_equal(g.get_colours(0), oo["colour"])
    assert st["sweeps"] == oo["sweeps"] == 150
    p = g.get_particles(0)
    assert np.max(np.abs(p["v"] - o.v)) <= vel_tol(o.v)
    assert st["residual"] == pytest.approx(oo["residual"], rel=2e-2, abs=1e-6)


def test_spread_tolerance_stops_with_the_oracle():
    spec = with_(settled_column(seed=9, n=500, footprint=0.7), tol=5e-3, max_sweeps=500)
    g = T.scene_from_specs(spec)
    g.set_solver_config(**SPREAD)
    st = g.step(1)[0]
    o = O.OracleScene(spec)
    oo = o.step()
    assert 1 < oo["sweeps"] < 500
    assert abs(st["sweeps"] - oo["sweeps"]) <= 1
    assert st["residual"] <= 5e-3
    assert np.max(np.abs(g.get_particles(0)["v"] - o.v)) <= vel_tol(o.v, rel=3e-3)


def test_spread_takes_one_env():
    specs = [settled_column(seed=4, n=300, footprint=0.5), settled_column(seed=5, n=300, footprint=0.5)]
    g = T.scene_from_specs(specs, cap_particles=300)
    with pytest.raises(T.TerrainError):
        g.set_solver_config(**SPREAD)
