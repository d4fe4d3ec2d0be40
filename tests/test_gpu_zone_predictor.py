"""Active-zone predictor on the HIP path against the FP64 oracle.

The predictor runs after the step's pose update, one thread per (tool, wedge),
in FP64 with the oracle's operations: the wedges' half-spaces must agree to
1e-9 (the bisection's last steps and the math library's last bits may
differ), the empty wedges exactly; the aggregates of particles held still
(no gravity, no sweeps) must equal the oracle's membership exactly; for a
layer of spheres on the terrain pushed by a moving blade the aggregates agree
to the dynamics' FP32 bar.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from helpers import with_
from paper_2011_00459_amd import scenegen as SG

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")

DT = 1.0 / 60.0


def terrain(h, nx=60, ny=60, ox=-3.0, oy=-3.0, l0=0.1):
    hh = np.asarray(h(ox + l0 * np.arange(nx)[None, :], oy + l0 * np.arange(ny)[:, None]), dtype=np.float32)
    return dict(pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), linvel=(0.0, 0.0, 0.0), angvel=(0.0, 0.0, 0.0),
                shapes=[dict(type="hfield", nx=nx, ny=ny, ox=ox, oy=oy, l0=l0, h=hh.ravel())])


def tool_body(pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), v=(1.0, 0.0, 0.0), w=(0.0, 0.0, 0.0)):
    return dict(pos=pos, quat=quat, linvel=v, angvel=w,
                shapes=[dict(type="box", half=(0.02, 0.6, 0.3), off=(-0.02, 0.0, 0.5))])


def scene_spec(bodies, tools, x=None, sweeps=0, g=(0.0, 0.0, 0.0)):
    x = SG.fp32([[2.5, 2.5, 1.5]] if x is None else x)  # (a scene holds at least one sphere)
    n = len(x)
    return dict(x=x, r=SG.fp32(np.full(n, 0.02)), v=np.zeros((n, 3)), w=np.zeros((n, 3)), id=np.arange(n), bodies=bodies,
                tools=tools, material=SG.material(0.5, 0.0), dt=DT, gravity=g, max_sweeps=sweeps, tol=0.0,
                warm_start="cold", grid_lo=(-1.5, -1.5, -0.5), grid_hi=(3.0, 3.0, 2.0), r_ref=0.05)


def advanced(body):
    # the oracle's pose update of one step (the predictor uses the end-of-step pose)
    sc = O.OracleScene(scene_spec([body], []))
    sc.step()
    (pose,) = sc.bb.poses()
    return dict(body, pos=tuple(pose["pos"]), quat=tuple(pose["quat"]))


def check_wedges(g, bodies, tool, body_id=1):
    gw = g.get_zone_wedges(0, body_id)
    ow = O.predict_wedges(tool, [bodies[0], advanced(bodies[1])])
    assert len(gw) == len(ow)
    for a, b in zip(gw, ow):
        assert a.shape == b.shape
        if len(a):
            assert np.max(np.abs(a - b)) <= 1e-9 * (1.0 + np.max(np.abs(b))), (a, b)
    return gw


PHI = math.radians(35.0)
CASES = {
    "level": (lambda x, y: 0 * x + 0 * y + 0.5, dict(edge0=(0, -0.5, 0.2), edge1=(0, 0.5, 0.2), n_c=(1, 0, 0))),
    "slope": (lambda x, y: 0.6 + 0.15 * x + 0.05 * y, dict(edge0=(0, -0.5, 0.25), edge1=(0, 0.5, 0.25), n_c=(1, 0, 0))),
    "step": (lambda x, y: np.where(y < 0.0, 0.5, 0.7) + 0 * x, dict(edge0=(0, -1, 0.2), edge1=(0, 1, 0.2), n_c=(1, 0, 0))),
    "fill": (lambda x, y: 0 * x + 0 * y + 0.5,
             dict(edge0=(0, -0.5, 0.2), edge1=(0, 0.5, 0.2), n_c=(0.5, 0, -math.sqrt(0.75)), n_tc=(0.98, 0, -0.2),
                  fill=0.35)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_wedges_match_oracle(case):
    h, geo = CASES[case]
    bodies = [terrain(h), tool_body()]
    tool = dict(body=1, n_wedges=6, phi=PHI, heap=0.05, **geo)
    g = T.scene_from_specs(scene_spec(bodies, [tool]))
    g.step(1)
    gw = check_wedges(g, bodies, tool)
    assert sum(len(w) > 0 for w in gw) == 6


def test_tilted_rotating_tool_and_deformer_gate():
    q = (math.cos(0.15), 0.0, math.sin(0.15), 0.0)  # pitched about y
    bodies = [terrain(lambda x, y: 0.55 + 0.1 * np.sin(2 * x) * np.cos(y)), tool_body(pos=(0.1, 0.0, 0.0), quat=q,
                                                                                       w=(0.0, 0.4, 0.2))]
    tool = dict(body=1, n_wedges=5, edge0=(0.0, -0.6, 0.2), edge1=(0.0, 0.6, 0.2), n_c=(1, 0, 0),
                n_tc=(0.9, 0, -0.4), fill=0.6, phi=PHI, heap=0.1)
    g = T.scene_from_specs(scene_spec(bodies, [tool]))
    g.step(1)
    check_wedges(g, bodies, tool)
    # a deformer slower than its threshold has no zone
    g2 = T.scene_from_specs(scene_spec(bodies, [dict(tool, v_min=5.0)]))
    g2.step(1)
    assert all(len(w) == 0 for w in g2.get_zone_wedges(0, 1))


def test_aggregates_of_still_particles_match_the_oracle_membership():
    rng = np.random.default_rng(5)
    x = SG.fp32(rng.uniform([-0.3, -0.7, 0.22], [1.2, 0.7, 0.75], (3000, 3)))
    bodies = [terrain(lambda x, y: 0.5 + 0.05 * x + 0 * y), tool_body(v=(0.0, 0.0, 0.0))]
    tool = dict(body=1, n_wedges=4, edge0=(0.0, -0.5, 0.2), edge1=(0.0, 0.5, 0.2), n_c=(1, 0, 0), phi=PHI, heap=0.1)
    spec = scene_spec(bodies, [tool], x=x)
    g = T.scene_from_specs(spec)
    g.step(1)
    out = O.OracleScene(spec).step()
    (oa,) = out["aggregates"]
    (ga,) = g.get_aggregates(0)
    assert oa["n_particles"] > 100
    assert ga["n_particles"] == oa["n_particles"]
    assert ga["M"] == pytest.approx(oa["M"], rel=1e-12)
    assert np.allclose(ga["x"], oa["x"], rtol=0, atol=1e-12)


def test_layer_on_terrain_with_moving_blade_tool_matches_oracle():
    # a layer of spheres resting on the terrain surface; the blade's edge cuts
    # 0.1 m below the surface, its zone reaches 0.2 m above it
    r, surf = 0.03, 0.3
    gx, gy, gz = np.meshgrid(np.arange(-0.4, 1.4, 2 * r), np.arange(-0.5, 0.5, 2 * r), np.arange(3), indexing="ij")
    rng = np.random.default_rng(2)
    x = np.stack([gx.ravel(), gy.ravel(), surf + r * (1 + 2 * gz.ravel()) - 1e-4], 1)
    x[:, :2] += rng.uniform(-1e-3, 1e-3, (len(x), 2))
    bodies = [terrain(lambda x, y: 0 * x + 0 * y + surf),
              tool_body(pos=(-0.5, 0.0, -0.3), v=(1.0, 0.0, 0.0))]
    tool = dict(body=1, n_wedges=4, edge0=(0.0, -0.6, 0.2), edge1=(0.0, 0.6, 0.2), n_c=(1, 0, 0),
                phi=math.atan(0.6), heap=0.2)
    spec = scene_spec(bodies, [tool], x=x, sweeps=40, g=(0.0, 0.0, -9.81))
    spec["r"] = SG.fp32(np.full(len(x), r))
    spec["material"] = SG.material(0.6, 0.0)
    g = T.scene_from_specs(spec)
    o = O.OracleScene(spec)
    for k in range(3):
        g.step(1)
        oo = o.step()
        (oa,) = oo["aggregates"]
        (ga,) = g.get_aggregates(0)
        assert oa["n_particles"] > 20
        # the states differ at the FP32 bar after a step: membership near a
        # boundary may flip for a particle or two
        assert abs(ga["n_particles"] - oa["n_particles"]) <= max(2, 0.01 * oa["n_particles"])
        assert ga["M"] == pytest.approx(oa["M"], rel=0.02)


def test_graph_replay_with_impacts_rolling_and_tool():
    # the step graphs capture the impact stage, the rolling rows and the
    # predictor; every replay is checked against eagerly launched steps
    r, surf = 0.03, 0.3
    gx, gy, gz = np.meshgrid(np.arange(-0.4, 1.0, 2 * r), np.arange(-0.4, 0.4, 2 * r), np.arange(3), indexing="ij")
    x = np.stack([gx.ravel(), gy.ravel(), surf + r + gz.ravel() * (2 * r - 2e-4) - 1e-4], 1)  # layers overlap
    v = np.zeros_like(x)
    v[x[:, 2] > surf + 3 * r, 2] = -2.0  # the top layer thrown down: impacts
    bodies = [terrain(lambda x, y: 0 * x + 0 * y + surf), tool_body(pos=(-0.5, 0.0, -0.3), v=(1.5, 0.0, 0.0))]
    tool = dict(body=1, n_wedges=3, edge0=(0.0, -0.6, 0.2), edge1=(0.0, 0.6, 0.2), n_c=(1, 0, 0),
                phi=math.atan(0.6), heap=0.2)
    spec = scene_spec(bodies, [tool], x=x, sweeps=20, g=(0.0, 0.0, -9.81))
    spec.update(r=SG.fp32(np.full(len(x), r)), v=SG.fp32(v), warm_start="prev",
                material=SG.material(0.6, 0.0, mu_r=0.1, restitution=0.3, v_imp=1.0))
    ga, gb = T.scene_from_specs(spec), T.scene_from_specs(spec)
    gb.set_step_graphs(False)
    for k in range(4):
        sa, sb = ga.step(1)[0], gb.step(1)[0]
        assert sa["impacts"] == sb["impacts"] and sa["contacts"] == sb["contacts"]
        if k == 0:
            assert sa["impacts"] > 0
        pa, pb = ga.get_particles(0), gb.get_particles(0)
        for q in ("x", "v", "w"):
            assert np.array_equal(pa[q], pb[q]), (k, q)
        (aa,), (ab,) = ga.get_aggregates(0), gb.get_aggregates(0)
        assert aa["n_particles"] == ab["n_particles"] and aa["M"] == ab["M"]
        assert np.array_equal(ga.get_rolling_impulses(0), gb.get_rolling_impulses(0))
        for wa, wb in zip(ga.get_zone_wedges(0, 1), gb.get_zone_wedges(0, 1)):
            assert np.array_equal(wa, wb)
