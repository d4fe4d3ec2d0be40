"""Active-zone predictor of the oracle (Eq. failure_plane on a heightfield).

Pins, each against geometry fixed independently of the predictor's code:
  - level terrain, vertical blade: the union of the lateral wedges is the
    host builder's single wedge (Rankine angle pi/4 - phi/2), and the failure
    line meets the surface at depth / tan(theta);
  - terrain sloped along the cut: beta and theta follow the surface, the
    meeting point solves the line-plane intersection in closed form;
  - the paper's worked angles (beta 42 deg -> theta 47, 45 -> 45 at
    phi = 44.5 deg, parity unpinned: the printed values are rounded);
  - the fill ratio moves the secondary separation plate between the
    primary plate and the inner face;
  - a step in the terrain across the edge gives the wedges on each side
    their own top; an edge above the surface and a slow deformer give none;
  - the oracle step aggregates exactly the particles inside the wedges.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG
from paper_2011_00459_amd import zones as Z


def terrain(h, nx=60, ny=60, ox=-3.0, oy=-3.0, l0=0.1):
    hh = np.asarray(h(ox + l0 * np.arange(nx)[None, :], oy + l0 * np.arange(ny)[:, None]), dtype=np.float32)
    return dict(pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0),
                shapes=[dict(type="hfield", nx=nx, ny=ny, ox=ox, oy=oy, l0=l0, h=hh.ravel())])


def blade_body(v=(1.0, 0.0, 0.0), pos=(0.0, 0.0, 0.0)):
    return dict(pos=pos, quat=(1.0, 0.0, 0.0, 0.0), linvel=v, angvel=(0.0, 0.0, 0.0), shapes=[])


def slope_of(W):
    """Angle of the failure plane (the wedge's second plane) against horizontal."""
    n = W[1, :3]
    return math.atan2(abs(n[0]), abs(n[2]))


def test_level_terrain_vertical_blade_is_the_rankine_wedge():
    phi = math.radians(35.0)
    surf, edge_z, heap, width = 0.5, 0.2, 0.1, 1.0
    bodies = [terrain(lambda x, y: 0 * x + 0 * y + surf), blade_body()]
    tool = dict(body=1, n_wedges=5, edge0=(0.0, -width / 2, edge_z), edge1=(0.0, width / 2, edge_z), n_c=(1, 0, 0),
                phi=phi, heap=heap)
    W = O.predict_wedges(tool, bodies)
    assert len(W) == 5 and all(len(w) == 5 for w in W)
    theta = math.pi / 4 - phi / 2
    for w in W:
        assert slope_of(w) == pytest.approx(theta, abs=1e-12)
        assert w[2, 3] == pytest.approx(surf + heap, abs=1e-9)  # where the failure line meets the surface, + heap
    # the union of the wedges is the host builder's wedge (away from slice borders)
    ref = Z.wedge_planes(edge_x=0.0, edge_z=edge_z, width=width, top_z=surf + heap, phi=phi)
    rng = np.random.default_rng(1)
    x = rng.uniform([-0.2, -0.7, 0.0], [1.2, 0.7, 0.8], (20000, 3))
    x = x[np.min(np.abs(x[:, 1:2] - np.linspace(-0.5, 0.5, 6)[None, :]), axis=1) > 1e-6]
    assert np.array_equal(O.inside_wedges(W, x), Z.inside(ref, x))
    assert np.sum(Z.inside(ref, x)) > 500


@pytest.mark.parametrize("alpha", [0.15, -0.1])
def test_sloped_terrain_along_the_cut(alpha):
    # surface z = h0 + alpha x; vertical blade: beta = pi/2 - atan(alpha), the
    # failure line leaves the edge at theta above the surface, i.e. at
    # theta + atan(alpha) above horizontal, and meets the plane where
    # edge_z + L sin(g) = h0 + alpha L cos(g)
    phi, h0, edge_z = math.radians(30.0), 0.6, 0.25
    bodies = [terrain(lambda x, y: h0 + alpha * x + 0 * y), blade_body()]
    tool = dict(body=1, n_wedges=1, edge0=(0.0, -0.3, edge_z), edge1=(0.0, 0.3, edge_z), n_c=(1, 0, 0), phi=phi)
    (w,) = O.predict_wedges(tool, bodies)
    a = math.atan(alpha)
    beta = math.pi / 2 - a
    theta = math.pi / 2 - (phi + beta) / 2
    g = theta + a
    # (the grid holds FP32 heights: the slope is exact to their rounding)
    assert slope_of(w) == pytest.approx(g, abs=2e-6)
    L = (h0 - edge_z) / (math.sin(g) - alpha * math.cos(g))
    assert w[2, 3] == pytest.approx(edge_z + L * math.sin(g), rel=2e-6)


@pytest.mark.parametrize("beta_deg,theta_printed", [(42.0, 47.0), (45.0, 45.0)])
def test_worked_angles_of_the_paper(beta_deg, theta_printed):
    # a plate leaning towards the zone at beta against level ground
    phi = math.radians(44.5)
    b = math.radians(beta_deg)
    n_c = (math.sin(b), 0.0, -math.cos(b))  # normal of a plate rising at beta towards +x
    bodies = [terrain(lambda x, y: 0 * x + 0 * y + 0.5), blade_body()]
    tool = dict(body=1, n_wedges=1, edge0=(0.0, -0.3, 0.2), edge1=(0.0, 0.3, 0.2), n_c=n_c, phi=phi)
    (w,) = O.predict_wedges(tool, bodies)
    theta = math.degrees(slope_of(w))
    assert theta == pytest.approx(90.0 - (44.5 + beta_deg) / 2, abs=1e-9)
    assert round(theta) == theta_printed


def test_fill_moves_the_separation_plate():
    phi = math.radians(35.0)
    bodies = [terrain(lambda x, y: 0 * x + 0 * y + 0.5), blade_body()]
    b0, b1 = math.radians(30.0), math.radians(80.0)
    n_c = (math.sin(b0), 0.0, -math.cos(b0))
    n_tc = (math.sin(b1), 0.0, -math.cos(b1))
    base = dict(body=1, n_wedges=1, edge0=(0.0, -0.3, 0.2), edge1=(0.0, 0.3, 0.2), n_c=n_c, n_tc=n_tc, phi=phi)
    for fill, beta in ((0.0, b0), (1.0, b1), (0.5, 0.5 * (b0 + b1))):
        (w,) = O.predict_wedges(dict(base, fill=fill), bodies)
        # half way between two unit normals is their bisector: beta averages
        assert slope_of(w) == pytest.approx(math.pi / 2 - (phi + beta) / 2, abs=1e-12)
    with pytest.raises(ValueError):
        O.predict_wedges(dict(base, fill=1.5), bodies)


def test_terrain_step_across_the_edge_and_empty_wedges():
    phi = math.radians(35.0)
    bodies = [terrain(lambda x, y: np.where(y < 0.0, 0.5, 0.7) + 0 * x), blade_body()]
    tool = dict(body=1, n_wedges=4, edge0=(0.0, -1.0, 0.2), edge1=(0.0, 1.0, 0.2), n_c=(1, 0, 0), phi=phi, heap=0.05)
    W = O.predict_wedges(tool, bodies)
    tops = [w[2, 3] for w in W]
    # (surface heights are FP32 values)
    assert tops[0] == pytest.approx(float(np.float32(0.5)) + 0.05, abs=1e-9)
    assert tops[3] == pytest.approx(float(np.float32(0.7)) + 0.05, abs=1e-9)
    # the edge above the surface: no zone
    high = dict(tool, edge0=(0.0, -1.0, 0.9), edge1=(0.0, 1.0, 0.9))
    assert all(len(w) == 0 for w in O.predict_wedges(high, bodies))
    # a deformer below its speed threshold: no zone; above it: the wedges
    assert all(len(w) == 0 for w in O.predict_wedges(dict(tool, v_min=2.0), bodies))
    fast = [terrain(lambda x, y: np.where(y < 0.0, 0.5, 0.7) + 0 * x), blade_body(v=(3.0, 0.0, 0.0))]
    assert all(len(w) == 5 for w in O.predict_wedges(dict(tool, v_min=2.0), fast))


def test_oracle_step_aggregates_the_particles_in_the_wedges():
    # particles held still (no gravity, no sweeps, no contacts between them):
    # the step's aggregate is the sum over the particles inside the wedges
    phi = math.radians(35.0)
    rng = np.random.default_rng(5)
    x = SG.fp32(rng.uniform([-0.3, -0.6, 0.25], [1.0, 0.6, 0.7], (400, 3)))
    bodies = [terrain(lambda x, y: 0 * x + 0 * y + 0.5), blade_body(v=(0.0, 0.0, 0.0))]
    tool = dict(body=1, n_wedges=3, edge0=(0.0, -0.5, 0.2), edge1=(0.0, 0.5, 0.2), n_c=(1, 0, 0), phi=phi, heap=0.1)
    spec = dict(x=x, r=np.full(400, 0.004), v=np.zeros((400, 3)), w=np.zeros((400, 3)), id=np.arange(400),
                bodies=bodies, tools=[tool], material=SG.material(0.5, 0.0), dt=1.0 / 60.0, gravity=(0.0, 0.0, 0.0),
                max_sweeps=0, tol=0.0, warm_start="cold", grid_lo=(-0.5, -0.8, 0.0), grid_hi=(1.2, 0.8, 1.0),
                r_ref=0.05)
    out = O.OracleScene(spec).step()
    W = O.predict_wedges(tool, bodies)
    inside = O.inside_wedges(W, x)
    assert inside.sum() > 20
    (agg,) = out["aggregates"]
    assert agg["zone"] == 1 and agg["n_particles"] == int(inside.sum())
    m = 2000.0 * 4.0 / 3.0 * math.pi * 0.004 ** 3
    assert agg["M"] == pytest.approx(m * inside.sum(), rel=1e-12)
    assert np.allclose(agg["x"], np.mean(x[inside], axis=0), rtol=0, atol=1e-12)
