"""Active-zone wedge builder (Eq. failure_plane) on the CPU.

  - the builder's failure angle is the oracle's theta(phi, beta) and reduces to
    Rankine's pi/4 - phi/2 for a vertical blade on level ground;
  - membership: points in front of the blade face and above the failure plane
    are inside, points below the plane, behind the face, above the top or
    beyond the sides are outside, and points on the plane's exact slope from
    the cutting edge sit on the boundary;
  - the oracle's aggregate of a zone built this way counts the particles that
    lie inside the wedge.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG
from paper_2011_00459_amd import zones as Z


@pytest.mark.parametrize("phi,beta", [(0.3, math.pi / 2), (0.6, math.pi / 2), (0.6, 1.2), (0.9, 1.8)])
def test_failure_angle_matches_oracle_and_rankine(phi, beta):
    assert Z.failure_angle(phi, beta) == pytest.approx(O.failure_angle(phi, beta), rel=1e-15)
    if beta == math.pi / 2:
        assert Z.failure_angle(phi, beta) == pytest.approx(math.pi / 4 - phi / 2, rel=1e-15)


def test_wedge_geometry():
    phi = Z.friction_angle(0.7)
    theta = Z.failure_angle(phi)
    planes = Z.wedge_planes(edge_x=0.025, edge_z=-0.3, width=1.5, top_z=0.5, phi=phi)
    assert len(planes) <= 8
    t = math.tan(theta)
    pts = np.array([
        [0.025 + 0.2, 0.0, -0.3 + 0.2 * t + 0.01],   # above the failure plane, in front: in
        [0.025 + 0.2, 0.0, -0.3 + 0.2 * t - 0.01],   # just below the plane: out
        [0.0, 0.0, 0.0],                             # behind the face: out
        [0.5, 0.0, 0.6],                             # above the top: out
        [0.025 + 0.2, 0.8, -0.3 + 0.2 * t + 0.01],   # beyond the side: out
        [0.025 + 0.1, -0.7, 0.2],                    # inside near the other side: in
    ])
    assert list(Z.inside(planes, pts)) == [True, False, False, False, False, True]
    # the failure plane passes through the cutting edge with slope tan(theta)
    n = np.array(planes[1][:3])
    d = planes[1][3]
    for s in (0.0, 0.3, 0.7):
        p = np.array([0.025 + s, 0.2, -0.3 + s * t])
        assert n @ p == pytest.approx(d, abs=1e-12)
    # a steeper separation plane (beta < pi/2, face leaning forward) steepens the wedge
    assert Z.failure_angle(phi, 1.2) > Z.failure_angle(phi, math.pi / 2)


def test_oracle_aggregate_of_a_built_zone_counts_the_wedge():
    rng = np.random.default_rng(3)
    blade = SG.box_blade(-1.0, 0.2, width=1.0, thick=0.05, height=0.6, vx=0.0)
    planes = Z.blade_zone(blade, mu=0.7, surface_z=0.8, heap=0.3)
    blade["zone_planes"] = planes
    # particles in the world around the blade (the blade frame is translated only)
    x = rng.uniform([-1.2, -0.8, 0.0], [0.2, 0.8, 1.2], (4000, 3))
    y = x - np.asarray(blade["pos"])
    expect = int(np.sum(Z.inside(planes, y)))
    agg = O.aggregates(x, np.zeros_like(x), np.zeros_like(x), [0.01] * len(x), [1.0] * len(x), [blade])
    assert expect > 100
    assert agg[0]["n_particles"] == expect
