"""Active-zone wedges of cutting tools as body-frame half-spaces.

The active zone in front of a cutting edge is a wedge bounded by the tool's
separation plane and the soil failure surface, approximated by a plane that
rises from the cutting edge to the free surface at the angle
theta(phi, beta) = pi/2 - (phi + beta)/2 against the terrain surface
(Eq. failure_plane: phi the soil's internal friction angle, beta the angle of
the separation plane against the terrain surface; a vertical blade on level
ground gives Rankine's pi/4 - phi/2).  Here the wedge is closed by a top
plane and two lateral planes at the tool's sides, which gives the up to 8
half-spaces `planes[k] . y <= d_k` that `set_kinematic_bodies` takes with a
body (the library moves them with the body's pose).

Body frame convention: the tool cuts along +x, z is up (the terrain surface
is the plane z = const of this frame), the cutting edge is the line
x = edge_x, z = edge_z, |y| <= width / 2.
"""
import math

import numpy as np


def failure_angle(phi, beta=math.pi / 2):
    """theta(phi, beta) of Eq. failure_plane (radians)."""
    return 0.5 * math.pi - 0.5 * (phi + beta)


def friction_angle(mu):
    """Internal friction angle from the contact friction coefficient: atan(mu)."""
    return math.atan(mu)


def wedge_planes(edge_x, edge_z, width, top_z, phi, beta=math.pi / 2):
    """Half-spaces (n, d) with n . y <= d of the active zone in front of a
    cutting edge, in the tool's body frame.

    - separation plane: through the edge at angle beta against the terrain,
      the zone on its front (+x) side;
    - failure plane: through the edge, rising towards +x at theta(phi, beta),
      the zone above it;
    - top: z <= top_z (the zone ends above the free surface, where the heap
      in front of the tool lies);
    - sides: |y| <= width / 2.
    """
    if not (0.0 < beta < math.pi):
        raise ValueError("beta must lie in (0, pi)")
    theta = failure_angle(phi, beta)
    if not (0.0 < theta < 0.5 * math.pi):
        raise ValueError(f"failure angle {theta} outside (0, pi/2) for phi={phi}, beta={beta}")
    e = np.array([edge_x, 0.0, edge_z])
    # separation plane: in-plane direction (cos beta, 0, sin beta) from the edge;
    # the zone lies where (sin beta, 0, -cos beta) . (y - e) >= 0
    n_sep = -np.array([math.sin(beta), 0.0, -math.cos(beta)])
    # failure plane: the zone lies where (sin theta, 0, -cos theta) . (y - e) <= 0
    n_fail = np.array([math.sin(theta), 0.0, -math.cos(theta)])
    planes = [
        (n_sep, float(n_sep @ e)),
        (n_fail, float(n_fail @ e)),
        (np.array([0.0, 0.0, 1.0]), float(top_z)),
        (np.array([0.0, 1.0, 0.0]), 0.5 * width),
        (np.array([0.0, -1.0, 0.0]), 0.5 * width),
    ]
    return [[float(n[0]), float(n[1]), float(n[2]), d] for n, d in planes]


def inside(planes, y):
    """Membership of body-frame points y (N x 3) in the zone."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    ok = np.ones(len(y), dtype=bool)
    for nx, ny, nz, d in planes:
        ok &= y @ np.array([nx, ny, nz]) <= d
    return ok


def blade_zone(blade, mu, surface_z, heap=0.5):
    """Zone half-spaces for a box blade description of scenegen (`box_blade`):
    the cutting edge is the blade's lower front edge, the separation plane its
    (vertical) front face, the soil friction angle atan(mu); the zone reaches
    `heap` above the free surface at `surface_z` (world z, level terrain, the
    blade upright)."""
    shape = blade["shapes"][0]
    half = np.asarray(shape["half"], dtype=np.float64)
    c = np.asarray(shape.get("off", (0.0, 0.0, 0.0)), dtype=np.float64)
    edge_x = c[0] + half[0]
    edge_z = c[2] - half[2]
    top = surface_z - blade["pos"][2] + heap
    return wedge_planes(edge_x, edge_z, 2.0 * half[1], top, friction_angle(mu))
