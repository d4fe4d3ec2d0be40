"""Seeded synthetic scene generators (numpy PCG64).

These build the inputs of both the GPU path and the FP64 oracle: particle
positions, radii and velocities rounded to FP32 (so both sides start from the
same state), the kinematic bodies with their shapes, and the step parameters.
The module holds none of the method's arithmetic: it only places spheres on
jittered lattices (non-overlapping by construction) and describes boundaries.

The workloads stand in for the paper's bulldozing and excavation beds (section
"Simulation tests": 45-55 mm spheres at 2200 kg/m^3, a 1.6 m blade cutting at
0.05 m depth, a 1.2 x 1.2 x 0.9 m bucket) at the sizes of the benchmark
configurations: a 1,000-sphere column, a 50,000-sphere bed with a box blade,
256 batched beds of log-uniform size, and a 500,000-sphere excavation bed.
"""
from __future__ import annotations

import math

import numpy as np

G = 9.81


def fp32(a):
    """Round to FP32 and return float64 holding exactly those values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def material(mu=0.6, c=1000.0, rho=2000.0, **kw):
    m = dict(rho=rho, mu_t=mu, mu_r=0.0, c_p=c, E=1e9, nu=0.15, restitution=0.0,
             tau_n=0.0, gamma_t=0.0, kappa_c=0.025, kappa_min=1e-4, v_imp=0.0)
    m.update(kw)
    return m


def walls_body(lx, ly, floor_z=0.0, walls=True, body_id=0):
    """Static body with a floor plane z = floor_z and four side walls."""
    shapes = [dict(type="plane", n=(0.0, 0.0, 1.0), d=floor_z)]
    if walls:
        shapes += [dict(type="plane", n=(1.0, 0.0, 0.0), d=-lx / 2),
                   dict(type="plane", n=(-1.0, 0.0, 0.0), d=-lx / 2),
                   dict(type="plane", n=(0.0, 1.0, 0.0), d=-ly / 2),
                   dict(type="plane", n=(0.0, -1.0, 0.0), d=-ly / 2)]
    return dict(id=body_id, pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), linvel=(0.0, 0.0, 0.0),
                angvel=(0.0, 0.0, 0.0), shapes=shapes)


def box_blade(x, z_bottom, width=1.5, thick=0.05, height=0.6, vx=1.0, body_id=1, heading=0.0,
              zone_planes=None):
    """Kinematic box blade: thickness along the heading, width across, bottom at z_bottom."""
    c, s = math.cos(heading / 2), math.sin(heading / 2)
    vel = (vx * math.cos(heading), vx * math.sin(heading), 0.0)
    b = dict(id=body_id, pos=(x, 0.0, z_bottom + height / 2), quat=(c, 0.0, 0.0, s),
             linvel=vel, angvel=(0.0, 0.0, 0.0),
             shapes=[dict(type="box", half=(thick / 2, width / 2, height / 2), off=(0.0, 0.0, 0.0))])
    if zone_planes is not None:
        b["zone_planes"] = zone_planes
    return b


def open_bucket(x, z_bottom, width=1.0, length=0.8, height=0.6, plate=0.02, vx=1.0, body_id=1,
                heading=0.0, zone_planes=None):
    """Open-box bucket: bottom, back and two side plates; open top and front (+x)."""
    c, s = math.cos(heading / 2), math.sin(heading / 2)
    vel = (vx * math.cos(heading), vx * math.sin(heading), 0.0)
    hw, hl, hh, hp = width / 2, length / 2, height / 2, plate / 2
    shapes = [
        dict(type="box", half=(hl, hw, hp), off=(0.0, 0.0, -hh + hp)),          # bottom
        dict(type="box", half=(hp, hw, hh), off=(-hl + hp, 0.0, 0.0)),          # back
        dict(type="box", half=(hl, hp, hh), off=(0.0, -hw + hp, 0.0)),          # side
        dict(type="box", half=(hl, hp, hh), off=(0.0, hw - hp, 0.0)),           # side
    ]
    b = dict(id=body_id, pos=(x, 0.0, z_bottom + hh), quat=(c, 0.0, 0.0, s), linvel=vel,
             angvel=(0.0, 0.0, 0.0), shapes=shapes)
    if zone_planes is not None:
        b["zone_planes"] = zone_planes
    return b


def lattice(rng, n, lx, ly, spacing, r, z0=0.0, jitter=True):
    """n non-overlapping sphere centres on a cubic lattice over an lx x ly
    footprint centred at the origin, layer by layer from z0, each jittered
    within its lattice cell by at most (spacing/2 - r)."""
    nx = max(1, int(lx // spacing))
    ny = max(1, int(ly // spacing))
    layers = int(math.ceil(n / (nx * ny)))
    i = np.arange(n)
    ix = i % nx
    iy = (i // nx) % ny
    iz = i // (nx * ny)
    x = -nx * spacing / 2 + spacing / 2 + ix * spacing
    y = -ny * spacing / 2 + spacing / 2 + iy * spacing
    z = z0 + spacing / 2 + iz * spacing
    pos = np.stack([x, y, z], axis=1)
    if jitter:
        room = np.maximum(spacing / 2 - r, 0.0)[:, None] * 0.98
        pos = pos + rng.uniform(-1.0, 1.0, size=(n, 3)) * room
    return pos, layers * spacing + z0


def _spec(x, r, bodies, mat, dt, sweeps, bounds, r_ref, v=None, tol=0.0, warm="cold"):
    n = len(x)
    return dict(x=fp32(x), v=fp32(v if v is not None else np.zeros((n, 3))), w=np.zeros((n, 3)),
                r=fp32(r), rho=None, id=np.arange(n, dtype=np.int64), bodies=bodies,
                material=mat, dt=dt, gravity=(0.0, 0.0, -G), max_sweeps=sweeps, tol=tol,
                warm_start=warm, grid_lo=tuple(bounds[0]), grid_hi=tuple(bounds[1]), r_ref=r_ref)


def column_scene(seed=1, n=1000, r0=0.05, spread=0.1, footprint=1.0, fill=0.3, mu=0.6, c=1000.0,
                 sweeps=100, dt=1.0 / 60.0, walls=True):
    """Loose random column: n spheres of radius r0 U(1-spread/2, 1+spread/2)
    over a square footprint with floor and four walls, volume fill `fill`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = r0 * rng.uniform(1 - spread, 1 + spread, size=n)
    rmax = r0 * (1 + spread)
    s = max((4.0 / 3.0 * math.pi * r0 ** 3 / fill) ** (1.0 / 3.0), 2.0 * rmax * 1.02)
    x, top = lattice(rng, n, footprint, footprint, s, r)
    bodies = [walls_body(footprint, footprint, 0.0, walls)]
    h = footprint / 2 + 2 * s
    bounds = ((-h, -h, -2 * s), (h, h, top + 2 * s))
    return _spec(x, r, bodies, material(mu, c), dt, sweeps, bounds, r0)


def bed_scene(seed=2, n=50000, r0=0.03, spread=0.1, lx=4.0, ly=2.0, mu=0.7, c=2000.0, sweeps=150,
              dt=1.0 / 60.0, tool="blade", tool_speed=1.0, depth=0.2, settled_top=None,
              tool_x=None, heading=0.0):
    """Dense bed of n spheres (r0 U(1-spread, 1+spread)) over lx x ly with floor
    and walls, and a kinematic tool (box blade or open bucket) cutting along
    the heading at `depth` below the bed top, moving at tool_speed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = r0 * rng.uniform(1 - spread, 1 + spread, size=n)
    rmax = r0 * (1 + spread)
    s = 2.0 * rmax * 1.01
    x, top = lattice(rng, n, lx, ly, s, r)
    bed_top = settled_top if settled_top is not None else top
    bodies = [walls_body(lx, ly, 0.0, True)]
    tx = tool_x if tool_x is not None else -lx / 2 + 0.4
    if tool == "blade":
        bodies.append(box_blade(tx, bed_top - depth, vx=tool_speed, heading=heading))
    elif tool == "bucket":
        bodies.append(open_bucket(tx, bed_top - depth, vx=tool_speed, heading=heading))
    bounds = ((-lx / 2 - 2 * s, -ly / 2 - 2 * s, -2 * s), (lx / 2 + 2 * s, ly / 2 + 2 * s, top + 0.5))
    return _spec(x, r, bodies, material(mu, c), dt, sweeps, bounds, r0)


def batch_specs(seed=3000, n_envs=256, nmin=500, nmax=20000, sweeps=100, dt=1.0 / 60.0):
    """Independent beds of log-uniform particle counts: each a 3 x 2 m
    footprint filled to 0.5 m at packing 0.6 (radius from N), mu 0.7,
    c 2 kPa, with a blade or an open bucket on a random heading, depth and
    speed."""
    return [batch_spec(seed, e, nmin, nmax, sweeps, dt) for e in range(n_envs)]


def batch_spec(seed, e, nmin=500, nmax=20000, sweeps=100, dt=1.0 / 60.0):
    """Bed e of batch_specs(seed, ...) alone."""
    rng = np.random.Generator(np.random.PCG64(seed + e))
    ns = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    rs = (0.6 * 3.0 * 3.0 / (4.0 * math.pi * ns)) ** (1.0 / 3.0)
    tool = "blade" if rng.uniform() < 0.5 else "bucket"
    heading = math.radians(rng.uniform(-20.0, 20.0))
    depth = rng.uniform(0.1, 0.3)
    speed = rng.uniform(0.3, 1.5)
    return bed_scene(seed=seed + e, n=ns, r0=rs, spread=0.1, lx=3.0, ly=2.0, mu=0.7, c=2000.0,
                     sweeps=sweeps, dt=dt, tool=tool, tool_speed=speed, depth=depth,
                     settled_top=0.5, tool_x=-1.1, heading=heading)


def excavation_scene(seed=5, n=500000, sweeps=200, dt=1.0 / 60.0):
    """500k spheres r 0.02 U(0.85, 1.15) over 8 x 4 m and a 1.2 x 1.0 x 0.8 bucket."""
    rng_probe = bed_scene(seed=seed, n=n, r0=0.02, spread=0.15, lx=8.0, ly=4.0, mu=0.7, c=2000.0,
                          sweeps=sweeps, dt=dt, tool="none")
    top = float(rng_probe["grid_hi"][2]) - 0.5
    bucket = open_bucket(-3.5, top - 0.4, width=1.2, length=1.0, height=0.8, vx=0.8)
    rng_probe["bodies"].append(bucket)
    return rng_probe


def jammed_bed(seed=21, nx=40, ny=20, nz=12, r0=0.03, spread=0.002, jitter=0.001, blade=True, sweeps=150,
               mu=0.7, c=2000.0, dt=1.0 / 60.0):
    """A dense cubic packing at spacing 2 r0 with radii r0 U(1-spread, 1+spread):
    about half of the lattice neighbours overlap by up to 2 spread r0 (a jammed
    bed resting on its floor), with a box blade cutting into its top."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = 2.0 * r0
    i = np.arange(nx * ny * nz)
    ix, iy, iz = i % nx, (i // nx) % ny, i // (nx * ny)
    x = np.stack([(ix - (nx - 1) / 2) * s, (iy - (ny - 1) / 2) * s, r0 + iz * s], axis=1)
    x += rng.uniform(-1, 1, x.shape) * jitter * r0
    n = len(x)
    r = r0 * rng.uniform(1 - spread, 1 + spread, n)
    lx, ly = nx * s, ny * s
    top = r0 + (nz - 1) * s + r0
    bodies = [walls_body(lx + 1e-3, ly + 1e-3, 0.0, True)]
    if blade:
        bodies.append(box_blade(-lx / 2 + 0.2, top - 0.1, width=0.6 * ly, height=0.4, vx=1.0))
    bounds = ((-lx / 2 - 2 * s, -ly / 2 - 2 * s, -2 * s), (lx / 2 + 2 * s, ly / 2 + 2 * s, top + 0.6))
    return _spec(x, r, bodies, material(mu, c), dt, sweeps, bounds, r0)


def ulp_nudge(x, seed):
    """x (FP32 values held in float64) with every coordinate moved by one FP32
    ulp up or down, the direction drawn per coordinate: an ensemble of starts
    that FP32 cannot tell apart, for statistics of chaotic trajectories."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x32 = np.asarray(x, dtype=np.float32)
    up = rng.integers(0, 2, x32.shape).astype(bool)
    out = np.where(up, np.nextafter(x32, np.float32(np.inf)), np.nextafter(x32, np.float32(-np.inf)))
    return out.astype(np.float64)


def voxel_workload(seed=11, dims=(256, 256, 128), l0=0.05, dt=1.0 / 60.0, rho_f=1600.0, courant=0.4):
    """Mesoscale grid of a dig site: fluidized soil (bulk density rho_f, in
    kg per voxel) filling an ellipsoidal zone ahead of a tool with a ragged
    fill fraction, zero elsewhere; the velocity is a swirl about the zone's
    axis plus noise, everywhere on the grid, scaled so that no face's Courant
    number exceeds `courant`.  Arrays shaped (nz, ny, nx) and (nz, ny, nx, 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    q = ((x - 0.5 * nx) / (0.3 * nx)) ** 2 + ((y - 0.5 * ny) / (0.2 * ny)) ** 2 + ((z - 0.3 * nz) / (0.25 * nz)) ** 2
    fill = np.clip(rng.uniform(0.0, 1.2, q.shape), 0.0, 1.0) * (q < 1.0)
    mf = rho_f * l0 ** 3 * fill
    u = np.empty(q.shape + (3,))
    u[..., 0] = -(y - 0.5 * ny) / ny + 0.2
    u[..., 1] = (x - 0.5 * nx) / nx
    u[..., 2] = 0.3 * np.sin(2 * np.pi * x / nx)
    u += rng.normal(0.0, 0.1, u.shape)
    u *= courant * l0 / dt / np.max(np.abs(u))  # a face's |u_f| is at most the larger of its two voxels'
    return dict(mf=mf, u=u, origin=(0.0, 0.0, 0.0), l0=l0, dims=dims, dt=dt)


def voxel_terrain(seed=12, dims=(256, 256, 128), l0=0.05, fluid_share=0.05, particle_share=0.3):
    """Resting soil on the voxel grid: columns filled to a rolling terrain
    height (a broad mound, ripples and noise, between 40 % and 75 % of the
    grid's height), compaction U(0.85, 1), fluidized mass (kg) in a random
    `fluid_share` of the voxels above the surface, and a particle density
    marker (1 where particles are, 0 elsewhere) in a random `particle_share`
    of those.  phi: the occupancy of columns filled to h from the grid's
    bottom.  Arrays shaped (nz, ny, nx); h (ny, nx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = dims
    y, x = np.meshgrid((np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx, indexing="ij")
    top = nz * l0
    h = top * (0.55 + 0.12 * np.exp(-((x - 0.6) ** 2 + (y - 0.4) ** 2) / 0.05) + 0.04 * np.sin(9 * x) * np.cos(7 * y))
    h = np.clip(h + rng.normal(0.0, 0.2 * l0, h.shape), 0.4 * top, 0.75 * top)
    h = np.asarray(h, dtype=np.float32).astype(np.float64)  # the heights a heightfield holds
    zb = l0 * np.arange(nz)
    phi = np.clip((h[None, :, :] - zb[:, None, None]) / l0, 0.0, 1.0)
    wc = rng.uniform(0.85, 1.0, phi.shape)
    above = phi == 0.0
    mf = np.where(above & (rng.uniform(size=phi.shape) < fluid_share), rng.uniform(0.0, 0.25, phi.shape), 0.0)
    rho_p = np.where((mf > 0) & (rng.uniform(size=phi.shape) < particle_share), 1.0, 0.0)
    return dict(phi=phi, wc=wc, mf=mf, rho_p=rho_p, h=h, origin=(0.0, 0.0, 0.0), l0=l0, dims=dims, rho_b=1800.0,
                w_dep=0.85)

