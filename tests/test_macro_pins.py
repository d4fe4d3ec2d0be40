"""Pins of the oracle's macroscale step: the aggregate body of a zone under
Eq. mdb:eqAgg with the constraints of Eqs. aggregateNormal and
aggregateTangent at its interfaces to the equipment (AB) and to the failure
surface (AC), four points each.

Expected values come from outside the oracle's code: hand-placed point sets
for the four-point reduction, closed forms of symmetric aggregates (a resting
aggregate, a cohesive one pulled away, one pushed by the equipment), the
momentum balance of the rigid body, and the optimality conditions of the
complementarity problem checked on the returned solution.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG

G = 9.81
DT = 1.0 / 60.0
R = 0.05
RHO = 2000.0


def sphere_mass(r=R):
    return RHO * 4.0 / 3.0 * math.pi * r ** 3


# ---------------------------------------------------------------------------
# the four-point reduction
# ---------------------------------------------------------------------------
def test_reduce4_picks_the_extremes_with_ties_to_the_smaller_index():
    # normal z: e1 = x, e2 = y
    pts = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [0.5, 0.5, 0]]
    assert O.reduce4(pts, [0, 0, 1]) == [1, 0, 2]      # +x: 1 (before 3), -x: 0, +y: 2, -y: 0 (kept once)
    # a cross: the four arm tips, in the order +e1, -e1, +e2, -e2
    cross = [[0, 0, 0], [2, 0, 0], [-2, 0, 0], [0, 3, 0], [0, -3, 0], [1, 0, 0]]
    assert O.reduce4(cross, [0, 0, 1]) == [1, 2, 3, 4]
    # normal x: the least aligned world axis is y (first of y, z), e1 = y, e2 = x * y = z
    pts = [[0, 0.2, 0.1], [0, -0.3, 0.0], [0, 0.0, 0.4], [0, 0.1, -0.5]]
    assert O.reduce4(pts, [1, 0, 0]) == [0, 1, 2, 3]
    # one candidate, none
    assert O.reduce4([[1, 2, 3]], [0, 0, 1]) == [0]
    assert O.reduce4(np.zeros((0, 3)), [0, 0, 1]) == []


# ---------------------------------------------------------------------------
# scenes: a blade at x = 0 (body 0 of the zone) with a box zone in front of it
# ---------------------------------------------------------------------------
ZONE = [[-1.0, 0.0, 0.0, 0.0],   # separation plate: x >= 0 (the blade face)
        [0.0, 0.0, -1.0, 0.0],   # failure plane: z >= 0 (level)
        [0.0, 0.0, 1.0, 1.0],    # top
        [0.0, 1.0, 0.0, 1.0],    # sides
        [0.0, -1.0, 0.0, 1.0],
        [1.0, 0.0, 0.0, 1.5]]    # front


def blade(linvel=(0.0, 0.0, 0.0)):
    return dict(pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), linvel=linvel, angvel=(0.0, 0.0, 0.0),
                shapes=[dict(type="box", half=(0.05, 1.0, 0.5), off=(-0.05, 0.0, 0.5))], zone_planes=ZONE)


def cross_layout(cx, cy, z, arms=2, s=2.2 * R):
    pts = [[cx, cy, z]]
    for k in range(1, arms + 1):
        pts += [[cx + k * s, cy, z], [cx - k * s, cy, z], [cx, cy + k * s, z], [cx, cy - k * s, z]]
    return pts


def spec_of(x, bodies, mu=0.5):
    n = len(x)
    return dict(x=np.asarray(x, dtype=np.float64), r=np.full(n, R), id=np.arange(n), bodies=bodies,
                material=SG.material(mu, 0.0), dt=DT, gravity=(0.0, 0.0, -G), max_sweeps=10, tol=0.0,
                warm_start="cold", grid_lo=(-2.0, -2.0, -2.0), grid_hi=(2.0, 2.0, 2.0), r_ref=R)


def resting_aggregate(cx=0.5, cy=0.1):
    # a bottom cross within R of the failure plane (the AC candidates) and a
    # second cross above it: symmetric about the aggregate's centre of mass
    z0 = 0.9 * R
    x = cross_layout(cx, cy, z0) + cross_layout(cx, cy, z0 + 3 * R)
    return np.asarray(x)


def test_resting_aggregate_closed_form():
    x = resting_aggregate()
    n = len(x)
    spec = spec_of(x, [blade()])
    out = O.macro_step(spec, x, np.zeros((n, 3)), np.zeros((n, 3)))
    assert len(out) == 1
    o = out[0]
    M = n * sphere_mass()
    assert o["M"] == pytest.approx(M, rel=1e-12)
    assert o["n_points"] == (0, 4) and o["n_cand"] == (0, 9)
    # the four arm tips of the bottom cross, projected onto the plane z = 0
    np.testing.assert_allclose(sorted(map(tuple, o["p"])), sorted([(0.5 + 2.2 * R * 2, 0.1, 0), (0.5 - 2.2 * R * 2, 0.1, 0),
                                                                   (0.5, 0.1 + 2.2 * R * 2, 0), (0.5, 0.1 - 2.2 * R * 2, 0)]),
                               atol=1e-15)
    np.testing.assert_allclose(o["n"], np.tile([0.0, 0.0, 1.0], (4, 1)))
    # interface area (cross sections of the candidates) and the regularisation
    # L / (c_as E_b A dt^2) with L the cube root of the solid volume
    A = 9 * math.pi * R * R
    L = (n * 4.0 / 3.0 * math.pi * R ** 3) ** (1.0 / 3.0)
    assert o["area"][1] == pytest.approx(A, rel=1e-12)
    gam = L / (0.001 * 1e7 * A * DT * DT)
    assert o["gamma"][1] == pytest.approx(gam, rel=1e-12)
    # four equal normal impulses: gamma lam + v_z = 0 with M v_z = -dt M g + 4 lam
    lam = DT * M * G / (M * gam + 4.0)
    np.testing.assert_allclose(o["lam"][:, 0], lam, rtol=1e-10)
    np.testing.assert_allclose(o["lam"][:, 1:], 0.0, atol=1e-12 * lam)
    np.testing.assert_allclose(o["v"], [0.0, 0.0, -gam * lam], rtol=1e-10, atol=1e-15)
    np.testing.assert_allclose(o["w"], 0.0, atol=1e-12)
    np.testing.assert_allclose(o["force_b"], 0.0, atol=1e-15)


@pytest.mark.parametrize("U,holds", [(0.25, True), (3.0, False)])
def test_cohesive_aggregate_pulled_off_the_failure_surface(U, holds):
    # moving up at U: the interface holds it with tension down to -c_b A dt / 4
    # per point, else it separates at that tension
    x = resting_aggregate()
    n = len(x)
    M = n * sphere_mass()
    v = np.tile([0.0, 0.0, U], (n, 1))
    c_b = 2000.0
    o = O.macro_step(spec_of(x, [blade()]), x, v, np.zeros((n, 3)), c_b=c_b)[0]
    gam = o["gamma"][1]
    lo = -c_b * o["area"][1] * DT / 4.0
    free = -M * (U - G * DT) / (4.0 + M * gam)
    if holds:
        assert lo < free < 0.0
        np.testing.assert_allclose(o["lam"][:, 0], free, rtol=1e-10)
        np.testing.assert_allclose(o["v"][2], -gam * free, rtol=1e-10)
    else:
        assert free < lo
        np.testing.assert_allclose(o["lam"][:, 0], lo, rtol=1e-12)
        np.testing.assert_allclose(o["v"][2], U - G * DT + 4.0 * lo / M, rtol=1e-10)


def test_equipment_pushing_a_frictionless_aggregate():
    # the blade moving at V along +x into the aggregate, frictionless on both
    # interfaces: the four AB points (a cross in the blade face, symmetric about
    # the centre of mass) give M v_x = 4 lam and v_x - V = -gamma_AB lam
    V = 0.8
    yc, zc = 0.0, 0.5
    s = 2.2 * R
    face = [[R - 0.01, yc, zc]] + [[R - 0.01, yc + d, zc] for d in (s, -s)] + \
           [[R - 0.01, yc, zc + d] for d in (s, -s)]
    back = [[p[0] + 4 * R, p[1], p[2]] for p in face]
    x = np.asarray(face + back)
    n = len(x)
    M = n * sphere_mass()
    o = O.macro_step(spec_of(x, [blade(linvel=(V, 0.0, 0.0))]), x, np.zeros((n, 3)), np.zeros((n, 3)),
                     mu_ab=0.0, mu_ac=0.0, c_b=0.0)[0]
    assert o["n_points"][0] == 4 and o["n_points"][1] == 0
    np.testing.assert_allclose(o["n"][:4], np.tile([1.0, 0.0, 0.0], (4, 1)), atol=1e-15)
    gam = o["gamma"][0]
    lam = V / (4.0 / M + gam)
    np.testing.assert_allclose(o["lam"][:4, 0], lam, rtol=1e-10)
    np.testing.assert_allclose(o["v"], [4.0 * lam / M, 0.0, -G * DT], rtol=1e-10, atol=1e-14)
    # the aggregate pushes back on the blade: -4 lam / dt along x
    np.testing.assert_allclose(o["force_b"], [-4.0 * lam / DT, 0.0, 0.0], rtol=1e-10, atol=1e-9)


def kkt_residuals(o, spec, mu_ab, mu_ac):
    """Optimality of the returned impulses: momentum balance of the rigid body
    and, per point, the normal complementarity and the friction disk with
    maximal dissipation (independent of how the problem was solved)."""
    M = o["M"]
    J = o["lam"][:, :1] * o["n"] + o["lam"][:, 1:]
    dv = o["v"] - o["v0"] - DT * np.array(spec["gravity"])
    assert np.allclose(M * dv, J.sum(axis=0), rtol=1e-9, atol=1e-12 * max(1.0, np.abs(J).max()))
    blade_b = spec["bodies"][0]
    errs = []
    for k in range(len(o["p"])):
        ab = k < o["n_points"][0]
        arm = o["p"][k] - o["x"]
        uo = np.asarray(blade_b["linvel"]) if ab else np.zeros(3)
        u = o["v"] + np.cross(o["w"], arm) - uo
        nn = o["n"][k]
        gam = o["gamma"][0 if ab else 1]
        mu = mu_ab if ab else mu_ac
        ln, lt = o["lam"][k][0], o["lam"][k][1:]
        rn = gam * ln + nn @ u
        rt = gam * lt + (u - (nn @ u) * nn)
        scale = max(abs(ln) * gam, 1e-12)
        errs.append(abs(rn) / scale if ln > 0 else max(-rn, 0.0) / scale)   # no cohesion here: lo = 0
        if ln == 0.0:
            errs.append(np.linalg.norm(lt))                                    # separated: no friction
        elif np.linalg.norm(lt) < mu * abs(ln) * (1 - 1e-9):
            errs.append(np.linalg.norm(rt) / scale)                            # sticking
        else:
            # sliding: on the disk, opposite to the residual slip
            errs.append(abs(np.linalg.norm(lt) - mu * abs(ln)) / max(abs(ln), 1e-30))
            if np.linalg.norm(rt) > 1e-12 * scale:
                errs.append(np.linalg.norm(lt / np.linalg.norm(lt) + rt / np.linalg.norm(rt)))
    return max(errs)


@pytest.mark.parametrize("V,mu_ac", [(0.3, 0.7), (2.0, 0.2)])
def test_pushed_aggregate_with_friction_satisfies_the_optimality_conditions(V, mu_ac):
    rng = np.random.default_rng(5)
    x = []
    s = 2.2 * R
    for ix in range(4):
        for iy in range(-2, 3):
            for iz in range(3):
                x.append([R - 0.01 + ix * s, iy * s, 0.9 * R + iz * s])
    x = np.asarray(x) + rng.uniform(-0.003, 0.003, (len(x), 3))
    n = len(x)
    spec = spec_of(x, [blade(linvel=(V, 0.0, 0.1))])
    v = np.tile([0.1, 0.05, -0.2], (n, 1))
    o = O.macro_step(spec, x, v, np.zeros((n, 3)), mu_ab=0.3, mu_ac=mu_ac, c_b=0.0)[0]
    assert o["n_points"] == (4, 4)
    assert o["sweeps"] < 200000
    assert kkt_residuals(o, spec, 0.3, mu_ac) < 1e-8
    # the angular momentum balance about the centre of mass
    J = o["lam"][:, :1] * o["n"] + o["lam"][:, 1:]
    torque = np.cross(o["p"] - o["x"], J).sum(axis=0)
    I = np.zeros((3, 3))
    m = sphere_mass()
    for p in x:
        rr = p - o["x"]
        I += (0.4 * m * R * R + m * rr @ rr) * np.eye(3) - m * np.outer(rr, rr)
    np.testing.assert_allclose(I @ (o["w"] - o["w0"]), torque, rtol=1e-8, atol=1e-10 * max(1.0, np.abs(torque).max()))


def test_mirror_symmetry():
    # mirroring the scene in y mirrors the solution
    rng = np.random.default_rng(8)
    x = resting_aggregate(cy=0.0) + rng.uniform(-0.002, 0.002, (18, 3))
    n = len(x)
    v = rng.normal(0, 0.1, (n, 3))
    spec = spec_of(x, [blade(linvel=(0.4, 0.0, 0.0))])
    a = O.macro_step(spec, x, v, np.zeros((n, 3)))[0]
    m = np.array([1.0, -1.0, 1.0])
    b = O.macro_step(spec, x * m, v * m, np.zeros((n, 3)))[0]
    np.testing.assert_allclose(b["v"], a["v"] * m, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(b["force_b"], a["force_b"] * m, rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------------------
# a dynamic equipment body (Eq. mdb:eqEq): mass, inertia and a drive
# ---------------------------------------------------------------------------
def plate_on_top(zb, half=0.4):
    """A horizontal plate whose bottom face (body z = -0.05) is the zone's
    separation plate, and whose zone reaches down to the level failure plane
    z = 0 (world); the plate is body 0 at height zb."""
    zone = [[0.0, 0.0, 1.0, -0.05],            # separation plate: below the plate's bottom face
            [0.0, 0.0, -1.0, zb],              # failure plane: world z >= 0
            [1.0, 0.0, 0.0, half], [-1.0, 0.0, 0.0, half], [0.0, 1.0, 0.0, half], [0.0, -1.0, 0.0, half]]
    return dict(pos=(0.0, 0.0, zb), quat=(1.0, 0.0, 0.0, 0.0), linvel=(0.0, 0.0, 0.0), angvel=(0.0, 0.0, 0.0),
                shapes=[dict(type="box", half=(half, half, 0.05), off=(0.0, 0.0, 0.0))], zone_planes=zone)


def box_inertia(m, a, b, c):
    return (m * (b * b + c * c) / 12.0, m * (a * a + c * c) / 12.0, m * (a * a + b * b) / 12.0, 0.0, 0.0, 0.0)


def stack(gap=0.004):
    """Two crosses of spheres: the bottom one within R of z = 0 (AC), the top
    one overlapping the plate's bottom face by `gap` (AB)."""
    z0 = 0.9 * R
    z1 = z0 + 3 * R
    x = np.asarray(cross_layout(0.0, 0.0, z0) + cross_layout(0.0, 0.0, z1))
    zb = z1 + R - gap + 0.05
    return x, zb


def test_drive_closed_forms_with_no_contact():
    # the plate far above a resting aggregate: its drive alone sets its motion
    x = resting_aggregate(cx=0.0, cy=0.0)
    n = len(x)
    mB, gd = 40.0, 1e-3
    plate = dict(plate_on_top(2.0), linvel=(0.3, -0.2, 0.1), angvel=(0.5, 0.0, -0.4))
    I = box_inertia(mB, 0.8, 0.8, 0.1)
    vt, wt = (1.0, 0.0, -0.5), (0.0, 2.0, 0.0)
    eq_free = dict(body=0, mass=mB, inertia=I, v_target=vt, w_target=wt, f_max=1e9, t_max=1e9, gamma_drive=gd)
    spec = spec_of(x, [plate])
    o = O.macro_step(spec, x, np.zeros((n, 3)), np.zeros((n, 3)), equipment=[eq_free])[0]
    v0 = np.array(plate["linvel"]) + DT * np.array([0.0, 0.0, -G])
    np.testing.assert_allclose(o["v_b"], (mB * v0 + np.array(vt) / gd) / (mB + 1.0 / gd), rtol=1e-12, atol=1e-15)
    Id = np.array(I[:3])
    np.testing.assert_allclose(o["w_b"], (Id * np.array(plate["angvel"]) + np.array(wt) / gd) / (Id + 1.0 / gd),
                               rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(o["lam_drive"][:3], mB * (o["v_b"] - v0), rtol=1e-12, atol=1e-15)
    # force-limited: each axis pushes at its limit toward the target
    fm, tm = 5.0, 0.01
    eq_lim = dict(eq_free, f_max=fm, t_max=tm)
    o2 = O.macro_step(spec, x, np.zeros((n, 3)), np.zeros((n, 3)), equipment=[eq_lim])[0]
    dirv = np.sign(np.array(vt) - v0)
    np.testing.assert_allclose(o2["v_b"], v0 + dirv * fm * DT / mB, rtol=1e-12)
    dirw = np.sign(np.array(wt) - np.array(plate["angvel"]))
    np.testing.assert_allclose(o2["w_b"], np.array(plate["angvel"]) + dirw * tm * DT / Id, rtol=1e-12)
    # the aggregate, touching only the terrain, is as with a kinematic plate
    ok = O.macro_step(spec, x, np.zeros((n, 3)), np.zeros((n, 3)))[0]
    np.testing.assert_allclose(o["v"], ok["v"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(o["lam"], ok["lam"], rtol=1e-12, atol=1e-15)


def test_free_plate_dropped_on_a_resting_aggregate():
    # drive off (zero limits): four equal AB impulses l1 between the plate and
    # the aggregate, four equal AC impulses l2 below it, from rest:
    #   M_A v_A = -M_A g dt - 4 l1 + 4 l2,   M_B v_B = -M_B g dt + 4 l1,
    #   gamma_AB l1 = v_A - v_B,             gamma_AC l2 = -v_A
    x, zb = stack()
    n = len(x)
    mB = 60.0
    eq = dict(body=0, mass=mB, inertia=box_inertia(mB, 0.8, 0.8, 0.1), f_max=0.0, t_max=0.0, gamma_drive=1e-3)
    spec = spec_of(x, [plate_on_top(zb)])
    o = O.macro_step(spec, x, np.zeros((n, 3)), np.zeros((n, 3)), equipment=[eq], c_b=0.0)[0]
    assert o["n_points"] == (4, 4)
    np.testing.assert_allclose(o["n"][:4], np.tile([0.0, 0.0, -1.0], (4, 1)))
    np.testing.assert_allclose(o["n"][4:], np.tile([0.0, 0.0, 1.0], (4, 1)))
    MA = n * sphere_mass()
    g1, g2 = o["gamma"]
    # unknowns (v_A, v_B, l1, l2)
    A = np.array([[MA, 0.0, 4.0, -4.0],
                  [0.0, mB, -4.0, 0.0],
                  [1.0, -1.0, -g1, 0.0],
                  [1.0, 0.0, 0.0, g2]])
    rhs = np.array([-MA * G * DT, -mB * G * DT, 0.0, 0.0])
    vA, vB, l1, l2 = np.linalg.solve(A, rhs)
    assert l1 > 0.0 and l2 > 0.0
    np.testing.assert_allclose(o["lam"][:4, 0], l1, rtol=1e-10)
    np.testing.assert_allclose(o["lam"][4:, 0], l2, rtol=1e-10)
    np.testing.assert_allclose(o["lam"][:, 1:], 0.0, atol=1e-12 * l2)
    np.testing.assert_allclose(o["v"], [0.0, 0.0, vA], atol=1e-12)
    np.testing.assert_allclose(o["v_b"], [0.0, 0.0, vB], atol=1e-12)
    np.testing.assert_allclose(o["w_b"], 0.0, atol=1e-12)
    np.testing.assert_allclose(o["lam_drive"], 0.0, atol=0.0)
    # the force of the aggregate on the plate: 4 l1 up
    np.testing.assert_allclose(o["force_b"], [0.0, 0.0, 4.0 * l1 / DT], rtol=1e-10, atol=1e-9)


def test_dynamic_equipment_momentum_balance_and_heavy_limit():
    # a rotated blade pushing a block, driven toward 0.6 m/s with a force
    # limit: the AB impulses cancel between the two bodies, so the momentum
    # change of A and B together is gravity plus the terrain's and the drive's
    # impulses
    rng = np.random.default_rng(21)
    s = 2.2 * R
    x = np.asarray([[R - 0.01 + ix * s, iy * s, 0.9 * R + iz * s]
                    for ix in range(4) for iy in range(-2, 3) for iz in range(3)]) + rng.uniform(-0.003, 0.003, (60, 3))
    n = len(x)
    c, sn = math.cos(0.05), math.sin(0.05)
    bl = dict(blade(linvel=(0.5, 0.0, 0.0)), quat=(c, 0.0, 0.0, sn), angvel=(0.0, 0.0, 0.2))
    mB = 30.0
    eq = dict(body=0, mass=mB, inertia=box_inertia(mB, 0.1, 2.0, 1.0), v_target=(0.6, 0.0, 0.0),
              w_target=(0.0, 0.0, 0.0), f_max=400.0, t_max=50.0, gamma_drive=1e-4)
    spec = spec_of(x, [bl])
    v = np.tile([0.1, 0.0, -0.1], (n, 1))
    o = O.macro_step(spec, x, v, np.zeros((n, 3)), equipment=[eq], mu_ab=0.3, mu_ac=0.6, c_b=500.0)[0]
    assert min(o["n_points"]) >= 3 and o["sweeps"] < 200000
    M = o["M"]
    gdt = DT * np.array([0.0, 0.0, -G])
    J = o["lam"][:, :1] * o["n"] + o["lam"][:, 1:]
    J_ac = J[o["n_points"][0]:].sum(axis=0)
    dp = M * (o["v"] - o["v0"] - gdt) + mB * (o["v_b"] - np.array(bl["linvel"]) - gdt)
    np.testing.assert_allclose(dp, J_ac + o["lam_drive"][:3], rtol=1e-9, atol=1e-9 * np.abs(J).max())
    assert np.all(np.abs(o["lam_drive"][:3]) <= 400.0 * DT * (1 + 1e-12))
    # a very heavy equipment driven at its own velocity is the kinematic case
    # (without gravity, so that the drive only has to hold the target)
    flat = dict(spec_of(x, [bl]), gravity=(0.0, 0.0, 0.0))
    heavy = dict(eq, mass=1e12, inertia=(1e12, 1e12, 1e12, 0.0, 0.0, 0.0), v_target=bl["linvel"],
                 w_target=bl["angvel"], f_max=1e20, t_max=1e20, gamma_drive=1e-6)
    oh = O.macro_step(flat, x, v, np.zeros((n, 3)), equipment=[heavy], mu_ab=0.3, mu_ac=0.6, c_b=500.0)[0]
    ok = O.macro_step(flat, x, v, np.zeros((n, 3)), mu_ab=0.3, mu_ac=0.6, c_b=500.0)[0]
    np.testing.assert_allclose(oh["v_b"], bl["linvel"], atol=1e-9)
    np.testing.assert_allclose(oh["w_b"], bl["angvel"], atol=1e-9)
    np.testing.assert_allclose(oh["v"], ok["v"], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(oh["lam"], ok["lam"], rtol=0, atol=1e-8 * np.abs(ok["lam"]).max())
