"""Parity of the macroscale step (C-ABI macro_step) against the FP64 oracle's
macroscale step: the aggregate body of each zone under Eq. mdb:eqAgg with the
constraints of Eqs. aggregateNormal and aggregateTangent at its equipment (AB)
and failure-surface (AC) interfaces, four points each.

Both sides get the same seeded FP32-representable particle state and the same
FP64 body poses; nothing the GPU produces is fed to the oracle.  Bars:
  - zone list, candidate counts, reduced-point particle indices: exact;
  - points and normals (same FP64 formulas on the same inputs): 1e-12 of the
    scene's length scale;
  - FP64 reductions (mass, centre of mass, area, regularisation): 1e-12
    relative (atomic summation order only);
  - the aggregate's angular velocity before the step (moments about the
    origin on the GPU, about the centre of mass in the oracle): 1e-9 of
    |v0| / extent;
  - the solved impulses, velocities and the force on the equipment (a strongly
    convex problem solved to 1e-15 relative change on both sides): 1e-8 of
    their largest magnitude.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG
from paper_2011_00459_amd import zones as Z

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")

DT = 1.0 / 60.0
MACRO = dict(E_b=1e7, c_b=2000.0, mu_ab=0.4, mu_ac=0.7, cas_ab=1.0, cas_ac=0.001)


def fp32_state(spec, seed, vscale=0.2, wscale=1.0):
    """spec with FP32-representable x, r and seeded FP32 velocities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(spec["x"])
    out = dict(spec)
    out["x"] = SG.fp32(spec["x"])
    out["r"] = SG.fp32(spec["r"])
    out["v"] = SG.fp32(rng.normal(0.0, vscale, (n, 3)))
    out["w"] = SG.fp32(rng.normal(0.0, wscale, (n, 3)))
    return out


def compare(g, o, scale):
    assert g["zone"] == o["zone"]
    assert g["n_points"] == o["n_points"]
    assert g["n_cand"] == o["n_cand"]
    assert list(g["src"]) == list(o["src"])
    np.testing.assert_allclose(g["p"], o["p"], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(g["n"], o["n"], rtol=0, atol=1e-15)
    assert g["M"] == pytest.approx(o["M"], rel=1e-12)
    np.testing.assert_allclose(g["x"], o["x"], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(g["area"], o["area"], rtol=1e-12)
    np.testing.assert_allclose(g["gamma"], o["gamma"], rtol=1e-12)
    vmag = max(float(np.max(np.abs(o["v0"]))), 9.81 * DT)
    np.testing.assert_allclose(g["v0"], o["v0"], rtol=0, atol=1e-12 * vmag)
    wmag = vmag / scale + float(np.max(np.abs(o["w0"])))
    np.testing.assert_allclose(g["w0"], o["w0"], rtol=0, atol=1e-9 * wmag)
    lmax = max(float(np.max(np.abs(o["lam"]))) if len(o["lam"]) else 0.0, 1e-300)
    np.testing.assert_allclose(g["lam"], o["lam"], rtol=0, atol=1e-8 * lmax)
    vmag = max(vmag, float(np.max(np.abs(o["v"]))))
    np.testing.assert_allclose(g["v"], o["v"], rtol=0, atol=1e-8 * vmag)
    wmag = vmag / scale + float(np.max(np.abs(o["w"])))
    np.testing.assert_allclose(g["w"], o["w"], rtol=0, atol=1e-8 * wmag)
    fmax = max(float(np.max(np.abs(o["force_b"]))), 1e-300)
    np.testing.assert_allclose(g["force"], o["force_b"], rtol=0, atol=1e-8 * fmax)
    tmax = max(float(np.max(np.abs(o["torque_b"]))), fmax * scale)
    np.testing.assert_allclose(g["torque"], o["torque_b"], rtol=0, atol=1e-8 * tmax)
    # the equipment's velocity after the step and its drive impulses (its own
    # velocity and zero when kinematic)
    vb = max(float(np.max(np.abs(o["v_b"]))), vmag)
    np.testing.assert_allclose(g["v_b"], o["v_b"], rtol=0, atol=1e-8 * vb)
    np.testing.assert_allclose(g["w_b"], o["w_b"], rtol=0, atol=1e-8 * (vb / scale + float(np.max(np.abs(o["w_b"])))))
    dmax = max(float(np.max(np.abs(o["lam_drive"]))), lmax)
    np.testing.assert_allclose(g["lam_drive"], o["lam_drive"], rtol=0, atol=1e-8 * dmax)


def run_both(spec, env=0, sc=None, equipment=None, **params):
    prm = dict(MACRO)
    prm.update(params)
    sc = sc or T.scene_from_specs(spec)
    gpu = sc.macro_step(env, equipment=equipment, **prm)       # body ids are the spec's body indices
    orc = O.macro_step(spec, spec["x"], spec["v"], spec["w"], equipment=equipment, **prm)
    return gpu, orc


def check(spec, expect_zones=None, equipment=None, **params):
    gpu, orc = run_both(spec, equipment=equipment, **params)
    scale = float(np.max(np.abs(spec["x"]))) + 1.0
    assert [g["zone"] for g in gpu] == [o["zone"] for o in orc]
    if expect_zones is not None:
        assert [o["zone"] for o in orc] == expect_zones
    for g, o in zip(gpu, orc):
        compare(g, o, scale)
    return gpu, orc


# ---------------------------------------------------------------------------
# small scenes: a box blade with a box-shaped zone in front of it
# ---------------------------------------------------------------------------
R0 = 0.05
BOX_ZONE = [[-1.0, 0.0, 0.0, 0.0],   # separation plate: the blade face x >= 0
            [0.0, 0.0, -1.0, 0.0],   # failure plane: z >= 0
            [0.0, 0.0, 1.0, 1.0], [0.0, 1.0, 0.0, 1.0], [0.0, -1.0, 0.0, 1.0], [1.0, 0.0, 0.0, 1.5]]


def small_spec(x, bodies, seed):
    n = len(x)
    spec = dict(x=np.asarray(x, dtype=np.float64), r=np.full(n, R0), id=np.arange(n), bodies=bodies,
                material=SG.material(0.5, 0.0), dt=DT, gravity=(0.0, 0.0, -9.81), max_sweeps=10, tol=0.0,
                warm_start="cold", grid_lo=(-2.0, -2.0, -2.0), grid_hi=(2.0, 2.0, 2.0), r_ref=R0)
    return fp32_state(spec, seed, vscale=0.1, wscale=0.5)


def small_blade(linvel=(0.0, 0.0, 0.0), angvel=(0.0, 0.0, 0.0), zone=BOX_ZONE):
    return dict(pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), linvel=linvel, angvel=angvel,
                shapes=[dict(type="box", half=(0.05, 1.0, 0.5), off=(-0.05, 0.0, 0.5))], zone_planes=zone)


def block(seed, nx=4, ny=5, nz=3):
    rng = np.random.default_rng(seed)
    s = 2.2 * R0
    x = [[R0 - 0.01 + ix * s, (iy - (ny - 1) / 2) * s, 0.9 * R0 + iz * s]
         for ix in range(nx) for iy in range(ny) for iz in range(nz)]
    return np.asarray(x) + rng.uniform(-0.003, 0.003, (len(x), 3))


@pytest.mark.parametrize("linvel,angvel,c_b", [((0.3, 0.0, 0.1), (0.0, 0.0, 0.0), 0.0),
                                               ((2.0, 0.1, -0.2), (0.0, 0.3, 0.1), 2000.0),
                                               ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 5000.0)])
def test_block_pushed_by_the_blade(linvel, angvel, c_b):
    spec = small_spec(block(5), [small_blade(linvel, angvel)], seed=11)
    gpu, orc = check(spec, expect_zones=[0], c_b=c_b)
    assert orc[0]["n_points"] == (4, 4)


def test_ties_along_a_lattice_go_to_the_smaller_particle():
    # an unjittered lattice: many candidates share the extreme projections
    s = 2.2 * R0
    x = [[R0 - 0.01 + ix * s, (iy - 2) * s, 0.9 * R0 + iz * s] for ix in range(4) for iy in range(5) for iz in range(3)]
    spec = small_spec(x, [small_blade((0.5, 0.0, 0.0))], seed=12)
    gpu, orc = check(spec, expect_zones=[0])
    assert orc[0]["n_cand"][1] == 20     # the bottom layer within R of z = 0


def test_zone_lists_two_zones_a_one_plane_body_and_an_empty_zone():
    x = np.concatenate([block(6), block(7) + [0.0, 1.5, 0.0]])
    b0 = small_blade((0.4, 0.0, 0.0))
    # a second blade at y = 1.5 with its own zone
    b1 = dict(small_blade((0.0, 0.5, 0.0)), pos=(0.0, 1.5, 0.0))
    b2 = dict(small_blade(), pos=(0.0, -1.5, 0.0), zone_planes=BOX_ZONE[:1])       # one half-space: no zone step
    b3 = dict(small_blade(), pos=(1.8, -1.8, 1.5))                                  # zone with no particle
    spec = small_spec(x, [b0, b1, b2, b3], seed=13)
    gpu, orc = check(spec, expect_zones=[0, 1])


def test_a_particle_in_two_zones_belongs_to_the_first():
    # two bodies whose zones overlap: the earlier body (its zone x >= 0.2)
    # takes the shared particles, the later one (x >= 0) the rest
    x = block(8)
    first = dict(small_blade((0.0, 0.0, 0.0)), pos=(0.2, 0.0, 0.0))
    second = small_blade((0.4, 0.0, 0.0))
    spec = small_spec(x, [first, second], seed=14)
    gpu, orc = check(spec, expect_zones=[0, 1])
    m = 2000.0 * 4.0 / 3.0 * math.pi * float(spec["r"][0]) ** 3
    assert orc[0]["M"] == pytest.approx(m * np.sum(spec["x"][:, 0] >= 0.2), rel=1e-12)
    assert orc[0]["M"] + orc[1]["M"] == pytest.approx(len(x) * m, rel=1e-12)


def test_no_zone_bodies():
    spec = small_spec(block(9), [dict(small_blade(), zone_planes=[])], seed=15)
    sc = T.scene_from_specs(spec)
    assert sc.macro_step(0, **MACRO) == []
    assert O.macro_step(spec, spec["x"], spec["v"], spec["w"], **MACRO) == []


def test_rejects_bad_parameters():
    spec = small_spec(block(9), [small_blade()], seed=16)
    sc = T.scene_from_specs(spec)
    for bad in (dict(E_b=0.0), dict(cas_ac=-1.0), dict(c_b=-1.0), dict(mu_ab=float("nan"))):
        prm = dict(MACRO)
        prm.update(bad)
        with pytest.raises(T.TerrainError):
            sc.macro_step(0, **prm)
    with pytest.raises(T.TerrainError):
        sc.macro_step(1, **MACRO)


# ---------------------------------------------------------------------------
# a dynamic equipment (Eq. mdb:eqEq): its mass, inertia and drive
# ---------------------------------------------------------------------------
def box_inertia(m, a, b, c):
    return (m * (b * b + c * c) / 12.0, m * (a * a + c * c) / 12.0, m * (a * a + b * b) / 12.0, 0.0, 0.0, 0.0)


@pytest.mark.parametrize("f_max,t_max", [(400.0, 50.0), (20.0, 2.0), (0.0, 0.0)])
def test_block_pushed_by_a_driven_blade(f_max, t_max):
    c, sn = math.cos(0.05), math.sin(0.05)
    bl = dict(small_blade((0.5, 0.0, 0.0), (0.0, 0.0, 0.2)), quat=(c, 0.0, 0.0, sn))
    spec = small_spec(block(5), [bl], seed=17)
    eq = [dict(body=0, mass=30.0, inertia=box_inertia(30.0, 0.1, 2.0, 1.0), v_target=(0.6, 0.0, 0.0),
               w_target=(0.0, 0.0, 0.0), f_max=f_max, t_max=t_max, gamma_drive=1e-4)]
    gpu, orc = check(spec, expect_zones=[0], equipment=eq)
    assert min(orc[0]["n_points"]) >= 3


def test_driven_bucket_in_a_bed_and_a_kinematic_second_tool():
    spec = bed_with_zone(61, 6000, 0.25, tool="bucket")
    # a second, kinematic blade with its own zone elsewhere in the bed
    blade2 = SG.box_blade(0.5, float(spec["bodies"][1]["pos"][2]) - 0.3, width=0.6, vx=-0.4, body_id=2)
    top = float(np.max(spec["x"][:, 2] + spec["r"]))
    blade2["zone_planes"] = Z.blade_zone(blade2, 0.7, top)
    spec["bodies"] = spec["bodies"] + [blade2]
    eq = [dict(body=1, mass=250.0, inertia=box_inertia(250.0, 0.8, 1.0, 0.6), v_target=(0.8, 0.0, -0.1),
               w_target=(0.0, 0.1, 0.0), f_max=3000.0, t_max=500.0, gamma_drive=2e-5)]
    gpu, orc = check(spec, equipment=eq)
    assert [o["zone"] for o in orc] == [1, 2]
    assert np.any(orc[0]["lam_drive"] != 0.0) and np.all(orc[1]["lam_drive"] == 0.0)


def test_rejects_bad_equipment():
    spec = small_spec(block(9), [small_blade()], seed=18)
    sc = T.scene_from_specs(spec)
    good = dict(body=0, mass=10.0, inertia=(1.0, 1.0, 1.0, 0.0, 0.0, 0.0), f_max=1.0, t_max=1.0, gamma_drive=1e-3)
    assert len(sc.macro_step(0, equipment=[good], **MACRO)) == 1
    for bad in (dict(body=5), dict(mass=0.0), dict(inertia=(1.0, 1.0, 1.0, 2.0, 0.0, 0.0)),
                dict(gamma_drive=0.0), dict(f_max=-1.0), dict(mass=float("inf"))):
        with pytest.raises(T.TerrainError):
            sc.macro_step(0, equipment=[dict(good, **bad)], **MACRO)
    with pytest.raises(T.TerrainError):
        sc.macro_step(0, equipment=[good, good], **MACRO)


# ---------------------------------------------------------------------------
# beds: a rotated moving blade with its failure-plane wedge, two envs
# ---------------------------------------------------------------------------
def bed_with_zone(seed, n, heading, tool="blade", speed=0.8):
    spec = SG.bed_scene(seed=seed, n=n, r0=0.03, spread=0.1, lx=1.6, ly=1.0, mu=0.7, c=2000.0, sweeps=20,
                        tool=tool, tool_speed=speed, depth=0.15, tool_x=-0.4, heading=heading)
    top = float(np.max(spec["x"][:, 2] + spec["r"]))
    tool_b = dict(spec["bodies"][1])
    if tool == "blade":
        tool_b["zone_planes"] = Z.blade_zone(tool_b, 0.7, top)
    else:
        hh = 0.3
        tool_b["zone_planes"] = Z.wedge_planes(0.4, -hh, 1.0, top - tool_b["pos"][2] + 0.3, Z.friction_angle(0.7))
    spec["bodies"] = [spec["bodies"][0], tool_b]
    return fp32_state(spec, seed + 100)


@pytest.mark.parametrize("heading,tool", [(0.0, "blade"), (0.35, "blade"), (-0.2, "bucket")])
def test_bed_with_a_moving_tool_and_its_wedge(heading, tool):
    spec = bed_with_zone(31, 6000, heading, tool)
    gpu, orc = check(spec, expect_zones=[1])
    o = orc[0]
    assert o["n_cand"][0] > 0 and o["n_cand"][1] > 4


@pytest.mark.parametrize("seed,heading", [(24, 0.0), (72, 0.3)])
def test_bed_where_newton_stalls_at_a_kink(seed, heading):
    # seeded beds whose damped Newton iteration stalls (no step of eight
    # halvings lowers the residual): a few Gauss-Seidel sweeps from its point
    # and a restart reach the oracle's fixed point, where Gauss-Seidel alone
    # needs thousands of sweeps
    spec = bed_with_zone(seed, 3000, heading, "blade")
    gpu, orc = check(spec, expect_zones=[1])
    assert orc[0]["sweeps"] > 1000
    assert gpu[0]["sweeps"] < 200


def test_second_env_of_a_two_env_scene():
    a = bed_with_zone(41, 3000, 0.1)
    b = bed_with_zone(42, 5000, -0.3, tool="bucket")
    sc = T.scene_from_specs([a, b], cap_particles=5000)
    for env, spec in ((1, b), (0, a)):
        gpu, orc = run_both(spec, env=env, sc=sc)
        assert [g["zone"] for g in gpu] == [o["zone"] for o in orc] == [1]
        compare(gpu[0], orc[0], float(np.max(np.abs(spec["x"]))) + 1.0)


def test_envs_loaded_out_of_order_go_through_the_id_map():
    # env 1's spheres added before env 0's: the slots are not in env order
    # until a step sorts them, so the macroscale step reads each env by id
    a = bed_with_zone(43, 3000, 0.1)
    b = bed_with_zone(44, 4000, -0.2, tool="bucket")
    ref = T.scene_from_specs([a, b], cap_particles=4000)
    sc = T.Scene(n_envs=2, dt=a["dt"], gravity=a["gravity"], max_sweeps=a["max_sweeps"], material=a["material"],
                 cap_particles=4000, cap_contacts=64000, r_ref=a["r_ref"],
                 env_bounds=[list(s["grid_lo"]) + list(s["grid_hi"]) for s in (a, b)])
    for env, spec in ((1, b), (0, a)):
        sc.add_particles(env, spec["x"], spec["r"], vel=spec["v"])
        sc.set_particles(env, w=spec["w"])
        sc.set_kinematic_bodies(env, [dict(bd, id=i) for i, bd in enumerate(spec["bodies"])])
    for env, spec in ((0, a), (1, b)):
        orc = O.macro_step(spec, spec["x"], spec["v"], spec["w"], **MACRO)
        for g in (sc.macro_step(env, **MACRO), ref.macro_step(env, **MACRO)):
            assert [q["zone"] for q in g] == [o["zone"] for o in orc] == [1]
            compare(g[0], orc[0], float(np.max(np.abs(spec["x"]))) + 1.0)


def test_after_steps_the_state_is_read_from_the_stepped_buffers():
    # macro_step reads the particles through the id map after the step's sort:
    # stepping then restoring the original state gives the original result
    spec = bed_with_zone(51, 4000, 0.2)
    sc = T.scene_from_specs(spec)
    before = sc.macro_step(0, **MACRO)
    sc.step(2)
    sc.set_particles(0, x=spec["x"], v=spec["v"], w=spec["w"])
    body = [dict(b, id=i) for i, b in enumerate(spec["bodies"])]
    sc.set_kinematic_bodies(0, body)
    after = sc.macro_step(0, **MACRO)
    orc = O.macro_step(spec, spec["x"], spec["v"], spec["w"], **MACRO)
    for g in (before, after):
        compare(g[0], orc[0], 2.0)


# ---------------------------------------------------------------------------
# full size: the 500,000-sphere excavation bed with the bucket in its wedge
# ---------------------------------------------------------------------------
def test_excavation_bed500k_bucket_zone_matches_oracle():
    spec = SG.excavation_scene(seed=5, n=500000, sweeps=200)
    floor, bucket = spec["bodies"][0], spec["bodies"][1]
    top = float(spec["grid_hi"][2]) - 0.5
    hh = 0.4
    bucket = dict(bucket, linvel=(0.8, 0.0, 0.0))
    bucket["zone_planes"] = Z.wedge_planes(0.5, -hh, 1.2, top - bucket["pos"][2] + 0.3, Z.friction_angle(0.7))
    spec = fp32_state(dict(spec, bodies=[floor, bucket]), 77, vscale=0.05, wscale=0.2)
    gpu, orc = check(spec, expect_zones=[1])
    assert orc[0]["n_points"] == (4, 4) and min(orc[0]["n_cand"]) >= 30
