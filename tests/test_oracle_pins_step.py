"""More pins of the FP64 oracle: the sweep residual, the force and torque on a
kinematic body, the kinematic pose step and contact-point velocity, the
edge and corner branches of the box geometry, and the learned-start inputs.

Each expected value comes from outside the oracle's own code: a hand-solved
single contact, the matrix form of Gauss-Seidel on a two-contact stack
(numpy), the exact rotation of a normalised first-order quaternion step
(scipy), hand-placed geometry, or a hand-built contact whose inputs are
simple numbers.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG

G = 9.81
DT = 1.0 / 60.0
ESTAR = 1e9 / (2.0 * (1.0 - 0.15 ** 2))
UPS = 1.0 / 9.0  # 1 / (1 + 4 tau / dt) with tau = 2 dt


def sphere_mass(r, rho=2000.0):
    return rho * 4.0 / 3.0 * math.pi * r ** 3


def spec_of(x, r, bodies, mu=0.0, c=0.0, sweeps=50, g=(0.0, 0.0, -G), v=None, w=None, warm="cold", **mat):
    n = len(x)
    return dict(x=np.asarray(x, dtype=np.float64).reshape(-1, 3), r=np.asarray(r, dtype=np.float64),
                v=np.zeros((n, 3)) if v is None else np.asarray(v, dtype=np.float64),
                w=np.zeros((n, 3)) if w is None else np.asarray(w, dtype=np.float64),
                id=np.arange(n), bodies=bodies, material=SG.material(mu, c, **mat), dt=DT, gravity=g,
                max_sweeps=sweeps, tol=0.0, warm_start=warm, grid_lo=(-5.0, -5.0, -5.0),
                grid_hi=(5.0, 5.0, 5.0), r_ref=0.05)


def plane_body(pos=(0.0, 0.0, 0.0), angvel=(0.0, 0.0, 0.0), linvel=(0.0, 0.0, 0.0)):
    return dict(pos=pos, quat=(1.0, 0.0, 0.0, 0.0), linvel=linvel, angvel=angvel,
                shapes=[dict(type="plane", n=(0, 0, 1), d=0.0)])


def wall_overlap_at_rest(m, r):
    """Overlap at which a sphere's weight balances the Hertz wall force."""
    kn = ESTAR * math.sqrt(2 * r) / 3.0
    return (m * G / kn) ** (2.0 / 3.0)


def sigma_of(kn, delta):
    """Compliance term of the scaled SPOOK row at overlap delta."""
    eps = 4.0 / (5.0 * kn * math.sqrt(delta))
    return (4.0 / DT ** 2) * eps * UPS


# --------------------------------------------------------------------------
# Sweep residual R_k (the energy-weighted change of the impulses in sweep k
# over their size)
# --------------------------------------------------------------------------
def test_residual_first_sweep_from_cold_start_is_one():
    spec = dict(SG.column_scene(seed=4, n=60, footprint=0.3, sweeps=6), warm_start="cold")
    sc = O.OracleScene(spec)
    for _ in range(25):
        sc.step()
    out = sc.step()
    assert out["contacts"] > 40
    # lambda^0 = 0, so the first sweep's change is the impulse itself
    assert out["resid"][0] == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("mu,vx", [(0.6, 0.05), (0.1, 1.5)])
def test_residual_single_contact_on_static_plane_is_solved_in_one_sweep(mu, vx):
    # one contact against a static body has a diagonal Delassus block and
    # decoupled normal and tangential rows: one sweep solves it exactly
    # (sticking for the slow sphere, sliding on the friction disk for the fast)
    r = 0.05
    m = sphere_mass(r)
    d0 = wall_overlap_at_rest(m, r)
    spec = spec_of([[0.0, 0.0, r - d0]], [r], [plane_body()], mu=mu, v=[[vx, 0.0, 0.0]], sweeps=6)
    out = O.OracleScene(spec).step()
    assert out["contacts"] == 1
    assert out["resid"][0] == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.abs(out["resid"][1:]) <= 1e-13)
    # the impulse is the hand-solved one: the weight over dt, and either the
    # sticking impulse or the disk limit
    lam = out["lam"][0]
    assert lam[0] == pytest.approx(m * G * DT, rel=1e-12)
    l2 = r - d0 / 2
    Wt = 1.0 / m + l2 * l2 / (0.4 * m * r * r)
    stick = vx / Wt
    assert -lam[1] == pytest.approx(min(stick, mu * m * G * DT), rel=1e-12)


def test_residual_two_contact_stack_follows_matrix_gauss_seidel():
    # floor - A - B stacked along z, frictionless, no cohesion: only the two
    # normal rows act and no bound is active, so the sweeps are Gauss-Seidel
    # on the 2x2 system (J M^-1 J^T + Sigma) lambda = q - J v*.  Its iterates
    # from the splitting (L + D) lambda^{k+1} = b - U lambda^k, taken in the
    # oracle's colour order, give every R_k.
    r = 0.05
    m = sphere_mass(r)
    d1, d2 = 4e-5, 3e-5
    zA = r - d1
    zB = zA + 2 * r - d2
    spec = spec_of([[0.0, 0.0, zA], [0.0, 0.0, zB]], [r, r], [plane_body()], sweeps=60)
    out = O.OracleScene(spec).step()
    keys = [int(k) for k in out["keys"]]
    assert len(keys) == 2
    pair = keys.index((0 << 32) | 1)
    floor = 1 - pair
    kn_wall = ESTAR * math.sqrt(2 * r) / 3.0
    kn_pair = ESTAR * math.sqrt(r) / 3.0
    # rows in the order (floor, pair); unknowns lambda = (floor, pair)
    J = np.array([[1.0, 0.0], [-1.0, 1.0]])               # u = J (vA_z, vB_z)
    Minv = np.diag([1.0 / m, 1.0 / m])
    Sig = np.diag([sigma_of(kn_wall, d1), sigma_of(kn_pair, d2)])
    A = J @ Minv @ J.T + Sig
    vstar = np.array([-G * DT, -G * DT])
    q = (4.0 / DT) * UPS * 0.8 * np.array([d1, d2])        # start at rest: no velocity term
    b = q - J @ vstar
    order = [0, 1] if out["colour"][floor] < out["colour"][pair] else [1, 0]
    P = np.eye(2)[order]                                   # permute to the sweep order
    Ap, bp = P @ A @ P.T, P @ b
    Lo, Up = np.tril(Ap), np.triu(Ap, 1)
    lam = np.zeros(2)
    Dw = np.diag(Ap)
    expect = []
    for _ in range(30):
        new = np.linalg.solve(Lo, bp - Up @ lam)
        d = new - lam
        expect.append(math.sqrt(np.sum(Dw * d * d)) / math.sqrt(np.sum(Dw * new * new)))
        lam = new
    assert np.all(lam > 0)  # no bound active
    got = out["resid"]
    np.testing.assert_allclose(got[:12], expect[:12], rtol=1e-9, atol=1e-15)
    # the asymptotic rate is the spectral radius of the 2x2 Gauss-Seidel
    # iteration, a12 a21 / (a11 a22)
    rho = A[0, 1] * A[1, 0] / (A[0, 0] * A[1, 1])
    assert got[24] / got[23] == pytest.approx(rho, rel=1e-5)
    # and the final impulses solve the system
    lam_oracle = np.array([out["lam"][floor][0], out["lam"][pair][0]])
    np.testing.assert_allclose(lam_oracle, np.linalg.solve(A, b), rtol=1e-12)


# --------------------------------------------------------------------------
# Force and torque on a kinematic body
# --------------------------------------------------------------------------
@pytest.mark.parametrize("yaw", [0.0, 0.7])
def test_body_torque_of_a_sphere_resting_off_centre_on_a_box(yaw):
    # a sphere at its resting overlap on the top face of a (yawed) box: one
    # sweep gives exactly the weight, so the mean force on the box is -m g z
    # and the torque about the box's position is arm x F, arm to the contact
    # point (the middle of the overlap)
    r = 0.05
    m = sphere_mass(r)
    d0 = wall_overlap_at_rest(m, r)
    half_z = 0.2
    box_pos = np.array([0.3, -0.1, 0.5])
    qz = (math.cos(yaw / 2), 0.0, 0.0, math.sin(yaw / 2))
    box = dict(pos=tuple(box_pos), quat=qz, linvel=(0, 0, 0), angvel=(0, 0, 0),
               shapes=[dict(type="box", half=(0.6, 0.5, half_z), off=(0.0, 0.0, 0.0))])
    ax, ay = 0.37, -0.21
    top = box_pos[2] + half_z
    xs = np.array([box_pos[0] + ax, box_pos[1] + ay, top + r - d0])
    spec = spec_of([xs], [r], [box], mu=0.5, sweeps=3)
    out = O.OracleScene(spec).step()
    assert out["contacts"] == 1
    F, T = out["body_ft"][0][:3], out["body_ft"][0][3:]
    np.testing.assert_allclose(F, [0.0, 0.0, -m * G], rtol=1e-9, atol=1e-9 * m * G)
    pz = top - d0 / 2 - box_pos[2]   # contact point above the box position
    np.testing.assert_allclose(T, [-m * G * ay, m * G * ax, 0.0], rtol=1e-9, atol=1e-9 * m * G)
    assert pz > 0


# --------------------------------------------------------------------------
# Kinematic pose step and the kinematic body's velocity at a contact
# --------------------------------------------------------------------------
def test_kinematic_pose_step_is_a_rotation_by_two_arctan_half_angle():
    # normalize(q + dt/2 (0, w) q) = (cos a + sin a w/|w|) q with tan a = dt |w| / 2:
    # a rotation by 2 atan(dt |w| / 2) about the world axis w, composed on the
    # left; the position moves by dt v
    q0 = Rotation.from_euler("xyz", [0.3, -0.5, 1.1])
    w = np.array([1.5, -2.0, 4.0])
    v = np.array([0.7, -0.2, 0.1])
    x0 = np.array([0.1, 0.2, 1.5])
    qx, qy, qz, qw = q0.as_quat()
    body = dict(pos=tuple(x0), quat=(qw, qx, qy, qz), linvel=tuple(v), angvel=tuple(w),
                shapes=[dict(type="box", half=(0.1, 0.1, 0.1), off=(0.0, 0.0, 0.0))])
    spec = spec_of([[3.0, 3.0, 3.0]], [0.05], [body], g=(0.0, 0.0, 0.0), sweeps=1)
    sc = O.OracleScene(spec)
    steps = 40
    for _ in range(steps):
        sc.step()
    pose = sc.bb.poses()[0]
    np.testing.assert_allclose(pose["pos"], x0 + steps * DT * v, rtol=0, atol=1e-13)
    wn = np.linalg.norm(w)
    ang = 2.0 * math.atan(0.5 * DT * wn)
    expect = Rotation.from_rotvec(steps * ang * w / wn) * q0
    got = Rotation.from_quat([pose["quat"][1], pose["quat"][2], pose["quat"][3], pose["quat"][0]])
    assert (got.inv() * expect).magnitude() < 1e-12
    # the step angle tends to the exact dt |w| (error (dt |w|)^3 / 12 per step)
    exact = Rotation.from_rotvec(steps * DT * w) * q0
    assert (got.inv() * exact).magnitude() == pytest.approx(steps * (DT * wn) ** 3 / 12.0, rel=1e-2)


@pytest.mark.parametrize("mu", [0.8, 0.02])
def test_sphere_on_a_spinning_plane_takes_the_plane_velocity_at_the_contact(mu):
    # the plane spins about z through its position; the relative velocity at
    # the contact is the sphere's minus v_B + w_B x (p - x_B) = (0, w R0, 0).
    # One sweep solves the single contact: sticking gives the tangential
    # impulse w R0 / W_t (W_t = 1/m + l^2/I), sliding the disk limit mu m g dt
    r, om, R0 = 0.05, 0.5, 0.2
    m = sphere_mass(r)
    I = 0.4 * m * r * r
    d0 = wall_overlap_at_rest(m, r)
    l2 = r - d0 / 2
    Wt = 1.0 / m + l2 * l2 / I
    body = plane_body(pos=(0.0, 0.0, 0.0), angvel=(0.0, 0.0, om))
    spec = spec_of([[R0, 0.0, r - d0]], [r], [body], mu=mu, sweeps=4)
    sc = O.OracleScene(spec)
    out = sc.step()
    J = min(om * R0 / Wt, mu * m * G * DT)
    np.testing.assert_allclose(out["lam"][0][1:], [0.0, J, 0.0], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(sc.v[0], [0.0, J / m, 0.0], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(sc.w[0], [l2 * J / I, 0.0, 0.0], rtol=1e-12, atol=1e-15)
    if J < mu * m * G * DT:
        # sticking: the contact point now moves with the plane
        cp = sc.v[0] + np.cross(sc.w[0], [0.0, 0.0, -l2])
        np.testing.assert_allclose(cp, [0.0, om * R0, 0.0], rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------
# Box geometry: edge and corner regions (closest point by clamping)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("region", ["edge", "corner"])
@pytest.mark.parametrize("yaw", [0.0, 0.9])
def test_box_edge_and_corner_overlap_and_normal(region, yaw):
    r = 0.05
    h = np.array([0.5, 0.4, 0.3])
    e = np.array([0.021, 0.017, 0.0]) if region == "edge" else np.array([0.013, 0.02, 0.011])
    local = h * np.array([1.0, 1.0, 1.0 if region == "corner" else 0.0]) + e
    if region == "edge":
        local[2] = 0.1            # beside the edge, within the face's z range
    rot = Rotation.from_euler("z", yaw)
    pos = np.array([0.2, -0.3, 0.4])
    x = pos + rot.apply(local)
    qx, qy, qz, qw = rot.as_quat()
    box = dict(pos=tuple(pos), quat=(qw, qx, qy, qz), linvel=(0, 0, 0), angvel=(0, 0, 0),
               shapes=[dict(type="box", half=tuple(h), off=(0.0, 0.0, 0.0))])
    spec = spec_of([x], [r], [box], g=(0.0, 0.0, 0.0), sweeps=1)
    keys, delta = O.detect(spec, O.BRUTE)
    dist = float(np.linalg.norm(e))
    assert len(keys) == 1
    assert delta[0] == pytest.approx(r - dist, rel=1e-11)
    # frictionless, no gravity, at rest: the step's impulse pushes the sphere
    # along the normal, from the closest point of the box towards the centre
    sc = O.OracleScene(spec)
    sc.step()
    nrm = rot.apply(e / dist)
    vdir = sc.v[0] / np.linalg.norm(sc.v[0])
    np.testing.assert_allclose(vdir, nrm, atol=1e-12)
    assert np.linalg.norm(sc.w[0]) < 1e-12  # a normal impulse through the centre
    # just out of range: no contact
    far = pos + rot.apply(h * np.array([1.0, 1.0, 1.0 if region == "corner" else 0.0]) +
                          (r * 1.0001) * e / dist + (np.array([0, 0, 0.1]) if region == "edge" else 0.0))
    keys, _ = O.detect(spec_of([far], [r], [box], g=(0.0, 0.0, 0.0)), O.BRUTE)
    assert len(keys) == 0


# --------------------------------------------------------------------------
# Learned-start inputs on a hand-built case
# --------------------------------------------------------------------------
def test_learned_features_of_a_hand_built_stack():
    # sphere A (id 0) resting on the floor, sphere B (id 1) straight above it
    # and overlapping, sphere C (id 2) alone in another column on the floor.
    # Velocities: A (0.3, 0, 0), B (0, 0, -0.1), C 0, no spin.  Previous-step
    # impulses are given for the pair (persistent) but not for the floor
    # contacts (new).
    rA, rB, rC = 0.05, 0.04, 0.045
    dA, dAB, dC = 2e-5, 3e-5, 1e-5
    zA = rA - dA
    zB = zA + rA + rB - dAB
    zC = rC - dC
    x = [[0.0, 0.0, zA], [0.0, 0.0, zB], [1.0, 0.7, zC]]
    v = [[0.3, 0.0, 0.0], [0.0, 0.0, -0.1], [0.0, 0.0, 0.0]]
    spec = spec_of(x, [rA, rB, rC], [plane_body()], mu=0.5, v=v, warm="prev")
    sc = O.OracleScene(spec)
    kAB = (0 << 32) | 1
    sc.prev_keys = np.array([kAB], dtype=np.uint64)
    lt_prev = np.array([0.02, 0.01, 0.003])          # its normal part is projected out
    sc.prev_lam = np.array([[0.5, *lt_prev]])
    F, frames, scale = sc.features()
    keys, _ = O.detect(spec, O.BRUTE)
    assert len(F) == 3
    kfA, kfC = (0 << 32) | 0x80000000, (2 << 32) | 0x80000000
    idx = {int(k): i for i, k in enumerate(keys)}
    mA, mB, mC = sphere_mass(rA), sphere_mass(rB), sphere_mass(rC)
    gdt = G * DT
    top = zB + rB                                     # top of the A-B column
    # pair A-B: n = +z, u = vB - vA = (-0.3, 0, -0.1); t1 = u_t/|u_t| = -x, t2 = n x t1 = -y
    f = F[idx[kAB]]
    ls = gdt / (1.0 / mA + 1.0 / mB)
    rbar = 0.5 * (rA + rB)
    expect = [dAB / rbar, -0.1 / gdt, 0.3 / gdt, 0.5 / ls, -0.02 / ls, -0.01 / ls,
              (top - zA) / rbar, (top - zB) / rbar, rA / 0.05, rB / 0.05, 0.0, 1.0]
    np.testing.assert_allclose(f, expect, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(frames[idx[kAB]], [-1, 0, 0, 0, -1, 0], atol=1e-15)
    assert scale[idx[kAB]] == pytest.approx(ls, rel=1e-12)
    # floor contact of A: body 1 is the plane, n = +z, u = vA = (0.3, 0, 0)
    f = F[idx[kfA]]
    ls = gdt * mA
    expect = [dA / rA, 0.0, 0.3 / gdt, 0.0, 0.0, 0.0, 0.0, (top - zA) / rA, 0.0, rA / 0.05, 1.0, 0.0]
    np.testing.assert_allclose(f, expect, rtol=1e-9, atol=1e-12)
    # floor contact of C: at rest, alone in its column (depth = its radius)
    f = F[idx[kfC]]
    expect = [dC / rC, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, rC / 0.05, 1.0, 0.0]
    np.testing.assert_allclose(f, expect, rtol=1e-9, atol=1e-12)
    # with no slip and no previous impulse the frame is the axis least
    # aligned with n, made orthogonal to it: x for n = z
    np.testing.assert_allclose(frames[idx[kfC]], [1, 0, 0, 0, 1, 0], atol=1e-15)


def test_depth_column_of_a_stack_and_the_column_decision():
    # a stack of five spheres in one column and two single spheres in the
    # neighbouring columns: every depth is the column top minus the centre.
    # The column is the detection cell (width h = 2 r_max (1 + kappa_c) 1.001
    # from the grid's low corner), decided in FP32 on the FP32 state; a sphere
    # a little inside either side of a cell boundary falls in its own cell.
    r = 0.05
    h = 2 * r * 1.025 * 1.001
    lo = -1.0
    cx = lo + 4.5 * h                       # centre of cell 4
    zs = [r + 2 * r * k for k in range(5)]
    x = [[cx, cx, z] for z in zs]
    x += [[lo + 4 * h + 1e-4, cx, 0.62], [lo + 4 * h - 1e-4, cx, 0.9]]   # cells 4 and 3
    x = SG.fp32(x)
    n = len(x)
    spec = spec_of(x, [r] * n, [plane_body(pos=(0, 0, -1.0))], c=1000.0, warm="cold")
    spec["grid_lo"] = (lo, lo, lo)
    spec["grid_hi"] = (1.0, 1.0, 1.0)
    # zero-velocity pairs along the stack give the depths through feature 6/7
    sc = O.OracleScene(spec)
    F, _, _ = sc.features()
    keys, _ = O.detect(spec, O.BRUTE)
    top4 = x[5][2] + r                      # cell 4 holds the stack and the sphere at x = +1e-4
    for k, f in zip(keys, F):
        a, b = int(k) >> 32, int(k) & 0xFFFFFFFF
        if b & 0x80000000:
            continue
        assert a < 5 and b < 5
        assert f[6] * r == pytest.approx(top4 - x[a][2], rel=1e-12)
        assert f[7] * r == pytest.approx(top4 - x[b][2], rel=1e-12)
    # the single sphere in cell 3 has no contact; its depth is checked through
    # a pair formed by moving a partner next to it in the same cell
    x2 = np.vstack([x, SG.fp32([[lo + 4 * h - 1e-4, cx, 0.9 + 2 * r - 1e-5]])])
    spec2 = dict(spec, x=x2, r=np.full(len(x2), r), v=np.zeros((len(x2), 3)), w=np.zeros((len(x2), 3)),
                 id=np.arange(len(x2)))
    F2, _, _ = O.OracleScene(spec2).features()
    keys2, _ = O.detect(spec2, O.BRUTE)
    i = [j for j, k in enumerate(keys2) if int(k) == ((6 << 32) | 7)]
    assert len(i) == 1
    top3 = x2[7][2] + r
    assert F2[i[0]][6] * r == pytest.approx(top3 - x2[6][2], rel=1e-12)
    assert F2[i[0]][7] * r == pytest.approx(r, rel=1e-12)


# --------------------------------------------------------------------------
# BF16 inference of the learned start (the precision the network runs in)
# --------------------------------------------------------------------------
def test_bf16_network_equals_a_torch_bfloat16_model():
    # torch's own float32 -> bfloat16 conversion (round to nearest even) as the
    # independent rounding: inputs x scale, weight matrices and hidden layers
    # rounded, biases and sums in double
    torch = pytest.importorskip("torch")

    def bf(a):
        t = torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64)
        return t.numpy()

    rng = np.random.default_rng(12)
    w = dict(W1=rng.normal(0, 0.4, (64, 12)), b1=rng.normal(0, 0.1, 64), W2=rng.normal(0, 0.2, (64, 64)),
             b2=rng.normal(0, 0.1, 64), W3=rng.normal(0, 0.2, (3, 64)), b3=rng.normal(0, 0.1, 3),
             in_scale=rng.uniform(0.5, 1.5, 12))
    feat = rng.normal(0, 1.0, (500, 12))
    x = bf(feat * w["in_scale"])
    z1 = x @ bf(w["W1"]).T + w["b1"]
    h1 = bf(z1 / (1.0 + np.exp(-z1)))
    z2 = h1 @ bf(w["W2"]).T + w["b2"]
    h2 = bf(z2 / (1.0 + np.exp(-z2)))
    ref = h2 @ bf(w["W3"]).T + w["b3"]
    got = O.mlp_forward(dict(w, bf16=True), feat)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    # and without the option the network is the plain double one
    z1 = (feat * w["in_scale"]) @ w["W1"].T + w["b1"]
    h1 = z1 / (1.0 + np.exp(-z1))
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = z2 / (1.0 + np.exp(-z2))
    np.testing.assert_allclose(O.mlp_forward(w, feat), h2 @ w["W3"].T + w["b3"], rtol=1e-12, atol=1e-12)
