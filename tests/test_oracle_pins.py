"""Pins of the FP64 oracle against what the paper and mechanics fix.

Each test checks the oracle against something other than its own formulas:
exact rational arithmetic, closed-form mechanics of one sphere or a column,
conservation laws, an independent round-based colouring, finite differences,
and the worked relations printed in the paper.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG

G = 9.81
DT = 1.0 / 60.0
ESTAR = 1e9 / (2.0 * (1.0 - 0.15 ** 2))


def sphere_mass(r, rho=2000.0):
    return rho * 4.0 / 3.0 * math.pi * r ** 3


def base_spec(x, r, bodies, mu=0.0, c=0.0, sweeps=50, g=(0.0, 0.0, -G), v=None, w=None, **mat):
    n = len(x)
    spec = dict(x=np.asarray(x, dtype=np.float64).reshape(-1, 3), r=np.asarray(r, dtype=np.float64),
                v=np.zeros((n, 3)) if v is None else np.asarray(v, dtype=np.float64),
                w=np.zeros((n, 3)) if w is None else np.asarray(w, dtype=np.float64),
                id=np.arange(n), bodies=bodies, material=SG.material(mu, c, **mat), dt=DT, gravity=g,
                max_sweeps=sweeps, tol=0.0, warm_start="cold", grid_lo=(-5.0, -5.0, -5.0), r_ref=0.05)
    return spec


def floor_body(z=0.0):
    return dict(pos=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0), shapes=[dict(type="plane", n=(0, 0, 1), d=z)])


# --------------------------------------------------------------------------
# Detection: cell list == brute force == exact rational predicate
# --------------------------------------------------------------------------
@pytest.mark.parametrize("cohesion", [0.0, 1000.0])
def test_detection_cells_equal_bruteforce(cohesion):
    rng = np.random.default_rng(7)
    n = 900
    r = SG.fp32(0.05 * rng.uniform(0.9, 1.1, n))
    x = SG.fp32(rng.uniform(-0.45, 0.45, (n, 3)) * np.array([1.0, 1.0, 1.0]))
    spec = base_spec(x, r, [SG.walls_body(1.0, 1.0, -0.45)], c=cohesion)
    kb, db = O.detect(spec, O.BRUTE)
    kc, dc = O.detect(spec, O.CELLS)
    assert len(kb) > 2 * n
    assert np.array_equal(kb, kc)
    assert np.array_equal(db, dc)
    assert np.all(np.diff(kb.astype(np.float64)) > 0)  # canonical, strictly sorted


def test_detection_matches_exact_rational_predicate():
    rng = np.random.default_rng(11)
    n = 300
    r = SG.fp32(0.05 * rng.uniform(0.9, 1.1, n))
    x = SG.fp32(rng.uniform(-0.3, 0.3, (n, 3)))
    kc = 0.025
    spec = base_spec(x, r, [], c=1000.0)
    keys, _ = O.detect(spec, O.BRUTE)
    got = set(int(k) for k in keys)
    kcf = Fraction(kc)
    undecided = 0
    for i in range(n):
        xi = [Fraction(float(v)) for v in x[i]]
        for j in range(i + 1, n):
            d2 = sum((Fraction(float(x[j, k])) - xi[k]) ** 2 for k in range(3))
            R = (Fraction(float(r[i])) + Fraction(float(r[j]))) * (1 + kcf)
            gap = d2 - R * R
            key = (i << 32) | j
            if abs(gap) <= Fraction(1, 10 ** 12) * R * R:
                undecided += 1
                continue
            assert (gap < 0) == (key in got), (i, j, float(gap))
    assert undecided < 3


def test_detection_boundary_cases_at_one_ulp():
    # two spheres of radius 0.5 at distance exactly 1: touching is not a contact
    spec = base_spec([[0, 0, 0], [1.0, 0, 0]], [0.5, 0.5], [])
    assert len(O.detect(spec, O.BRUTE)[0]) == 0
    spec = base_spec([[0, 0, 0], [np.nextafter(1.0, 0.0), 0, 0]], [0.5, 0.5], [])
    assert len(O.detect(spec, O.BRUTE)[0]) == 1
    # a sphere exactly resting on a plane is not in contact; one ulp lower is
    spec = base_spec([[0, 0, 0.5]], [0.5], [floor_body()])
    assert len(O.detect(spec, O.BRUTE)[0]) == 0
    spec = base_spec([[0, 0, np.nextafter(0.5, 0.0)]], [0.5], [floor_body()])
    k, d = O.detect(spec, O.BRUTE)
    assert len(k) == 1 and int(k[0]) == (0x80000000 | 0) and d[0] > 0.0


def test_box_face_equals_plane_and_inside_rule():
    # a sphere under the top face of an axis-aligned box sees the same overlap
    # as against the equivalent plane
    r = 0.05
    z = 0.5 + r - 1e-4
    box = dict(pos=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0), shapes=[dict(type="box", half=(1.0, 1.0, 0.5))])
    plane = dict(pos=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0), shapes=[dict(type="plane", n=(0, 0, 1), d=0.5)])
    kb, db = O.detect(base_spec([[0.1, -0.2, z]], [r], [box]), O.BRUTE)
    kp, dp = O.detect(base_spec([[0.1, -0.2, z]], [r], [plane]), O.BRUTE)
    assert len(kb) == 1 and len(kp) == 1
    assert db[0] == pytest.approx(dp[0], rel=1e-12, abs=1e-15)
    # centre inside: least-penetration face (+z here), overlap r + depth
    k, d = O.detect(base_spec([[0.3, 0.2, 0.45]], [r], [box]), O.BRUTE)
    assert d[0] == pytest.approx(r + 0.05, rel=1e-12)


# --------------------------------------------------------------------------
# Hertz / SPOOK mapping: resting column (closed form)
# --------------------------------------------------------------------------
def test_resting_column_impulses_and_overlaps():
    K, r = 5, 0.05
    m = sphere_mass(r)
    x = [[0.0, 0.0, r + 2 * r * k] for k in range(K)]
    spec = base_spec(x, [r] * K, [floor_body()], mu=0.0, c=0.0, sweeps=300)
    sc = O.OracleScene(spec)
    for _ in range(400):
        out = sc.step()
    keys, lam = out["keys"], out["lam"]
    kn_pair = ESTAR * math.sqrt(r) / 3.0          # d* = (1/2r + 1/2r)^-1 = r
    kn_wall = ESTAR * math.sqrt(2 * r) / 3.0      # d* = 2r
    assert kn_pair == pytest.approx(3.81e7, rel=2e-3)   # printed-scale check of k_n
    assert kn_wall == pytest.approx(5.39e7, rel=2e-3)
    found = 0
    for key, l in zip(keys, lam):
        a, b = int(key) >> 32, int(key) & 0xFFFFFFFF
        if b & 0x80000000:
            assert a == 0
            assert l[0] == pytest.approx(K * m * G * DT, rel=1e-7)
            delta = r - sc.x[0, 2]
            assert delta == pytest.approx((K * m * G / kn_wall) ** (2.0 / 3.0), rel=1e-5)
            found += 1
        else:
            k_above = K - b  # contacts from the top carry k m g dt
            assert l[0] == pytest.approx(k_above * m * G * DT, rel=1e-7)
            delta = 2 * r - (sc.x[b, 2] - sc.x[a, 2])
            assert delta == pytest.approx((k_above * m * G / kn_pair) ** (2.0 / 3.0), rel=1e-5)
            found += 1
    assert found == K
    assert np.max(np.abs(sc.v)) < 1e-9


def test_spook_tau_to_zero_limit():
    # Ideal stiff constraint: G v_{n+1} = -(4/dt) g (scaled row: g' = -4/5 delta)
    r, delta = 0.05, 1e-4
    spec = base_spec([[0.0, 0.0, r - delta]], [r], [floor_body()], g=(0.0, 0.0, 0.0), sweeps=1,
                     E=1e18, tau_n=1e-14)
    sc = O.OracleScene(spec)
    sc.step()
    assert sc.v[0, 2] == pytest.approx((4.0 / DT) * 0.8 * delta, rel=1e-6)


def test_zero_restitution_drop_does_not_rebound():
    # restitution 0 and tau_n = 2 dt: an impact is damped out, no rebound
    # (the damping of the printed SPOOK form is strong at tau = 2 dt)
    r, h0 = 0.05, 0.3
    spec = base_spec([[0.0, 0.0, r + h0]], [r], [floor_body()], mu=0.5, sweeps=5)
    sc = O.OracleScene(spec)
    touched, peak_after = False, -1.0
    for _ in range(150):
        out = sc.step()
        if out["contacts"] > 0:
            touched = True
        if touched:
            peak_after = max(peak_after, sc.x[0, 2] - r)
    assert touched
    assert peak_after < 0.01 * h0
    assert abs(sc.v[0, 2]) < 1e-6


# --------------------------------------------------------------------------
# Coulomb friction: sliding sphere (closed form, exact per step)
# --------------------------------------------------------------------------
def test_sliding_sphere_stick_slip():
    r, mu, v0 = 0.05, 0.3, 2.0
    m = sphere_mass(r)
    kn = ESTAR * math.sqrt(2 * r) / 3.0
    d0 = (m * G / kn) ** (2.0 / 3.0)
    spec = base_spec([[0.0, 0.0, r - d0]], [r], [floor_body()], mu=mu, v=[[v0, 0.0, 0.0]], sweeps=1)
    sc = O.OracleScene(spec)
    l2 = r - d0 / 2
    I = 0.4 * m * r * r
    kappa = m * l2 * l2 / I
    vprev, wprev = v0, 0.0
    slipping_steps = 0
    for _ in range(120):
        sc.step()
        vx, wy = sc.v[0, 0], sc.w[0, 1]
        slip_prev = vprev - l2 * wprev
        if slip_prev > mu * G * DT * (1 + kappa) * (1 + 1e-9):
            assert vx - vprev == pytest.approx(-mu * G * DT, rel=1e-9)
            assert wy - wprev == pytest.approx(mu * G * DT * m * l2 / I, rel=1e-9)
            slipping_steps += 1
        vprev, wprev = vx, wy
    assert slipping_steps > 10
    assert sc.v[0, 0] == pytest.approx(v0 * kappa / (1 + kappa), rel=1e-9)
    assert sc.v[0, 0] == pytest.approx(5.0 / 7.0 * v0, rel=2e-3)
    assert abs(sc.v[0, 0] - l2 * sc.w[0, 1]) < 1e-12


# --------------------------------------------------------------------------
# Heightfield: incline rolls or slips per the closed form; flat == plane
# --------------------------------------------------------------------------
def incline_hfield(tan_theta=0.5):
    l0, n = 0.25, 17
    ox = oy = -2.0
    xs = ox + l0 * np.arange(n)
    h = np.tile((-tan_theta * xs).astype(np.float32), (n, 1))  # h[j, i]
    return dict(pos=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0),
                shapes=[dict(type="hfield", nx=n, ny=n, ox=ox, oy=oy, l0=l0, h=h.ravel())])


@pytest.mark.parametrize("mu,rolls", [(0.3, True), (0.1, False)])
def test_incline_roll_or_slip(mu, rolls):
    tan_t = 0.5
    th = math.atan(tan_t)
    r = 0.05
    m = sphere_mass(r)
    kn = ESTAR * math.sqrt(2 * r) / 3.0
    d0 = (m * G * math.cos(th) / kn) ** (2.0 / 3.0)
    nrm = np.array([math.sin(th), 0.0, math.cos(th)])
    x0 = (r - d0) * nrm  # surface passes through the origin
    spec = base_spec([x0], [r], [incline_hfield(tan_t)], mu=mu, sweeps=1)
    sc = O.OracleScene(spec)
    sdir = np.array([math.cos(th), 0.0, -math.sin(th)])  # down-slope
    l2 = r - d0 / 2
    I = 0.4 * m * r * r
    vs_prev = 0.0
    for k in range(20):
        sc.step()
        vs = float(sc.v[0] @ sdir)
        dv = vs - vs_prev
        if rolls:
            expect = G * math.sin(th) * DT / (1.0 + I / (m * l2 * l2))
        else:
            expect = G * (math.sin(th) - mu * math.cos(th)) * DT
        assert dv == pytest.approx(expect, rel=2e-6), k
        vs_prev = vs
    if rolls:
        assert (5.0 / 7.0) * G * math.sin(th) * DT == pytest.approx(expect, rel=3e-3)


def test_tilted_hfield_matches_plane():
    tan_t = 0.5
    th = math.atan(tan_t)
    r = 0.05
    nrm = (math.sin(th), 0.0, math.cos(th))
    plane = dict(pos=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0), shapes=[dict(type="plane", n=nrm, d=0.0)])
    x0 = (r - 3e-5) * np.array(nrm)
    a = O.OracleScene(base_spec([x0], [r], [incline_hfield(tan_t)], mu=0.3, sweeps=1))
    b = O.OracleScene(base_spec([x0], [r], [plane], mu=0.3, sweeps=1))
    for _ in range(10):
        a.step()
        b.step()
    assert np.allclose(a.v, b.v, rtol=1e-6, atol=1e-9)
    assert np.allclose(a.x, b.x, rtol=1e-9, atol=1e-12)


def test_flat_hfield_equals_plane_exactly():
    spec = SG.column_scene(seed=4, n=120, footprint=0.6, sweeps=20)
    flat = np.zeros(8 * 8, dtype=np.float32)
    hf = dict(type="hfield", nx=8, ny=8, ox=-2.0, oy=-2.0, l0=0.5, h=flat)
    spec_hf = dict(spec)
    walls = dict(spec["bodies"][0])
    walls_hf = dict(walls)
    walls_hf["shapes"] = [hf] + walls["shapes"][1:]
    spec_hf["bodies"] = [walls_hf]
    a, b = O.OracleScene(spec), O.OracleScene(spec_hf)
    for _ in range(30):
        oa, ob = a.step(), b.step()
        assert np.array_equal(oa["keys"], ob["keys"])
    assert np.array_equal(a.x, b.x)
    assert np.array_equal(a.v, b.v)
    assert np.array_equal(oa["lam"], ob["lam"])


# --------------------------------------------------------------------------
# Cohesion: a hanging sphere holds iff m g < c_p pi r^2
# --------------------------------------------------------------------------
@pytest.mark.parametrize("c,holds", [(1000.0, False), (2000.0, True)])
def test_hanging_cohesive_sphere(c, holds):
    r = 0.05
    m = sphere_mass(r)
    assert (m * G < c * math.pi * r * r) == holds
    ceiling = dict(pos=(0.0, 0.0, 0.0), quat=(1, 0, 0, 0), shapes=[dict(type="plane", n=(0, 0, -1), d=-1.0)])
    # sphere just touching the ceiling z = 1 from below
    spec = base_spec([[0.0, 0.0, 1.0 - r]], [r], [ceiling], mu=0.5, c=c, sweeps=5)
    sc = O.OracleScene(spec)
    for _ in range(60):
        out = sc.step()
    gap = (1.0 - r) - sc.x[0, 2]
    if holds:
        assert gap < 2 * 0.025 * r
        assert len(out["keys"]) == 1
        assert out["lam"][0, 0] == pytest.approx(-m * G * DT, rel=1e-6)
    else:
        assert gap > 0.5
        assert len(out["keys"]) == 0


# --------------------------------------------------------------------------
# Conservation: no gravity, no boundaries
# --------------------------------------------------------------------------
def test_momentum_and_angular_momentum_conserved():
    rng = np.random.default_rng(5)
    n = 200
    r = SG.fp32(0.05 * rng.uniform(0.9, 1.1, n))
    x, _ = SG.lattice(rng, n, 0.6, 0.6, 0.098, r)
    v = rng.normal(0, 0.5, (n, 3))
    w = rng.normal(0, 3.0, (n, 3))
    spec = base_spec(x, r, [], mu=0.5, c=1000.0, g=(0.0, 0.0, 0.0), v=v, w=w, sweeps=30)
    sc = O.OracleScene(spec)
    m = sphere_mass(r)
    I = 0.4 * m * r * r

    def moments():
        p = (m[:, None] * sc.v).sum(0)
        L = (m[:, None] * np.cross(sc.x, sc.v)).sum(0) + (I[:, None] * sc.w).sum(0)
        return p, L

    p0, L0 = moments()
    total = 0
    for _ in range(20):
        total += sc.step()["contacts"]
    p1, L1 = moments()
    assert total > 100
    scale_p = (m[:, None] * np.abs(sc.v)).sum()
    assert np.allclose(p0, p1, rtol=0, atol=1e-12 * scale_p)
    scale_L = (m[:, None] * np.abs(np.cross(sc.x, sc.v))).sum() + (I[:, None] * np.abs(sc.w)).sum()
    assert np.allclose(L0, L1, rtol=0, atol=1e-12 * scale_L)


# --------------------------------------------------------------------------
# Colouring: valid, order independent, equal to parallel Jones-Plassmann
# --------------------------------------------------------------------------
def splitmix64(x):
    M = (1 << 64) - 1
    z = (x + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def parts(key):
    a, b = key >> 32, key & 0xFFFFFFFF
    return (a,) if b & 0x80000000 else (a, b)


def jones_plassmann_rounds(keys):
    """Parallel JP: each round, every uncoloured vertex that beats all its
    uncoloured neighbours takes the least colour free among its coloured ones."""
    keys = [int(k) for k in keys]
    pr = {k: (splitmix64(k), k) for k in keys}
    inc = {}
    for k in keys:
        for p in parts(k):
            inc.setdefault(p, []).append(k)
    nbr = {k: set(e for p in parts(k) for e in inc[p] if e != k) for k in keys}
    col = {}
    rounds = 0
    while len(col) < len(keys):
        rounds += 1
        winners = [k for k in keys if k not in col and all(e in col or pr[e] < pr[k] for e in nbr[k])]
        new = {}
        for k in winners:
            used = {col[e] for e in nbr[k] if e in col}
            c = 0
            while c in used:
                c += 1
            new[k] = c
        col.update(new)
    return col, rounds, nbr


def settled(seed, n, steps, sweeps=10, footprint=0.5):
    spec = SG.column_scene(seed=seed, n=n, footprint=footprint, fill=0.45, sweeps=sweeps)
    sc = O.OracleScene(spec)
    for _ in range(steps):
        sc.step()
    out = dict(spec)
    out.update(x=sc.x.copy(), v=sc.v.copy(), w=sc.w.copy())
    return out


def test_colouring_valid_and_equal_to_parallel_jp():
    spec = settled(9, 400, 60)
    out = O.OracleScene(spec).step()
    keys, colour = out["keys"], out["colour"]
    assert len(keys) > 300
    jp, rounds, nbr = jones_plassmann_rounds(keys)
    for k, c in zip(keys, colour):
        assert jp[int(k)] == c
        for e in nbr[int(k)]:
            assert jp[e] != c
    assert out["colours"] == max(colour) + 1
    assert rounds >= 3


def test_colouring_independent_of_input_order():
    spec = settled(10, 300, 60)
    a = O.OracleScene(spec)
    oa = a.step()
    perm = np.random.default_rng(0).permutation(len(spec["x"]))
    spec_p = dict(spec)
    for k in ("x", "v", "w"):
        spec_p[k] = spec[k][perm]
    spec_p["r"] = spec["r"][perm]
    spec_p["id"] = spec["id"][perm]
    b = O.OracleScene(spec_p)
    ob = b.step()
    assert np.array_equal(oa["keys"], ob["keys"])
    assert np.array_equal(oa["colour"], ob["colour"])
    assert np.array_equal(oa["lam"], ob["lam"])
    inv = np.argsort(perm)
    assert np.array_equal(a.v, b.v[inv])


# --------------------------------------------------------------------------
# PGS convergence: the natural-map residual goes to zero
# --------------------------------------------------------------------------
def test_natural_residual_vanishes_with_sweeps():
    spec = SG.column_scene(seed=12, n=150, footprint=0.4, fill=0.5, sweeps=40)
    sc = O.OracleScene(spec)
    for _ in range(40):
        sc.step()
    res = []
    for sweeps in (5, 500, 20000):
        s2 = dict(spec)
        s2.update(x=sc.x.copy(), v=sc.v.copy(), w=sc.w.copy(), max_sweeps=sweeps)
        t = O.OracleScene(s2)
        x0, v0, w0 = t.x.copy(), t.v.copy(), t.w.copy()
        out = t.step()
        res.append(t.natural_residual(x0, v0, w0, out["lam"]))
    assert res[0] > res[1] > res[2]
    assert res[2] < 1e-6


def test_prev_warm_start_speeds_up_convergence():
    spec = SG.column_scene(seed=13, n=200, footprint=0.4, fill=0.5, sweeps=60)
    spec["warm_start"] = "prev"
    sc = O.OracleScene(spec)
    for _ in range(40):
        out = sc.step()
    s_cold = dict(spec)
    s_cold.update(x=sc.x.copy(), v=sc.v.copy(), w=sc.w.copy(), warm_start="cold", max_sweeps=1)
    cold = O.OracleScene(s_cold).step()
    warm = O.OracleScene(dict(s_cold, warm_start="prev"))
    warm.prev_keys, warm.prev_lam = sc.prev_keys.copy(), sc.prev_lam.copy()
    ow = warm.step()
    assert ow["r1"] < 0.5 * cold["r1"]


# --------------------------------------------------------------------------
# Aggregates (Eqs. aggregate_mass .. aggregate_rot_vel): closed forms
# --------------------------------------------------------------------------
BIG_ZONE = [[1, 0, 0, 10], [-1, 0, 0, 10], [0, 1, 0, 10], [0, -1, 0, 10], [0, 0, 1, 10], [0, 0, -1, 10]]


def zone_body(planes=BIG_ZONE, pos=(0.0, 0.0, 0.0)):
    return dict(pos=pos, quat=(1, 0, 0, 0), zone_planes=planes, shapes=[])


def test_aggregate_single_sphere_and_dumbbell():
    r, m = 0.05, 1.7
    a = O.aggregates([[0.3, -0.1, 0.2]], np.zeros((1, 3)), np.zeros((1, 3)), [r], [m], [zone_body()])[0]
    Is = 0.4 * m * r * r
    assert a["M"] == m and a["n_particles"] == 1
    assert np.allclose(a["I"], [Is, Is, Is, 0, 0, 0], rtol=1e-14, atol=1e-18)
    d = 0.4
    a = O.aggregates([[d, 0, 0], [-d, 0, 0]], np.zeros((2, 3)), np.zeros((2, 3)), [r, r], [m, m],
                     [zone_body()])[0]
    assert np.allclose(a["x"], 0.0)
    assert np.allclose(a["I"], [2 * Is, 2 * Is + 2 * m * d * d, 2 * Is + 2 * m * d * d, 0, 0, 0], rtol=1e-13)


def test_aggregate_rigid_motion():
    rng = np.random.default_rng(3)
    n = 50
    x = rng.uniform(-1, 1, (n, 3))
    r = rng.uniform(0.02, 0.06, n)
    m = rng.uniform(0.5, 2.0, n)
    vt = np.array([0.3, -1.2, 0.5])
    a = O.aggregates(x, np.tile(vt, (n, 1)), np.zeros((n, 3)), r, m, [zone_body()])[0]
    assert np.allclose(a["v"], vt, rtol=1e-14)
    assert np.allclose(a["w"], 0.0, atol=1e-14)
    om = np.array([0.7, -0.2, 1.9])
    c = np.array([0.1, 0.2, -0.3])
    v = vt + np.cross(om, x - c)
    a = O.aggregates(x, v, np.tile(om, (n, 1)), r, m, [zone_body()])[0]
    assert np.allclose(a["w"], om, rtol=1e-12)
    assert np.allclose(a["v"], vt + np.cross(om, a["x"] - c), rtol=1e-12)


def test_zone_membership_first_body_wins():
    x = np.array([[0.0, 0, 0], [2.0, 0, 0], [5.0, 0, 0]])
    b1 = zone_body([[1, 0, 0, 1.0]])          # x <= 1
    b2 = zone_body([[1, 0, 0, 3.0]])          # x <= 3
    aggs = O.aggregates(x, np.zeros((3, 3)), np.zeros((3, 3)), [0.05] * 3, [1.0] * 3, [b1, b2])
    assert [a["n_particles"] for a in aggs] == [1, 1]
    # zone planes move with the body pose
    b3 = zone_body([[1, 0, 0, 0.0]], pos=(4.0, 0.0, 0.0))  # x <= 4 in the world
    assert O.aggregates(x, np.zeros((3, 3)), np.zeros((3, 3)), [0.05] * 3, [1.0] * 3, [b3])[0]["n_particles"] == 2


def test_failure_plane_reduces_to_rankine():
    for phi_deg in (20, 30, 40, 44.5):
        phi = math.radians(phi_deg)
        assert O.failure_angle(phi, math.pi / 2) == pytest.approx(math.pi / 4 - phi / 2, rel=1e-15)
    # a sloped separation plate steepens the wedge by half the slope
    assert O.failure_angle(0.7, 0.5) - O.failure_angle(0.7, 0.6) == pytest.approx(0.05, rel=1e-12)


# --------------------------------------------------------------------------
# MLP: FP64 gradients against central finite differences
# --------------------------------------------------------------------------
def random_mlp(seed=0):
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(0, 0.4, (64, 12)), b1=rng.normal(0, 0.1, 64), W2=rng.normal(0, 0.15, (64, 64)),
                b2=rng.normal(0, 0.1, 64), W3=rng.normal(0, 0.15, (3, 64)), b3=rng.normal(0, 0.1, 3),
                in_scale=rng.uniform(0.5, 2.0, 12))


def test_mlp_gradient_matches_finite_differences():
    net = random_mlp(1)
    rng = np.random.default_rng(2)
    feat = rng.normal(0, 1, (7, 12))
    label = rng.normal(0, 1, (7, 3))
    loss, grads = O.mlp_loss_grad(net, feat, label)
    y = O.mlp_forward(net, feat)
    assert loss == pytest.approx(0.5 * np.mean(np.sum((y - label) ** 2, axis=1)), rel=1e-13)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = net[name].reshape(-1)
        for idx in rng.choice(len(flat), size=min(6, len(flat)), replace=False):
            orig = flat[idx]
            flat[idx] = orig + eps
            lp, _ = O.mlp_loss_grad(net, feat, label)
            flat[idx] = orig - eps
            lm, _ = O.mlp_loss_grad(net, feat, label)
            flat[idx] = orig
            fd = (lp - lm) / (2 * eps)
            assert grads[name].reshape(-1)[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10), (name, idx)


# --------------------------------------------------------------------------
# Learned start (residual form): special cases that reduce to the previous-
# step start
# --------------------------------------------------------------------------
def _fork(src, spec, mlp=None, **kw):
    """A scene in src's state (positions, velocities, contact cache)."""
    from helpers import with_
    o = O.OracleScene(with_(spec, **kw), mlp=mlp)
    o.x, o.v, o.w = src.x.copy(), src.v.copy(), src.w.copy()
    o.prev_keys, o.prev_lam = src.prev_keys.copy(), src.prev_lam.copy()
    return o


def _zero_net():
    net = random_mlp(3)
    net["W3"] = np.zeros((3, 64))
    net["b3"] = np.zeros(3)
    return net


def test_learned_start_with_zero_output_is_the_previous_step_start():
    from helpers import settled_column, with_
    spec = with_(settled_column(seed=31, n=250, footprint=0.5), max_sweeps=30)
    src = O.OracleScene(with_(spec, warm_start="prev"))
    src.step()  # builds the contact cache
    a = _fork(src, spec, warm_start="prev")
    b = _fork(src, spec, mlp=_zero_net(), warm_start="learned")
    oa, ob = a.step(), b.step()
    assert np.array_equal(oa["keys"], ob["keys"]) and oa["sweeps"] == ob["sweeps"]
    # both trial starts are the previous-step impulses: equal first-sweep residuals
    r1l, r1p = ob["r1_trial"]
    assert r1p > 0 and abs(r1l - r1p) <= 1e-12 * r1p
    scale = max(np.max(np.abs(a.v)), 1e-9)
    assert np.max(np.abs(a.v - b.v)) <= 1e-12 * scale
    assert np.max(np.abs(oa["lam"] - ob["lam"])) <= 1e-12 * max(np.max(np.abs(oa["lam"])), 1e-12)


def test_learned_start_nonfinite_output_falls_back_to_previous_step_exactly():
    from helpers import settled_column, with_
    spec = with_(settled_column(seed=32, n=250, footprint=0.5), max_sweeps=20)
    src = O.OracleScene(with_(spec, warm_start="prev"))
    src.step()
    net = _zero_net()
    net["b3"] = np.array([np.inf, 0.0, 0.0])
    a = _fork(src, spec, warm_start="prev")
    b = _fork(src, spec, mlp=net, warm_start="learned")
    oa, ob = a.step(), b.step()
    assert ob["fallback_used"] == 1 and ob["learned_used"] == 0
    assert np.array_equal(a.v, b.v) and np.array_equal(a.w, b.w)
    assert np.array_equal(oa["lam"], ob["lam"])


# --------------------------------------------------------------------------
# Rolling resistance (Eq. signCoul3): closed forms of one sphere, conservation
# --------------------------------------------------------------------------
def test_rolling_resistance_decelerates_a_rolling_sphere():
    r, mu_t, mu_r, v0 = 0.05, 0.5, 0.1, 1.5
    m = sphere_mass(r)
    I = 0.4 * m * r * r
    kn = ESTAR * math.sqrt(2 * r) / 3.0
    d0 = (m * G / kn) ** (2.0 / 3.0)
    l = r - d0 / 2
    spec = base_spec([[0.0, 0.0, r - d0]], [r], [floor_body()], mu=mu_t, v=[[v0, 0.0, 0.0]],
                     w=[[0.0, v0 / l, 0.0]], sweeps=400, mu_r=mu_r)
    sc = O.OracleScene(spec)
    # the rolling couple r mu_r lambda_n (lambda_n = m g dt) against the rolling
    # inertia about the contact point: dv = -l r mu_r m g dt / (I + m l^2)
    expect = -l * r * mu_r * m * G * DT / (I + m * l * l)
    assert expect == pytest.approx(-5.0 / 7.0 * mu_r * G * DT, rel=2e-3)
    vprev = v0
    for k in range(25):
        out = sc.step()
        assert sc.v[0, 0] - vprev == pytest.approx(expect, rel=1e-6), k
        assert abs(sc.v[0, 0] - l * sc.w[0, 1]) < 1e-9  # still rolling without slip
        lr = out["lr"][0]
        assert np.linalg.norm(lr) == pytest.approx(r * mu_r * m * G * DT, rel=1e-6)  # the bound is active
        vprev = sc.v[0, 0]


def test_rolling_resistance_stops_a_spinning_sphere():
    # spin about the contact normal: no slip at the contact point, only the
    # rolling row acts: d omega_z = -r mu_r m g dt / I = -(5/2) mu_r g dt / r
    r, mu_r, w0 = 0.05, 0.2, 30.0
    m = sphere_mass(r)
    kn = ESTAR * math.sqrt(2 * r) / 3.0
    d0 = (m * G / kn) ** (2.0 / 3.0)
    spec = base_spec([[0.0, 0.0, r - d0]], [r], [floor_body()], mu=0.5, w=[[0.0, 0.0, w0]], sweeps=5, mu_r=mu_r)
    sc = O.OracleScene(spec)
    step = 2.5 * mu_r * G * DT / r
    wprev = w0
    for k in range(int(w0 / step) + 3):
        sc.step()
        expect = max(wprev - step, 0.0)
        assert sc.w[0, 2] == pytest.approx(expect, rel=1e-9, abs=1e-9), k
        wprev = sc.w[0, 2]
    assert sc.w[0, 2] == 0.0 or abs(sc.w[0, 2]) < 1e-9


@pytest.mark.parametrize("mu_r,tan_t,rolls", [(0.3, 0.2, False), (0.1, 0.5, True)])
def test_rolling_resistance_on_an_incline(mu_r, tan_t, rolls):
    th = math.atan(tan_t)
    r = 0.05
    m = sphere_mass(r)
    I = 0.4 * m * r * r
    kn = ESTAR * math.sqrt(2 * r) / 3.0
    d0 = (m * G * math.cos(th) / kn) ** (2.0 / 3.0)
    nrm = np.array([math.sin(th), 0.0, math.cos(th)])
    x0 = (r - d0) * nrm
    spec = base_spec([x0], [r], [incline_hfield(tan_t)], mu=0.8, sweeps=400, mu_r=mu_r)
    sc = O.OracleScene(spec)
    sdir = np.array([math.cos(th), 0.0, -math.sin(th)])
    l = r - d0 / 2
    a = (m * G * math.sin(th) * DT - r * mu_r * m * G * math.cos(th) * DT / l) / (m + I / (l * l))
    assert (a > 0) == rolls
    vs_prev = 0.0
    for k in range(15):
        sc.step()
        vs = float(sc.v[0] @ sdir)
        if rolls:
            assert vs - vs_prev == pytest.approx(a, rel=1e-5), k
        else:
            assert abs(vs) < 1e-9 * G * DT, k  # held by the rolling couple
        vs_prev = vs


def test_rolling_couples_conserve_angular_momentum():
    # two overlapping spheres in free space with opposite spins: the rolling
    # couples are equal and opposite, friction forces act at a shared point
    r = 0.05
    x = [[0.0, 0.0, 0.0], [2 * r - 2e-4, 0.0, 0.0]]
    w = [[3.0, 5.0, -2.0], [-4.0, 1.0, 6.0]]
    v = [[0.1, 0.0, 0.2], [-0.1, 0.05, 0.0]]
    spec = base_spec(x, [r, r], [], mu=0.5, g=(0.0, 0.0, 0.0), v=v, w=w, sweeps=20, mu_r=0.2)
    sc = O.OracleScene(spec)
    m = sphere_mass(r)
    I = 0.4 * m * r * r

    def ang():
        return sum(m * np.cross(sc.x[i], sc.v[i]) + I * sc.w[i] for i in range(2))
    for k in range(3):
        L0 = ang()
        out = sc.step()
        if k == 0:  # in contact on the first step (they separate afterwards)
            assert np.linalg.norm(out["lr"][0]) > 0.0
        # positions advanced with the new velocities: compare at the same positions
        x_new = sc.x.copy()
        sc.x = x_new - DT * sc.v
        L1 = ang()
        sc.x = x_new
        assert np.allclose(L1, L0, rtol=0, atol=1e-12 * (np.linalg.norm(L0) + 1e-9))


# --------------------------------------------------------------------------
# Impact stage (Newton law before the main solve): closed forms of collisions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("e", [0.25, 0.5, 1.0])
def test_impact_stage_bounce_off_the_floor(e):
    # a sphere touching the floor approaches at v0 > v_imp: it leaves at e v0,
    # then gravity acts over the step (the separating contact carries no load)
    r, v0 = 0.05, 3.0
    m = sphere_mass(r)
    spec = base_spec([[0.0, 0.0, r - 1e-6]], [r], [floor_body()], mu=0.5, v=[[0.0, 0.0, -v0]], sweeps=20,
                     restitution=e, v_imp=1.0)
    sc = O.OracleScene(spec)
    out = sc.step()
    assert out["impacts"] == 1 and out["impact_sweeps"] == 20
    assert sc.v[0, 2] == pytest.approx(e * v0 - G * DT, rel=1e-12)
    assert abs(sc.v[0, 0]) < 1e-15 and abs(sc.v[0, 1]) < 1e-15
    # the floor received the impact impulse m (1 + e) v0 (reported as impulse / dt)
    assert out["body_ft"][0][2] == pytest.approx(-m * (1.0 + e) * v0 / DT, rel=1e-12)


def test_impact_stage_threshold_and_disabled_agree_below_threshold():
    # no contact approaches faster than v_imp: the step is the plain step, bit for bit
    spec = SG.column_scene(seed=4, n=300, sweeps=15, footprint=0.5, c=0.0, mu=0.5)
    plain = O.OracleScene(spec)
    gated = O.OracleScene(dict(spec, material=dict(spec["material"], restitution=0.5, v_imp=50.0)))
    for _ in range(3):
        a, b = plain.step(), gated.step()
        assert b["impacts"] == 0 and b["impact_sweeps"] == 0
        assert np.array_equal(plain.v, gated.v) and np.array_equal(plain.w, gated.w)
        assert np.array_equal(a["lam"], b["lam"])


@pytest.mark.parametrize("e", [0.0, 0.3, 1.0])
def test_impact_stage_head_on_pair(e):
    # two spheres of different mass, approaching along their line of centres:
    # Newton's law with momentum conservation, and (e = 1) kinetic energy kept
    r1, r2, U1, U2 = 0.05, 0.04, 1.5, 0.7
    m1, m2 = sphere_mass(r1), sphere_mass(r2)
    spec = base_spec([[0.0, 0.0, 0.0], [r1 + r2 - 1e-6, 0.0, 0.0]], [r1, r2], [], mu=0.4, g=(0.0, 0.0, 0.0),
                     v=[[U1, 0.0, 0.0], [-U2, 0.0, 0.0]], sweeps=10, restitution=e, v_imp=0.5)
    sc = O.OracleScene(spec)
    out = sc.step()
    assert out["impacts"] == 1
    P = (1.0 + e) * (U1 + U2) / (1.0 / m1 + 1.0 / m2)
    if e > 0.0:
        # separating after the impact: the main solve adds nothing
        assert sc.v[0, 0] == pytest.approx(U1 - P / m1, rel=1e-12)
        assert sc.v[1, 0] == pytest.approx(-U2 + P / m2, rel=1e-12)
        assert sc.v[1, 0] - sc.v[0, 0] == pytest.approx(e * (U1 + U2), rel=1e-12)
    assert m1 * sc.v[0, 0] + m2 * sc.v[1, 0] == pytest.approx(m1 * U1 - m2 * U2, rel=1e-12)
    if e == 1.0:
        ke0 = 0.5 * (m1 * U1 ** 2 + m2 * U2 ** 2)
        ke1 = 0.5 * (m1 * sc.v[0, 0] ** 2 + m2 * sc.v[1, 0] ** 2)
        assert ke1 == pytest.approx(ke0, rel=1e-12)


@pytest.mark.parametrize("vx,mu,sticks", [(0.4, 0.5, True), (4.0, 0.2, False)])
def test_impact_stage_oblique_impact_with_friction(vx, mu, sticks):
    # a non-spinning sphere hits the floor obliquely: normal impulse P_n = m (1+e) v0;
    # the friction impulse stops the slip when that needs no more than mu P_n
    # (then v_x' = v_x (m l^2/I) / (1 + m l^2/I), 5/7 v_x for l = r), else slides
    r, v0, e = 0.05, 2.0, 0.4
    m = sphere_mass(r)
    I = 0.4 * m * r * r
    d0 = 1e-6
    l = r - d0 / 2
    spec = base_spec([[0.0, 0.0, r - d0]], [r], [floor_body()], mu=mu, v=[[vx, 0.0, -v0]], sweeps=20,
                     restitution=e, v_imp=1.0)
    sc = O.OracleScene(spec)
    sc.step()
    Pn = m * (1.0 + e) * v0
    Pstick = vx / (1.0 / m + l * l / I)
    assert (Pstick <= mu * Pn) == sticks
    Pt = Pstick if sticks else mu * Pn
    assert sc.v[0, 0] == pytest.approx(vx - Pt / m, rel=1e-12)
    assert sc.w[0, 1] == pytest.approx(l * Pt / I, rel=1e-12)
    assert sc.v[0, 2] == pytest.approx(e * v0 - G * DT, rel=1e-12)
    if sticks:
        assert sc.v[0, 0] == pytest.approx(vx * (m * l * l / I) / (1.0 + m * l * l / I), rel=1e-12)
        assert abs(sc.v[0, 0] - l * sc.w[0, 1]) < 1e-12  # rolling without slip


def test_impact_stage_conserves_momentum_in_a_cluster():
    # a jittered cluster flying apart and together in free space: the impact
    # stage and the main solve exchange only pair impulses and couples
    rng = np.random.default_rng(12)
    r = 0.05
    g = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = SG.fp32(g * (2 * r - 0.004) + rng.uniform(-0.001, 0.001, (27, 3)))
    v = SG.fp32(rng.normal(0.0, 2.0, (27, 3)))
    w = SG.fp32(rng.normal(0.0, 5.0, (27, 3)))
    spec = base_spec(x, [r] * 27, [], mu=0.5, g=(0.0, 0.0, 0.0), v=v, w=w, sweeps=30, restitution=0.4,
                     v_imp=0.5, mu_r=0.1)
    sc = O.OracleScene(spec)
    m = sphere_mass(r)
    I = 0.4 * m * r * r
    p0 = m * np.sum(sc.v, axis=0)
    L0 = np.sum(m * np.cross(sc.x, sc.v) + I * sc.w, axis=0)
    out = sc.step()
    assert out["impacts"] > 0
    p1 = m * np.sum(sc.v, axis=0)
    assert np.allclose(p1, p0, rtol=0, atol=1e-12 * m * np.sum(np.abs(v)))
    xs = sc.x - DT * sc.v  # the start-of-step positions
    L1 = np.sum(m * np.cross(xs, sc.v) + I * sc.w, axis=0)
    assert np.allclose(L1, L0, rtol=0, atol=1e-12 * (np.linalg.norm(L0) + m * r))


def test_restitution_outside_unit_interval_is_rejected():
    spec = base_spec([[0.0, 0.0, 0.04]], [0.05], [floor_body()], restitution=1.5, v_imp=1.0)
    with pytest.raises(RuntimeError):
        O.OracleScene(spec).step()


def test_impact_stage_inelastic_then_resting_row_uses_post_impact_velocity():
    # e = 0: the impact stops the approach; the main solve's SPOOK row then sees
    # the post-impact normal velocity 0 (its target is the overlap term alone),
    # so one contact's closed form holds: v = v* + W (q - v*) / (W + Sigma),
    # v* = -g dt, q = (4/dt) Ups 0.8 delta, Ups = 1/(1 + 4 tau/dt), tau = 2 dt
    r, v0, d0 = 0.05, 3.0, 1e-6
    m = sphere_mass(r)
    spec = base_spec([[0.0, 0.0, r - d0]], [r], [floor_body()], mu=0.5, v=[[0.0, 0.0, -v0]], sweeps=20,
                     restitution=0.0, v_imp=1.0)
    sc = O.OracleScene(spec)
    sc.step()
    ups = 1.0 / (1.0 + 8.0)
    kn = ESTAR * math.sqrt(2 * r) / 3.0
    de = max(d0, 1e-4 * 2 * r)
    sig = (4.0 / DT ** 2) * (4.0 / (5.0 * kn * math.sqrt(de))) * ups
    q = (4.0 / DT) * ups * 0.8 * d0
    vstar = -G * DT
    W = 1.0 / m
    expect = vstar + W * (q - vstar) / (W + sig)
    assert sc.v[0, 2] == pytest.approx(expect, rel=1e-9)
    assert abs(sc.v[0, 2]) < 0.01 * v0  # the approach v0 is gone, not a ninth of it


def test_impact_stage_keeps_the_resting_contacts():
    # sphere B falls on sphere A resting on the floor: the A-floor contact is no
    # impact but keeps G_n v+ >= 0 in the stage, so A stays and B leaves at e v0
    r, v0, e = 0.05, 2.0, 0.6
    spec = base_spec([[0.0, 0.0, r - 1e-6], [0.0, 0.0, 3 * r - 3e-6]], [r, r], [floor_body()], mu=0.3,
                     v=[[0.0, 0.0, 0.0], [0.0, 0.0, -v0]], sweeps=80, restitution=e, v_imp=1.0)
    sc = O.OracleScene(spec)
    out = sc.step()
    assert out["impacts"] == 1 and out["contacts"] == 2
    assert sc.v[1, 2] == pytest.approx(e * v0 - G * DT, rel=1e-9)
    assert abs(sc.v[0, 2]) < 1e-3 * v0
