"""Conversion between resting solid and fluidized mass in the oracle (the
passage on converting overlapping soil; Eq. surface).

Pins, each against geometry or arithmetic fixed outside the oracle's code:
  - Eq. surface on hand-built columns (full, partial, empty);
  - a hand-written Rankine wedge over level ground: the liberated mass is the
    sum over the cut columns of rho_b l0^2 (h0 - z_fail(x)), the new surface
    is z_fail there, every other column keeps h0;
  - a deposit raises the surface by m / (w_dep rho_b l0^2), whatever the voxel
    boundaries crossed, with the mass-weighted compaction of a voxel being
    filled; fluid beside particles or inside a zone stays; a full column
    keeps what does not fit;
  - cut followed by deposit with no zone and no particles is the identity;
  - solid plus fluid mass is conserved to rounding on random terrain with the
    predictor's wedges;
  - particle growth (Eq. eqmotmb): the mass bound 3 m d'_max / d is a diameter
    rate d'_max (Taylor expansion), growth stops at d_max and outside the
    grid, scarce fluid is used up and shared in the ratio of the bounds
    ((r1/r2)^2), particle plus fluid mass is conserved.
"""
import math

import numpy as np
import pytest

import pyoracle as O

L0 = 0.1
DIMS = (24, 10, 12)  # nx, ny, nz
ORIGIN = (-1.0, -0.5, 0.0)
RHO_B = 1800.0
V0 = L0 ** 3


def columns(h):
    """Occupancy of columns filled to the heights h (ny, nx) from the grid's bottom."""
    zb = ORIGIN[2] + L0 * np.arange(DIMS[2])
    return np.clip((np.asarray(h)[None, :, :] - zb[:, None, None]) / L0, 0.0, 1.0)


def solid_mass(phi, wc):
    return float(np.sum(wc * phi) * RHO_B * V0)


def test_surface_heights_closed_forms():
    phi = np.zeros((DIMS[2], DIMS[1], DIMS[0]))
    phi[:3, 0, 0] = 1.0
    phi[3, 0, 0] = 0.25       # three full voxels and a quarter
    phi[:, 1, 0] = 1.0        # a full column
    phi[0, 2, 0] = 0.5        # half a voxel
    h = O.surface_heights(phi, ORIGIN, L0, DIMS)
    assert h[0, 0] == pytest.approx(ORIGIN[2] + 3.25 * L0, abs=1e-15)
    assert h[1, 0] == pytest.approx(ORIGIN[2] + DIMS[2] * L0, abs=1e-15)
    assert h[2, 0] == pytest.approx(ORIGIN[2] + 0.5 * L0, abs=1e-15)
    assert h[3, 0] == ORIGIN[2]  # empty column: the grid's bottom
    hh = np.random.default_rng(1).uniform(0.05, 1.15, (DIMS[1], DIMS[0]))
    assert np.allclose(O.surface_heights(columns(hh), ORIGIN, L0, DIMS), hh, rtol=0, atol=1e-14)


def rankine_wedge(ex, ez, theta, top, half_width):
    # in front of the plate x >= ex, above the failure line z >= ez + (x - ex) tan(theta),
    # below the top, between the lateral planes
    t = math.tan(theta)
    return np.array([[-1.0, 0.0, 0.0, -ex],
                     [t, 0.0, -1.0, t * ex - ez],
                     [0.0, 0.0, 1.0, top],
                     [0.0, 1.0, 0.0, half_width],
                     [0.0, -1.0, 0.0, half_width]])


def test_cut_of_level_ground_by_a_rankine_wedge():
    h0, ex, ez, theta, top, hw = 0.83, -0.35, 0.41, math.radians(27.5), 0.9, 0.25
    phi = columns(np.full((DIMS[1], DIMS[0]), h0))
    wc = np.ones_like(phi)
    mf = np.zeros_like(phi)
    W = rankine_wedge(ex, ez, theta, top, hw)
    phi2, mf2, lib = O.convert_cut(phi, wc, mf, [W], ORIGIN, L0, DIMS, RHO_B)
    xc = ORIGIN[0] + L0 * (np.arange(DIMS[0]) + 0.5)
    yc = ORIGIN[1] + L0 * (np.arange(DIMS[1]) + 0.5)
    zf = ez + (xc - ex) * math.tan(theta)
    cut_x = (xc >= ex) & (zf <= top)
    cut_y = np.abs(yc) <= hw
    expect_h = np.full((DIMS[1], DIMS[0]), h0)
    for j in np.nonzero(cut_y)[0]:
        for i in np.nonzero(cut_x)[0]:
            expect_h[j, i] = min(h0, zf[i])
    assert np.sum(expect_h < h0) > 10
    h = O.surface_heights(phi2, ORIGIN, L0, DIMS)
    assert np.allclose(h, expect_h, rtol=0, atol=1e-13)
    assert lib == pytest.approx(RHO_B * L0 ** 2 * np.sum(h0 - expect_h), rel=1e-12)
    # the liberated mass sits in the voxels that held it
    assert np.sum(mf2) == pytest.approx(lib, rel=1e-14)
    assert np.all(mf2[phi2 >= phi] == 0.0)
    assert solid_mass(phi2, wc) + np.sum(mf2) == pytest.approx(solid_mass(phi, wc), rel=1e-14)


def test_deposit_raises_the_surface():
    h0, w_dep = 0.43, 0.8
    phi = columns(np.full((DIMS[1], DIMS[0]), h0))
    wc = np.ones_like(phi)
    mf = np.zeros_like(phi)
    rho_p = np.zeros_like(phi)
    m = 2.5 * w_dep * RHO_B * L0 ** 2 * L0  # 2.5 voxels' worth at the loose density
    mf[9, 3, 5] = m                          # high above the surface, no particles
    mf[9, 4, 5] = 1.0
    rho_p[9, 4, 5] = 10.0                    # beside particles: stays
    mf[9, 5, 5] = 1.0                        # inside a zone: stays
    W = np.array([[1.0, 0, 0, ORIGIN[0] + 5.9 * L0], [-1.0, 0, 0, -(ORIGIN[0] + 5.1 * L0)],
                  [0, 1.0, 0, ORIGIN[1] + 5.9 * L0], [0, -1.0, 0, -(ORIGIN[1] + 5.1 * L0)],
                  [0, 0, -1.0, -0.0]])
    phi2, wc2, mf2, dep = O.convert_deposit(phi, wc, mf, rho_p, [W], ORIGIN, L0, DIMS, RHO_B, w_dep)
    h = O.surface_heights(phi2, ORIGIN, L0, DIMS)
    assert dep == pytest.approx(m, rel=1e-14)
    assert h[3, 5] == pytest.approx(h0 + m / (w_dep * RHO_B * L0 ** 2), rel=1e-13)
    assert mf2[9, 3, 5] == 0.0 and mf2[9, 4, 5] == 1.0 and mf2[9, 5, 5] == 1.0
    # the voxel that was partly full holds the mass-weighted compaction
    k = int((h0 - ORIGIN[2]) // L0)
    f0 = (h0 - ORIGIN[2]) / L0 - k
    assert wc2[k, 3, 5] == pytest.approx((f0 * 1.0 + (1 - f0) * w_dep) / 1.0, rel=1e-13)
    assert wc2[k + 1, 3, 5] == pytest.approx(w_dep, rel=1e-15)
    assert solid_mass(phi2, wc2) + np.sum(mf2) == pytest.approx(solid_mass(phi, wc) + np.sum(mf), rel=1e-14)
    # a full column keeps the rest as fluid
    full = np.ones_like(phi)
    mf3 = np.zeros_like(phi)
    mf3[-1, 0, 0] = 3.0
    phi4, _, mf4, dep4 = O.convert_deposit(full, wc, mf3, rho_p, [], ORIGIN, L0, DIMS, RHO_B, w_dep)
    assert dep4 == 0.0 and mf4[-1, 0, 0] == 3.0 and np.array_equal(phi4, full)


def test_cut_then_deposit_is_the_identity():
    rng = np.random.default_rng(4)
    h0 = rng.uniform(0.3, 1.0, (DIMS[1], DIMS[0]))
    phi = columns(h0)
    wc = np.ones_like(phi)
    W = rankine_wedge(-0.6, 0.2, math.radians(30), 1.1, 0.3)
    phi2, mf2, lib = O.convert_cut(phi, wc, np.zeros_like(phi), [W], ORIGIN, L0, DIMS, RHO_B)
    assert lib > 0
    phi3, wc3, mf3, dep = O.convert_deposit(phi2, wc, mf2, np.zeros_like(phi), [], ORIGIN, L0, DIMS, RHO_B, 1.0)
    assert dep == pytest.approx(lib, rel=1e-13) and not mf3.any()
    assert np.allclose(O.surface_heights(phi3, ORIGIN, L0, DIMS), h0, rtol=0, atol=1e-13)
    assert np.allclose(wc3, 1.0, rtol=1e-13)


def test_mass_conserved_with_predicted_wedges():
    rng = np.random.default_rng(9)
    nx, ny = DIMS[0], DIMS[1]
    hh = 0.6 + 0.08 * np.sin(np.linspace(0, 3, nx))[None, :] + 0.02 * rng.normal(size=(ny, nx))
    # the heightfield of the predictor shares the columns' centres
    terrain = dict(pos=(0, 0, 0), quat=(1, 0, 0, 0), linvel=(0, 0, 0), angvel=(0, 0, 0),
                   shapes=[dict(type="hfield", nx=nx, ny=ny, ox=ORIGIN[0] + 0.5 * L0, oy=ORIGIN[1] + 0.5 * L0, l0=L0,
                                h=np.float32(hh).ravel())])
    blade = dict(pos=(0, 0, 0), quat=(1, 0, 0, 0), linvel=(1.0, 0, 0), angvel=(0, 0, 0), shapes=[])
    tool = dict(body=1, n_wedges=4, edge0=(-0.5, -0.3, 0.35), edge1=(-0.5, 0.3, 0.35), n_c=(1, 0, 0),
                phi=math.radians(33), heap=0.1)
    wedges = O.predict_wedges(tool, [terrain, blade])
    assert sum(len(w) > 0 for w in wedges) == 4
    phi = columns(np.float32(hh).astype(np.float64))
    wc = rng.uniform(0.8, 1.0, phi.shape)
    mf = np.where(rng.uniform(size=phi.shape) < 0.1, rng.uniform(0, 0.5, phi.shape), 0.0)
    m0 = solid_mass(phi, wc) + np.sum(mf)
    phi2, mf2, lib = O.convert_cut(phi, wc, mf, wedges, ORIGIN, L0, DIMS, RHO_B)
    assert lib > 0.5
    rho_p = np.where(rng.uniform(size=phi.shape) < 0.3, 1.0, 0.0)
    phi3, wc3, mf3, dep = O.convert_deposit(phi2, wc, mf2, rho_p, wedges, ORIGIN, L0, DIMS, RHO_B, 0.85)
    assert dep > 0
    assert solid_mass(phi3, wc3) + np.sum(mf3) == pytest.approx(m0, rel=1e-13)
    assert np.all(phi3 >= 0.0) and np.all(phi3 <= 1.0) and np.all(mf3 >= 0.0)


RHO_P = 2000.0


def pmass(r):
    return RHO_P * 4.0 / 3.0 * math.pi * np.asarray(r) ** 3


def test_growth_rate_is_the_diameter_rate():
    # ample fluid: over a short dt the diameter grows by d'_max dt (to first order)
    mf = np.zeros((DIMS[2], DIMS[1], DIMS[0]))
    x = np.array([[0.05, 0.05, 0.55]])
    v = (5, 5, 10)  # its voxel (k, j, i)
    mf[v] = 10.0
    for dt in (1e-3, 1e-5):
        r2, mf2, grown = O.grow_particles(x, [0.02], RHO_P, mf, ORIGIN, L0, DIMS, dt, 0.1, 0.2)
        # a mass rate 3 m d' / d is a diameter rate d': (1 + 3 e)^(1/3) = 1 + e - e^2 + ..., e = d' dt / d
        e = 0.1 * dt / 0.04
        assert (2 * r2[0] - 0.04) / (0.1 * dt) == pytest.approx(1.0 - e, abs=2 * e * e + 1e-9)
        assert grown == pytest.approx(pmass(r2[0]) - pmass(0.02), rel=1e-9)
        assert mf[v] - mf2[v] == pytest.approx(grown, rel=1e-12)


def test_growth_stops_at_d_max_and_outside():
    mf = np.full((DIMS[2], DIMS[1], DIMS[0]), 5.0)
    x = np.array([[0.05, 0.05, 0.55], [5.0, 0.0, 0.0], [0.25, 0.05, 0.55]])
    r = np.array([0.0299, 0.02, 0.01])
    r2, mf2, grown = O.grow_particles(x, r, RHO_P, mf, ORIGIN, L0, DIMS, 1.0, 1.0, 0.06)
    assert r2[0] == pytest.approx(0.03, rel=1e-14)   # reached d_max / 2
    assert r2[1] == 0.02                               # outside the grid
    assert r2[2] == pytest.approx(0.03, rel=1e-14)
    assert grown == pytest.approx(pmass(0.03) * 2 - pmass(0.0299) - pmass(0.01), rel=1e-10)


def test_scarce_fluid_is_shared_by_the_bounds():
    # two particles in one voxel: the bound 3 m d' dt / d grows as r^2, so the
    # gains are in the ratio (r1 / r2)^2 and the voxel's fluid is used up
    mf = np.zeros((DIMS[2], DIMS[1], DIMS[0]))
    v = (5, 5, 10)
    mf[v] = 1e-4
    x = np.array([[0.03, 0.02, 0.53], [0.07, 0.08, 0.57]])
    r = np.array([0.01, 0.02])
    r2, mf2, grown = O.grow_particles(x, r, RHO_P, mf, ORIGIN, L0, DIMS, 0.1, 0.5, 1.0)
    g = pmass(r2) - pmass(r)
    assert grown == pytest.approx(1e-4, rel=1e-12)
    assert abs(mf2[v]) <= 1e-18
    assert g[0] / g[1] == pytest.approx((0.01 / 0.02) ** 2, rel=1e-9)


def test_growth_conserves_mass():
    rng = np.random.default_rng(6)
    n = 3000
    x = rng.uniform(ORIGIN, np.add(ORIGIN, np.multiply(DIMS, L0)), (n, 3))
    r = rng.uniform(0.01, 0.03, n)
    mf = np.where(rng.uniform(size=(DIMS[2], DIMS[1], DIMS[0])) < 0.5, rng.uniform(0, 2e-3, (DIMS[2], DIMS[1], DIMS[0])), 0.0)
    r2, mf2, grown = O.grow_particles(x, r, RHO_P, mf, ORIGIN, L0, DIMS, 1.0 / 60, 0.2, 0.07)
    assert grown > 0 and np.all(r2 >= r) and np.all(r2 <= 0.035 * (1 + 1e-15))
    assert np.all(mf2 >= -1e-18)
    assert np.sum(pmass(r2)) + np.sum(mf2) == pytest.approx(np.sum(pmass(r)) + np.sum(mf), rel=1e-13)


def test_particle_formation():
    # a zone over the grid's middle; fluid in four voxels of it and one outside
    W = np.array([[1.0, 0, 0, 0.5], [-1.0, 0, 0, 0.5], [0, 1.0, 0, 0.3], [0, -1.0, 0, 0.3], [0, 0, 1.0, 1.0]])
    sh = (DIMS[2], DIMS[1], DIMS[0])
    mf = np.zeros(sh)
    rho_p = np.zeros(sh)
    u = np.zeros(sh + (3,))
    d_min, d_max, phi_max = 0.02, 0.05, 0.6
    m_of = lambda d: RHO_P * math.pi / 6 * d ** 3
    mf[2, 5, 10] = 3 * m_of(d_max)           # plenty: a d_max particle
    u[2, 5, 10] = (0.1, -0.2, 0.3)
    mf[3, 5, 10] = 0.5 * (m_of(d_min) + m_of(d_max))  # all of it in one particle
    mf[4, 5, 10] = 0.9 * m_of(d_min)         # too little
    mf[5, 5, 10] = m_of(d_max)
    rho_p[5, 5, 10] = 0.55 * RHO_P           # no room: 0.55 + 0.065 > 0.6
    mf[2, 5, 20] = m_of(d_max)               # outside the zone (x = 1.05)
    mf2, P = O.form_particles(mf, rho_p, u, [W], ORIGIN, L0, DIMS, RHO_P, d_min, d_max, phi_max)
    assert len(P["r"]) == 2
    vox = [np.ravel_multi_index(t, sh) for t in ((2, 5, 10), (3, 5, 10))]
    assert list(P["voxel"]) == vox
    assert P["r"][0] == pytest.approx(0.5 * d_max, rel=1e-15)
    assert np.allclose(P["x"][0], [ORIGIN[0] + 10.5 * L0, ORIGIN[1] + 5.5 * L0, ORIGIN[2] + 2.5 * L0], rtol=0, atol=1e-15)
    assert np.allclose(P["v"][0], [0.1, -0.2, 0.3], rtol=0, atol=0)
    assert mf2[2, 5, 10] == pytest.approx(2 * m_of(d_max), rel=1e-14)
    assert m_of(2 * P["r"][1]) == pytest.approx(mf[3, 5, 10], rel=1e-14) and abs(mf2[3, 5, 10]) <= 1e-15
    for t in ((4, 5, 10), (5, 5, 10), (2, 5, 20)):
        assert mf2[t] == mf[t]
    # conservation on a random field
    rng = np.random.default_rng(8)
    mfr = np.where(rng.uniform(size=sh) < 0.3, rng.uniform(0, 2 * m_of(d_max), sh), 0.0)
    rpr = np.where(rng.uniform(size=sh) < 0.3, rng.uniform(0, 0.6 * RHO_P, sh), 0.0)
    mf3, P3 = O.form_particles(mfr, rpr, np.zeros(sh + (3,)), [W], ORIGIN, L0, DIMS, RHO_P, d_min, d_max, phi_max)
    assert len(P3["r"]) > 10 and np.all(np.diff(P3["voxel"]) > 0)
    assert np.all((2 * P3["r"] >= d_min * (1 - 1e-12)) & (2 * P3["r"] <= d_max))
    assert np.sum(mf3) + np.sum(m_of(2 * P3["r"])) == pytest.approx(np.sum(mfr), rel=1e-13)


def test_particles_at_rest_outside_the_zone_settle():
    # slow particles outside the zone give their mass to their voxel's fluid;
    # with no particle left there, the deposit turns it into solid: the
    # column rises by m / (w_dep rho_b l0^2)
    W = np.array([[1.0, 0, 0, 0.0], [-1.0, 0, 0, 0.5], [0, 0, 1.0, 1.0]])  # -0.5 <= x <= 0, z <= 1
    x = np.array([[0.55, 0.05, 0.45], [0.55, 0.05, 0.47], [-0.25, 0.05, 0.45], [0.35, 0.05, 0.45], [5.0, 0, 0]])
    v = np.array([[0.0, 0.01, 0.0], [0.02, 0.0, 0.0], [0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0, 0, 0]])
    m = np.array([0.3, 0.2, 0.4, 0.5, 0.6])
    sh = (DIMS[2], DIMS[1], DIMS[0])
    mf = np.zeros(sh)
    mf2, gone, tot = O.settle_particles(x, v, m, mf, [W], ORIGIN, L0, DIMS, 0.05)
    # 0, 1: slow, outside the zone, same voxel; 2: inside the zone; 3: moving; 4: outside the grid
    assert list(gone) == [True, True, False, False, False]
    assert tot == pytest.approx(0.5, rel=1e-15) and mf2[4, 5, 15] == pytest.approx(0.5, rel=1e-15)
    h0 = 0.23
    phi = columns(np.full((DIMS[1], DIMS[0]), h0))
    wc = np.ones_like(phi)
    phi3, wc3, mf3, dep = O.convert_deposit(phi, wc, mf2, np.zeros(sh), [W], ORIGIN, L0, DIMS, RHO_B, 0.8)
    assert dep == pytest.approx(0.5, rel=1e-14) and not mf3.any()
    h = O.surface_heights(phi3, ORIGIN, L0, DIMS)
    assert h[5, 15] == pytest.approx(h0 + 0.5 / (0.8 * RHO_B * L0 ** 2), rel=1e-13)
