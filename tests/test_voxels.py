"""Mesoscale voxel fields of the oracle: coarse-graining (Eq. cg_velocity) and
the conserved advection of fluidized mass (Eq. advection).

Pins against facts that do not depend on the oracle's code:
  - Heaviside kernel: the voxel masses sum to the particle mass (the paper's
    "preserve mass precisely"), one particle lands in its own voxel with its
    momentum, and a rigid translation gives u = v wherever there is mass;
  - Gaussian kernel: one particle at a voxel centre gives m (sqrt(2 pi) R)^-3
    there, the field is symmetric, the mass inside the 3R cut is the
    Gaussian's 3-sigma share, and u = v for a rigid translation;
  - advection: zero velocity changes nothing; a uniform velocity at Courant
    number 1 moves the field exactly one voxel; at 1/2 every interior voxel
    becomes the mean of itself and its upwind neighbour (donor cell); closed
    walls keep every kilogram; the total is conserved to rounding for a
    random field.
"""
import math

import numpy as np
import pytest

import pyoracle as O

DIMS = (8, 6, 5)
L0 = 0.1
ORIGIN = (-0.4, -0.3, 0.0)


def test_heaviside_conserves_mass_and_momentum():
    rng = np.random.default_rng(1)
    x = rng.uniform(ORIGIN, np.add(ORIGIN, np.multiply(DIMS, L0)), (500, 3))
    v = rng.normal(0, 1, (500, 3))
    m = rng.uniform(0.5, 2.0, 500)
    rho, mom, u = O.coarse_grain(x, v, m, ORIGIN, L0, DIMS)
    V0 = L0 ** 3
    assert np.sum(rho) * V0 == pytest.approx(np.sum(m), rel=1e-13)
    assert np.allclose(np.sum(mom, axis=(0, 1, 2)) * V0, m @ v, rtol=1e-12, atol=1e-12)
    # one particle: its own voxel
    rho1, mom1, u1 = O.coarse_grain([[0.05, 0.15, 0.25]], [[1.0, -2.0, 0.5]], [3.0], ORIGIN, L0, DIMS)
    k, j, i = 2, 4, 4  # z 0.25 -> k 2; y 0.15 + 0.3 -> j 4; x 0.05 + 0.4 -> i 4
    assert rho1[k, j, i] == pytest.approx(3.0 / V0, rel=1e-14) and np.count_nonzero(rho1) == 1
    assert np.allclose(u1[k, j, i], [1.0, -2.0, 0.5], rtol=1e-14)
    # rigid translation
    vv = np.tile([0.3, -0.1, 0.7], (500, 1))
    _, _, ut = O.coarse_grain(x, vv, m, ORIGIN, L0, DIMS)
    occupied = rho > 0
    assert np.allclose(ut[occupied], [0.3, -0.1, 0.7], rtol=1e-13, atol=0)


def test_gaussian_kernel_closed_forms():
    R = 0.08
    centre = [ORIGIN[0] + 4.5 * L0, ORIGIN[1] + 3.5 * L0, ORIGIN[2] + 2.5 * L0]
    rho, mom, u = O.coarse_grain([centre], [[0.0, 1.0, 0.0]], [2.0], ORIGIN, L0, DIMS, kernel="gauss", R=R)
    peak = 2.0 / (math.sqrt(2 * math.pi) * R) ** 3
    assert rho[2, 3, 4] == pytest.approx(peak, rel=1e-13)
    assert rho[2, 3, 5] == pytest.approx(peak * math.exp(-L0 ** 2 / (2 * R ** 2)), rel=1e-13)
    assert rho[2, 3, 3] == pytest.approx(rho[2, 3, 5], rel=1e-13) and rho[1, 3, 4] == pytest.approx(rho[3, 3, 4], rel=1e-13)
    assert np.allclose(u[rho > 0], [0.0, 1.0, 0.0], rtol=1e-13, atol=0)
    # the kernel is cut at 3R: a sum over voxels recovers the Gaussian's mass
    # inside radius 3 sigma, P(chi^2_3 <= 9) = erf(3/sqrt2) - 3 sqrt(2/pi) e^-4.5
    # (about 0.9707; 0.74 for a 2R cut, 1 for none), up to the voxel sum
    dims = (40, 40, 40)
    o = (-2.0, -2.0, -2.0)
    rho2, _, _ = O.coarse_grain([[0.0, 0.0, 0.0]], [[0, 0, 0]], [1.0], o, L0, dims, kernel="gauss", R=0.15)
    inside = math.erf(3 / math.sqrt(2)) - 3 * math.sqrt(2 / math.pi) * math.exp(-4.5)
    assert np.sum(rho2) * L0 ** 3 == pytest.approx(inside, abs=1e-2)


def test_advection_zero_and_unit_courant():
    rng = np.random.default_rng(2)
    mf = rng.uniform(0, 1, (DIMS[2], DIMS[1], DIMS[0]))
    u0 = np.zeros(mf.shape + (3,))
    out, cfl = O.advect(mf, u0, ORIGIN, L0, DIMS, 0.01)
    assert cfl == 0.0 and np.array_equal(out, mf)
    # uniform +x velocity, Courant 1: one voxel downstream, the last column
    # keeps what it had plus what arrived (closed wall), the first empties
    dt = 0.01
    u = np.zeros(mf.shape + (3,))
    u[..., 0] = L0 / dt
    out, cfl = O.advect(mf, u, ORIGIN, L0, DIMS, dt)
    assert cfl == pytest.approx(1.0)
    assert np.allclose(out[..., 1:-1], mf[..., :-2], rtol=1e-14, atol=1e-15)
    assert np.allclose(out[..., 0], 0.0, atol=1e-15)
    assert np.allclose(out[..., -1], mf[..., -1] + mf[..., -2], rtol=1e-14)


def test_advection_half_courant_donor_cell_and_conservation():
    rng = np.random.default_rng(3)
    mf = rng.uniform(0, 1, (DIMS[2], DIMS[1], DIMS[0]))
    dt = 0.01
    u = np.zeros(mf.shape + (3,))
    u[..., 1] = -0.5 * L0 / dt  # towards -y, Courant 1/2
    out, cfl = O.advect(mf, u, ORIGIN, L0, DIMS, dt)
    assert cfl == pytest.approx(0.5)
    assert np.allclose(out[:, 1:-1, :], 0.5 * mf[:, 1:-1, :] + 0.5 * mf[:, 2:, :], rtol=1e-14)
    assert np.allclose(out[:, 0, :], mf[:, 0, :] + 0.5 * mf[:, 1, :], rtol=1e-14)
    # a random velocity field: every kilogram stays, to rounding
    ur = rng.normal(0, 1, mf.shape + (3,)) * (0.4 * L0 / dt)
    out2, cfl2 = O.advect(mf, ur, ORIGIN, L0, DIMS, dt)
    assert cfl2 < 1.5
    assert np.sum(out2) == pytest.approx(np.sum(mf), rel=1e-14)
