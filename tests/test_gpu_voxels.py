"""Mesoscale voxel fields on the HIP path against the FP64 oracle.

Coarse-graining (Eq. cg_velocity) sums in FP64 with atomics, so only the order
of the additions differs from the oracle: the fields agree to 1e-12 of their
largest value (Heaviside: the same voxel for every particle, the mass exactly
conserved to rounding; Gaussian: the math library's exp may differ in the last
bit).  The advection step (Eq. advection) evaluates every face with the
oracle's operations and sums each voxel's fluxes in the oracle's order: the
result and the Courant number are bit-exact, on a ragged grid and at the full
size of the timed workload.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")
D = pytest.importorskip("paper_2011_00459_amd.devmem")


def particle_masses(r, rho):
    # the library's mass: FP32 density and radius, FP64 arithmetic in this order
    r = np.asarray(r, dtype=np.float64)
    return np.float64(np.float32(rho)) * (4.0 / 3.0) * math.pi * r * r * r


def stepped_column(seed=3, n=2000):
    """A scene whose particle state is set from seeded inputs after one step
    (the step builds the library's tables); both sides take the FP32 values."""
    spec = SG.column_scene(seed=seed, n=n, footprint=0.6, sweeps=20)
    g = T.scene_from_specs(spec)
    g.step(1)
    rng = np.random.default_rng(seed)
    x = SG.fp32(np.asarray(spec["x"]) + rng.uniform(-0.01, 0.01, (n, 3)))
    v = SG.fp32(rng.normal(0.0, 0.5, (n, 3)))
    g.set_particles(0, x=x, v=v, w=np.zeros((n, 3)))
    p = dict(x=x, v=v, r=np.asarray(SG.fp32(spec["r"]), dtype=np.float64))
    return g, spec, p


def gpu_coarse_grain(g, origin, l0, dims, kernel="heaviside", R=0.0):
    nv = int(np.prod(dims))
    rho, mom, u = D.DeviceArray((nv,), np.float64), D.DeviceArray((nv, 3), np.float64), D.DeviceArray((nv, 3), np.float64)
    g.coarse_grain(0, origin, l0, dims, rho.ptr, mom.ptr, u.ptr, kernel=kernel, R=R)
    sh = (dims[2], dims[1], dims[0])
    return rho.get().reshape(sh), mom.get().reshape(sh + (3,)), u.get().reshape(sh + (3,))


@pytest.mark.parametrize("kernel", ["heaviside", "gauss"])
def test_coarse_grain_matches_oracle(kernel):
    g, spec, p = stepped_column()
    m = particle_masses(p["r"], spec["material"]["rho"])
    # a ragged grid that cuts through the column: some particles fall outside
    origin, l0, dims = (-0.37, -0.29, 0.013), 0.045, (13, 11, 9)
    R = 2.0 * float(np.max(p["r"]))
    got = gpu_coarse_grain(g, origin, l0, dims, kernel, R)
    ref = O.coarse_grain(p["x"], p["v"], m, origin, l0, dims, kernel=kernel, R=R)
    for a, b in zip(got, ref):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), kernel
    rho = got[0]
    assert np.count_nonzero(rho) > 50
    if kernel == "heaviside":
        assert np.array_equal(rho > 0, ref[0] > 0)
        inside = np.all((p["x"] >= origin) & (p["x"] < np.add(origin, np.multiply(dims, l0))), axis=1)
        assert 0 < inside.sum() < len(m)
        assert np.sum(rho) * l0 ** 3 == pytest.approx(np.sum(m[inside]), rel=1e-12)


def test_coarse_grain_empty_grid_and_errors():
    g, spec, p = stepped_column(n=300)
    # a grid far from every particle: all fields zero
    rho, mom, u = gpu_coarse_grain(g, (50.0, 50.0, 50.0), 0.1, (4, 3, 2))
    assert not rho.any() and not mom.any() and not u.any()
    buf = D.DeviceArray((24,), np.float64)
    with pytest.raises(T.TerrainError):
        g.coarse_grain(0, (0, 0, 0), 0.0, (2, 2, 2), buf.ptr, buf.ptr)
    with pytest.raises(T.TerrainError):
        g.coarse_grain(0, (0, 0, 0), 0.1, (2, 2, 2), buf.ptr, buf.ptr, kernel="gauss", R=0.0)
    with pytest.raises(T.TerrainError):
        g.coarse_grain(3, (0, 0, 0), 0.1, (2, 2, 2), buf.ptr, buf.ptr)


def gpu_advect(g, mf, u, origin, l0, dims, dt):
    a, b, uu = D.DeviceArray.from_host(mf, np.float64), D.DeviceArray(np.shape(mf), np.float64), \
        D.DeviceArray.from_host(u, np.float64)
    cfl = g.advect_fluid(origin, l0, dims, dt, uu.ptr, a.ptr, b.ptr)
    return b.get(), cfl


@pytest.mark.parametrize("dims", [(1, 1, 1), (7, 5, 3), (37, 29, 23)])
def test_advection_bit_exact(dims):
    g, _, _ = stepped_column(n=300)
    rng = np.random.default_rng(sum(dims))
    sh = (dims[2], dims[1], dims[0])
    l0, dt = 0.05, 1.0 / 60.0
    mf = rng.uniform(0.0, 2.0, sh)
    mf[rng.uniform(size=sh) < 0.3] = 0.0
    u = rng.normal(0.0, 0.35 * l0 / dt, sh + (3,))
    got, cfl = gpu_advect(g, mf, u, (0.0, 0.0, 0.0), l0, dims, dt)
    ref, cfl_ref = O.advect(mf, u, (0.0, 0.0, 0.0), l0, dims, dt)
    assert np.array_equal(got, ref)
    assert cfl == cfl_ref
    assert np.sum(got) == pytest.approx(np.sum(mf), rel=1e-13)
    # the alias of input and output is refused
    a = D.DeviceArray.from_host(mf, np.float64)
    uu = D.DeviceArray.from_host(u, np.float64)
    with pytest.raises(T.TerrainError):
        g.advect_fluid((0.0, 0.0, 0.0), l0, dims, dt, uu.ptr, a.ptr, a.ptr)


def test_advection_full_workload_bit_exact():
    # the size the benchmark times: 256 x 256 x 128 voxels
    from paper_2011_00459_amd import scenegen as SG2
    g, _, _ = stepped_column(n=300)
    w = SG2.voxel_workload(seed=11)
    got, cfl = gpu_advect(g, w["mf"], w["u"], w["origin"], w["l0"], w["dims"], w["dt"])
    ref, cfl_ref = O.advect(w["mf"], w["u"], w["origin"], w["l0"], w["dims"], w["dt"])
    assert cfl == cfl_ref and cfl < 1.0
    assert np.array_equal(got, ref)


def test_coarse_grained_velocity_feeds_advection():
    # the chain of the two: u of the particles drives their own mass density;
    # the GPU u differs from the oracle's by rounding, so the chain agrees to
    # a tolerance, and the mass stays
    g, spec, p = stepped_column()
    m = particle_masses(p["r"], spec["material"]["rho"])
    origin, l0, dims = (-0.4, -0.4, 0.0), 0.05, (16, 16, 12)
    rho, _, u = gpu_coarse_grain(g, origin, l0, dims)
    mf = rho * l0 ** 3
    out, cfl = gpu_advect(g, mf, u, origin, l0, dims, spec["dt"])
    orho, _, ou = O.coarse_grain(p["x"], p["v"], m, origin, l0, dims)
    ref, cfl_ref = O.advect(orho * l0 ** 3, ou, origin, l0, dims, spec["dt"])
    assert np.max(np.abs(out - ref)) <= 1e-11 * np.max(ref)
    assert cfl == pytest.approx(cfl_ref, rel=1e-9, abs=1e-15)
    assert np.sum(out) == pytest.approx(np.sum(mf), rel=1e-13)
