"""Soil library and the polygon rolling-resistance relation (CPU).

  - mu_r = tan(pi / 2n) / 4 gives the values the paper prints next to
    Eq. signCoul3 (0.05 for an octagon, 0.1 for a square, 0 for a sphere) and
    decreases with the number of sides;
  - the library's particle materials step on the oracle, and a library soil's
    bulk friction angle gives the active-zone failure angle of Eq. failure_plane.
"""
import math

import numpy as np
import pytest

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG
from paper_2011_00459_amd import soils as S
from paper_2011_00459_amd import zones as Z


def test_polygon_rolling_resistance_matches_the_printed_values():
    assert S.rolling_resistance_of_polygon(8) == pytest.approx(0.05, abs=5e-4)
    assert S.rolling_resistance_of_polygon(4) == pytest.approx(0.1, abs=5e-3)
    assert S.rolling_resistance_of_polygon(math.inf) == 0.0
    vals = [S.rolling_resistance_of_polygon(n) for n in range(3, 40)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    with pytest.raises(ValueError):
        S.rolling_resistance_of_polygon(2)


def test_library_has_fifteen_soils_with_si_materials():
    assert len(S.SOIL_LIBRARY) == 15
    m = S.material("wet-sand-1")
    assert m["c_p"] == 30e3 and m["mu_t"] == 0.3 and m["mu_r"] == 0.1 and m["rho"] == 2200.0
    b = S.bulk("dirt-3")
    assert b["c"] == 21e3 and b["phi"] == pytest.approx(math.radians(35.0))
    # frictional soils carry no particle cohesion, cohesive ones do
    for name, (_, cb, _, _, _, _, cp) in S.SOIL_LIBRARY.items():
        assert (cb == 0.0) == (cp == 0.0) or name == "frictionless"


def test_library_material_steps_on_the_oracle_and_gives_zone_angles():
    spec = SG.column_scene(seed=3, n=200, sweeps=10, footprint=0.4)
    spec = dict(spec, material=S.material("dirt-1"))
    sc = O.OracleScene(spec)
    out = sc.step()
    assert out["contacts"] > 0 and np.all(np.isfinite(sc.v))
    phi = S.bulk("dirt-1")["phi"]
    assert Z.failure_angle(phi) == pytest.approx(math.radians(25.0), rel=1e-12)  # pi/4 - 40deg/2


def test_effective_friction_adds_the_dilatancy_angle():
    assert S.effective_friction("gravel-1") == pytest.approx(math.tan(math.radians(55.0)), rel=1e-12)
    assert S.effective_friction("frictionless") == pytest.approx(math.tan(math.radians(7.0)), rel=1e-12)
