"""Calibrated soil materials and the rolling-resistance coefficient of a polygon.

The paper calibrates 15 soils with a virtual triaxial test and lists, for each,
the bulk parameters (internal friction angle phi_b [deg], cohesion c_b [kPa],
dilatancy angle psi_b [deg], bulk modulus E_b [MPa]) and the particle
parameters that reproduce them (friction mu_t, rolling resistance mu_r,
particle cohesion c_p [kPa]) (Table soil_library).  All library particles share
Young's modulus 1e9 Pa, Poisson's ratio 0.15, density 2200 kg/m^3 and zero
restitution (section "Soil library").

An n-sided polygon's angularity maps to a rolling-resistance coefficient
mu_r = tan(pi / (2 n)) / 4 (the relation the paper cites next to
Eq. signCoul3): about 0.05 for an octagon, 0.1 for a square, 0 for a sphere.
"""
from __future__ import annotations

import math

# name: (phi_b deg, c_b kPa, psi_b deg, E_b MPa, mu_t, mu_r, c_p kPa)  -- Table soil_library
SOIL_LIBRARY = {
    "gravel-1": (44.0, 0.0, 11.0, 4.6, 0.4, 0.3, 0.0),
    "sand-1": (39.0, 0.0, 9.0, 4.5, 0.3, 0.1, 0.0),
    "sand-2": (32.0, 0.0, 8.0, 3.5, 0.3, 0.02, 0.0),
    "wet-sand-1": (33.0, 8.7, 8.0, 4.0, 0.3, 0.1, 30.0),
    "dirt-1": (40.0, 2.1, 13.0, 6.5, 0.4, 0.1, 2.5),
    "dirt-2": (37.0, 4.9, 10.0, 4.6, 0.4, 0.1, 12.7),
    "dirt-3": (35.0, 21.0, 10.0, 5.8, 0.4, 0.1, 63.7),
    "fs-strong": (42.0, 0.0, 13.0, 3.8, 0.5, 0.1, 0.0),
    "fs-weak": (35.0, 0.0, 8.0, 2.8, 0.3, 0.05, 0.0),
    "cfs-strong": (32.0, 7.1, 7.0, 4.6, 0.3, 0.05, 23.0),
    "cfs-medium": (32.0, 4.3, 7.0, 4.2, 0.3, 0.05, 12.0),
    "cfs-weak": (21.0, 4.8, 6.0, 3.0, 0.15, 0.025, 23.0),
    "cfs-weakest": (12.0, 2.4, 1.0, 1.0, 0.06, 0.01, 23.0),
    "cs-weak": (5.0, 3.1, 2.0, 0.7, 0.0, 0.0, 50.0),
    "frictionless": (6.0, 0.0, 1.0, 0.25, 0.0, 0.0, 0.0),
}

LIBRARY_PARTICLE = dict(E=1e9, nu=0.15, rho=2200.0, restitution=0.0)


def rolling_resistance_of_polygon(n_sides: float) -> float:
    """mu_r of an n-sided polygon, tan(pi / (2 n)) / 4; n = inf gives 0 (a sphere)."""
    if not n_sides >= 3:
        raise ValueError("a polygon has at least 3 sides")
    if math.isinf(n_sides):
        return 0.0
    return 0.25 * math.tan(math.pi / (2.0 * n_sides))


def bulk(name: str) -> dict:
    """Bulk parameters of a library soil (angles in radians, stresses in Pa)."""
    phi, c, psi, E, *_ = SOIL_LIBRARY[name]
    return dict(phi=math.radians(phi), c=c * 1e3, psi=math.radians(psi), E=E * 1e6)


def material(name: str, **overrides) -> dict:
    """Particle material of a library soil, in the field names of the
    library's tr_material (and the oracle's), SI units."""
    *_, mu_t, mu_r, c_p = SOIL_LIBRARY[name]
    m = dict(rho=LIBRARY_PARTICLE["rho"], mu_t=mu_t, mu_r=mu_r, c_p=c_p * 1e3, E=LIBRARY_PARTICLE["E"],
             nu=LIBRARY_PARTICLE["nu"], restitution=LIBRARY_PARTICLE["restitution"], tau_n=0.0, gamma_t=0.0,
             kappa_c=0.025, kappa_min=1e-4, v_imp=0.0)
    m.update(overrides)
    return m


def effective_friction(name: str) -> float:
    """Effective internal friction of a library soil with its dilatancy,
    mu = tan(phi_b + psi_b) (Eq. effective_internal_friction)."""
    b = bulk(name)
    return math.tan(b["phi"] + b["psi"])
