"""Shared test inputs: seeded scenes, settled by the oracle where a realistic
contact network is needed (inputs only; expected values are always computed
by the oracle from the same input)."""
from __future__ import annotations

import functools

import numpy as np

import pyoracle as O
from paper_2011_00459_amd import scenegen as SG


@functools.lru_cache(maxsize=None)
def settled_column(seed=1, n=1000, steps=80, settle_sweeps=20, footprint=1.0, c=1000.0, mu=0.6):
    """A column poured and settled by the oracle (state rounded to FP32)."""
    spec = SG.column_scene(seed=seed, n=n, sweeps=settle_sweeps, footprint=footprint, c=c, mu=mu)
    sc = O.OracleScene(spec)
    for _ in range(steps):
        sc.step()
    out = dict(spec)
    out.update(x=SG.fp32(sc.x), v=SG.fp32(sc.v), w=SG.fp32(sc.w))
    return out


def with_(spec, **kw):
    out = dict(spec)
    out.update(kw)
    return out


jammed_bed = SG.jammed_bed


def vel_tol(v_ref, g=9.81, dt=1.0 / 60.0, rel=1e-4):
    """Parity bound on velocities: rel * max(|v|_inf, g dt)."""
    return rel * max(float(np.max(np.abs(v_ref))), g * dt)
