"""ctypes wrapper of the FP64 CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It marshals
a plain scene description (numpy arrays and dicts, see ``scenegen``) into the
oracle's own C structs; it contains none of the method's arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

PLANE, BOX, HFIELD = 0, 1, 2
COLD, PREV, LEARNED = 0, 1, 2
BRUTE, CELLS = 0, 1
_SHAPE_CODES = {"plane": PLANE, "box": BOX, "hfield": HFIELD}
_WARM_CODES = {"cold": COLD, "prev": PREV, "learned": LEARNED}


def build(verbose: bool = False) -> str:
    """Compile the oracle with -O2 -ffp-contract=off (plain C, libm only)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall", "-fPIC", "-shared",
           os.path.join(HERE, "oracle.c"), "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Material(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("rho", "mu_t", "mu_r", "c_p", "E", "nu", "restitution", "tau_n",
                 "gamma_t", "kappa_c", "kappa_min", "v_imp")]


class Tool(C.Structure):
    _fields_ = [("body", C.c_int32), ("n_wedges", C.c_int32), ("edge0", C.c_double * 3), ("edge1", C.c_double * 3),
                ("n_c", C.c_double * 3), ("n_tc", C.c_double * 3), ("fill", C.c_double), ("phi", C.c_double),
                ("heap", C.c_double), ("v_min", C.c_double)]


class Wedge(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad", C.c_int32), ("planes", (C.c_double * 4) * 5)]


MAX_WEDGES = 16


class VoxelGrid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("l0", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("pad", C.c_int32)]


def voxel_grid(origin, l0, dims) -> VoxelGrid:
    g = VoxelGrid()
    for k in range(3):
        g.origin[k] = origin[k]
    g.l0 = l0
    g.nx, g.ny, g.nz = (int(d) for d in dims)
    return g


class Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("g", C.c_double * 3), ("grid_lo", C.c_double * 3),
                ("grid_hi", C.c_double * 3), ("r_ref", C.c_double), ("max_sweeps", C.c_int32), ("tol", C.c_double),
                ("warm", C.c_int32), ("detect", C.c_int32), ("m", Material), ("ntools", C.c_int32),
                ("tools", C.POINTER(Tool))]


def tool_struct(t: dict) -> Tool:
    """A tool dict (body index, n_wedges, edge0, edge1, n_c, n_tc, fill, phi,
    heap, v_min; geometry in the body frame) as the oracle's struct."""
    T = Tool()
    T.body = int(t["body"])
    T.n_wedges = int(t.get("n_wedges", 1))
    for k in range(3):
        T.edge0[k] = t["edge0"][k]
        T.edge1[k] = t["edge1"][k]
        T.n_c[k] = t["n_c"][k]
        T.n_tc[k] = t.get("n_tc", t["n_c"])[k]
    T.fill = t.get("fill", 0.0)
    T.phi = t["phi"]
    T.heap = t.get("heap", 0.0)
    T.v_min = t.get("v_min", 0.0)
    return T


class Body(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("quat", C.c_double * 4), ("linvel", C.c_double * 3),
                ("angvel", C.c_double * 3), ("nplanes", C.c_int32), ("planes", (C.c_double * 4) * 8)]


class Shape(C.Structure):
    _fields_ = [("type", C.c_int32), ("body", C.c_int32), ("n", C.c_double * 3), ("d", C.c_double),
                ("half", C.c_double * 3), ("off", C.c_double * 3), ("nx", C.c_int32), ("ny", C.c_int32),
                ("ox", C.c_double), ("oy", C.c_double), ("l0", C.c_double), ("h", C.POINTER(C.c_float))]


class Mlp(C.Structure):
    _fields_ = [("W1", C.POINTER(C.c_double)), ("b1", C.POINTER(C.c_double)),
                ("W2", C.POINTER(C.c_double)), ("b2", C.POINTER(C.c_double)),
                ("W3", C.POINTER(C.c_double)), ("b3", C.POINTER(C.c_double)),
                ("in_scale", C.c_double * 12), ("bf16", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("contacts", C.c_int64), ("pair_contacts", C.c_int64), ("colours", C.c_int32),
                ("sweeps", C.c_int32), ("residual", C.c_double), ("fallback_used", C.c_int32),
                ("learned_used", C.c_int32), ("r1_first", C.c_double), ("r1_trial", C.c_double * 2),
                ("impacts", C.c_int32), ("impact_sweeps", C.c_int32)]


class Aggregate(C.Structure):
    _fields_ = [("zone", C.c_int32), ("n_particles", C.c_int64), ("M", C.c_double),
                ("x", C.c_double * 3), ("v", C.c_double * 3), ("I", C.c_double * 6),
                ("w", C.c_double * 3), ("L", C.c_double * 3)]


class MacroParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_b", "c_b", "mu_ab", "mu_ac", "cas_ab", "cas_ac")]


class MacroEquipment(C.Structure):
    _fields_ = [("body", C.c_int32), ("mass", C.c_double), ("inertia", C.c_double * 6),
                ("v_target", C.c_double * 3), ("w_target", C.c_double * 3), ("f_max", C.c_double),
                ("t_max", C.c_double), ("gamma_drive", C.c_double)]


class MacroOut(C.Structure):
    _fields_ = [("zone", C.c_int32), ("n_points", C.c_int32 * 2), ("n_cand", C.c_int64 * 2),
                ("area", C.c_double * 2), ("gamma", C.c_double * 2), ("p", (C.c_double * 3) * 8),
                ("n", (C.c_double * 3) * 8), ("src", C.c_int64 * 8), ("lam", (C.c_double * 4) * 8),
                ("M", C.c_double), ("x", C.c_double * 3), ("v0", C.c_double * 3), ("w0", C.c_double * 3),
                ("v", C.c_double * 3), ("w", C.c_double * 3), ("force_b", C.c_double * 3),
                ("torque_b", C.c_double * 3), ("sweeps", C.c_int32), ("v_b", C.c_double * 3),
                ("w_b", C.c_double * 3), ("lam_drive", C.c_double * 6)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "oracle.c")
        if not os.path.exists(LIB_PATH) or (os.path.exists(src) and os.path.getmtime(src) > os.path.getmtime(LIB_PATH)):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        u64p = C.POINTER(C.c_uint64)
        L.orc_detect.restype = C.c_int64
        L.orc_detect.argtypes = [C.POINTER(Params), C.c_int64, i64p, dp, dp, C.c_int32, C.POINTER(Body),
                                 C.c_int32, C.POINTER(Shape), C.c_int64, u64p, dp]
        L.orc_step.restype = C.c_int64
        L.orc_step.argtypes = [C.POINTER(Params), C.c_int64, i64p, dp, dp, dp, dp, dp,
                               C.c_int32, C.POINTER(Body), C.c_int32, C.POINTER(Shape),
                               C.c_int64, u64p, dp, dp, C.POINTER(Mlp),
                               C.c_int64, u64p, dp, dp, C.POINTER(C.c_int32), C.POINTER(Stats), dp,
                               C.POINTER(Aggregate), C.POINTER(C.c_int32), dp]
        L.orc_aggregates.restype = C.c_int32
        L.orc_aggregates.argtypes = [C.c_int64, dp, dp, dp, dp, dp, C.c_int32, C.POINTER(Body),
                                     C.POINTER(Aggregate)]
        L.orc_features.restype = C.c_int64
        L.orc_features.argtypes = [C.POINTER(Params), C.c_int64, i64p, dp, dp, dp, dp, dp,
                                   C.c_int32, C.POINTER(Body), C.c_int32, C.POINTER(Shape),
                                   C.c_int64, u64p, dp, C.c_int64, dp, dp, dp]
        L.orc_natural_residual.restype = C.c_double
        L.orc_natural_residual.argtypes = [C.POINTER(Params), C.c_int64, i64p, dp, dp, dp, dp, dp,
                                           C.c_int32, C.POINTER(Body), C.c_int32, C.POINTER(Shape),
                                           C.c_int64, dp]
        L.orc_mlp_forward.restype = None
        L.orc_mlp_forward.argtypes = [C.POINTER(Mlp), C.c_int64, dp, dp]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_mlp_loss_grad.argtypes = [C.POINTER(Mlp), C.c_int64, dp, dp, dp]
        L.orc_predict_wedges.restype = C.c_int32
        L.orc_predict_wedges.argtypes = [C.POINTER(Tool), C.POINTER(Body), C.POINTER(Shape), C.POINTER(Wedge)]
        L.orc_coarse_grain.restype = C.c_int32
        L.orc_coarse_grain.argtypes = [C.c_int64, dp, dp, dp, C.POINTER(VoxelGrid), C.c_int32, C.c_double, dp, dp, dp]
        L.orc_advect.restype = C.c_double
        L.orc_advect.argtypes = [C.POINTER(VoxelGrid), C.c_double, dp, dp]
        L.orc_surface_heights.restype = C.c_int32
        L.orc_surface_heights.argtypes = [C.POINTER(VoxelGrid), dp, dp]
        L.orc_convert_cut.restype = C.c_double
        L.orc_convert_cut.argtypes = [C.POINTER(VoxelGrid), C.c_double, C.c_int32, C.POINTER(Wedge), dp, dp, dp]
        L.orc_settle_particles.restype = C.c_double
        L.orc_settle_particles.argtypes = [C.c_int64, dp, dp, dp, C.POINTER(VoxelGrid), C.c_double, C.c_int32,
                                           C.POINTER(Wedge), dp, C.POINTER(C.c_int32)]
        L.orc_form_particles.restype = C.c_int64
        L.orc_form_particles.argtypes = [C.POINTER(VoxelGrid), C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_int32, C.POINTER(Wedge), dp, dp, dp, C.c_int64,
                                         C.POINTER(C.c_int64), dp, dp, dp]
        L.orc_grow_particles.restype = C.c_double
        L.orc_grow_particles.argtypes = [C.c_int64, dp, dp, C.c_double, C.POINTER(VoxelGrid), C.c_double, C.c_double,
                                         C.c_double, dp]
        L.orc_convert_deposit.restype = C.c_double
        L.orc_convert_deposit.argtypes = [C.POINTER(VoxelGrid), C.c_double, C.c_double, C.c_int32, C.POINTER(Wedge),
                                          dp, dp, dp, dp]
        L.orc_reduce4.restype = C.c_int32
        L.orc_reduce4.argtypes = [C.c_int64, dp, dp, C.POINTER(C.c_int64)]
        L.orc_macro_step.restype = C.c_int32
        L.orc_macro_step.argtypes = [C.POINTER(Params), C.c_int64, dp, dp, dp, dp, dp, C.c_int32, C.POINTER(Body),
                                     C.c_int32, C.POINTER(Shape), C.POINTER(MacroParams), C.c_int32,
                                     C.POINTER(MacroEquipment), C.c_int32, C.POINTER(MacroOut)]
        L.orc_failure_angle.restype = C.c_double
        L.orc_failure_angle.argtypes = [C.c_double, C.c_double]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


DEFAULT_MATERIAL = dict(rho=2000.0, mu_t=0.6, mu_r=0.0, c_p=1000.0, E=1e9, nu=0.15, restitution=0.0,
                        tau_n=0.0, gamma_t=0.0, kappa_c=0.025, kappa_min=1e-4, v_imp=0.0)


def make_params(spec: dict, detect: int = CELLS) -> Params:
    P = Params()
    P.dt = spec["dt"]
    for k in range(3):
        P.g[k] = spec["gravity"][k]
        P.grid_lo[k] = spec.get("grid_lo", (0.0, 0.0, 0.0))[k]
        P.grid_hi[k] = spec.get("grid_hi", (1.0, 1.0, 1.0))[k]
    P.r_ref = spec.get("r_ref", 0.05)
    P.max_sweeps = spec["max_sweeps"]
    P.tol = spec.get("tol", 0.0)
    P.warm = _WARM_CODES[spec.get("warm_start", "cold")]
    P.detect = detect
    mat = dict(DEFAULT_MATERIAL)
    mat.update(spec.get("material", {}))
    for k, v in mat.items():
        setattr(P.m, k, v)
    tools = spec.get("tools", [])
    if tools:
        arr = (Tool * len(tools))(*[tool_struct(t) for t in tools])
        P.ntools = len(tools)
        P.tools = C.cast(arr, C.POINTER(Tool))
        P._tools_keep = arr  # the array lives as long as the params
    return P


class _Bodies:
    """Holds the ctypes arrays for bodies and shapes (and the heightfields)."""

    def __init__(self, bodies: list):
        self.keep = []
        nb = len(bodies)
        self.nb = nb
        self.bodies = (Body * max(nb, 1))()
        shapes = []
        for bi, b in enumerate(bodies):
            B = self.bodies[bi]
            for k in range(3):
                B.pos[k] = b["pos"][k]
                B.linvel[k] = b.get("linvel", (0, 0, 0))[k]
                B.angvel[k] = b.get("angvel", (0, 0, 0))[k]
            q = b.get("quat", (1.0, 0.0, 0.0, 0.0))
            for k in range(4):
                B.quat[k] = q[k]
            planes = np.asarray(b.get("zone_planes", np.zeros((0, 4))), dtype=np.float64).reshape(-1, 4)
            B.nplanes = len(planes)
            for p in range(len(planes)):
                for k in range(4):
                    B.planes[p][k] = planes[p, k]
            for s in b.get("shapes", []):
                shapes.append((bi, s))
        self.ns = len(shapes)
        self.shapes = (Shape * max(self.ns, 1))()
        for si, (bi, s) in enumerate(shapes):
            S = self.shapes[si]
            S.type = _SHAPE_CODES[s["type"]]
            S.body = bi
            for k in range(3):
                S.n[k] = s.get("n", (0, 0, 1))[k]
                S.half[k] = s.get("half", (0, 0, 0))[k]
                S.off[k] = s.get("off", (0, 0, 0))[k]
            S.d = s.get("d", 0.0)
            if s["type"] == "hfield":
                h = np.ascontiguousarray(s["h"], dtype=np.float32)
                self.keep.append(h)
                S.nx, S.ny = int(s["nx"]), int(s["ny"])
                S.ox, S.oy, S.l0 = s["ox"], s["oy"], s["l0"]
                S.h = h.ctypes.data_as(C.POINTER(C.c_float))

    def poses(self):
        out = []
        for bi in range(self.nb):
            B = self.bodies[bi]
            out.append(dict(pos=np.array(B.pos[:]), quat=np.array(B.quat[:])))
        return out


def detect(spec: dict, method: int = CELLS, cap: int | None = None):
    """Sorted contact keys and overlaps of the spec's particle state."""
    L = lib()
    P = make_params(spec, method)
    x = _c64(spec["x"]).reshape(-1, 3)
    n = len(x)
    r = _c64(spec["r"])
    ids = np.ascontiguousarray(spec.get("id", np.arange(n)), dtype=np.int64)
    bb = _Bodies(spec.get("bodies", []))
    cap = cap or max(64, 16 * n + 64)
    keys = np.zeros(cap, dtype=np.uint64)
    delta = np.zeros(cap, dtype=np.float64)
    nc = L.orc_detect(C.byref(P), n, ids.ctypes.data_as(C.POINTER(C.c_int64)), _dp(x), _dp(r),
                      bb.nb, bb.bodies, bb.ns, bb.shapes, cap,
                      keys.ctypes.data_as(C.POINTER(C.c_uint64)), _dp(delta))
    if nc < 0:
        raise RuntimeError(f"orc_detect failed ({nc})")
    return keys[:nc].copy(), delta[:nc].copy()


def mlp_struct(weights: dict):
    """Build an Mlp struct from a dict of float64 arrays (kept alive by the caller)."""
    m = Mlp()
    keep = {}
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        a = np.ascontiguousarray(weights[k], dtype=np.float64)
        keep[k] = a
        setattr(m, k, _dp(a))
    sc = np.asarray(weights.get("in_scale", np.ones(12)), dtype=np.float64)
    for i in range(12):
        m.in_scale[i] = sc[i]
    m.bf16 = 1 if weights.get("bf16", False) else 0
    return m, keep


class OracleScene:
    """A single-environment scene stepped by the oracle; holds its own state."""

    def __init__(self, spec: dict, detect_method: int = CELLS, mlp: dict | None = None):
        self.spec = spec
        self.P = make_params(spec, detect_method)
        self.x = _c64(spec["x"]).reshape(-1, 3).copy()
        n = len(self.x)
        self.n = n
        self.v = _c64(spec.get("v", np.zeros((n, 3)))).reshape(-1, 3).copy()
        self.w = _c64(spec.get("w", np.zeros((n, 3)))).reshape(-1, 3).copy()
        self.r = _c64(spec["r"]).copy()
        self.rho = None if spec.get("rho") is None else _c64(spec["rho"]).copy()
        self.ids = np.ascontiguousarray(spec.get("id", np.arange(n)), dtype=np.int64)
        self.bb = _Bodies(spec.get("bodies", []))
        self.prev_keys = np.zeros(0, dtype=np.uint64)
        self.prev_lam = np.zeros((0, 4), dtype=np.float64)
        self.prev_lr = np.zeros((0, 3), dtype=np.float64)
        self.mlp = None
        if mlp is not None:
            self.mlp, self._mlp_keep = mlp_struct(mlp)
        self.cap = max(1024, 16 * n + 1024)
        self.last = None

    def step(self):
        L = lib()
        cap = self.cap
        keys = np.zeros(cap, dtype=np.uint64)
        lam = np.zeros((cap, 4), dtype=np.float64)
        lr = np.zeros((cap, 3), dtype=np.float64)
        col = np.zeros(cap, dtype=np.int32)
        st = Stats()
        nb = self.bb.nb
        ft = np.zeros((max(nb, 1), 6), dtype=np.float64)
        agg = (Aggregate * max(nb, 1))()
        nagg = C.c_int32(0)
        resid = np.zeros(max(self.P.max_sweeps, 1) + 1, dtype=np.float64)
        rho_p = _dp(self.rho) if self.rho is not None else C.POINTER(C.c_double)()
        mlp_p = C.byref(self.mlp) if self.mlp is not None else C.POINTER(Mlp)()
        pk = np.ascontiguousarray(self.prev_keys)
        pl = np.ascontiguousarray(self.prev_lam)
        plr = np.ascontiguousarray(self.prev_lr if len(self.prev_lr) == len(pk) else np.zeros((len(pk), 3)))
        nc = L.orc_step(C.byref(self.P), self.n, self.ids.ctypes.data_as(C.POINTER(C.c_int64)),
                        _dp(self.r), rho_p, _dp(self.x), _dp(self.v), _dp(self.w),
                        nb, self.bb.bodies, self.bb.ns, self.bb.shapes,
                        len(pk), pk.ctypes.data_as(C.POINTER(C.c_uint64)), _dp(pl), _dp(plr), mlp_p,
                        cap, keys.ctypes.data_as(C.POINTER(C.c_uint64)), _dp(lam), _dp(lr),
                        col.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(st), _dp(ft),
                        agg, C.byref(nagg), _dp(resid))
        if nc < 0:
            raise RuntimeError(f"orc_step failed ({nc})")
        if nagg.value < 0:
            raise RuntimeError("orc_step: a tool was rejected")
        self.prev_keys = keys[:nc].copy()
        self.prev_lam = lam[:nc].copy()
        self.prev_lr = lr[:nc].copy()
        aggs = []
        for a in agg[: nagg.value]:
            aggs.append(dict(zone=a.zone, n_particles=a.n_particles, M=a.M, x=np.array(a.x[:]),
                             v=np.array(a.v[:]), I=np.array(a.I[:]), w=np.array(a.w[:]),
                             L=np.array(a.L[:])))
        self.last = dict(keys=keys[:nc].copy(), lam=lam[:nc].copy(), lr=lr[:nc].copy(), colour=col[:nc].copy(),
                         contacts=st.contacts, pair_contacts=st.pair_contacts, colours=st.colours,
                         sweeps=st.sweeps, residual=st.residual, fallback_used=st.fallback_used,
                         learned_used=st.learned_used, r1=st.r1_first, r1_trial=tuple(st.r1_trial),
                         impacts=st.impacts, impact_sweeps=st.impact_sweeps,
                         resid=resid[: st.sweeps].copy(), body_ft=ft[:nb].copy(), aggregates=aggs)
        return self.last

    def features(self):
        """Learned-start features, frames and impulse scales of the current
        state and cache (the inputs the next step's learned start sees)."""
        L = lib()
        cap = self.cap
        feat = np.zeros((cap, 12)); frame = np.zeros((cap, 6)); scale = np.zeros(cap)
        rho_p = _dp(self.rho) if self.rho is not None else C.POINTER(C.c_double)()
        pk = np.ascontiguousarray(self.prev_keys)
        pl = np.ascontiguousarray(self.prev_lam)
        nc = L.orc_features(C.byref(self.P), self.n, self.ids.ctypes.data_as(C.POINTER(C.c_int64)),
                            _dp(self.r), rho_p, _dp(self.x), _dp(self.v), _dp(self.w),
                            self.bb.nb, self.bb.bodies, self.bb.ns, self.bb.shapes,
                            len(pk), pk.ctypes.data_as(C.POINTER(C.c_uint64)), _dp(pl),
                            cap, _dp(feat), _dp(frame), _dp(scale))
        if nc < 0:
            raise RuntimeError(f"orc_features failed ({nc})")
        return feat[:nc].copy(), frame[:nc].copy(), scale[:nc].copy()

    def natural_residual(self, x, v, w, lam):
        L = lib()
        x = _c64(x); v = _c64(v); w = _c64(w); lam = _c64(lam)
        rho_p = _dp(self.rho) if self.rho is not None else C.POINTER(C.c_double)()
        return L.orc_natural_residual(C.byref(self.P), self.n, self.ids.ctypes.data_as(C.POINTER(C.c_int64)),
                                      _dp(self.r), rho_p, _dp(x), _dp(v), _dp(w),
                                      self.bb.nb, self.bb.bodies, self.bb.ns, self.bb.shapes,
                                      len(lam), _dp(lam))


def predict_wedges(tool: dict, bodies: list):
    """Wedges of a tool at its body's pose on the first heightfield of
    `bodies`: a list (one per wedge) of (k x 4) plane arrays, k = 0 for an
    empty wedge (world frame, inside iff n . x <= d for every row)."""
    bb = _Bodies(bodies)
    terrain = None
    for k in range(bb.ns):
        if bb.shapes[k].type == _SHAPE_CODES["hfield"]:
            terrain = C.pointer(bb.shapes[k])
            break
    T = tool_struct(tool)
    out = (Wedge * MAX_WEDGES)()
    nw = lib().orc_predict_wedges(C.byref(T), bb.bodies, terrain if terrain is not None else C.POINTER(Shape)(), out)
    if nw < 0:
        raise ValueError("bad tool")
    return [np.array([[out[w].planes[p][q] for q in range(4)] for p in range(out[w].n)]).reshape(-1, 4)
            for w in range(nw)]


def inside_wedges(wedges, x):
    """Membership of points in the union of wedges."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    ok = np.zeros(len(x), dtype=bool)
    for W in wedges:
        if len(W):
            ok |= np.all(x @ W[:, :3].T - W[:, 3] <= 0.0, axis=1)
    return ok


def aggregates(x, v, w, r, mass, bodies: list):
    """Aggregate bodies of the zones of `bodies` for the given particle state."""
    x = _c64(x).reshape(-1, 3)
    n = len(x)
    v = _c64(v).reshape(-1, 3)
    w = _c64(w).reshape(-1, 3)
    r = _c64(r)
    im = 1.0 / _c64(mass)
    bb = _Bodies(bodies)
    agg = (Aggregate * max(bb.nb, 1))()
    na = lib().orc_aggregates(n, _dp(r), _dp(im), _dp(x), _dp(v), _dp(w), bb.nb, bb.bodies, agg)
    return [dict(zone=a.zone, n_particles=a.n_particles, M=a.M, x=np.array(a.x[:]), v=np.array(a.v[:]),
                 I=np.array(a.I[:]), w=np.array(a.w[:]), L=np.array(a.L[:])) for a in agg[:na]]


def mlp_forward(weights: dict, feat: np.ndarray) -> np.ndarray:
    m, keep = mlp_struct(weights)
    f = _c64(feat).reshape(-1, 12)
    out = np.zeros((len(f), 3))
    lib().orc_mlp_forward(C.byref(m), len(f), _dp(f), _dp(out))
    return out


N_MLP_PARAMS = 64 * 12 + 64 + 64 * 64 + 64 + 3 * 64 + 3


def mlp_loss_grad(weights: dict, feat: np.ndarray, label: np.ndarray):
    m, keep = mlp_struct(weights)
    f = _c64(feat).reshape(-1, 12)
    lb = _c64(label).reshape(-1, 3)
    g = np.zeros(N_MLP_PARAMS)
    loss = lib().orc_mlp_loss_grad(C.byref(m), len(f), _dp(f), _dp(lb), _dp(g))
    o = 0
    out = {}
    for k, shp in (("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
                   ("W3", (3, 64)), ("b3", (3,))):
        sz = int(np.prod(shp))
        out[k] = g[o:o + sz].reshape(shp)
        o += sz
    return loss, out


def failure_angle(phi: float, beta: float) -> float:
    return lib().orc_failure_angle(phi, beta)


CG_KERNELS = {"heaviside": 0, "gauss": 1}


def coarse_grain(x, v, m, origin, l0, dims, kernel="heaviside", R=0.0):
    """Mass density, momentum density and velocity on a voxel grid (arrays
    shaped (nz, ny, nx), (nz, ny, nx, 3), (nz, ny, nx, 3))."""
    x = _c64(x).reshape(-1, 3)
    v = _c64(v).reshape(-1, 3)
    m = _c64(m)
    g = voxel_grid(origin, l0, dims)
    nv = int(np.prod(dims))
    rho = np.zeros(nv); mom = np.zeros((nv, 3)); u = np.zeros((nv, 3))
    rc = lib().orc_coarse_grain(len(x), _dp(x), _dp(v), _dp(m), C.byref(g), CG_KERNELS[kernel], R, _dp(rho),
                                _dp(mom), _dp(u))
    if rc != 0:
        raise ValueError("bad grid or kernel")
    sh = (dims[2], dims[1], dims[0])
    return rho.reshape(sh), mom.reshape(sh + (3,)), u.reshape(sh + (3,))


def advect(mf, u, origin, l0, dims, dt):
    """One step of conserved donor-cell advection; returns (new mf, largest Courant number)."""
    g = voxel_grid(origin, l0, dims)
    m = _c64(mf).ravel().copy()
    uu = _c64(u).reshape(-1, 3)
    cfl = lib().orc_advect(C.byref(g), dt, _dp(uu), _dp(m))
    if cfl < 0:
        raise ValueError("bad grid")
    return m.reshape(np.shape(mf)), cfl


def _wedge_array(wedges):
    arr = (Wedge * max(1, len(wedges)))()
    for k, W in enumerate(wedges):
        W = np.asarray(W, dtype=np.float64).reshape(-1, 4)
        arr[k].n = len(W)
        for p in range(len(W)):
            for q in range(4):
                arr[k].planes[p][q] = W[p, q]
    return arr


def surface_heights(phi, origin, l0, dims):
    """Eq. surface per column: (ny, nx) heights of the solid occupancy phi (nz, ny, nx)."""
    g = voxel_grid(origin, l0, dims)
    f = _c64(phi).ravel()
    h = np.zeros(dims[0] * dims[1])
    if lib().orc_surface_heights(C.byref(g), _dp(f), _dp(h)) != 0:
        raise ValueError("bad grid")
    return h.reshape(dims[1], dims[0])


def convert_cut(phi, wc, mf, wedges, origin, l0, dims, rho_b):
    """Liberate the solid above the zone's bottom into fluidized mass; returns
    (phi, mf, liberated mass) (new arrays)."""
    g = voxel_grid(origin, l0, dims)
    f, w, m = _c64(phi).ravel().copy(), _c64(wc).ravel().copy(), _c64(mf).ravel().copy()
    tot = lib().orc_convert_cut(C.byref(g), rho_b, len(wedges), _wedge_array(wedges), _dp(f), _dp(w), _dp(m))
    if tot < 0:
        raise ValueError("bad grid")
    sh = np.shape(phi)
    return f.reshape(sh), m.reshape(sh), tot


def convert_deposit(phi, wc, mf, rho_p, wedges, origin, l0, dims, rho_b, w_dep):
    """Deposit particle-free fluidized mass outside the zones onto the column
    surfaces; returns (phi, wc, mf, deposited mass) (new arrays)."""
    g = voxel_grid(origin, l0, dims)
    f, w, m = _c64(phi).ravel().copy(), _c64(wc).ravel().copy(), _c64(mf).ravel().copy()
    rp = _c64(rho_p).ravel()
    tot = lib().orc_convert_deposit(C.byref(g), rho_b, w_dep, len(wedges), _wedge_array(wedges), _dp(rp), _dp(f),
                                    _dp(w), _dp(m))
    if tot < 0:
        raise ValueError("bad grid or w_dep")
    sh = np.shape(phi)
    return f.reshape(sh), w.reshape(sh), m.reshape(sh), tot


def grow_particles(x, r, rho, mf, origin, l0, dims, dt, dprime_max, d_max):
    """Particles grow from their voxel's fluidized mass (Eq. eqmotmb); returns
    (new radii, new mf, grown mass) (new arrays)."""
    g = voxel_grid(origin, l0, dims)
    x = _c64(x).reshape(-1, 3)
    rr = _c64(r).copy()
    m = _c64(mf).ravel().copy()
    tot = lib().orc_grow_particles(len(x), _dp(x), _dp(rr), rho, C.byref(g), dt, dprime_max, d_max, _dp(m))
    if tot < 0:
        raise ValueError("bad grid or parameter")
    return rr, m.reshape(np.shape(mf)), tot


def form_particles(mf, rho_p, u, wedges, origin, l0, dims, rho, d_min, d_max, phi_max):
    """New particles from the fluid inside the zones; returns (new mf, dict of
    voxel, x, v, r arrays in increasing voxel order)."""
    g = voxel_grid(origin, l0, dims)
    m = _c64(mf).ravel().copy()
    rp = _c64(rho_p).ravel()
    uu = _c64(u).reshape(-1, 3)
    cap = int(np.count_nonzero(m > 0)) + 1
    vox = np.zeros(cap, dtype=np.int64)
    x = np.zeros((cap, 3)); v = np.zeros((cap, 3)); r = np.zeros(cap)
    n = lib().orc_form_particles(C.byref(g), rho, d_min, d_max, phi_max, len(wedges), _wedge_array(wedges), _dp(rp),
                                 _dp(uu), _dp(m), cap, vox.ctypes.data_as(C.POINTER(C.c_int64)), _dp(x), _dp(v),
                                 _dp(r))
    if n < 0:
        raise ValueError("bad grid or parameter")
    return m.reshape(np.shape(mf)), dict(voxel=vox[:n], x=x[:n], v=v[:n], r=r[:n])


def settle_particles(x, v, m, mf, wedges, origin, l0, dims, v_rest):
    """Particles at rest outside the zones give their mass to their voxel's
    fluid; returns (new mf, removed mask, converted mass)."""
    g = voxel_grid(origin, l0, dims)
    x = _c64(x).reshape(-1, 3)
    v = _c64(v).reshape(-1, 3)
    mm = _c64(m)
    f = _c64(mf).ravel().copy()
    gone = np.zeros(len(x), dtype=np.int32)
    tot = lib().orc_settle_particles(len(x), _dp(x), _dp(v), _dp(mm), C.byref(g), v_rest, len(wedges),
                                     _wedge_array(wedges), _dp(f), gone.ctypes.data_as(C.POINTER(C.c_int32)))
    if tot < 0:
        raise ValueError("bad grid or v_rest")
    return f.reshape(np.shape(mf)), gone.astype(bool), tot



def reduce4(points, normal):
    """Indices of at most four of the points extreme along +-e1, +-e2 of the plane with this normal."""
    pts = _c64(points).reshape(-1, 3)
    nrm = _c64(normal)
    idx = (C.c_int64 * 4)()
    m = lib().orc_reduce4(len(pts), _dp(pts), _dp(nrm), idx)
    return [int(idx[k]) for k in range(m)]


MACRO_DEFAULTS = dict(E_b=1e7, c_b=0.0, mu_ab=0.4, mu_ac=0.7, cas_ab=1.0, cas_ac=0.001)


def macro_step(spec: dict, x, v, w, bodies=None, equipment=None, **params):
    """The oracle's macroscale step of every zone of spec's bodies for the
    particle state (x, v, w): a list of dicts (zone, points, normals, impulses,
    the aggregate's velocity after the step, the force on its body).
    equipment: dicts (body index, mass, inertia (xx, yy, zz, xy, xz, yz, body
    frame), v_target, w_target, f_max, t_max, gamma_drive) of the bodies that
    are dynamic; the others are kinematic."""
    L = lib()
    P = make_params(spec)
    x = _c64(x).reshape(-1, 3); v = _c64(v).reshape(-1, 3); w = _c64(w).reshape(-1, 3)
    r = _c64(spec["r"])
    rho = None if spec.get("rho") is None else _c64(spec["rho"])
    bb = _Bodies(bodies if bodies is not None else spec.get("bodies", []))
    mp = MacroParams()
    prm = dict(MACRO_DEFAULTS)
    prm.update(params)
    for k, val in prm.items():
        setattr(mp, k, val)
    eqs = list(equipment or [])
    eq = (MacroEquipment * max(len(eqs), 1))()
    for k, e in enumerate(eqs):
        eq[k].body = int(e["body"])
        eq[k].mass = e["mass"]
        for j in range(6):
            eq[k].inertia[j] = e["inertia"][j]
        for j in range(3):
            eq[k].v_target[j] = e.get("v_target", (0.0, 0.0, 0.0))[j]
            eq[k].w_target[j] = e.get("w_target", (0.0, 0.0, 0.0))[j]
        eq[k].f_max = e.get("f_max", 0.0)
        eq[k].t_max = e.get("t_max", 0.0)
        eq[k].gamma_drive = e.get("gamma_drive", 1e-6)
    out = (MacroOut * max(bb.nb, 1))()
    m = L.orc_macro_step(C.byref(P), len(x), _dp(r), _dp(rho) if rho is not None else C.POINTER(C.c_double)(),
                         _dp(x), _dp(v), _dp(w), bb.nb, bb.bodies, bb.ns, bb.shapes, C.byref(mp), len(eqs), eq,
                         bb.nb, out)
    res = []
    for o in out[:m]:
        np_ = (o.n_points[0], o.n_points[1])
        sel = list(range(np_[0])) + [4 + j for j in range(np_[1])]
        res.append(dict(zone=o.zone, n_points=np_, n_cand=(o.n_cand[0], o.n_cand[1]), area=(o.area[0], o.area[1]),
                        gamma=(o.gamma[0], o.gamma[1]), p=np.array([o.p[k][:] for k in sel]),
                        n=np.array([o.n[k][:] for k in sel]), src=[o.src[k] for k in sel],
                        lam=np.array([o.lam[k][:] for k in sel]), M=o.M, x=np.array(o.x[:]), v0=np.array(o.v0[:]),
                        w0=np.array(o.w0[:]), v=np.array(o.v[:]), w=np.array(o.w[:]),
                        force_b=np.array(o.force_b[:]), torque_b=np.array(o.torque_b[:]), sweeps=o.sweeps,
                        v_b=np.array(o.v_b[:]), w_b=np.array(o.w_b[:]), lam_drive=np.array(o.lam_drive[:])))
    return res
