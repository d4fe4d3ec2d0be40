"""ctypes binding of libterrain.so (include/terrain.h): argument marshalling only.

Every step of the particle system runs in the library's HIP kernels; this
module converts numpy arrays and plain dicts to the C structs, optionally
hands the library PyTorch's caching allocator and current stream, and turns
error codes into exceptions.  It raises at import when the built library is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libterrain.so")

TR_OK, TR_E_INVAL, TR_E_NOMEM, TR_E_DEVICE, TR_E_STATE, TR_E_CAPACITY, TR_E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
WARM = {"cold": 0, "prev": 1, "learned": 2}
SHAPE = {"plane": 0, "box": 1, "hfield": 2}
MLP_PARAMS = 64 * 12 + 64 + 64 * 64 + 64 + 3 * 64 + 3 + 12
EXPORTS = ("create_scene", "destroy_scene", "add_particles", "set_kinematic_bodies", "step",
           "get_contact_forces", "get_aggregates", "get_last_error", "get_contacts", "get_particles",
           "set_particles", "set_mlp_weights", "get_phase_times", "set_learned_precision", "get_learn_samples", "set_learn_capture",
           "mlp_forward", "mlp_grad_scratch_floats", "mlp_loss_grad", "mlp_adam_step", "set_solver_config",
           "get_solver_config", "set_step_graphs", "set_warm_start", "save_state", "load_state", "autotune",
           "get_rolling_impulses", "set_tool", "get_zone_wedges", "coarse_grain", "advect_fluid",
           "terrain_from_voxels", "convert_cut", "convert_deposit", "grow_particles", "form_particles",
           "remove_particles", "settle_particles", "get_colours", "mlp_loss_grad_noalloc", "macro_step")
CG_KERNEL = {"heaviside": 0, "gauss": 1}
PGS_MODE = {"grouped": 0, "per_env": 1, "spread": 2}
CLUSTER_NONE = -1  # TR_CLUSTER_NONE: per-env solves of one block each
MLP_TRAINABLE = MLP_PARAMS - 12


class TerrainError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"terrain error {code}: {msg}")
        self.code = code


class tr_material(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("rho", "mu_t", "mu_r", "c_p", "E", "nu", "restitution", "tau_n", "gamma_t", "kappa_c", "kappa_min",
                 "v_imp")]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class tr_macro_params(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_b", "c_b", "mu_ab", "mu_ac", "cas_ab", "cas_ac")]


class tr_macro_result(C.Structure):
    _fields_ = [("zone", C.c_int32), ("n_points", C.c_int32 * 2), ("sweeps", C.c_int32),
                ("n_cand", C.c_int64 * 2), ("area", C.c_double * 2), ("gamma", C.c_double * 2),
                ("p", C.c_double * 24), ("n", C.c_double * 24), ("src", C.c_int64 * 8), ("lam", C.c_double * 32),
                ("M", C.c_double), ("x", C.c_double * 3), ("v0", C.c_double * 3), ("w0", C.c_double * 3),
                ("v", C.c_double * 3), ("w", C.c_double * 3), ("force", C.c_double * 3),
                ("torque", C.c_double * 3), ("v_b", C.c_double * 3), ("w_b", C.c_double * 3),
                ("lam_drive", C.c_double * 6)]


class tr_macro_equipment(C.Structure):
    _fields_ = [("body_id", C.c_int32), ("pad", C.c_int32), ("mass", C.c_double), ("inertia", C.c_double * 6),
                ("v_target", C.c_double * 3), ("w_target", C.c_double * 3), ("f_max", C.c_double),
                ("t_max", C.c_double), ("gamma_drive", C.c_double)]


class tr_scene_desc(C.Structure):
    _fields_ = [("n_envs", C.c_int32), ("dt", C.c_double), ("gravity", C.c_double * 3),
                ("max_sweeps", C.c_int32), ("tol", C.c_double), ("warm_start", C.c_int32),
                ("material", tr_material), ("cap_particles", C.c_int64), ("cap_contacts", C.c_int64),
                ("env_bounds", C.POINTER(C.c_double)), ("r_ref", C.c_double), ("stream", C.c_void_p),
                ("alloc_fn", ALLOC_FN), ("free_fn", FREE_FN), ("alloc_ctx", C.c_void_p)]


class tr_shape_desc(C.Structure):
    _fields_ = [("type", C.c_int32), ("normal", C.c_double * 3), ("offset", C.c_double),
                ("half", C.c_double * 3), ("center", C.c_double * 3), ("nx", C.c_int32), ("ny", C.c_int32),
                ("origin", C.c_double * 2), ("l0", C.c_double), ("heights", C.POINTER(C.c_float))]


class tr_body_desc(C.Structure):
    _fields_ = [("id", C.c_int32), ("pos", C.c_double * 3), ("quat", C.c_double * 4),
                ("linvel", C.c_double * 3), ("angvel", C.c_double * 3), ("n_shapes", C.c_int32),
                ("shapes", C.POINTER(tr_shape_desc)), ("n_halfspaces", C.c_int32),
                ("planes", (C.c_double * 4) * 8)]


MAX_WEDGES = 16


class tr_tool_desc(C.Structure):
    _fields_ = [("n_wedges", C.c_int32), ("pad", C.c_int32), ("edge0", C.c_double * 3), ("edge1", C.c_double * 3),
                ("n_c", C.c_double * 3), ("n_tc", C.c_double * 3), ("fill", C.c_double), ("phi", C.c_double),
                ("heap", C.c_double), ("v_min", C.c_double)]


class tr_voxel_grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("l0", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("pad", C.c_int32)]


def voxel_grid(origin, l0, dims):
    g = tr_voxel_grid()
    for k in range(3):
        g.origin[k] = origin[k]
    g.l0 = l0
    g.nx, g.ny, g.nz = (int(d) for d in dims)
    return g


class tr_step_stats(C.Structure):
    _fields_ = [("contacts", C.c_int64), ("pair_contacts", C.c_int64), ("colours", C.c_int32),
                ("sweeps", C.c_int32), ("residual", C.c_double), ("residual_first", C.c_double),
                ("fallback_used", C.c_int32), ("overflow", C.c_int32), ("impacts", C.c_int32),
                ("impact_sweeps", C.c_int32)]


class tr_solver_config(C.Structure):
    _fields_ = [("mode", C.c_int32), ("blocks_per_xcd", C.c_int32), ("lds_particles", C.c_int32),
                ("cluster_particles", C.c_int32), ("dataflow", C.c_int32)]


class tr_aggregate(C.Structure):
    _fields_ = [("zone", C.c_int32), ("pad", C.c_int32), ("n_particles", C.c_int64), ("M", C.c_double),
                ("x", C.c_double * 3), ("v", C.c_double * 3), ("I", C.c_double * 6), ("w", C.c_double * 3)]


_lib = None


def torch_first():
    """Import PyTorch before the library is loaded, so that the library binds
    to the HIP runtime the PyTorch wheel carries (one runtime in the process:
    PyTorch's tensors, caching allocator and streams are then the library's
    device memory and streams).  Loading the library first gives the process
    a second runtime that PyTorch's devices are not visible to.  Returns the
    torch module; raises if the library is already loaded."""
    if _lib is not None:
        raise RuntimeError("libterrain is already loaded: call torch_first() before anything else uses it")
    import torch
    return torch


def torch_allocator(device=0):
    """ALLOC_FN / FREE_FN over PyTorch's caching allocator (after torch_first())."""
    import torch

    def alloc(ctx, nbytes, stream):
        with torch.cuda.device(device):
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0)

    def free(ctx, ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(alloc), FREE_FN(free)


def lib():
    """Load libterrain.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2011_00459_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.create_scene.argtypes = [C.POINTER(tr_scene_desc), C.POINTER(C.c_void_p)]
        L.destroy_scene.argtypes = [P]
        L.add_particles.argtypes = [P, C.c_int32, C.c_int64, dp, dp, dp, dp, C.POINTER(C.c_int64)]
        L.set_kinematic_bodies.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(tr_body_desc)]
        L.step.argtypes = [P, C.c_int32, C.POINTER(tr_step_stats)]
        L.get_contact_forces.argtypes = [P, C.c_int32, C.c_int32, dp, dp]
        L.set_tool.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(tr_tool_desc)]
        L.get_zone_wedges.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, dp, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
        L.get_aggregates.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(tr_aggregate), C.POINTER(C.c_int32)]
        L.get_last_error.argtypes = [P]
        L.get_last_error.restype = C.c_char_p
        L.get_contacts.argtypes = [P, C.c_int32, C.c_int64, C.POINTER(C.c_uint64), C.POINTER(C.c_float),
                                   C.POINTER(C.c_int64)]
        L.get_particles.argtypes = [P, C.c_int32, dp, dp, dp, dp, C.POINTER(C.c_int64)]
        L.set_particles.argtypes = [P, C.c_int32, dp, dp, dp]
        L.set_mlp_weights.argtypes = [P, C.POINTER(C.c_float), C.c_int64]
        L.get_phase_times.argtypes = [P, C.POINTER(C.c_float), C.c_int32]
        L.set_learned_precision.argtypes = [P, C.c_int32]
        L.set_learn_capture.argtypes = [P, C.c_int32]
        fp = C.POINTER(C.c_float)
        L.get_learn_samples.argtypes = [P, C.c_int32, C.c_int64, fp, fp, C.POINTER(C.c_int64)]
        L.mlp_forward.argtypes = [P, P, C.c_int64, P, C.c_int32, P]
        L.mlp_loss_grad.argtypes = [P, P, P, C.c_int64, P, P, P, C.c_int64, P]
        L.mlp_loss_grad_noalloc.argtypes = [P, P, P, C.c_int64, P, P, P]
        L.mlp_adam_step.argtypes = [P, P, P, P, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32, P]
        L.set_solver_config.argtypes = [P, C.POINTER(tr_solver_config)]
        L.get_solver_config.argtypes = [P, C.POINTER(tr_solver_config)]
        L.set_step_graphs.argtypes = [P, C.c_int32]
        L.set_warm_start.argtypes = [P, C.c_int32]
        L.save_state.argtypes = [P, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
        L.load_state.argtypes = [P, C.c_void_p, C.c_int64]
        L.autotune.argtypes = [P, C.c_int32, C.c_char_p, C.POINTER(tr_solver_config), C.POINTER(C.c_float)]
        L.get_rolling_impulses.argtypes = [P, C.c_int32, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_int64)]
        L.get_colours.argtypes = [P, C.c_int32, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.macro_step.argtypes = [P, C.c_int32, C.POINTER(tr_macro_params), C.c_int32, C.POINTER(tr_macro_equipment),
                                 C.c_int32, C.POINTER(tr_macro_result), C.POINTER(C.c_int32)]
        L.coarse_grain.argtypes = [P, C.c_int32, C.POINTER(tr_voxel_grid), C.c_int32, C.c_double, P, P, P]
        L.advect_fluid.argtypes = [P, C.POINTER(tr_voxel_grid), C.c_double, P, P, P, C.POINTER(C.c_double)]
        L.remove_particles.argtypes = [P, C.c_int32, C.c_int64, C.POINTER(C.c_int64)]
        L.settle_particles.argtypes = [P, C.c_int32, C.POINTER(tr_voxel_grid), C.c_double, C.c_int32,
                                       C.POINTER(C.c_int32), dp, P, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.form_particles.argtypes = [P, C.c_int32, C.POINTER(tr_voxel_grid), C.c_double, C.c_double, C.c_double,
                                     C.c_int32, C.POINTER(C.c_int32), dp, P, P, P, C.c_int64, C.POINTER(C.c_int64)]
        L.grow_particles.argtypes = [P, C.c_int32, C.POINTER(tr_voxel_grid), C.c_double, C.c_double, C.c_double, P,
                                     P, C.POINTER(C.c_double)]
        L.terrain_from_voxels.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(tr_voxel_grid), P, P]
        L.convert_cut.argtypes = [P, C.c_int32, C.POINTER(tr_voxel_grid), C.c_double, C.c_int32,
                                  C.POINTER(C.c_int32), dp, P, P, P, C.POINTER(C.c_double)]
        L.convert_deposit.argtypes = [P, C.c_int32, C.POINTER(tr_voxel_grid), C.c_double, C.c_double, C.c_int32,
                                      C.POINTER(C.c_int32), dp, P, P, P, P, C.POINTER(C.c_double)]
        for name in EXPORTS:
            if name != "get_last_error":
                getattr(L, name).restype = C.c_int
        L.mlp_grad_scratch_floats.argtypes = [C.c_int64]
        L.mlp_grad_scratch_floats.restype = C.c_int64
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


MATERIAL_DEFAULTS = dict(rho=2000.0, mu_t=0.6, mu_r=0.0, c_p=1000.0, E=1e9, nu=0.15, restitution=0.0,
                         tau_n=0.0, gamma_t=0.0, kappa_c=0.025, kappa_min=1e-4, v_imp=0.0)


class Scene:
    """One libterrain scene (n_envs independent environments)."""

    def __init__(self, n_envs=1, dt=1.0 / 60.0, gravity=(0.0, 0.0, -9.81), max_sweeps=100, tol=0.0,
                 warm_start="cold", material=None, cap_particles=1024, cap_contacts=16384, env_bounds=None,
                 r_ref=0.0, stream=None, alloc_fn=None, free_fn=None, alloc_ctx=None):
        """stream: a hipStream_t (int) the scene runs on; alloc_fn / free_fn:
        ALLOC_FN / FREE_FN callbacks for its device buffers (kept alive with
        the scene)."""
        L = lib()
        d = tr_scene_desc()
        d.n_envs = n_envs
        d.dt = dt
        for k in range(3):
            d.gravity[k] = gravity[k]
        d.max_sweeps = max_sweeps
        d.tol = tol
        d.warm_start = WARM[warm_start] if isinstance(warm_start, str) else int(warm_start)
        mat = dict(MATERIAL_DEFAULTS)
        mat.update(material or {})
        for k, v in mat.items():
            setattr(d.material, k, v)
        d.cap_particles = cap_particles
        d.cap_contacts = cap_contacts
        self._bounds = np.ascontiguousarray(np.asarray(env_bounds, dtype=np.float64).reshape(n_envs, 6))
        d.env_bounds = self._bounds.ctypes.data_as(C.POINTER(C.c_double))
        d.r_ref = r_ref
        if stream is not None:
            d.stream = stream
        if (alloc_fn is None) != (free_fn is None):
            raise ValueError("alloc_fn and free_fn go together")
        if alloc_fn is not None:
            d.alloc_fn = alloc_fn
            d.free_fn = free_fn
            d.alloc_ctx = alloc_ctx
        self._callbacks = (alloc_fn, free_fn)
        self.n_envs = n_envs
        self.max_sweeps = max_sweeps
        h = C.c_void_p()
        rc = L.create_scene(C.byref(d), C.byref(h))
        if rc != TR_OK:
            raise TerrainError(rc, "create_scene failed")
        self.h = h
        self._desc = d

    def _check(self, rc, what):
        if rc != TR_OK:
            msg = lib().get_last_error(self.h)
            raise TerrainError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            lib().destroy_scene(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_particles(self, env, pos, radius, vel=None, density=None):
        pos = _c64(pos, (-1, 3))
        n = len(pos)
        radius = _c64(radius, (n,))
        vel = _c64(vel, (n, 3))
        density = _c64(density, (n,))
        first = C.c_int64()
        self._check(lib().add_particles(self.h, env, n, _dp(pos), _dp(vel), _dp(radius), _dp(density),
                                        C.byref(first)), "add_particles")
        return first.value

    def set_kinematic_bodies(self, env, bodies):
        keep = []
        arr = (tr_body_desc * max(len(bodies), 1))()
        for i, b in enumerate(bodies):
            B = arr[i]
            B.id = int(b.get("id", i))
            for k in range(3):
                B.pos[k] = b["pos"][k]
                B.linvel[k] = b.get("linvel", (0, 0, 0))[k]
                B.angvel[k] = b.get("angvel", (0, 0, 0))[k]
            q = b.get("quat", (1.0, 0.0, 0.0, 0.0))
            for k in range(4):
                B.quat[k] = q[k]
            planes = np.asarray(b.get("zone_planes", np.zeros((0, 4))), dtype=np.float64).reshape(-1, 4)
            B.n_halfspaces = len(planes)
            for p in range(len(planes)):
                for k in range(4):
                    B.planes[p][k] = planes[p, k]
            shapes = b.get("shapes", [])
            sa = (tr_shape_desc * max(len(shapes), 1))()
            for j, s in enumerate(shapes):
                S = sa[j]
                S.type = SHAPE[s["type"]]
                for k in range(3):
                    S.normal[k] = s.get("n", (0, 0, 1))[k]
                    S.half[k] = s.get("half", (0, 0, 0))[k]
                    S.center[k] = s.get("off", (0, 0, 0))[k]
                S.offset = s.get("d", 0.0)
                if s["type"] == "hfield":
                    h = np.ascontiguousarray(s["h"], dtype=np.float32)
                    keep.append(h)
                    S.nx, S.ny = int(s["nx"]), int(s["ny"])
                    S.origin[0], S.origin[1] = s["ox"], s["oy"]
                    S.l0 = s["l0"]
                    S.heights = h.ctypes.data_as(C.POINTER(C.c_float))
            keep.append(sa)
            B.n_shapes = len(shapes)
            B.shapes = C.cast(sa, C.POINTER(tr_shape_desc))
        self._check(lib().set_kinematic_bodies(self.h, env, len(bodies), arr), "set_kinematic_bodies")

    def step(self, n_steps=1, stats=True):
        if not stats:
            self._check(lib().step(self.h, n_steps, None), "step")
            return None
        st = (tr_step_stats * self.n_envs)()
        self._check(lib().step(self.h, n_steps, st), "step")
        return [dict(contacts=s.contacts, pair_contacts=s.pair_contacts, colours=s.colours, sweeps=s.sweeps,
                     residual=s.residual, residual_first=s.residual_first, fallback_used=s.fallback_used,
                     overflow=s.overflow, impacts=s.impacts, impact_sweeps=s.impact_sweeps) for s in st]

    def set_tool(self, env, body_id, tool):
        """Attach a zone predictor tool (dict: n_wedges, edge0, edge1, n_c,
        n_tc, fill, phi, heap, v_min; body frame) to a body; None removes it."""
        if tool is None:
            self._check(lib().set_tool(self.h, env, body_id, None), "set_tool")
            return
        T = tr_tool_desc()
        T.n_wedges = int(tool.get("n_wedges", 1))
        for k in range(3):
            T.edge0[k] = tool["edge0"][k]
            T.edge1[k] = tool["edge1"][k]
            T.n_c[k] = tool["n_c"][k]
            T.n_tc[k] = tool.get("n_tc", tool["n_c"])[k]
        T.fill = tool.get("fill", 0.0)
        T.phi = tool["phi"]
        T.heap = tool.get("heap", 0.0)
        T.v_min = tool.get("v_min", 0.0)
        self._check(lib().set_tool(self.h, env, body_id, C.byref(T)), "set_tool")

    def get_zone_wedges(self, env, body_id):
        """The last step's wedges of a body's tool: a list of (k x 4) arrays of
        half-spaces (n, d), world frame, k = 0 for an empty wedge."""
        planes = np.zeros(MAX_WEDGES * 20)
        counts = (C.c_int32 * MAX_WEDGES)()
        n = C.c_int32()
        self._check(lib().get_zone_wedges(self.h, env, body_id, MAX_WEDGES, _dp(planes), counts, C.byref(n)),
                    "get_zone_wedges")
        return [planes[w * 20:w * 20 + 4 * counts[w]].reshape(-1, 4) for w in range(n.value)]

    def coarse_grain(self, env, origin, l0, dims, rho_ptr, mom_ptr, u_ptr=None, kernel="heaviside", R=0.0):
        """Density, momentum density and velocity of env's particles on a voxel
        grid (dims = (nx, ny, nz)), into caller-owned device arrays given as
        pointers (nx ny nz doubles for rho, three times that for mom and u)."""
        g = voxel_grid(origin, l0, dims)
        self._check(lib().coarse_grain(self.h, env, C.byref(g), CG_KERNEL[kernel], R, rho_ptr, mom_ptr, u_ptr),
                    "coarse_grain")

    def advect_fluid(self, origin, l0, dims, dt, u_ptr, mf_in_ptr, mf_out_ptr, sync=True):
        """One conserved donor-cell step of the fluidized mass on device arrays;
        returns the largest Courant number (None with sync=False: the step is
        only enqueued)."""
        g = voxel_grid(origin, l0, dims)
        cfl = C.c_double()
        self._check(lib().advect_fluid(self.h, C.byref(g), dt, u_ptr, mf_in_ptr, mf_out_ptr,
                                       C.byref(cfl) if sync else None), "advect_fluid")
        return cfl.value if sync else None

    def remove_particles(self, env, ids):
        """Remove particles by id; env's remaining particles are renumbered in order."""
        a = np.ascontiguousarray(ids, dtype=np.int64)
        self._check(lib().remove_particles(self.h, env, len(a), a.ctypes.data_as(C.POINTER(C.c_int64))),
                    "remove_particles")

    def settle_particles(self, env, origin, l0, dims, v_rest, mf_ptr, wedges=None):
        """Particles at rest outside the zones into their voxels' fluid (and out
        of the scene); returns (count, mass)."""
        g = voxel_grid(origin, l0, dims)
        n, counts, planes = self._wedge_args(wedges)
        cnt, mass = C.c_int64(), C.c_double()
        self._check(lib().settle_particles(self.h, env, C.byref(g), v_rest, n, counts, _dp(planes), mf_ptr,
                                           C.byref(cnt), C.byref(mass)), "settle_particles")
        return cnt.value, mass.value

    def form_particles(self, env, origin, l0, dims, d_min, d_max, phi_max, rho_p_ptr, u_ptr, mf_ptr, max_new,
                       wedges=None):
        """Form new particles from the fluid inside the zones (appended to env
        in increasing voxel order); returns their number."""
        g = voxel_grid(origin, l0, dims)
        n, counts, planes = self._wedge_args(wedges)
        out = C.c_int64()
        self._check(lib().form_particles(self.h, env, C.byref(g), d_min, d_max, phi_max, n, counts, _dp(planes),
                                         rho_p_ptr, u_ptr, mf_ptr, max_new, C.byref(out)), "form_particles")
        return out.value

    def grow_particles(self, env, origin, l0, dims, dt, dprime_max, d_max, mf_ptr, work_ptr, sync=True):
        """Grow env's particles from their voxels' fluidized mass (work: 2 nx ny
        nz device doubles); returns the mass grown (None with sync=False)."""
        g = voxel_grid(origin, l0, dims)
        tot = C.c_double()
        self._check(lib().grow_particles(self.h, env, C.byref(g), dt, dprime_max, d_max, mf_ptr, work_ptr,
                                         C.byref(tot) if sync else None), "grow_particles")
        return tot.value if sync else None

    def terrain_from_voxels(self, env, origin, l0, dims, phi_ptr, h_ptr=None, body_id=-1):
        """Eq. surface per column into h (device, may be None) and, with a body
        id, into that body's heightfield."""
        g = voxel_grid(origin, l0, dims)
        self._check(lib().terrain_from_voxels(self.h, env, body_id, C.byref(g), phi_ptr, h_ptr),
                    "terrain_from_voxels")

    @staticmethod
    def _wedge_args(wedges):
        if wedges is None:
            return 0, None, None
        counts = (C.c_int32 * max(1, len(wedges)))()
        planes = np.zeros(max(1, len(wedges)) * 20)
        for k, W in enumerate(wedges):
            W = np.asarray(W, dtype=np.float64).reshape(-1, 4)
            counts[k] = len(W)
            planes[k * 20:k * 20 + W.size] = W.ravel()
        return len(wedges), counts, planes

    def convert_cut(self, env, origin, l0, dims, rho_b, phi_ptr, wc_ptr, mf_ptr, wedges=None, sync=True):
        """Liberate the solid above the zones' bottoms (wedges: a list of (k x 4)
        plane arrays, or None for the last step's predicted wedges of env's
        tools); returns the liberated mass (None with sync=False)."""
        g = voxel_grid(origin, l0, dims)
        n, counts, planes = self._wedge_args(wedges)
        tot = C.c_double()
        self._check(lib().convert_cut(self.h, env, C.byref(g), rho_b, n, counts, _dp(planes), phi_ptr, wc_ptr, mf_ptr,
                                      C.byref(tot) if sync else None), "convert_cut")
        return tot.value if sync else None

    def convert_deposit(self, env, origin, l0, dims, rho_b, w_dep, rho_p_ptr, phi_ptr, wc_ptr, mf_ptr, wedges=None,
                        sync=True):
        """Deposit particle-free fluidized mass outside the zones onto the
        column surfaces; returns the deposited mass (None with sync=False)."""
        g = voxel_grid(origin, l0, dims)
        n, counts, planes = self._wedge_args(wedges)
        tot = C.c_double()
        self._check(lib().convert_deposit(self.h, env, C.byref(g), rho_b, w_dep, n, counts, _dp(planes), rho_p_ptr,
                                          phi_ptr, wc_ptr, mf_ptr, C.byref(tot) if sync else None), "convert_deposit")
        return tot.value if sync else None

    def get_contact_forces(self, env, body_id):
        f = np.zeros(3)
        t = np.zeros(3)
        self._check(lib().get_contact_forces(self.h, env, body_id, _dp(f), _dp(t)), "get_contact_forces")
        return f, t

    def macro_step(self, env, E_b, c_b, mu_ab, mu_ac, cas_ab, cas_ac, equipment=None, cap=8):
        """The macroscale step of env's zones for the current state (the C-ABI
        macro_step); one dict per zone, arrays per interface point.
        equipment: dicts (body id, mass, inertia (xx, yy, zz, xy, xz, yz, body
        frame), v_target, w_target, f_max, t_max, gamma_drive) of the bodies
        that move with their aggregate; the others are kinematic."""
        mp = tr_macro_params(E_b, c_b, mu_ab, mu_ac, cas_ab, cas_ac)
        eqs = list(equipment or [])
        eq = (tr_macro_equipment * max(len(eqs), 1))()
        for k, e in enumerate(eqs):
            eq[k].body_id = int(e["body"])
            eq[k].mass = e["mass"]
            for j in range(6):
                eq[k].inertia[j] = e["inertia"][j]
            for j in range(3):
                eq[k].v_target[j] = e.get("v_target", (0.0, 0.0, 0.0))[j]
                eq[k].w_target[j] = e.get("w_target", (0.0, 0.0, 0.0))[j]
            eq[k].f_max = e.get("f_max", 0.0)
            eq[k].t_max = e.get("t_max", 0.0)
            eq[k].gamma_drive = e.get("gamma_drive", 1e-6)
        out = (tr_macro_result * cap)()
        n = C.c_int32()
        self._check(lib().macro_step(self.h, env, C.byref(mp), len(eqs), eq, cap, out, C.byref(n)), "macro_step")
        res = []
        for o in out[: min(n.value, cap)]:
            npt = (o.n_points[0], o.n_points[1])
            sel = list(range(npt[0])) + [4 + j for j in range(npt[1])]   # AB points, then AC points
            p = np.array(o.p[:]).reshape(8, 3)
            nn = np.array(o.n[:]).reshape(8, 3)
            lam = np.array(o.lam[:]).reshape(8, 4)
            res.append(dict(zone=o.zone, n_points=npt, sweeps=o.sweeps, n_cand=(o.n_cand[0], o.n_cand[1]),
                            area=(o.area[0], o.area[1]), gamma=(o.gamma[0], o.gamma[1]), p=p[sel], n=nn[sel],
                            src=[o.src[k] for k in sel], lam=lam[sel], M=o.M, x=np.array(o.x[:]),
                            v0=np.array(o.v0[:]), w0=np.array(o.w0[:]), v=np.array(o.v[:]), w=np.array(o.w[:]),
                            force=np.array(o.force[:]), torque=np.array(o.torque[:]), v_b=np.array(o.v_b[:]),
                            w_b=np.array(o.w_b[:]), lam_drive=np.array(o.lam_drive[:])))
        return res

    def get_aggregates(self, env, cap=8):
        out = (tr_aggregate * cap)()
        n = C.c_int32()
        self._check(lib().get_aggregates(self.h, env, cap, out, C.byref(n)), "get_aggregates")
        return [dict(zone=a.zone, n_particles=a.n_particles, M=a.M, x=np.array(a.x[:]), v=np.array(a.v[:]),
                     I=np.array(a.I[:]), w=np.array(a.w[:])) for a in out[: min(n.value, cap)]]

    def get_contacts(self, env, cap=None):
        n = C.c_int64()
        self._check(lib().get_contacts(self.h, env, 0, None, None, C.byref(n)), "get_contacts")
        cap = n.value if cap is None else cap
        keys = np.zeros(max(cap, 1), dtype=np.uint64)
        lam = np.zeros((max(cap, 1), 4), dtype=np.float32)
        self._check(lib().get_contacts(self.h, env, cap, keys.ctypes.data_as(C.POINTER(C.c_uint64)),
                                       lam.ctypes.data_as(C.POINTER(C.c_float)), C.byref(n)), "get_contacts")
        m = min(n.value, cap)
        return keys[:m], lam[:m]

    def get_colours(self, env):
        """Colour of each contact of the last step, in get_contacts order."""
        n = C.c_int64()
        self._check(lib().get_colours(self.h, env, 0, None, C.byref(n)), "get_colours")
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        self._check(lib().get_colours(self.h, env, n.value, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                      C.byref(n)), "get_colours")
        return out[:n.value]

    def get_rolling_impulses(self, env):
        n = C.c_int64()
        self._check(lib().get_rolling_impulses(self.h, env, 0, None, C.byref(n)), "get_rolling_impulses")
        out = np.zeros((max(n.value, 1), 3), dtype=np.float32)
        self._check(lib().get_rolling_impulses(self.h, env, n.value, out.ctypes.data_as(C.POINTER(C.c_float)),
                                               C.byref(n)), "get_rolling_impulses")
        return out[:n.value]

    def get_particles(self, env):
        n = C.c_int64()
        self._check(lib().get_particles(self.h, env, None, None, None, None, C.byref(n)), "get_particles")
        m = n.value
        x = np.zeros((m, 3)); v = np.zeros((m, 3)); w = np.zeros((m, 3)); r = np.zeros(m)
        self._check(lib().get_particles(self.h, env, _dp(x), _dp(v), _dp(w), _dp(r), C.byref(n)), "get_particles")
        return dict(x=x, v=v, w=w, r=r)

    def set_particles(self, env, x=None, v=None, w=None):
        self._check(lib().set_particles(self.h, env, _dp(_c64(x, (-1, 3))), _dp(_c64(v, (-1, 3))),
                                        _dp(_c64(w, (-1, 3)))), "set_particles")

    def set_mlp_weights(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(lib().set_mlp_weights(self.h, flat.ctypes.data_as(C.POINTER(C.c_float)), len(flat)),
                    "set_mlp_weights")

    def set_learned_precision(self, bf16=True):
        self._check(lib().set_learned_precision(self.h, 1 if bf16 else 0), "set_learned_precision")

    def set_learn_capture(self, on=True):
        """Write the learned start's inputs in every following step (for get_learn_samples)."""
        self._check(lib().set_learn_capture(self.h, 1 if on else 0), "set_learn_capture")

    def get_learn_samples(self, env):
        n = C.c_int64()
        self._check(lib().get_learn_samples(self.h, env, 0, None, None, C.byref(n)), "get_learn_samples")
        m = n.value
        feat = np.zeros((max(m, 1), 12), dtype=np.float32)
        lab = np.zeros((max(m, 1), 3), dtype=np.float32)
        fp = C.POINTER(C.c_float)
        self._check(lib().get_learn_samples(self.h, env, m, feat.ctypes.data_as(fp), lab.ctypes.data_as(fp),
                                            C.byref(n)), "get_learn_samples")
        return feat[:m], lab[:m]

    def get_solver_config(self):
        c = tr_solver_config()
        self._check(lib().get_solver_config(self.h, C.byref(c)), "get_solver_config")
        mode = {v: k for k, v in PGS_MODE.items()}[c.mode]
        return dict(mode=mode, blocks_per_xcd=c.blocks_per_xcd, lds_particles=c.lds_particles,
                    cluster_particles=c.cluster_particles, dataflow=c.dataflow)

    def set_solver_config(self, mode=None, blocks_per_xcd=None, lds_particles=None, cluster_particles=None,
                          dataflow=None):
        """Change the PGS schedule; fields left None keep their value."""
        cur = self.get_solver_config()
        new = dict(mode=mode, blocks_per_xcd=blocks_per_xcd, lds_particles=lds_particles,
                   cluster_particles=cluster_particles, dataflow=None if dataflow is None else int(dataflow))
        cur.update({k: v for k, v in new.items() if v is not None})
        c = tr_solver_config(PGS_MODE[cur["mode"]], cur["blocks_per_xcd"], cur["lds_particles"],
                             cur["cluster_particles"], cur["dataflow"])
        self._check(lib().set_solver_config(self.h, C.byref(c)), "set_solver_config")

    def set_warm_start(self, mode):
        self._check(lib().set_warm_start(self.h, WARM[mode] if isinstance(mode, str) else int(mode)), "set_warm_start")

    def save_state(self):
        """The scene's state as bytes (see load_state)."""
        n = C.c_int64()
        self._check(lib().save_state(self.h, None, 0, C.byref(n)), "save_state")
        buf = C.create_string_buffer(n.value)
        self._check(lib().save_state(self.h, buf, n.value, C.byref(n)), "save_state")
        return buf.raw[:n.value]

    def load_state(self, state):
        buf = C.create_string_buffer(bytes(state), len(state))
        self._check(lib().load_state(self.h, buf, len(state)), "load_state")

    def autotune(self, steps=3, cache_path=None):
        """Pick the fastest PGS schedule (see the C header); returns (config, ms per step or -1 if cached)."""
        c = tr_solver_config()
        ms = C.c_float()
        path = None if cache_path is None else os.fspath(cache_path).encode()
        self._check(lib().autotune(self.h, steps, path, C.byref(c), C.byref(ms)), "autotune")
        return self.get_solver_config(), float(ms.value)

    def set_step_graphs(self, enable=True):
        self._check(lib().set_step_graphs(self.h, 1 if enable else 0), "set_step_graphs")

    def get_phase_times(self):
        """Device ms of the last step's phases; NaN per phase after a step-graph replay (only "step" is timed)."""
        t = (C.c_float * 5)()
        self._check(lib().get_phase_times(self.h, t, 5), "get_phase_times")
        return dict(detect=t[0], rows=t[1], pgs=t[2], finish=t[3], step=t[4])


def _check_rc(rc, what):
    if rc != TR_OK:
        raise TerrainError(rc, what)


def mlp_forward(weights_ptr, feat_ptr, B, out_ptr, bf16=True, stream=None):
    """Device-pointer network forward (pointers as ints, e.g. tensor.data_ptr())."""
    _check_rc(lib().mlp_forward(weights_ptr, feat_ptr, B, out_ptr, 1 if bf16 else 0, stream), "mlp_forward")


def mlp_grad_scratch_floats(B):
    return lib().mlp_grad_scratch_floats(B)


MLP_NOALLOC_MAX_BATCH = 8192  # TR_MLP_NOALLOC_MAX_BATCH


def mlp_loss_grad_noalloc(weights_ptr, feat_ptr, label_ptr, B, grad_ptr, loss_ptr, stream=None):
    """mlp_loss_grad with the library's own fixed scratch (no allocation; B <= 8192)."""
    _check_rc(lib().mlp_loss_grad_noalloc(weights_ptr, feat_ptr, label_ptr, B, grad_ptr, loss_ptr, stream),
              "mlp_loss_grad_noalloc")


def mlp_loss_grad(weights_ptr, feat_ptr, label_ptr, B, grad_ptr, loss_ptr, scratch_ptr, scratch_floats, stream=None):
    _check_rc(lib().mlp_loss_grad(weights_ptr, feat_ptr, label_ptr, B, grad_ptr, loss_ptr, scratch_ptr,
                                  scratch_floats, stream), "mlp_loss_grad")


def mlp_adam_step(weights_ptr, grad_ptr, m_ptr, v_ptr, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check_rc(lib().mlp_adam_step(weights_ptr, grad_ptr, m_ptr, v_ptr, lr, beta1, beta2, eps, t, stream),
              "mlp_adam_step")


def scene_from_specs(specs, cap_particles=None, cap_contacts=None, **kw):
    """Build a Scene holding one env per spec (see scenegen) and load it."""
    if isinstance(specs, dict):
        specs = [specs]
    s0 = specs[0]
    nmax = max(len(s["x"]) for s in specs)
    cap_p = cap_particles or nmax
    cap_c = cap_contacts or max(16 * nmax, 1024)
    bounds = np.array([list(s["grid_lo"]) + list(s["grid_hi"]) for s in specs], dtype=np.float64)
    args = dict(n_envs=len(specs), dt=s0["dt"], gravity=s0["gravity"], max_sweeps=s0["max_sweeps"],
                tol=s0.get("tol", 0.0), warm_start=s0.get("warm_start", "cold"), material=s0["material"],
                cap_particles=cap_p, cap_contacts=cap_c, env_bounds=bounds, r_ref=s0.get("r_ref", 0.0))
    args.update(kw)
    sc = Scene(**args)
    for e, s in enumerate(specs):
        sc.add_particles(e, s["x"], s["r"], vel=s.get("v"), density=s.get("rho"))
        if s.get("w") is not None and np.any(s["w"]):
            sc.set_particles(e, w=s["w"])
        bodies = [dict(b, id=i) for i, b in enumerate(s.get("bodies", []))]  # id = body index
        sc.set_kinematic_bodies(e, bodies)
        for t in s.get("tools", []):  # tools name their body by index (= id here)
            sc.set_tool(e, int(t["body"]), t)
    return sc
