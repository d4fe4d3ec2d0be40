"""A scene on a caller's stream with the caller's allocator callbacks: the
device buffers come from alloc_fn (every one handed back to free_fn exactly
once, with the scene's stream), the work runs on that stream, and the steps
give the same state, bit for bit, as a scene on the null stream with
hipMalloc."""
import ctypes as C

import numpy as np
import pytest

from helpers import settled_column

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")
D = pytest.importorskip("paper_2011_00459_amd.devmem")


class CountingAllocator:
    """alloc_fn / free_fn over hipMalloc / hipFree that record every call."""

    def __init__(self):
        self.live = {}
        self.freed = []
        self.streams = set()
        hip = D.hip()

        def alloc(ctx, nbytes, stream):
            p = C.c_void_p()
            if hip.hipMalloc(C.byref(p), C.c_size_t(nbytes)) != 0:
                return None
            self.live[p.value] = nbytes
            self.streams.add(stream)
            return p.value

        def free(ctx, ptr, stream):
            assert ptr in self.live, "free of a block the allocator did not hand out"
            self.freed.append(ptr)
            del self.live[ptr]
            self.streams.add(stream)
            hip.hipFree(C.c_void_p(ptr))

        self.alloc_fn = T.ALLOC_FN(alloc)
        self.free_fn = T.FREE_FN(free)


def make_stream():
    hip = D.hip()
    hip.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
    s = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(s)) == 0
    return s.value


def destroy_stream(s):
    hip = D.hip()
    hip.hipStreamDestroy.argtypes = [C.c_void_p]
    assert hip.hipStreamDestroy(C.c_void_p(s)) == 0


def scene_kwargs(spec):
    n = len(spec["x"])
    bounds = np.array([list(spec["grid_lo"]) + list(spec["grid_hi"])], dtype=np.float64)
    return dict(n_envs=1, dt=spec["dt"], gravity=spec["gravity"], max_sweeps=spec["max_sweeps"],
                tol=spec.get("tol", 0.0), warm_start="prev", material=spec["material"], cap_particles=n,
                cap_contacts=16 * n, env_bounds=bounds, r_ref=spec.get("r_ref", 0.0))


def load(sc, spec):
    sc.add_particles(0, spec["x"], spec["r"], vel=spec.get("v"))
    sc.set_kinematic_bodies(0, [dict(b, id=i) for i, b in enumerate(spec["bodies"])])


def test_caller_stream_and_allocator_give_the_same_steps():
    spec = settled_column(n=600, footprint=0.5)
    ref = T.Scene(**scene_kwargs(spec))
    load(ref, spec)
    st_ref = ref.step(4)
    p_ref = ref.get_particles(0)
    k_ref, l_ref = ref.get_contacts(0)
    ref.close()

    stream = make_stream()
    alloc = CountingAllocator()
    try:
        sc = T.Scene(**scene_kwargs(spec), stream=stream, alloc_fn=alloc.alloc_fn, free_fn=alloc.free_fn)
        n_blocks = len(alloc.live)
        assert n_blocks > 20                      # every device buffer of the scene
        load(sc, spec)
        st = sc.step(4)
        p = sc.get_particles(0)
        k, lam = sc.get_contacts(0)
        assert st[0]["contacts"] == st_ref[0]["contacts"] and st[0]["sweeps"] == st_ref[0]["sweeps"]
        assert np.array_equal(k, k_ref) and np.array_equal(lam, l_ref)
        for key in ("x", "v", "w"):
            assert np.array_equal(p[key], p_ref[key]), key
        assert alloc.streams == {stream}          # the callbacks see the scene's stream
        sc.close()
        assert not alloc.live                     # destroy_scene frees every block once
        assert len(alloc.freed) == len(set(alloc.freed)) >= n_blocks
    finally:
        destroy_stream(stream)


def test_allocator_failure_is_reported_not_crashed():
    spec = settled_column(n=200, footprint=0.5)
    fail = T.ALLOC_FN(lambda ctx, n, s: None)
    noop = T.FREE_FN(lambda ctx, p, s: None)
    with pytest.raises(T.TerrainError) as e:
        T.Scene(**scene_kwargs(spec), alloc_fn=fail, free_fn=noop)
    assert e.value.code == T.TR_E_NOMEM


def test_alloc_without_free_is_rejected():
    spec = settled_column(n=200, footprint=0.5)
    alloc = CountingAllocator()
    d_kw = scene_kwargs(spec)
    sc = None
    with pytest.raises(ValueError):
        sc = T.Scene(**d_kw, alloc_fn=alloc.alloc_fn)
    assert sc is None and not alloc.live
