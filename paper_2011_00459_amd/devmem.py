"""Device buffers from the HIP runtime that libterrain itself links.

The PyTorch wheel carries its own copy of the HIP and HSA runtimes; a process
that initialises both copies gets two runtimes on one GPU, and the second one
finds no device.  Buffers handed to the library's device-pointer entry points
(the network kernels) therefore come from here: hipMalloc / hipMemcpy of the
runtime that is already loaded with libterrain.
"""
import ctypes as C

import numpy as np

from . import terrain as T

_hip = None


def hip():
    global _hip
    if _hip is None:
        T.lib()  # load libterrain first: its libamdhip64.so.7 is the one resolved below
        h = C.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        h.hipFree.argtypes = [C.c_void_p]
        h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        h.hipMemset.argtypes = [C.c_void_p, C.c_int, C.c_size_t]
        _hip = h
    return _hip


def _ck(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed (HIP error {rc})")


class DeviceArray:
    """A device allocation with a numpy shape and dtype."""

    def __init__(self, shape, dtype=np.float32):
        self.shape = tuple(np.atleast_1d(shape)) if not isinstance(shape, tuple) else shape
        self.dtype = np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        p = C.c_void_p()
        _ck(hip().hipMalloc(C.byref(p), C.c_size_t(max(self.nbytes, 4))), "hipMalloc")
        self.ptr = p.value

    @classmethod
    def from_host(cls, a, dtype=np.float32):
        a = np.ascontiguousarray(a, dtype=dtype)
        d = cls(a.shape, dtype)
        d.upload(a)
        return d

    def upload(self, a, offset_bytes=0):
        a = np.ascontiguousarray(a, dtype=self.dtype)
        if offset_bytes + a.nbytes > self.nbytes:
            raise ValueError("upload past the end of the buffer")
        _ck(hip().hipMemcpy(C.c_void_p(self.ptr + offset_bytes), a.ctypes.data_as(C.c_void_p), a.nbytes, 1),
            "hipMemcpy H2D")

    def zero(self):
        _ck(hip().hipMemset(C.c_void_p(self.ptr), 0, self.nbytes), "hipMemset")

    def get(self):
        out = np.empty(self.shape, dtype=self.dtype)
        _ck(hip().hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(self.ptr), self.nbytes, 2), "hipMemcpy D2H")
        return out

    def at(self, row):
        """Device address of row `row` (first axis)."""
        return self.ptr + row * (self.nbytes // self.shape[0])

    def free(self):
        if getattr(self, "ptr", None):
            hip().hipFree(C.c_void_p(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
