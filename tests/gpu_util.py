"""Helpers for the GPU parity tests."""
import numpy as np


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def rows_rel(got, ref):
    """max over vectors of the normwise relative error of each vector"""
    got = np.atleast_2d(got)
    ref = np.atleast_2d(ref)
    return max(normwise(g, r) for g, r in zip(got, ref))


class DeviceArrays:
    """Device buffers through the HIP runtime the library itself loads (for
    the entry points that take device pointers); freed on close."""

    def __init__(self):
        import ctypes as C
        self.C = C
        self.hip = C.CDLL("/opt/rocm/lib/libamdhip64.so")
        self.ptrs = []

    def _ok(self, e):
        if e != 0:
            raise RuntimeError("HIP error %d" % e)

    def upload(self, a):
        C = self.C
        a = np.ascontiguousarray(a)
        p = C.c_void_p()
        self._ok(self.hip.hipMalloc(C.byref(p), C.c_size_t(max(a.nbytes, 256))))
        self.ptrs.append(p)
        self._ok(self.hip.hipMemcpy(p, a.ctypes.data_as(C.c_void_p), C.c_size_t(a.nbytes), 1))  # host to device
        return p.value

    def empty_like(self, a, fill):
        return self.upload(np.full_like(np.asarray(a), fill))

    def download(self, ptr, like):
        C = self.C
        out = np.empty_like(np.asarray(like))
        self._ok(self.hip.hipDeviceSynchronize())
        self._ok(self.hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), C.c_size_t(out.nbytes), 2))
        return out

    def close(self):
        self.hip.hipDeviceSynchronize()
        for p in self.ptrs:
            self.hip.hipFree(p)
        self.ptrs = []
