"""ctypes view of the 3-D CPU oracle ``libaskref3.so`` (test infrastructure only).

A volume is any object with attributes ``x0, x1, y0, y1, z0, z1`` (the box of
points), ``W, H, L`` (voxels per axis), ``D`` (maximum dwell) and ``c`` (the
pair (cr, ci) of the quaternion Julia set). Volumes come back as
``numpy.uint32`` arrays of shape ``(L, H, W)``.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

MAX_LEVELS = 32
CANONICAL, MORTON = 0, 1
ORDERS = {"canonical": CANONICAL, "morton": MORTON}


class Stats(C.Structure):
    _fields_ = [("levels", C.c_uint32), ("pad_", C.c_uint32),
                ("regions", C.c_uint64 * MAX_LEVELS),
                ("fills", C.c_uint64 * MAX_LEVELS),
                ("splits", C.c_uint64 * MAX_LEVELS),
                ("leaves", C.c_uint64 * MAX_LEVELS),
                ("iters_surface", C.c_uint64), ("iters_leaf", C.c_uint64)]

    def as_dict(self):
        n = self.levels
        d = {"levels": n, "iters_surface": self.iters_surface, "iters_leaf": self.iters_leaf}
        for k in ("regions", "fills", "splits", "leaves"):
            d[k] = list(getattr(self, k)[:n])
        return d


_lib = None


def lib():
    """Load the 3-D oracle library, compiling it first if it is not built."""
    global _lib
    if _lib is None:
        path = os.environ.get("ASKREF3_LIB")  # planted-mistake builds in tests
        if path is None:
            path = _build.LIB3
            if not os.path.exists(path):
                _build.build3()
        L = C.CDLL(path)
        d, u32, u64, i32 = C.c_double, C.c_uint32, C.c_uint64, C.c_int
        p32, pd = C.POINTER(C.c_uint32), C.POINTER(C.c_double)
        L.askref3_dwell.argtypes = [d, d, d, d, d, u32]
        L.askref3_dwell.restype = u32
        L.askref3_voxel_dwell.argtypes = [pd, u32, u32, u32, d, d, u32, u32, u32, u32]
        L.askref3_voxel_dwell.restype = u32
        L.askref3_exhaustive.argtypes = [pd, u32, u32, u32, d, d, u32, p32]
        L.askref3_exhaustive.restype = i32
        L.askref3_canonical.argtypes = [u64, p32]
        L.askref3_canonical.restype = u64
        L.askref3_canonical_inv.argtypes = [u64, u64, p32]
        L.askref3_canonical_inv.restype = None
        L.askref3_morton.argtypes = [p32]
        L.askref3_morton.restype = u64
        L.askref3_morton_inv.argtypes = [u64, p32]
        L.askref3_morton_inv.restype = None
        L.askref3_cell_lo.argtypes = [u64, u64, u32]
        L.askref3_cell_lo.restype = u32
        L.askref3_subdiv.argtypes = [pd, u32, u32, u32, d, d, u32, u32, u32, u32, i32, p32,
                                     C.POINTER(Stats)]
        L.askref3_subdiv.restype = C.c_int64
        _lib = L
    return _lib


def _box(v):
    return (C.c_double * 6)(float(v.x0), float(v.x1), float(v.y0), float(v.y1),
                            float(v.z0), float(v.z1))


def _p32(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def dwell(a, b, e, cr, ci, D):
    return int(lib().askref3_dwell(float(a), float(b), float(e), float(cr), float(ci), int(D)))


def voxel_dwell(v, px, py, pz):
    return int(lib().askref3_voxel_dwell(_box(v), v.W, v.H, v.L, float(v.c[0]), float(v.c[1]),
                                         v.D, int(px), int(py), int(pz)))


def exhaustive(v):
    out = np.empty((v.L, v.H, v.W), dtype=np.uint32)
    if lib().askref3_exhaustive(_box(v), v.W, v.H, v.L, float(v.c[0]), float(v.c[1]), v.D,
                                _p32(out)) != 0:
        raise ValueError("askref3_exhaustive rejected the volume")
    return out


def subdiv(v, g, r, B, order="canonical"):
    """(volume, stats dict) of the subdivision volume."""
    out = np.empty((v.L, v.H, v.W), dtype=np.uint32)
    st = Stats()
    rc = lib().askref3_subdiv(_box(v), v.W, v.H, v.L, float(v.c[0]), float(v.c[1]), v.D,
                              int(g), int(r), int(B), ORDERS[order], _p32(out), C.byref(st))
    if rc < 0:
        raise ValueError("askref3_subdiv rejected its arguments (%d)" % rc)
    return out, st.as_dict()


def canonical(G, p):
    a = (C.c_uint32 * 3)(*p)
    return int(lib().askref3_canonical(int(G), a))


def canonical_inv(G, s):
    a = (C.c_uint32 * 3)()
    lib().askref3_canonical_inv(int(G), int(s), a)
    return tuple(a)


def morton(p):
    a = (C.c_uint32 * 3)(*p)
    return int(lib().askref3_morton(a))


def morton_inv(s):
    a = (C.c_uint32 * 3)()
    lib().askref3_morton_inv(int(s), a)
    return tuple(a)


def cell_lo(j, G, n):
    return int(lib().askref3_cell_lo(int(j), int(G), int(n)))
