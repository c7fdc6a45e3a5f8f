"""ctypes view of the CPU oracle ``libaskref.so`` (test infrastructure only).

A window is any object with attributes ``x0, x1, y0, y1, W, H, D`` (the
complex rectangle, the image size in pixels and the maximum dwell) and,
optionally, ``julia``: None for the Mandelbrot set (a pixel's point is c), or
the pair (cr, ci) of the filled Julia set whose points z0 the pixels are.
Images come back as ``numpy.uint32`` arrays of shape ``(H, W)``, row 0 on the
``y0`` side.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

MAX_LEVELS = 64


class Stats(C.Structure):
    _fields_ = [
        ("levels", C.c_uint32), ("pad_", C.c_uint32),
        ("regions", C.c_uint64 * MAX_LEVELS),
        ("fills", C.c_uint64 * MAX_LEVELS),
        ("splits", C.c_uint64 * MAX_LEVELS),
        ("leaves", C.c_uint64 * MAX_LEVELS),
        ("ring_px", C.c_uint64), ("leaf_px", C.c_uint64), ("fill_px", C.c_uint64),
        ("iters_ring", C.c_uint64), ("iters_leaf", C.c_uint64),
        ("iters_ring_new", C.c_uint64), ("iters_leaf_inner", C.c_uint64),
        ("iters_ring_filled", C.c_uint64),
    ]

    def as_dict(self):
        n = self.levels
        d = {k: getattr(self, k) for k in ("levels", "ring_px", "leaf_px", "fill_px",
                                            "iters_ring", "iters_leaf",
                                            "iters_ring_new", "iters_leaf_inner",
                                            "iters_ring_filled")}
        for k in ("regions", "fills", "splits", "leaves"):
            d[k] = list(getattr(self, k)[:n])
        d["iters_alg"] = self.iters_ring + self.iters_leaf
        return d


class Set(C.Structure):
    _fields_ = [("julia", C.c_uint32), ("pad_", C.c_uint32),
                ("cr", C.c_double), ("ci", C.c_double)]


REGION_DTYPE = np.dtype([("x", "<u4"), ("y", "<u4"), ("w", "<u4"), ("h", "<u4"),
                         ("level", "<u4"), ("kind", "<u4"), ("value", "<u4"),
                         ("pad", "<u4")])
KIND_FILL, KIND_LEAF, KIND_SPLIT = 1, 2, 3

_lib = None


def lib():
    """Load the oracle library, compiling it first if it is not built."""
    global _lib
    if _lib is None:
        path = os.environ.get("ASKREF_LIB")  # planted-mistake builds in tests
        if path is None:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = C.CDLL(path)
        d, u32, u64, i32 = C.c_double, C.c_uint32, C.c_uint64, C.c_int
        p32, p64 = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
        L.askref_map.argtypes = [d, d, d, d, u32, u32, C.POINTER(d)]
        L.askref_map.restype = None
        L.askref_pixel_c.argtypes = [C.POINTER(d), u32, u32, u32, u32,
                                     C.POINTER(d), C.POINTER(d)]
        L.askref_pixel_c.restype = None
        L.askref_dwell.argtypes = [d, d, u32]
        L.askref_dwell.restype = u32
        L.askref_exhaustive.argtypes = [d, d, d, d, u32, u32, u32, p32, p64, i32]
        L.askref_exhaustive.restype = i32
        L.askref_subdiv.argtypes = [d, d, d, d, u32, u32, u32, u32, u32, u32, i32, i32,
                                    p32, C.POINTER(Stats), C.c_void_p, u64]
        L.askref_subdiv.restype = C.c_int64
        L.askref_subdiv_pixels.argtypes = [d, d, d, d, u32, u32, u32, u32, u32, u32,
                                           u64, p32, p32, p32]
        L.askref_subdiv_pixels.restype = i32
        L.askref_dwell_pixels.argtypes = [d, d, d, d, u32, u32, u32, u64, p32, p32, p32]
        L.askref_dwell_pixels.restype = None
        ps = C.POINTER(Set)
        L.askref_dwell_julia.argtypes = [d, d, d, d, u32]
        L.askref_dwell_julia.restype = u32
        L.askref_exhaustive_set.argtypes = [d, d, d, d, u32, u32, u32, ps, p32, p64, i32]
        L.askref_exhaustive_set.restype = i32
        L.askref_subdiv_set.argtypes = [d, d, d, d, u32, u32, u32, ps, u32, u32, u32, i32, i32,
                                        p32, C.POINTER(Stats), C.c_void_p, u64]
        L.askref_subdiv_set.restype = C.c_int64
        L.askref_subdiv_pixels_set.argtypes = [d, d, d, d, u32, u32, u32, ps, u32, u32, u32,
                                               u64, p32, p32, p32]
        L.askref_subdiv_pixels_set.restype = i32
        L.askref_dwell_pixels_set.argtypes = [d, d, d, d, u32, u32, u32, ps, u64, p32, p32, p32]
        L.askref_dwell_pixels_set.restype = None
        _lib = L
    return _lib


def _win(w):
    return (float(w.x0), float(w.x1), float(w.y0), float(w.y1), int(w.W), int(w.H), int(w.D))


def _set(w):
    """The window's set as the oracle's struct, or None for the Mandelbrot set."""
    j = getattr(w, "julia", None)
    if j is None:
        return None
    return C.byref(Set(1, 0, float(j[0]), float(j[1])))


def _p32(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def mapping(w):
    """(cxm, cym, hx, hy) of a window."""
    m = (C.c_double * 4)()
    x0, x1, y0, y1, W, H, _ = _win(w)
    lib().askref_map(x0, x1, y0, y1, W, H, m)
    return tuple(m)


def pixel_c(w, px, py):
    m = (C.c_double * 4)(*mapping(w))
    cr, ci = C.c_double(), C.c_double()
    lib().askref_pixel_c(m, int(w.W), int(w.H), int(px), int(py), C.byref(cr), C.byref(ci))
    return cr.value, ci.value


def dwell(cr, ci, D):
    return int(lib().askref_dwell(float(cr), float(ci), int(D)))


def dwell_julia(zr0, zi0, cr, ci, D):
    return int(lib().askref_dwell_julia(float(zr0), float(zi0), float(cr), float(ci), int(D)))


def exhaustive(w, threads=0):
    """(image, sum of dwells) of the exhaustive image."""
    x0, x1, y0, y1, W, H, D = _win(w)
    out = np.empty((H, W), dtype=np.uint32)
    it = C.c_uint64()
    rc = lib().askref_exhaustive_set(x0, x1, y0, y1, W, H, D, _set(w), _p32(out), C.byref(it),
                                     int(threads))
    if rc != 0:
        raise ValueError("askref_exhaustive rejected the window")
    return out, it.value


def subdiv(w, g, r, B, order="bfs", threads=0, records=False):
    """(image, stats dict[, region records]) of the subdivision image."""
    x0, x1, y0, y1, W, H, D = _win(w)
    out = np.empty((H, W), dtype=np.uint32)
    st = Stats()
    o = {"bfs": 0, "dfs": 1}[order]
    recs, cap = None, 0
    if records:
        cap = 1 << 12
    while True:
        if records:
            recs = np.zeros(cap, dtype=REGION_DTYPE)
        rc = lib().askref_subdiv_set(x0, x1, y0, y1, W, H, D, _set(w), int(g), int(r), int(B),
                                     o, int(threads), _p32(out), C.byref(st),
                                     recs.ctypes.data if records else None, cap)
        if rc < 0:
            raise ValueError("askref_subdiv rejected its arguments")
        if not records:
            return out, st.as_dict()
        if rc <= cap:
            return out, st.as_dict(), recs[:rc].copy()
        cap = int(rc)


def subdiv_pixels(w, g, r, B, px, py):
    """Subdivision-image values at sampled pixels."""
    x0, x1, y0, y1, W, H, D = _win(w)
    px = np.ascontiguousarray(px, dtype=np.uint32)
    py = np.ascontiguousarray(py, dtype=np.uint32)
    out = np.empty(px.shape, dtype=np.uint32)
    rc = lib().askref_subdiv_pixels_set(x0, x1, y0, y1, W, H, D, _set(w), int(g), int(r),
                                        int(B), px.size, _p32(px), _p32(py), _p32(out))
    if rc != 0:
        raise ValueError("askref_subdiv_pixels rejected its arguments")
    return out


def dwell_pixels(w, px, py):
    """Exhaustive-image values at sampled pixels."""
    x0, x1, y0, y1, W, H, D = _win(w)
    px = np.ascontiguousarray(px, dtype=np.uint32)
    py = np.ascontiguousarray(py, dtype=np.uint32)
    out = np.empty(px.shape, dtype=np.uint32)
    lib().askref_dwell_pixels_set(x0, x1, y0, y1, W, H, D, _set(w), px.size, _p32(px), _p32(py),
                                  _p32(out))
    return out
