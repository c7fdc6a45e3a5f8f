"""Python binding of ``libask.so`` (include/ask.h): argument marshalling only.

Every call goes straight to the C ABI; all of the work runs in the gfx950
kernels. Device memory and streams come from PyTorch: pass a tensor's
``data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``. There is no
fallback: if the library is not built, importing this module raises.
"""
import ctypes as C
import os

# PyTorch ships its own HIP runtime with the same soname as the system one.
# Loading it first makes libask.so bind to that same runtime, so that the
# streams and device pointers PyTorch hands over are valid in the library.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libask.so")

MAX_LEVELS = 64
OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW, EBUSY, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
FORM_LEVELS, FORM_LEVELS_READBACK, FORM_PERSISTENT = 0, 1, 2
FORMS = {"levels": FORM_LEVELS, "levels_readback": FORM_LEVELS_READBACK,
         "persistent": FORM_PERSISTENT}


class AskError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class ask_window(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("W", C.c_uint32), ("H", C.c_uint32), ("D", C.c_uint32), ("set", C.c_uint32),
                ("cr", C.c_double), ("ci", C.c_double)]


class ask_params(C.Structure):
    _fields_ = [("g", C.c_uint32), ("r", C.c_uint32), ("B", C.c_uint32), ("form", C.c_uint32),
                ("band", C.c_uint32), ("tile_w", C.c_uint32), ("tile_h", C.c_uint32)]


class ask_server_cfg(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("waves_per_cu", C.c_uint32), ("pool_bytes", C.c_uint64)]


class ask_stats(C.Structure):
    _fields_ = [("levels", C.c_uint32), ("overflow", C.c_uint32),
                ("regions", C.c_uint64 * MAX_LEVELS), ("fills", C.c_uint64 * MAX_LEVELS),
                ("splits", C.c_uint64 * MAX_LEVELS), ("leaves", C.c_uint64 * MAX_LEVELS),
                ("iters_ring", C.c_uint64), ("iters_leaf", C.c_uint64),
                ("ring_px", C.c_uint64), ("leaf_px", C.c_uint64), ("fill_px", C.c_uint64)]

    def as_dict(self):
        n = self.levels
        d = {"levels": n, "overflow": self.overflow, "iters_ring": self.iters_ring,
             "iters_leaf": self.iters_leaf, "ring_px": self.ring_px, "leaf_px": self.leaf_px,
             "fill_px": self.fill_px}
        for k in ("regions", "fills", "splits", "leaves"):
            d[k] = list(getattr(self, k)[:n])
        return d


CURVE_CANONICAL, CURVE_MORTON = 0, 1
CURVES = {"canonical": CURVE_CANONICAL, "morton": CURVE_MORTON}
MAX_LEVELS3 = 32
EXHAUSTIVE3_WORK_BYTES = 1024  # ASK3_EXHAUSTIVE_WORK_BYTES


class ask_volume(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("z0", C.c_double), ("z1", C.c_double), ("W", C.c_uint32), ("H", C.c_uint32),
                ("L", C.c_uint32), ("D", C.c_uint32), ("cr", C.c_double), ("ci", C.c_double)]


class ask3_params(C.Structure):
    _fields_ = [("g", C.c_uint32), ("r", C.c_uint32), ("B", C.c_uint32), ("curve", C.c_uint32)]


class ask3_stats(C.Structure):
    _fields_ = [("levels", C.c_uint32), ("overflow", C.c_uint32),
                ("regions", C.c_uint64 * MAX_LEVELS3), ("fills", C.c_uint64 * MAX_LEVELS3),
                ("splits", C.c_uint64 * MAX_LEVELS3), ("leaves", C.c_uint64 * MAX_LEVELS3)]

    def as_dict(self):
        n = self.levels
        d = {"levels": n, "overflow": self.overflow}
        for k in ("regions", "fills", "splits", "leaves"):
            d[k] = list(getattr(self, k)[:n])
        return d


# Every symbol include/ask.h and include/ask3d.h declare, with its C signature.
_P = C.c_void_p
SIGNATURES = {
    "ask_status_str": (C.c_char_p, [C.c_int]),
    "ask_last_error": (C.c_char_p, [_P]),
    "ask_create": (C.c_int, [C.POINTER(_P), C.c_int, C.c_size_t]),
    "ask_destroy": (C.c_int, [_P]),
    "ask_validate": (C.c_int, [C.POINTER(ask_window), C.POINTER(ask_params)]),
    "ask_mapping": (C.c_int, [C.POINTER(ask_window), C.POINTER(C.c_double)]),
    "ask_level_count": (C.c_int, [C.POINTER(ask_window), C.POINTER(ask_params),
                                  C.POINTER(C.c_uint32)]),
    "ask_dwell_exhaustive": (C.c_int, [_P, C.POINTER(ask_window), C.POINTER(ask_params), _P,
                                       _P]),
    "ask_dwell_subdiv": (C.c_int, [_P, C.POINTER(ask_window), C.POINTER(ask_params), _P, _P,
                                   C.POINTER(ask_stats)]),
    "ask_dwell_subdiv_noalloc": (C.c_int, [C.POINTER(ask_window), C.POINTER(ask_params), _P,
                                           _P]),
    "ask_dwell_batch": (C.c_int, [_P, C.c_uint32, C.POINTER(ask_window), C.POINTER(ask_params),
                                  C.c_uint32, C.POINTER(C.c_void_p), _P, C.POINTER(ask_stats)]),
    "ask_synchronize": (C.c_int, [_P, _P]),
    "ask_set_wait_limit": (C.c_int, [_P, C.c_double]),
    "ask_enable_timing": (C.c_int, [_P, C.c_int]),
    "ask_last_kernel_ms": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "ask_kernel_times": (C.c_int, [_P, C.POINTER(C.c_float), C.c_uint32, C.POINTER(C.c_uint32)]),
    "ask_server_create": (C.c_int, [_P, C.POINTER(ask_server_cfg), C.POINTER(_P)]),
    "ask_server_submit": (C.c_int, [_P, C.POINTER(ask_window), C.POINTER(ask_params), _P,
                                    C.POINTER(C.c_uint64)]),
    "ask_server_reap": (C.c_int, [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_int32), C.c_uint32,
                                  C.POINTER(C.c_uint32)]),
    "ask_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "ask_server_in_flight": (C.c_int, [_P, C.POINTER(C.c_uint32)]),
    "ask_server_destroy": (C.c_int, [_P]),
    "ask3_validate": (C.c_int, [C.POINTER(ask_volume), C.POINTER(ask3_params)]),
    "ask3_workspace_bytes": (C.c_int, [C.POINTER(ask_volume), C.POINTER(ask3_params),
                                       C.POINTER(C.c_uint64)]),
    "ask3_dwell_exhaustive": (C.c_int, [C.POINTER(ask_volume), _P, _P, C.c_uint64, _P]),
    "ask3_dwell_subdiv": (C.c_int, [C.POINTER(ask_volume), C.POINTER(ask3_params), _P, _P,
                                    C.c_uint64, _P, C.POINTER(ask3_stats)]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libask.so is not built (expected at %s); build it with "
                          "paper_2206_02255_amd.build.build()" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def status_str(s):
    return lib.ask_status_str(s).decode()


SET_MANDELBROT, SET_JULIA = 0, 1


def window(w):
    """ask_window from any object with x0, x1, y0, y1, W, H, D and optionally
    julia: None (the Mandelbrot set) or the fixed c (cr, ci) of a filled
    Julia set."""
    j = getattr(w, "julia", None)
    if j is None:
        return ask_window(float(w.x0), float(w.x1), float(w.y0), float(w.y1),
                          int(w.W), int(w.H), int(w.D), SET_MANDELBROT, 0.0, 0.0)
    return ask_window(float(w.x0), float(w.x1), float(w.y0), float(w.y1),
                      int(w.W), int(w.H), int(w.D), SET_JULIA, float(j[0]), float(j[1]))


BAND_DEFAULT, BAND_NONE = 1024, 0xffffffff


def params(g, r, B, form="levels", band=0, tile=(0, 0)):
    """ask_params; band: pixels per leaf band (0: BAND_DEFAULT; BAND_NONE:
    every leaf computed whole by the wave that decides it); tile: the wave's
    pixel tile (tile_w, tile_h), (0, 0) for the defaults."""
    return ask_params(int(g), int(r), int(B), FORMS[form] if isinstance(form, str) else int(form),
                      int(band), int(tile[0]), int(tile[1]))


def tile_params(tile):
    """ask_params that carry only a wave tile, for ask_dwell_exhaustive."""
    return params(1, 2, 1, "levels", 0, tile)


def _check(s, ctx=None):
    if s != OK:
        msg = status_str(s)
        if ctx:
            detail = lib.ask_last_error(ctx)
            if detail:
                msg += ": " + detail.decode()
        raise AskError(s, msg)


def ask_validate(win, prm=None):
    return lib.ask_validate(C.byref(win), C.byref(prm) if prm is not None else None)


def ask_mapping(win):
    m = (C.c_double * 4)()
    _check(lib.ask_mapping(C.byref(win), m))
    return tuple(m)


def ask_level_count(win, prm):
    n = C.c_uint32()
    _check(lib.ask_level_count(C.byref(win), C.byref(prm), C.byref(n)))
    return n.value


def ask_create(device=0, queue_bytes=0):
    h = _P()
    _check(lib.ask_create(C.byref(h), int(device), int(queue_bytes)))
    return h


def ask_destroy(ctx):
    _check(lib.ask_destroy(ctx))


def ask_dwell_exhaustive(ctx, win, d_out, stream=0, tile=None):
    """tile: None (the default 16 x 4 wave tile) or (tile_w, tile_h)."""
    prm = tile_params(tile) if tile is not None else None
    _check(lib.ask_dwell_exhaustive(ctx, C.byref(win), C.byref(prm) if prm is not None else None,
                                    _P(d_out), _P(stream)), ctx)


def ask_dwell_subdiv(ctx, win, prm, d_out, stream=0, want_stats=False):
    st = ask_stats() if want_stats else None
    _check(lib.ask_dwell_subdiv(ctx, C.byref(win), C.byref(prm), _P(d_out), _P(stream),
                                C.byref(st) if st is not None else None), ctx)
    return st.as_dict() if st is not None else None


NOALLOC_SCRATCH_BYTES = 64 << 20


def ask_dwell_subdiv_noalloc(win, prm, d_out, stream=0):
    """The subdivision image without a context and without allocating (the
    render works in the library's fixed device array of the current device)."""
    _check(lib.ask_dwell_subdiv_noalloc(C.byref(win), C.byref(prm), _P(d_out), _P(stream)))


def ask_synchronize(ctx, stream=0):
    _check(lib.ask_synchronize(ctx, _P(stream)), ctx)


def ask_set_wait_limit(ctx, seconds):
    _check(lib.ask_set_wait_limit(ctx, float(seconds)), ctx)


def ask_enable_timing(ctx, on=True):
    _check(lib.ask_enable_timing(ctx, 1 if on else 0), ctx)


def ask_last_kernel_ms(ctx):
    ms = C.c_float()
    _check(lib.ask_last_kernel_ms(ctx, C.byref(ms)), ctx)
    return ms.value


def ask_kernel_times(ctx, cap=256):
    """Device times (ms) of the renders timed since ask_enable_timing, oldest
    first (at most the last 256)."""
    ms = (C.c_float * cap)()
    n = C.c_uint32()
    _check(lib.ask_kernel_times(ctx, ms, int(cap), C.byref(n)), ctx)
    return list(ms[:n.value])


def ask_dwell_batch(ctx, wins, prms, d_outs, stream=0, want_stats=False):
    """wins: sequence of ask_window; prms: one ask_params or one per window;
    d_outs: device pointers (ints)."""
    n = len(wins)
    if isinstance(prms, ask_params):
        prms = [prms]
    W = (ask_window * n)(*wins)
    P = (ask_params * len(prms))(*prms)
    O = (C.c_void_p * n)(*[int(p) for p in d_outs])
    st = ask_stats() if want_stats else None
    _check(lib.ask_dwell_batch(ctx, n, W, P, len(prms), O, _P(stream),
                               C.byref(st) if st is not None else None), ctx)
    return st.as_dict() if st is not None else None


# Servers still running when the interpreter exits are stopped first, so
# that no server kernel outlives the process's last HIP call.
_live_servers = {}


def ask_server_create(ctx, slots=64, waves_per_cu=0, pool_bytes=0):
    cfg = ask_server_cfg(int(slots), int(waves_per_cu), int(pool_bytes))
    h = _P()
    _check(lib.ask_server_create(ctx, C.byref(cfg), C.byref(h)), ctx)
    _live_servers[h.value] = ctx
    return h


def ask_server_submit(sv, win, prm, d_out):
    """Ticket of the posted request, or None when the server is busy
    (no free slot or pool memory right now)."""
    t = C.c_uint64()
    s = lib.ask_server_submit(sv, C.byref(win), C.byref(prm), _P(d_out), C.byref(t))
    if s == EBUSY:
        return None
    _check(s, _live_servers.get(sv.value))
    return t.value


def ask_server_reap(sv, cap=256):
    """[(ticket, status)] of requests finished since the last reap."""
    T = (C.c_uint64 * cap)()
    S = (C.c_int32 * cap)()
    n = C.c_uint32()
    _check(lib.ask_server_reap(sv, T, S, cap, C.byref(n)), _live_servers.get(sv.value))
    return [(T[i], S[i]) for i in range(n.value)]


def ask_server_poll(sv, ticket):
    """(done, status, latency in s or None while running) of one request."""
    d = C.c_int()
    lat = C.c_double()
    s = lib.ask_server_poll(sv, int(ticket), C.byref(d), C.byref(lat))
    if s == EINVAL:
        _check(s, _live_servers.get(sv.value))
    return bool(d.value), s, (lat.value if lat.value >= 0 else None)


def ask_server_in_flight(sv):
    n = C.c_uint32()
    _check(lib.ask_server_in_flight(sv, C.byref(n)))
    return n.value


def ask_server_destroy(sv):
    ctx = _live_servers.pop(sv.value, None)
    _check(lib.ask_server_destroy(sv), ctx)


def volume(v):
    """ask_volume of a volume description (x0..z1, W, H, L, D, c = (cr, ci))."""
    return ask_volume(float(v.x0), float(v.x1), float(v.y0), float(v.y1), float(v.z0),
                      float(v.z1), int(v.W), int(v.H), int(v.L), int(v.D), float(v.c[0]),
                      float(v.c[1]))


def params3(g, r, B, curve="canonical"):
    return ask3_params(int(g), int(r), int(B), CURVES[curve] if isinstance(curve, str) else curve)


def ask3_validate(vol, prm=None):
    return lib.ask3_validate(C.byref(vol), C.byref(prm) if prm is not None else None)


def ask3_workspace_bytes(vol, prm):
    n = C.c_uint64()
    _check(lib.ask3_workspace_bytes(C.byref(vol), C.byref(prm), C.byref(n)))
    return n.value


def ask3_dwell_exhaustive(vol, d_out, d_work, work_bytes=None, stream=0):
    """d_work: device memory of at least EXHAUSTIVE3_WORK_BYTES bytes."""
    nbytes = EXHAUSTIVE3_WORK_BYTES if work_bytes is None else work_bytes
    _check(lib.ask3_dwell_exhaustive(C.byref(vol), _P(d_out), _P(d_work), nbytes, _P(stream)))


def ask3_dwell_subdiv(vol, prm, d_out, d_work, work_bytes, stream=0, want_stats=False):
    st = ask3_stats() if want_stats else None
    _check(lib.ask3_dwell_subdiv(C.byref(vol), C.byref(prm), _P(d_out), _P(d_work),
                                 int(work_bytes), _P(stream),
                                 C.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def _stop_servers():
    for h in list(_live_servers):
        lib.ask_server_destroy(_P(h))
        _live_servers.pop(h, None)


import atexit  # noqa: E402

atexit.register(_stop_servers)
