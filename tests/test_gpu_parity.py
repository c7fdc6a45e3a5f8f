"""GPU parity: images from the C ABI equal the CPU oracle's bit for bit.

Dwell images are integers, so the bar is exact equality of every pixel (and
of the work counters) against the oracle on the same seeded inputs: small
ragged windows that span several tiles and regions, the 1024 x 1024 paper
window, a 4096 x 4096 window, and sampled pixels of the 16384 x 16384 window.
"""
import math

import numpy as np
import pytest

from workloads import (LARGE, LARGE_DEFAULT, LARGE_DEFAULT_FORM, SMALL, SMALL_PARAMS, Window,
                       paper_window, random_params, random_windows)

pytestmark = pytest.mark.gpu

FORMS = ("levels", "levels_readback", "persistent")


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2206_02255_amd import ask
    assert torch.cuda.is_available()
    ctx = ask.ask_create(0)
    yield ask, ctx, torch
    ask.ask_destroy(ctx)


def _out(torch, w):
    return torch.zeros(w.H * w.W, dtype=torch.int32, device="cuda")


def _host(torch, t, w):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32).reshape(w.H, w.W)


def gpu_exhaustive(gpu, w, tile=None):
    ask, ctx, torch = gpu
    out = _out(torch, w)
    ask.ask_dwell_exhaustive(ctx, ask.window(w), out.data_ptr(),
                             torch.cuda.current_stream().cuda_stream, tile=tile)
    return _host(torch, out, w)


def gpu_subdiv(gpu, w, g, r, B, form, stats=True, band=0, tile=(0, 0)):
    ask, ctx, torch = gpu
    out = _out(torch, w)
    st = ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(g, r, B, form, band, tile),
                              out.data_ptr(), torch.cuda.current_stream().cuda_stream,
                              want_stats=stats)
    return _host(torch, out, w), st


def assert_same_stats(st, ref_st, no_bands=False):
    n = ref_st["levels"]
    assert st["levels"] == n
    for k in ("regions", "fills", "splits", "leaves"):
        assert st[k][:n] == ref_st[k][:n], k
    # A ring scan stops once the ring is known to be mixed, so the GPU computes
    # at most the oracle's ring iterations and at least those of the rings of
    # filled regions, which must be computed whole. A leaf keeps its ring's
    # dwells and computes its inside; a leaf cut into bands computes every
    # pixel of its bands.
    assert ref_st["iters_ring_filled"] <= st["iters_ring"] <= ref_st["iters_ring"]
    assert ref_st["iters_leaf_inner"] <= st["iters_leaf"] <= ref_st["iters_leaf"]
    if no_bands:
        # every leaf's ring is computed whole, once, and its inside once
        leaf_rings = ref_st["iters_leaf"] - ref_st["iters_leaf_inner"]
        assert st["iters_leaf"] == ref_st["iters_leaf_inner"]
        assert ref_st["iters_ring_filled"] + leaf_rings <= st["iters_ring"]
    for k in ("ring_px", "leaf_px", "fill_px"):
        assert st[k] == ref_st[k], k
    assert st["overflow"] == 0


EDGE_WINDOWS = [
    Window(-1.5, 0.5, -1.0, 1.0, 1, 1, 100),
    Window(-1.5, 0.5, -1.0, 1.0, 1, 77, 100),
    Window(-1.5, 0.5, -1.0, 1.0, 93, 1, 100),
    Window(-1.5, 0.5, -1.0, 1.0, 17, 300, 1),    # D = 1
    Window(-1.5, 0.5, -1.0, 1.0, 130, 70, 15),   # D below the test stride
    Window(-1.5, 0.5, -1.0, 1.0, 130, 70, 16),
    Window(-1.5, 0.5, -1.0, 1.0, 130, 70, 17),
]


def adversarial_windows():
    """Windows where the escape test is delicate: around c = -2 (orbits that
    hover at |z| = 2), on the circle |c| = 2, and across |c|^2 = 3.99, where
    the fast loop hands over to the plain one."""
    out = []
    for span in (1e-15, 1e-12, 1e-8, 1e-4):
        out.append(Window(-2 - span, -2 + span, -span, span, 67, 61, 3000))
    for th in np.linspace(0.1, math.pi, 9):
        cx, cy = 2 * math.cos(th), 2 * math.sin(th)
        for span in (1e-13, 1e-6):
            out.append(Window(cx - span, cx + span, cy - span, cy + span, 33, 35, 500))
    rad = math.sqrt(3.99)
    for th in (0.3, 1.7, 2.9, 3.1):
        cx, cy = rad * math.cos(th), rad * math.sin(th)
        out.append(Window(cx - 1e-9, cx + 1e-9, cy - 1e-9, cy + 1e-9, 40, 40, 2000))
    return out


def test_exhaustive_edge_windows(gpu, ref):
    for w in EDGE_WINDOWS:
        print("exhaustive", w, flush=True)
        assert np.array_equal(gpu_exhaustive(gpu, w), ref.exhaustive(w)[0])


def test_exhaustive_adversarial_windows(gpu, ref):
    for w in adversarial_windows():
        print("exhaustive", w, flush=True)
        assert np.array_equal(gpu_exhaustive(gpu, w), ref.exhaustive(w)[0])


def test_exhaustive_random_windows(gpu, ref):
    for w in random_windows(31, 40, max_side=200, max_dwell=3000):
        print("exhaustive", w, flush=True)
        assert np.array_equal(gpu_exhaustive(gpu, w), ref.exhaustive(w)[0])


def test_exhaustive_small_paper_window(gpu, ref):
    img = gpu_exhaustive(gpu, SMALL)
    want, iters = ref.exhaustive(SMALL)
    assert np.array_equal(img, want)
    assert int(img.astype(np.uint64).sum()) == iters


def test_exhaustive_4096(gpu, ref):
    w = paper_window(4096, 2048)
    assert np.array_equal(gpu_exhaustive(gpu, w), ref.exhaustive(w)[0])


@pytest.mark.parametrize("form", FORMS)
def test_subdiv_edge_windows(gpu, ref, form):
    for w in EDGE_WINDOWS:
        for g, r, B in [(1, 2, 1), (1, 3, 4), (min(w.W, w.H), 2, 2)]:
            print(form, w, g, r, B, flush=True)
            img, st = gpu_subdiv(gpu, w, g, r, B, form)
            want, ref_st = ref.subdiv(w, g, r, B)
            assert np.array_equal(img, want)
            assert_same_stats(st, ref_st)


@pytest.mark.parametrize("form", FORMS)
def test_subdiv_random_windows(gpu, ref, form):
    for i, w in enumerate(random_windows(41, 25, max_side=160, max_dwell=2000)):
        for p in random_params(300 + i, w, 3):
            print(form, w, p, flush=True)
            img, st = gpu_subdiv(gpu, w, p.g, p.r, p.B, form)
            want, ref_st = ref.subdiv(w, p.g, p.r, p.B)
            assert np.array_equal(img, want)
            assert_same_stats(st, ref_st)


@pytest.mark.parametrize("form", FORMS)
def test_subdiv_small_paper_window(gpu, ref, form):
    p = SMALL_PARAMS
    img, st = gpu_subdiv(gpu, SMALL, p.g, p.r, p.B, form)
    want, ref_st = ref.subdiv(SMALL, p.g, p.r, p.B)
    assert np.array_equal(img, want)
    assert_same_stats(st, ref_st, no_bands=True)  # B = 32: 1024-pixel leaves, no bands


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("g,r,B", [(32, 4, 16), (16, 2, 32), (2, 8, 128), (64, 2, 16)])
def test_subdiv_4096(gpu, ref, form, g, r, B):
    w = paper_window(4096, 2048)
    img, st = gpu_subdiv(gpu, w, g, r, B, form)
    want, ref_st = ref.subdiv(w, g, r, B)
    assert np.array_equal(img, want)
    assert_same_stats(st, ref_st)


# Levels whose rings have 512 pixels or more run a workgroup per region in
# the per-level form: ragged regions that split, leaf-size regions whose
# inside the four waves stream together (no bands), leaf-size regions cut
# into bands, and a Julia set.
WORKGROUP_CASES = [
    (Window(-1.5, 0.5, -1.0, 1.0, 1500, 900, 600), 2, 2, 64, 0),
    (Window(-1.5, 0.5, -1.0, 1.0, 1500, 900, 600), 2, 2, 800, 0xffffffff),
    (Window(-1.5, 0.5, -1.0, 1.0, 1500, 900, 600), 2, 2, 800, 0),
    (Window(-0.8, -0.6, 0.05, 0.2, 1111, 777, 1500), 1, 3, 40, 0),
    (Window(-1.7, 1.7, -1.7, 1.7, 1200, 1200, 800, julia=(-1.0, 0.0)), 2, 4, 300, 0xffffffff),
]


@pytest.mark.parametrize("w,g,r,B,band", WORKGROUP_CASES)
def test_levels_workgroup_regions(gpu, ref, w, g, r, B, band):
    img, st = gpu_subdiv(gpu, w, g, r, B, "levels", band=band)
    want, ref_st = ref.subdiv(w, g, r, B)
    assert np.array_equal(img, want)
    assert_same_stats(st, ref_st, no_bands=band == 0xffffffff)


def test_subdiv_without_stats_equals_with_stats(gpu):
    w = paper_window(2048, 1024)
    for form in FORMS:
        a, _ = gpu_subdiv(gpu, w, 8, 2, 16, form, stats=True)
        b, _ = gpu_subdiv(gpu, w, 8, 2, 16, form, stats=False)
        assert np.array_equal(a, b)


# Windows whose 180 x 150 border (one level-0 region at g = 1) is mixed while
# every 11th border pixel, counted along the ring (first row, last row, first
# column, last column), has one dwell: a long ring's first 64 evenly spaced
# pixels then agree, and only the rest of the ring shows that it is mixed.
PROBE_UNIFORM_WINDOWS = [
    Window(-0.70645, -0.18018, -0.18604, 0.25252, 180, 150, 96),
    Window(0.21974, 0.30202, -0.44334, -0.37477, 180, 150, 96),
    Window(0.15577, 0.32353, 0.04127, 0.18107, 180, 150, 96),
]


def _ring_dwells(E):
    H, W = E.shape
    return np.concatenate([E[0, :], E[H - 1, :], E[1:H - 1, 0], E[1:H - 1, W - 1]])


@pytest.mark.parametrize("form", FORMS)
def test_mixed_ring_whose_spread_sample_is_uniform(gpu, ref, form):
    for w in PROBE_UNIFORM_WINDOWS:
        E, _ = ref.exhaustive(w)
        ring = _ring_dwells(np.asarray(E).reshape(w.H, w.W))
        p = (len(ring) + 63) // 64
        assert len(np.unique(ring[::p])) == 1 and len(np.unique(ring)) > 1
        for B in (16, 64):
            want, ref_st = ref.subdiv(w, 1, 2, B)
            img, st = gpu_subdiv(gpu, w, 1, 2, B, form)
            assert np.array_equal(img, want), (w, B)
            assert_same_stats(st, ref_st)


def test_persistent_repeated_calls(gpu, ref):
    # Queue slots are reused across calls; tags of older calls must never be
    # taken for new entries.
    ws = random_windows(51, 6, max_side=120, max_dwell=600)
    for rep in range(3):
        for w in ws:
            img, _ = gpu_subdiv(gpu, w, 2, 2, 4, "persistent", stats=False)
            assert np.array_equal(img, ref.subdiv(w, 2, 2, 4)[0])


@pytest.mark.parametrize("form,g,r,B", [
    ("levels", 32, 4, 16), ("persistent", 32, 4, 16),
    (LARGE_DEFAULT_FORM, LARGE_DEFAULT.g, LARGE_DEFAULT.r, LARGE_DEFAULT.B)])
def test_large_paper_window_sampled(gpu, ref, form, g, r, B):
    # 16384 x 16384, D = 2048: sampled pixels against the oracle's tree
    # descent, plus the counters that hold at any size (the last case is the
    # benchmark's launch configuration).
    w = LARGE
    img, st = gpu_subdiv(gpu, w, g, r, B, form)
    rng = np.random.default_rng(77)
    px = rng.integers(0, w.W, 150)
    py = rng.integers(0, w.H, 150)
    assert np.array_equal(img[py, px], ref.subdiv_pixels(w, g, r, B, px, py))
    assert st["overflow"] == 0
    assert st["regions"][0] == g * g
    for lv in range(st["levels"] - 1):
        assert st["regions"][lv + 1] <= st["splits"][lv] * r * r
        assert st["regions"][lv] == st["fills"][lv] + st["leaves"][lv] + st["splits"][lv]
    assert (img >= 1).all() and (img <= w.D).all()
    # the window is symmetric about the real axis and every partition of
    # 16384 used here is exact, so the image is too
    assert np.array_equal(img[:64], img[::-1][:64])


def test_deep_window_sampled(gpu, ref):
    # 32768 x 32768 around a boundary point, width 1e-6, D = 8192, in the
    # bench's launch configuration: sampled pixels against the oracle's tree
    # descent (subdivision) and dwell (exhaustive).
    import workloads
    ask, ctx, torch = gpu
    w = workloads.deep_window()
    p = workloads.DEEP_PARAMS
    rng = np.random.default_rng(17)
    px = rng.integers(0, w.W, 120)
    py = rng.integers(0, w.H, 120)
    out = torch.empty(w.W * w.H, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    idx = torch.as_tensor(py * w.W + px, device="cuda")

    def sample():
        torch.cuda.synchronize()
        return out[idx].cpu().numpy().view(np.uint32)

    ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(p.g, p.r, p.B, "persistent"),
                         out.data_ptr(), s)
    ask.ask_synchronize(ctx, s)
    assert np.array_equal(sample(), ref.subdiv_pixels(w, p.g, p.r, p.B, px, py))
    ask.ask_dwell_exhaustive(ctx, ask.window(w), out.data_ptr(), s)
    assert np.array_equal(sample(), ref.dwell_pixels(w, px, py))


def test_large_exhaustive_sampled(gpu, ref):
    w = LARGE
    img = gpu_exhaustive(gpu, w)
    rng = np.random.default_rng(78)
    px = rng.integers(0, w.W, 400)
    py = rng.integers(0, w.H, 400)
    assert np.array_equal(img[py, px], ref.dwell_pixels(w, px, py))
    assert np.array_equal(img[:32], img[::-1][:32])


def test_persistent_wait_limit_reports_timeout(gpu, ref):
    # Host-forced failure: with a zero wait limit every wave that has to wait
    # records a timeout and leaves; the render reports ASK_ETIMEOUT, and the
    # next render on the same context is whole again.
    ask, ctx, torch = gpu
    w = paper_window(512, 256)
    stream = torch.cuda.current_stream().cuda_stream
    out = _out(torch, w)
    ask.ask_set_wait_limit(ctx, 0.0)
    try:
        ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(2, 2, 8, "persistent"),
                             out.data_ptr(), stream)
        with pytest.raises(ask.AskError) as e:
            ask.ask_synchronize(ctx, stream)
        assert e.value.status == ask.ETIMEOUT
    finally:
        ask.ask_set_wait_limit(ctx, 10.0)
    img, _ = gpu_subdiv(gpu, w, 2, 2, 8, "persistent")
    assert np.array_equal(img, ref.subdiv(w, 2, 2, 8)[0])
    ask.ask_synchronize(ctx, stream)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("band", [0xffffffff, 64, 200, 4096])
def test_leaf_bands(gpu, ref, form, band):
    """Leaf work shared by several waves (row bands of `band` pixels, queued
    or put in the next level's table) or kept on the deciding wave
    (0xffffffff): the same image and counters in every form."""
    ask, ctx, torch = gpu
    cases = [(Window(-1.5, 0.5, -1.0, 1.0, 600, 517, 700), 4, 2, 128),
             (Window(-0.75, -0.73, 0.1, 0.12, 400, 300, 3000), 2, 3, 200),
             (Window(-1.6, 1.6, -1.6, 1.6, 512, 512, 400, julia=(-1.0, 0.0)), 8, 2, 64)]
    for w, g, r, B in cases:
        print(band, w, (g, r, B), flush=True)
        out = _out(torch, w)
        st = ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(g, r, B, form, band),
                                  out.data_ptr(), torch.cuda.current_stream().cuda_stream,
                                  want_stats=True)
        want, rst = ref.subdiv(w, g, r, B)
        assert np.array_equal(_host(torch, out, w), want), (w, band)
        assert_same_stats(st, rst, no_bands=band == 0xffffffff or B * B <= band)


TILES = [(4, 16), (8, 8), (16, 4), (32, 2), (64, 1)]


@pytest.mark.parametrize("tile", TILES)
def test_exhaustive_wave_tiles(gpu, ref, tile):
    """Every wave tile gives the oracle's image: ragged windows (partial
    tiles on the right and bottom edges) and the 1024 x 1024 paper window."""
    for w in EDGE_WINDOWS + random_windows(33, 8, max_side=200, max_dwell=1000) + [SMALL]:
        assert np.array_equal(gpu_exhaustive(gpu, w, tile), ref.exhaustive(w)[0]), (tile, w)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("tile", [(4, 16), (8, 8), (32, 2), (64, 1)])
def test_subdiv_wave_tiles(gpu, ref, form, tile):
    """Leaf pixels streamed tile by tile: the oracle's image and counters,
    for whole leaves and for leaf bands."""
    cases = [(w, p) for i, w in enumerate(random_windows(43, 6, max_side=160, max_dwell=1500))
             for p in random_params(900 + i, w, 2)]
    cases.append((SMALL, SMALL_PARAMS))
    for w, p in cases:
        want, rst = ref.subdiv(w, p.g, p.r, p.B)
        for band in (0xffffffff, 64, 0):
            img, st = gpu_subdiv(gpu, w, p.g, p.r, p.B, form, band=band, tile=tile)
            assert np.array_equal(img, want), (tile, w, p, band)
            assert_same_stats(st, rst)


def test_kernel_times_of_consecutive_renders(gpu):
    """The context times the dominant kernel of every timed render: one
    positive device time per render, in order, no more than the ring holds."""
    ask, ctx, torch = gpu
    w = paper_window(1024, 512)
    out = _out(torch, w)
    s = torch.cuda.current_stream().cuda_stream
    ask.ask_enable_timing(ctx, True)
    try:
        for _ in range(5):
            ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(8, 2, 16, "persistent"),
                                 out.data_ptr(), s)
        ms = ask.ask_kernel_times(ctx)
        assert len(ms) == 5 and all(m > 0 for m in ms)
        assert ask.ask_last_kernel_ms(ctx) == ms[-1]
        for _ in range(300):
            ask.ask_dwell_exhaustive(ctx, ask.window(paper_window(64, 16)), out.data_ptr(), s)
        assert len(ask.ask_kernel_times(ctx, cap=1000)) == 256
        assert len(ask.ask_kernel_times(ctx, cap=3)) == 3
    finally:
        ask.ask_enable_timing(ctx, False)
        ask.ask_synchronize(ctx, s)


def test_context_with_preallocated_queues(ref):
    """A context created with queue memory set aside renders the same images."""
    import torch
    from paper_2206_02255_amd import ask
    ctx = ask.ask_create(0, queue_bytes=8 << 20)
    try:
        g = (ask, ctx, torch)
        for form in FORMS:
            img, st = gpu_subdiv(g, SMALL, 4, 2, 32, form)
            want, rst = ref.subdiv(SMALL, 4, 2, 32)
            assert np.array_equal(img, want)
            assert_same_stats(st, rst)
    finally:
        ask.ask_destroy(ctx)


@pytest.mark.parametrize("form,band", [("persistent", 0xffffffff), ("levels", 0)])
def test_one_leaf_of_65536_squared(gpu, ref, form, band):
    """W = H = 65536, g = 1, B = 65536: the whole image is one leaf of 2^32
    pixels (cut into bands of 2^24 pixels even without banding). Every pixel is written
    and sampled pixels equal the oracle's (the paper's largest n, Sec. 6.1)."""
    ask, ctx, torch = gpu
    w = paper_window(65536, 24)
    out = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    print(form, band, w, flush=True)
    st = ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(1, 2, 65536, form, band),
                              out.data_ptr(), s, want_stats=True)
    assert st["leaves"][0] == 1 and st["leaf_px"] == 1 << 32 and st["overflow"] == 0
    assert int((out == 0).sum().item()) == 0
    rng = np.random.default_rng(65536)
    px = rng.integers(0, w.W, 2000).astype(np.int64)
    py = rng.integers(0, w.H, 2000).astype(np.int64)
    idx = torch.as_tensor(py * w.W + px, device="cuda")
    got = out[idx].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref.subdiv_pixels(w, 1, 2, 65536, px, py))
    corners = torch.as_tensor([0, w.W - 1, (w.H - 1) * w.W, w.W * w.H - 1], device="cuda")
    cpx, cpy = np.array([0, w.W - 1, 0, w.W - 1]), np.array([0, 0, w.H - 1, w.H - 1])
    assert np.array_equal(out[corners].cpu().numpy().view(np.uint32),
                          ref.subdiv_pixels(w, 1, 2, 65536, cpx, cpy))
    del out
