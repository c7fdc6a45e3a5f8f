"""GPU parity for filled Julia sets (the pixel is z0, c is fixed): every form,
the batch and the server give the oracle's images bit for bit, on ragged
windows that cross the set's boundary, on the degenerate cases (one pixel,
one row, the real segment of c = -2, c = 0, |c|^2 > 3.99 where every pixel
takes the checked loop), mixed with Mandelbrot images in one batch, and at
the 16384 x 16384 basilica size on sampled pixels."""
import time

import numpy as np
import pytest

from workloads import JULIA, JULIA_PARAMS, Window, paper_window

pytestmark = pytest.mark.gpu

FORMS = ("levels", "levels_readback", "persistent")

WINDOWS = [
    Window(-1.7, 1.7, -1.7, 1.7, 300, 211, 500, julia=(-1.0, 0.0)),
    Window(-1.6, 1.6, -1.2, 1.2, 257, 190, 800, julia=(-0.123, 0.745)),
    Window(-1.6, 1.6, -1.0, 1.0, 200, 125, 300, julia=(-0.8, 0.156)),
    Window(-2.5, 2.5, -2.5, 2.5, 131, 97, 200, julia=(-2.0, 0.0)),
    Window(-1.5, 1.5, -1.5, 1.5, 77, 64, 150, julia=(2.1, 0.3)),
    Window(-0.05, 0.05, 0.6, 0.7, 128, 128, 4000, julia=(-0.123, 0.745)),
    Window(-1.0, 1.0, -1.0, 1.0, 1, 1, 10, julia=(0.0, 0.0)),
    Window(-1.3, 1.3, -1.3, 1.3, 97, 1, 64, julia=(0.0, 0.0)),
]
PARAMS = [(4, 2, 8), (3, 3, 5), (1, 2, 1)]


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2206_02255_amd import ask
    assert torch.cuda.is_available()
    ctx = ask.ask_create(0)
    ask.ask_set_wait_limit(ctx, 5.0)
    yield ask, ctx, torch
    ask.ask_destroy(ctx)


def _host(torch, t, w):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32).reshape(w.H, w.W)


def exhaustive(gpu, w):
    ask, ctx, torch = gpu
    out = torch.zeros(w.H * w.W, dtype=torch.int32, device="cuda")
    ask.ask_dwell_exhaustive(ctx, ask.window(w), out.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    return _host(torch, out, w)


def subdiv(gpu, w, g, r, B, form, stats=True):
    ask, ctx, torch = gpu
    out = torch.zeros(w.H * w.W, dtype=torch.int32, device="cuda")
    st = ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(g, r, B, form), out.data_ptr(),
                              torch.cuda.current_stream().cuda_stream, want_stats=stats)
    return _host(torch, out, w), st


def test_window_set_fields(gpu):
    ask = gpu[0]
    aw = ask.window(WINDOWS[0])
    assert aw.set == ask.SET_JULIA and (aw.cr, aw.ci) == (-1.0, 0.0)
    assert ask.window(paper_window(8, 8)).set == ask.SET_MANDELBROT
    bad = ask.window(WINDOWS[0])
    bad.cr = float("nan")
    assert ask.ask_validate(bad) == ask.EINVAL


def test_julia_exhaustive(gpu, ref):
    for w in WINDOWS:
        print("exhaustive", w, flush=True)
        want, _ = ref.exhaustive(w)
        assert np.array_equal(exhaustive(gpu, w), want), w


@pytest.mark.parametrize("form", FORMS)
def test_julia_subdiv(gpu, ref, form):
    for w in WINDOWS:
        for g, r, B in PARAMS:
            g = min(g, w.W, w.H)
            print(form, w, (g, r, B), flush=True)
            img, st = subdiv(gpu, w, g, r, B, form)
            want, rst = ref.subdiv(w, g, r, B)
            assert np.array_equal(img, want), (w, g, r, B)
            n = rst["levels"]
            assert st["levels"] == n
            for k in ("regions", "fills", "splits", "leaves"):
                assert st[k][:n] == rst[k][:n], k
            assert rst["iters_ring_filled"] <= st["iters_ring"] <= rst["iters_ring"]
            assert rst["iters_leaf_inner"] <= st["iters_leaf"] <= rst["iters_leaf"]
            assert st["overflow"] == 0


@pytest.mark.parametrize("form", ["levels", "persistent"])
def test_batch_mixes_mandelbrot_and_julia(gpu, ref, form):
    ask, ctx, torch = gpu
    ws = [WINDOWS[0], paper_window(300, 200), WINDOWS[1],
          Window(-1.5, 0.5, -1.0, 1.0, 181, 97, 700), WINDOWS[3], WINDOWS[6]]
    ps = [(4, 2, 8), (3, 2, 16), (2, 4, 8), (5, 3, 7), (4, 2, 4), (1, 2, 1)]
    outs = [torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda") for w in ws]
    ask.ask_dwell_batch(ctx, [ask.window(w) for w in ws],
                        [ask.params(g, r, B, form) for g, r, B in ps],
                        [o.data_ptr() for o in outs], torch.cuda.current_stream().cuda_stream)
    for w, (g, r, B), o in zip(ws, ps, outs):
        want, _ = ref.subdiv(w, g, r, B)
        assert np.array_equal(_host(torch, o, w), want), (w, g, r, B)


def test_server_serves_julia_requests(gpu, ref):
    ask, ctx, torch = gpu
    reqs = [(WINDOWS[0], 4, 2, 8), (WINDOWS[2], 3, 3, 5), (paper_window(400, 300), 4, 2, 16),
            (WINDOWS[1], 2, 2, 16), (WINDOWS[4], 2, 2, 4)]
    outs = [torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda") for w, *_ in reqs]
    torch.cuda.synchronize()
    sv = ask.ask_server_create(ctx, slots=8, pool_bytes=64 << 20)
    try:
        tickets = {}
        for i, (w, g, r, B) in enumerate(reqs):
            t = ask.ask_server_submit(sv, ask.window(w), ask.params(g, r, B), outs[i].data_ptr())
            assert t is not None
            tickets[t] = i
        got = {}
        t0 = time.time()
        while len(got) < len(tickets):
            assert time.time() - t0 < 60, "requests did not finish"
            for t, st in ask.ask_server_reap(sv):
                got[t] = st
            time.sleep(0.0005)
        assert all(st == 0 for st in got.values())
    finally:
        ask.ask_server_destroy(sv)
    for i, (w, g, r, B) in enumerate(reqs):
        want, _ = ref.subdiv(w, g, r, B)
        assert np.array_equal(outs[i].cpu().numpy().view(np.uint32).reshape(w.H, w.W), want), w


def test_julia_large_sampled(gpu, ref):
    """The basilica at 16384 x 16384, D = 2048, in the benchmarked form and
    parameters, and the exhaustive image, on 4096 sampled pixels each."""
    ask, ctx, torch = gpu
    w, p = JULIA, JULIA_PARAMS
    rng = np.random.default_rng(2206)
    px = rng.integers(0, w.W, 4096).astype(np.uint32)
    py = rng.integers(0, w.H, 4096).astype(np.uint32)
    out = torch.zeros(w.H * w.W, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    print("julia 16384 persistent", flush=True)
    ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(p.g, p.r, p.B, "persistent"),
                         out.data_ptr(), s)
    torch.cuda.synchronize()
    flat = (py.astype(np.int64) * w.W + px).astype(np.int64)
    got = out[torch.from_numpy(flat).cuda()].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref.subdiv_pixels(w, p.g, p.r, p.B, px, py))
    print("julia 16384 exhaustive", flush=True)
    ask.ask_dwell_exhaustive(ctx, ask.window(w), out.data_ptr(), s)
    torch.cuda.synchronize()
    got = out[torch.from_numpy(flat).cuda()].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref.dwell_pixels(w, px, py))
