"""GPU parity at the full sizes of the benchmark's workloads.

* The 16384 x 16384 paper window (Sec. 6.1, D = 2048): every point of the
  (g, r, B) sweep of Sec. 6.2 in the per-level form, the benchmark's
  (64, 4, 16) in the persistent form too, and the exhaustive image, each
  compared whole with the oracle through the SHA-256 digest of its pixels
  (tests/golden/fullsize_mandelbrot16384_D2048.txt, written by
  make_fullsize_digests.py from the oracle alone), and the pixel count where
  each subdivision image differs from the exhaustive one.
* The deep zoom (32768 x 32768, width 1e-6, D = 8192): 12 blocks of 32 x 32
  pixels (12 288 pixels) against the oracle's tree descent, for the
  subdivision and the exhaustive image.
* The 256-image batch, rendered in one launch and captured into a graph: an
  8 x 8 block of every image against the oracle, and the replays against the
  eager batch.
* Served requests: an 8 x 8 block of every request of one second of the
  serving schedule against the oracle.
"""
import concurrent.futures
import hashlib
import os

import numpy as np
import pytest

import workloads
from workloads import LARGE, LARGE_DEFAULT, Params

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fullsize_mandelbrot16384_D2048.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "exhaustive":
                out["exhaustive"] = (parts[1], int(parts[2]))
            else:
                g, r, B = (int(x) for x in parts[:3])
                out[(g, r, B)] = (parts[3], int(parts[4]), int(parts[5]))
    return out


GOLD = _golden()
CONFIGS = [(p.g, p.r, p.B) for p in workloads.LARGE_SWEEP]


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2206_02255_amd import ask
    ctx = ask.ask_create(0)
    yield ask, ctx, torch
    ask.ask_destroy(ctx)


def _digest(t):
    return hashlib.sha256(t.cpu().numpy().astype("<i4", copy=False).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def exhaustive(env):
    ask, ctx, torch = env
    e = torch.empty(LARGE.pixels, dtype=torch.int32, device="cuda")
    ask.ask_dwell_exhaustive(ctx, ask.window(LARGE), e.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    yield e
    del e


def test_exhaustive_image_whole(env, exhaustive):
    ask, ctx, torch = env
    want, iters = GOLD["exhaustive"]
    assert _digest(exhaustive) == want
    assert int(exhaustive.to(torch.int64).sum().item()) == iters


def _subdiv_whole(env, exhaustive, g, r, B, form):
    ask, ctx, torch = env
    want, _, mismatch = GOLD[(g, r, B)]
    out = torch.zeros(LARGE.pixels, dtype=torch.int32, device="cuda")
    print(form, g, r, B, flush=True)
    ask.ask_dwell_subdiv(ctx, ask.window(LARGE), ask.params(g, r, B, form), out.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    ask.ask_synchronize(ctx, torch.cuda.current_stream().cuda_stream)
    assert _digest(out) == want, (form, g, r, B)
    assert int((out != exhaustive).sum().item()) == mismatch
    del out


@pytest.mark.parametrize("g,r,B", CONFIGS)
def test_sweep_image_whole(env, exhaustive, g, r, B):
    _subdiv_whole(env, exhaustive, g, r, B, "levels")


@pytest.mark.parametrize("form", ["persistent", "levels"])
def test_benchmark_configuration_whole(env, exhaustive, form):
    p = LARGE_DEFAULT
    _subdiv_whole(env, exhaustive, p.g, p.r, p.B, form)


def _blocks(rng, W, H, n, side):
    """n blocks of side x side pixels at random places: pixel coordinates."""
    px, py = [], []
    for _ in range(n):
        x0 = int(rng.integers(0, max(1, W - side + 1)))
        y0 = int(rng.integers(0, max(1, H - side + 1)))
        yy, xx = np.mgrid[y0:min(H, y0 + side), x0:min(W, x0 + side)]
        px.append(xx.ravel())
        py.append(yy.ravel())
    return px, py


def _parallel(fn, jobs):
    with concurrent.futures.ThreadPoolExecutor(16) as ex:
        return list(ex.map(lambda a: fn(*a), jobs))


def test_deep_zoom_blocks(env, ref):
    """12 288 pixels of the deep zoom in 32 x 32 blocks (each block shares
    its region tree, so the oracle's descent stays cheap), in the
    benchmark's parameters and the autotuner's, and the exhaustive image."""
    from paper_2206_02255_amd import autotune
    ask, ctx, torch = env
    w = workloads.deep_window()
    win = ask.window(w)
    params = [workloads.DEEP_PARAMS]
    hit = autotune.lookup(autotune.workload_key(win, "persistent"))
    if hit and "tile" in hit and Params(hit["g"], hit["r"], hit["B"]) != params[0]:
        params.append(Params(hit["g"], hit["r"], hit["B"]))
    rng = np.random.default_rng(33)
    px, py = _blocks(rng, w.W, w.H, 12, 32)
    allx, ally = np.concatenate(px), np.concatenate(py)
    idx = torch.as_tensor(ally.astype(np.int64) * w.W + allx, device="cuda")
    out = torch.empty(w.W * w.H, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for p in params:
        print("deep", p, flush=True)
        ask.ask_dwell_subdiv(ctx, win, ask.params(p.g, p.r, p.B, "persistent"), out.data_ptr(), s)
        ask.ask_synchronize(ctx, s)
        got = out[idx].cpu().numpy().view(np.uint32)
        want = np.concatenate(_parallel(lambda x, y: ref.subdiv_pixels(w, p.g, p.r, p.B, x, y),
                                        list(zip(px, py))))
        assert np.array_equal(got, want), p
    ask.ask_dwell_exhaustive(ctx, win, out.data_ptr(), s)
    torch.cuda.synchronize()
    got = out[idx].cpu().numpy().view(np.uint32)
    want = np.concatenate(_parallel(lambda x, y: ref.dwell_pixels(w, x, y), list(zip(px, py))))
    assert np.array_equal(got, want)
    del out


def test_batch_of_256_boundary_images(env, ref):
    """The benchmark's batch in one persistent launch with the autotuner's
    per-image rule: an 8 x 8 block of every image against the oracle, the
    one-by-one renders, and four replays of the batch captured into a graph."""
    from paper_2206_02255_amd import autotune
    ask, ctx, torch = env
    ims = workloads.batch_images()
    hit = autotune.lookup(autotune.BATCH_KEY)
    rule = hit["rule"] if hit else {"s0": 256, "r": 2, "B": 128, "tile": [0, 0]}
    prms = [workloads.rule_params(w.W, rule["s0"], rule["r"], rule["B"]) for w in ims]
    sizes = [w.pixels for w in ims]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = torch.zeros(int(sum(sizes)), dtype=torch.int32, device="cuda")
    ptrs = [out.data_ptr() + 4 * int(o) for o in offs]
    wins = [ask.window(w) for w in ims]
    pers = [ask.params(p.g, p.r, p.B, "persistent", 0, tuple(rule["tile"])) for p in prms]
    s = torch.cuda.current_stream().cuda_stream
    print("batch", rule, flush=True)
    st = ask.ask_dwell_batch(ctx, wins, pers, ptrs, s, want_stats=True)
    assert st["overflow"] == 0
    rng = np.random.default_rng(44)
    blocks = [_blocks(rng, w.W, w.H, 1, 8) for w in ims]
    px = [b[0][0] for b in blocks]
    py = [b[1][0] for b in blocks]
    idx = torch.as_tensor(np.concatenate([o + y.astype(np.int64) * w.W + x
                                          for o, w, x, y in zip(offs, ims, px, py)]),
                          device="cuda")

    def sample():
        torch.cuda.synchronize()
        return out[idx].cpu().numpy().view(np.uint32)

    got = sample()
    want = np.concatenate(_parallel(lambda w, p, x, y: ref.subdiv_pixels(w, p.g, p.r, p.B, x, y),
                                    list(zip(ims, prms, px, py))))
    assert np.array_equal(got, want)
    eager = out.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ask.ask_dwell_batch(ctx, wins, pers, ptrs, torch.cuda.current_stream().cuda_stream)
    for rep in range(4):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        assert np.array_equal(sample(), want), rep
    del graph
    # one by one, both forms
    for form in ("persistent", "levels"):
        out.zero_()
        for wn, p, ptr in zip(wins, prms, ptrs):
            ask.ask_dwell_subdiv(ctx, wn, ask.params(p.g, p.r, p.B, form), ptr, s)
        ask.ask_synchronize(ctx, s)
        assert torch.equal(out, eager), form
    del out, eager


def test_served_requests_blocks(env, ref):
    """One second of the serving schedule through the server kernel: an
    8 x 8 block of every request against the oracle."""
    from paper_2206_02255_amd import serve
    ask, ctx, torch = env
    sched = workloads.serving_requests(seconds=1.0)
    rng = np.random.default_rng(55)
    blocks = [_blocks(rng, w.W, w.H, 1, 8) for _, w in sched]
    px = [b[0][0] for b in blocks]
    py = [b[1][0] for b in blocks]
    params_of = lambda w: workloads.batch_params(w.W)  # noqa: E731

    def probe(j, flat):
        w = sched[j][1]
        i = torch.as_tensor(py[j].astype(np.int64) * w.W + px[j], device="cuda")
        return flat[i].cpu().numpy().view(np.uint32)

    res = serve.serve(ctx, sched, params_of, slots=64, probe=probe)
    assert res["failed"] == 0 and len(res["probes"]) == len(sched)
    want = _parallel(lambda w, x, y: ref.subdiv_pixels(w, params_of(w).g, params_of(w).r,
                                                       params_of(w).B, x, y),
                     [(w, px[j], py[j]) for j, (_, w) in enumerate(sched)])
    for j in range(len(sched)):
        assert np.array_equal(res["probes"][j], want[j]), (j, sched[j][1])
