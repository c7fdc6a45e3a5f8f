"""GPU parity of batched rendering: many images of different sizes, windows,
dwell limits and parameters in one launch sequence over one region queue.
Each image must equal the oracle's subdivision image and the image the same
window gives when rendered alone, bit for bit."""
import numpy as np
import pytest

from workloads import Window, paper_window, random_params, random_windows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    from paper_2206_02255_amd import ask
    ctx = ask.ask_create(0)
    yield ask, ctx, torch
    ask.ask_destroy(ctx)


def batch(gpu, ws, ps, form, stats=False):
    ask, ctx, torch = gpu
    outs = [torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda") for w in ws]
    prms = [ask.params(p.g, p.r, p.B, form) for p in ps]
    st = ask.ask_dwell_batch(ctx, [ask.window(w) for w in ws], prms if len(prms) > 1 else prms[0],
                             [o.data_ptr() for o in outs], torch.cuda.current_stream().cuda_stream,
                             want_stats=stats)
    torch.cuda.synchronize()
    return [o.cpu().numpy().view(np.uint32).reshape(w.H, w.W) for o, w in zip(outs, ws)], st


def alone(gpu, w, p, form):
    ask, ctx, torch = gpu
    out = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
    ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(p.g, p.r, p.B, form), out.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32).reshape(w.H, w.W)


@pytest.mark.parametrize("form", ["levels", "persistent"])
def test_batch_of_random_windows(gpu, ref, form):
    ws = random_windows(61, 40, max_side=180, max_dwell=2500)
    ps = [random_params(400 + i, w, 1)[0] for i, w in enumerate(ws)]
    print(form, len(ws), "images", flush=True)
    imgs, st = batch(gpu, ws, ps, form, stats=True)
    it_ring = it_filled = it_leaf = it_inner = 0
    for w, p, img in zip(ws, ps, imgs):
        want, rst = ref.subdiv(w, p.g, p.r, p.B)
        assert np.array_equal(img, want), (w, p)
        assert np.array_equal(img, alone(gpu, w, p, form)), (w, p)
        it_ring += rst["iters_ring"]
        it_filled += rst["iters_ring_filled"]
        it_leaf += rst["iters_leaf"]
        it_inner += rst["iters_leaf_inner"]
    assert it_filled <= st["iters_ring"] <= it_ring
    assert it_inner <= st["iters_leaf"] <= it_leaf
    assert st["overflow"] == 0


def test_batch_shared_parameters_and_sizes(gpu, ref):
    from workloads import Params
    ws = [paper_window(n, d) for n, d in [(512, 256), (777, 1024), (1024, 512), (300, 4096)]]
    ws.append(Window(-0.7452, -0.7448, 0.1101, 0.1105, 640, 480, 2000))
    p = Params(8, 2, 16)
    for form in ("levels", "persistent"):
        imgs, _ = batch(gpu, ws, [p], form)
        for w, img in zip(ws, imgs):
            assert np.array_equal(img, ref.subdiv(w, p.g, p.r, p.B)[0]), (form, w)


def test_repeated_batches_of_different_lengths(gpu, ref):
    ws = random_windows(62, 12, max_side=100, max_dwell=500)
    ps = [random_params(500 + i, w, 1)[0] for i, w in enumerate(ws)]
    want = [ref.subdiv(w, p.g, p.r, p.B)[0] for w, p in zip(ws, ps)]
    for rep in range(4):
        k = 3 + 3 * rep  # batches of different lengths, back to back
        imgs, _ = batch(gpu, ws[:k], ps[:k], "persistent")
        for img, wt in zip(imgs, want[:k]):
            assert np.array_equal(img, wt)


def test_batch_argument_errors(gpu):
    ask, ctx, torch = gpu
    w = paper_window(64, 100)
    out = torch.zeros(64 * 64, dtype=torch.int32, device="cuda")
    mixed = [ask.params(4, 2, 8, "levels"), ask.params(4, 2, 8, "persistent")]
    with pytest.raises(ask.AskError) as e:
        ask.ask_dwell_batch(ctx, [ask.window(w)] * 2, mixed, [out.data_ptr()] * 2)
    assert e.value.status == ask.EINVAL
    with pytest.raises(ask.AskError) as e:
        ask.ask_dwell_batch(ctx, [ask.window(w)], ask.params(65, 2, 8), [out.data_ptr()])
    assert e.value.status == ask.EINVAL
