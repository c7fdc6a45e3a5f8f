"""Renders captured into HIP graphs (stream capture through torch.cuda.graph):
every replay gives the oracle's image, with eager renders and clears in
between, for single images and for batches; capture refuses what it cannot
replay."""
import numpy as np
import pytest

from workloads import Window, paper_window

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2206_02255_amd import ask
    assert torch.cuda.is_available()
    ctx = ask.ask_create(0)
    yield ask, ctx, torch
    ask.ask_destroy(ctx)


def _img(torch, t, w):
    torch.cuda.current_stream().synchronize()
    return t.cpu().numpy().view(np.uint32).reshape(w.H, w.W)


@pytest.mark.parametrize("form", ["levels", "persistent"])
def test_replays_equal_the_eager_render(env, ref, form):
    ask, ctx, torch = env
    w = paper_window(2048, 1024)
    other = Window(-0.7454, -0.7446, 0.1126, 0.1134, 640, 480, 1200)
    prm = ask.params(16, 2, 32, form)
    out = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
    out2 = torch.zeros(other.W * other.H, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    ask.ask_dwell_subdiv(ctx, ask.window(w), prm, out.data_ptr(), s.cuda_stream)  # sizes the queues
    ask.ask_synchronize(ctx, s.cuda_stream)
    want = ref.subdiv(w, 16, 2, 32)[0]
    assert np.array_equal(_img(torch, out, w), want)
    want2 = ref.subdiv(other, 4, 2, 16)[0]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ask.ask_dwell_subdiv(ctx, ask.window(w), prm, out.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    for rep in range(4):
        out.zero_()
        g.replay()
        assert np.array_equal(_img(torch, out, w), want), rep
        # eager work of the same context between replays
        ask.ask_dwell_subdiv(ctx, ask.window(other), ask.params(4, 2, 16, form), out2.data_ptr(),
                             s.cuda_stream)
        ask.ask_synchronize(ctx, s.cuda_stream)
        assert np.array_equal(_img(torch, out2, other), want2), rep
    del g


def test_capture_refuses_what_it_cannot_replay(env):
    ask, ctx, torch = env
    w = paper_window(256, 128)
    out = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(4, 2, 16, "persistent"), out.data_ptr(),
                         s.cuda_stream)
    ask.ask_synchronize(ctx, s.cuda_stream)
    bad = [
        lambda st: ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(4, 2, 16, "persistent"),
                                        out.data_ptr(), st, want_stats=True),
        lambda st: ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(4, 2, 16, "levels_readback"),
                                        out.data_ptr(), st),
    ]
    for call in bad:
        g = torch.cuda.CUDAGraph()
        with pytest.raises(ask.AskError):
            with torch.cuda.graph(g):
                call(torch.cuda.current_stream().cuda_stream)
        del g


@pytest.mark.parametrize("form", ["levels", "persistent"])
def test_batch_replays_equal_the_oracle(env, ref, form):
    """A batch captured whole (its image table written by kernels of the
    graph): every replay gives the oracle's images, with eager batches of
    other images on the same context between the replays."""
    from workloads import random_params, random_windows
    ask, ctx, torch = env
    ws = random_windows(71, 10, max_side=300, max_dwell=1500) + [paper_window(700, 600)]
    ps = [random_params(700 + i, w, 1)[0] for i, w in enumerate(ws)]
    others = random_windows(72, 7, max_side=200, max_dwell=900)
    ops = [random_params(800 + i, w, 1)[0] for i, w in enumerate(others)]
    want = [ref.subdiv(w, p.g, p.r, p.B)[0] for w, p in zip(ws, ps)]
    want_o = [ref.subdiv(w, p.g, p.r, p.B)[0] for w, p in zip(others, ops)]
    outs = [torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda") for w in ws]
    outs_o = [torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda") for w in others]
    wins = [ask.window(w) for w in ws]
    prms = [ask.params(p.g, p.r, p.B, form) for p in ps]
    wins_o = [ask.window(w) for w in others]
    prms_o = [ask.params(p.g, p.r, p.B, form) for p in ops]
    s = torch.cuda.current_stream()
    ask.ask_dwell_batch(ctx, wins, prms, [o.data_ptr() for o in outs], s.cuda_stream)
    ask.ask_synchronize(ctx, s.cuda_stream)  # the queues are sized outside the capture
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ask.ask_dwell_batch(ctx, wins, prms, [o.data_ptr() for o in outs],
                            torch.cuda.current_stream().cuda_stream)
    for rep in range(4):
        for o in outs:
            o.zero_()
        g.replay()
        for o, w, wt in zip(outs, ws, want):
            assert np.array_equal(_img(torch, o, w), wt), (rep, w)
        ask.ask_dwell_batch(ctx, wins_o, prms_o, [o.data_ptr() for o in outs_o], s.cuda_stream)
        ask.ask_synchronize(ctx, s.cuda_stream)
        for o, w, wt in zip(outs_o, others, want_o):
            assert np.array_equal(_img(torch, o, w), wt), (rep, w)
    del g
