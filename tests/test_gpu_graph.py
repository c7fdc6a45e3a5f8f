"""Renders captured into HIP graphs (stream capture through torch.cuda.graph):
every replay gives the eager image, with eager renders and clears in
between; capture refuses what it cannot replay."""
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
    want = _img(torch, out, w)
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
        lambda st: ask.ask_dwell_batch(ctx, [ask.window(w)] * 2, ask.params(4, 2, 16, "persistent"),
                                       [out.data_ptr(), out.data_ptr()], st),
    ]
    for call in bad:
        g = torch.cuda.CUDAGraph()
        with pytest.raises(ask.AskError):
            with torch.cuda.graph(g):
                call(torch.cuda.current_stream().cuda_stream)
        del g
