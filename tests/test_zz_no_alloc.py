"""The allocation-free subdivision entry point (ask_dwell_subdiv_noalloc):
called through the C ABI twice in a row, the second time with a smaller
image, each image equal bit for bit to the one ask_dwell_subdiv gives for the
same window and parameters, and to the oracle's; sizes beyond its fixed
device array are refused."""
import numpy as np
import pytest

from workloads import Window, paper_window

pytestmark = pytest.mark.gpu


def _img(torch, t, w):
    torch.cuda.current_stream().synchronize()
    return t.cpu().numpy().view(np.uint32).reshape(w.H, w.W)


@pytest.mark.parametrize("form", ["persistent", "levels"])
def test_noalloc_equals_the_context_render(ref, form):
    import torch
    from paper_2206_02255_amd import ask
    s = torch.cuda.current_stream().cuda_stream
    ctx = ask.ask_create(0)
    try:
        cases = [(paper_window(1024, 512), (4, 2, 32)),
                 (Window(-0.7454, -0.7446, 0.1126, 0.1134, 333, 250, 1500), (3, 3, 16))]
        for w, (g, r, B) in cases:
            print(form, w, (g, r, B), flush=True)
            prm = ask.params(g, r, B, form)
            a = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
            b = torch.full((w.W * w.H,), -1, dtype=torch.int32, device="cuda")
            ask.ask_dwell_subdiv(ctx, ask.window(w), prm, a.data_ptr(), s)
            ask.ask_synchronize(ctx, s)
            ask.ask_dwell_subdiv_noalloc(ask.window(w), prm, b.data_ptr(), s)
            want = _img(torch, a, w)
            assert np.array_equal(_img(torch, b, w), want), (form, w)
            assert np.array_equal(want, ref.subdiv(w, g, r, B)[0])
    finally:
        ask.ask_destroy(ctx)


def test_noalloc_refuses_what_does_not_fit():
    import torch
    from paper_2206_02255_amd import ask
    out = torch.zeros(16, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    # 65536^2 with tiny leaves: its worst-case queue is far beyond the array
    big = ask.window(paper_window(65536, 100))
    for form in ("persistent", "levels"):
        with pytest.raises(ask.AskError) as e:
            ask.ask_dwell_subdiv_noalloc(big, ask.params(1024, 2, 1, form), out.data_ptr(), s)
        assert e.value.status == ask.EINVAL
    with pytest.raises(ask.AskError) as e:
        ask.ask_dwell_subdiv_noalloc(ask.window(paper_window(64, 100)),
                                     ask.params(4, 2, 8, "levels_readback"), out.data_ptr(), s)
    assert e.value.status == ask.EINVAL
