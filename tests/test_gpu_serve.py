"""Serving on the GPU: requests posted to a running server kernel give the
images they give alone, bit for bit, while they overlap with each other on
the device; admission by slots and pool memory; the kernel's idle exit and
relaunch; destroy with requests in flight.

While a server kernel runs, these tests wait on single streams only (a
device-wide synchronisation would wait for the server kernel itself).
"""
import time

import numpy as np
import pytest

from workloads import Window, paper_window, random_windows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2206_02255_amd import ask
    assert torch.cuda.is_available()
    ctx = ask.ask_create(0)
    ask.ask_set_wait_limit(ctx, 5.0)
    yield ask, ctx, torch
    ask.ask_destroy(ctx)


def _alone(env, w, g, r, B):
    ask, ctx, torch = env
    out = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(g, r, B, "persistent"), out.data_ptr(),
                         s.cuda_stream)
    ask.ask_synchronize(ctx, s.cuda_stream)
    return out.cpu().numpy().view(np.uint32).reshape(w.H, w.W)


def _host(t, w):
    return t.cpu().numpy().view(np.uint32).reshape(w.H, w.W)


def _wait(ask, sv, tickets, limit=60.0):
    """Reap until every ticket has finished; returns {ticket: status} and the
    largest number of requests seen in flight at once."""
    got, peak = {}, 0
    t0 = time.time()
    while len(got) < len(tickets):
        assert time.time() - t0 < limit, "requests did not finish"
        peak = max(peak, ask.ask_server_in_flight(sv))
        for t, st in ask.ask_server_reap(sv):
            got[t] = st
        time.sleep(0.0005)
    return got, peak


def _requests():
    # Sizes and depths spread like a serving mix (a large deep image first,
    # so that the smaller ones arrive while it runs), plus ragged windows.
    reqs = [(paper_window(4096, 4096), 16, 2, 32),
            (Window(-0.7454, -0.7446, 0.1126, 0.1134, 1000, 700, 1500), 8, 2, 16),
            (paper_window(1024, 512), 4, 2, 32),
            (Window(-1.5, 0.5, -1.0, 1.0, 517, 333, 300), 4, 3, 16),
            (Window(-0.2, 0.1, -0.15, 0.15, 300, 260, 200), 2, 2, 16)]
    for i, w in enumerate(random_windows(77, 10, max_side=200, max_dwell=800)):
        lim = min(w.W, w.H)
        reqs.append((w, max(1, min(lim, 1 + i % 4)), 2 + i % 3, 1 + (7 * i) % 33))
    return reqs


def test_results_equal_alone_and_in_the_mix(env, ref):
    ask, ctx, torch = env
    reqs = _requests()
    alone = [_alone(env, w, g, r, B) for w, g, r, B in reqs]
    for (w, g, r, B), img in list(zip(reqs, alone))[2:]:  # the alone path against the oracle
        assert np.array_equal(img, ref.subdiv(w, g, r, B)[0])
    sv = ask.ask_server_create(ctx, slots=8)
    try:
        outs = [torch.full((w.W * w.H,), -1, dtype=torch.int32, device="cuda") for w, *_ in reqs]
        torch.cuda.current_stream().synchronize()
        tickets, order, peak = {}, list(range(len(reqs))), 0
        t0 = time.time()
        while order:  # post as slots free up
            assert time.time() - t0 < 60
            i = order[0]
            w, g, r, B = reqs[i]
            t = ask.ask_server_submit(sv, ask.window(w), ask.params(g, r, B), outs[i].data_ptr())
            peak = max(peak, ask.ask_server_in_flight(sv))
            if t is None:
                time.sleep(0.0005)
                continue
            tickets[t] = i
            order.pop(0)
        got, peak2 = _wait(ask, sv, list(tickets))
        assert all(st == 0 for st in got.values())
        assert max(peak, peak2) >= 2  # requests were on the device together
        for t, i in tickets.items():
            w = reqs[i][0]
            assert np.array_equal(_host(outs[i], w), alone[i]), i
            done, st, lat = ask.ask_server_poll(sv, t)
            assert done and st == 0
            assert lat is not None and 0.0 <= lat < 60.0
    finally:
        ask.ask_server_destroy(sv)


def test_busy_when_slots_are_taken_then_admitted(env):
    ask, ctx, torch = env
    w = paper_window(4096, 4096)  # tens of milliseconds each
    alone = _alone(env, w, 8, 2, 32)
    sv = ask.ask_server_create(ctx, slots=2)
    try:
        outs = [torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda") for _ in range(4)]
        torch.cuda.current_stream().synchronize()
        prm = ask.params(8, 2, 32)
        t1 = ask.ask_server_submit(sv, ask.window(w), prm, outs[0].data_ptr())
        t2 = ask.ask_server_submit(sv, ask.window(w), prm, outs[1].data_ptr())
        assert t1 is not None and t2 is not None
        if ask.ask_server_in_flight(sv) == 2:
            assert ask.ask_server_submit(sv, ask.window(w), prm, outs[2].data_ptr()) is None
        tickets = [t1, t2]
        for k in (2, 3):
            t0 = time.time()
            while True:
                t = ask.ask_server_submit(sv, ask.window(w), prm, outs[k].data_ptr())
                if t is not None:
                    break
                assert time.time() - t0 < 30
                time.sleep(0.0005)
            tickets.append(t)
        got, _ = _wait(ask, sv, tickets)
        assert sorted(got) == sorted(tickets) and all(st == 0 for st in got.values())
        for o in outs:
            assert np.array_equal(_host(o, w), alone)
    finally:
        ask.ask_server_destroy(sv)


def test_admission_by_pool_memory(env):
    ask, ctx, torch = env
    sv = ask.ask_server_create(ctx, slots=8, pool_bytes=2 << 20)
    try:
        big = paper_window(16384, 64)
        out = torch.zeros(64, dtype=torch.int32, device="cuda")
        with pytest.raises(ask.AskError) as e:  # its worst case exceeds the whole pool
            ask.ask_server_submit(sv, ask.window(big), ask.params(64, 2, 4), out.data_ptr())
        assert e.value.status == ask.ENOMEM
        # A request whose worst case takes most of the 2 MiB pool (about
        # 100k queue entries of the 114k): a second one waits for its memory,
        # not for a slot.
        w = paper_window(5000, 8192)
        prm = ask.params(8, 2, 64)
        outs = [torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda") for _ in range(2)]
        torch.cuda.current_stream().synchronize()
        t1 = ask.ask_server_submit(sv, ask.window(w), prm, outs[0].data_ptr())
        assert t1 is not None
        t2 = ask.ask_server_submit(sv, ask.window(w), prm, outs[1].data_ptr())
        if t2 is None:
            _wait(ask, sv, [t1])
            t2 = ask.ask_server_submit(sv, ask.window(w), prm, outs[1].data_ptr())
            assert t2 is not None
            _wait(ask, sv, [t2])
        else:  # only if the first had already finished
            assert ask.ask_server_poll(sv, t1)[0]
            _wait(ask, sv, [t2])
        assert np.array_equal(_host(outs[0], w), _host(outs[1], w))
    finally:
        ask.ask_server_destroy(sv)


def test_idle_exit_and_relaunch(env, ref):
    ask, ctx, torch = env
    ask.ask_set_wait_limit(ctx, 1.0)  # the kernel leaves after 1 s with nothing to do
    sv = ask.ask_server_create(ctx, slots=2)
    try:
        w = Window(-1.5, 0.5, -1.0, 1.0, 300, 200, 400)
        want = ref.subdiv(w, 4, 2, 16)[0]
        for rep in range(3):
            out = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
            torch.cuda.current_stream().synchronize()
            t = ask.ask_server_submit(sv, ask.window(w), ask.params(4, 2, 16), out.data_ptr())
            _wait(ask, sv, [t], limit=30)
            assert np.array_equal(_host(out, w), want), rep
            time.sleep(1.6)
    finally:
        ask.ask_server_destroy(sv)
        ask.ask_set_wait_limit(ctx, 5.0)


def test_destroy_waits_for_requests_in_flight(env):
    ask, ctx, torch = env
    w = paper_window(2048, 1024)
    alone = _alone(env, w, 16, 2, 32)
    sv = ask.ask_server_create(ctx, slots=4)
    out = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
    torch.cuda.current_stream().synchronize()
    t = ask.ask_server_submit(sv, ask.window(w), ask.params(16, 2, 32), out.data_ptr())
    assert t is not None
    ask.ask_server_destroy(sv)
    assert np.array_equal(_host(out, w), alone)


def test_other_kernels_run_beside_the_server(env):
    ask, ctx, torch = env
    sv = ask.ask_server_create(ctx, slots=2)
    try:
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
        y = (x * 2.0 + 1.0).sum()
        torch.cuda.current_stream().synchronize()
        assert float(y) == pytest.approx(float(1 << 40), rel=1e-4)
    finally:
        ask.ask_server_destroy(sv)


def test_server_argument_errors(env):
    ask, ctx, torch = env
    for slots, waves in [(0, 0), (65, 0), (4, 3)]:
        with pytest.raises(ask.AskError):
            ask.ask_server_create(ctx, slots=slots, waves_per_cu=waves)
    sv = ask.ask_server_create(ctx, slots=1)
    try:
        with pytest.raises(ask.AskError):  # one server per context
            ask.ask_server_create(ctx, slots=1)
        w = paper_window(64, 64)
        with pytest.raises(ask.AskError):
            ask.ask_server_submit(sv, ask.window(w), ask.params(0, 2, 4), 0)
        with pytest.raises(ask.AskError):
            ask.ask_server_poll(sv, 12345)
    finally:
        ask.ask_server_destroy(sv)
