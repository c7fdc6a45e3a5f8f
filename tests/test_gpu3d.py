"""GPU parity of the 3-D extension: the exhaustive and the subdivision
volumes of quaternion Julia sets equal the 3-D oracle's bit for bit, with the
same per-level counts, for both curves, on ragged volumes, degenerate ones
(one voxel, one line, one slice, g above every side) and the benchmarked
512^3 volume; the z = 0 slice equals the library's own 2-D Julia image; a
render captured into a HIP graph gives the oracle's volume on every replay."""
import numpy as np
import pytest

from workloads import VOLUME, VOLUME_PARAMS, Volume, Window

pytestmark = pytest.mark.gpu

CURVES = ("canonical", "morton")

VOLUMES = [
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 40, 40, 40, 256, c=(-0.2, 0.6)), 4, 2, 4),
    (Volume(-1.5, 1.4, -1.3, 1.2, -0.9, 1.1, 37, 29, 23, 300, c=(-1.0, 0.0)), 3, 3, 2),
    (Volume(-0.8, 0.4, -0.2, 0.9, -0.5, 0.5, 26, 31, 19, 400, c=(-0.125, 0.65)), 5, 2, 3),
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 24, 24, 24, 128, c=(-0.2, 0.6)), 2, 4, 1),
    (Volume(-1.3, 1.1, -1.2, 1.2, -1.1, 1.3, 131, 97, 75, 256, c=(-0.2, 0.6)), 8, 2, 8),
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 128, 128, 128, 256, c=(-0.2, 0.6)), 16, 2, 8),
    (Volume(-0.1, 0.1, -0.1, 0.1, -0.1, 0.1, 1, 1, 1, 50, c=(-0.2, 0.6)), 4, 2, 1),
    (Volume(-1.6, 1.6, -0.01, 0.01, -0.01, 0.01, 57, 1, 1, 100, c=(-1.0, 0.0)), 3, 2, 2),
    (Volume(-1.6, 1.6, -1.2, 1.2, -0.01, 0.01, 90, 70, 1, 200, c=(-0.2, 0.6)), 4, 2, 4),
    (Volume(-1.0, 1.0, -1.0, 1.0, -1.0, 1.0, 3, 5, 2, 60, c=(-0.2, 0.6)), 8, 2, 1),
    # long orbits: many refill rounds per voxel, surfaces at D
    (Volume(-1.4, 1.4, -1.3, 1.3, -0.7, 0.7, 70, 66, 35, 3000, c=(-0.125, 0.65)), 4, 2, 5),
    # c beyond |c| = 2: every orbit escapes at once or never starts close
    (Volume(-2.5, 2.5, -2.5, 2.5, -2.5, 2.5, 33, 30, 27, 100, c=(2.1, 0.3)), 3, 2, 4),
    # boxes whose surface a whole workgroup scans: 32^3 boxes split into 16^3
    # leaf boxes; ragged 44 x 32 x 25 boxes and their leaf children; thin
    # 50 x 45 x 2 leaf boxes (all surface); |c| > 2 on 30^3 leaf boxes
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 96, 96, 96, 256, c=(-0.2, 0.6)), 3, 2, 16),
    (Volume(-1.3, 1.1, -1.2, 1.2, -1.1, 1.3, 131, 97, 75, 256, c=(-0.2, 0.6)), 3, 2, 24),
    (Volume(-1.5, 1.5, -1.5, 1.5, -0.02, 0.02, 100, 90, 2, 300, c=(-1.0, 0.0)), 2, 2, 64),
    (Volume(-2.5, 2.5, -2.5, 2.5, -2.5, 2.5, 60, 60, 60, 100, c=(2.1, 0.3)), 2, 2, 30),
    # dwell limits at or below the steps tested when a lane takes a voxel:
    # with D = 1 every dwell is 1 and every box is filled; D = 2 and 3 on
    # wave boxes and on workgroup boxes
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 30, 27, 25, 1, c=(-0.2, 0.6)), 3, 2, 4),
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 30, 27, 25, 2, c=(-0.2, 0.6)), 3, 2, 4),
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 96, 96, 96, 2, c=(-0.2, 0.6)), 3, 2, 16),
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 96, 96, 96, 3, c=(-0.2, 0.6)), 3, 2, 16),
]


@pytest.fixture(scope="module")
def lib3():
    import torch
    from paper_2206_02255_amd import ask
    assert torch.cuda.is_available()
    return ask, torch


@pytest.fixture(scope="module")
def ref3():
    from oracle import askref3
    askref3.lib()
    return askref3


def gpu_exhaustive(lib3, v):
    ask, torch = lib3
    out = torch.zeros(v.voxels, dtype=torch.int32, device="cuda")
    work = torch.empty(ask.EXHAUSTIVE3_WORK_BYTES, dtype=torch.uint8, device="cuda")
    ask.ask3_dwell_exhaustive(ask.volume(v), out.data_ptr(), work.data_ptr(),
                              stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out


def gpu_subdiv(lib3, v, g, r, B, curve, stats=True):
    ask, torch = lib3
    vol, prm = ask.volume(v), ask.params3(g, r, B, curve)
    nbytes = ask.ask3_workspace_bytes(vol, prm)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(v.voxels, dtype=torch.int32, device="cuda")
    st = ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(), nbytes,
                               torch.cuda.current_stream().cuda_stream, want_stats=stats)
    torch.cuda.synchronize()
    return out, st


def host(t, v):
    return t.cpu().numpy().view(np.uint32).reshape(v.L, v.H, v.W)


def test_exhaustive_volumes(lib3, ref3):
    for v, *_ in VOLUMES:
        print("exhaustive3", v, flush=True)
        assert np.array_equal(host(gpu_exhaustive(lib3, v), v), ref3.exhaustive(v)), v


@pytest.mark.parametrize("curve", CURVES)
def test_subdivision_volumes(lib3, ref3, curve):
    for v, g, r, B in VOLUMES:
        print("subdiv3", curve, v, (g, r, B), flush=True)
        out, st = gpu_subdiv(lib3, v, g, r, B, curve)
        want, rst = ref3.subdiv(v, g, r, B, curve)
        assert np.array_equal(host(out, v), want), (v, g, r, B)
        assert st["overflow"] == 0
        for k in ("levels", "regions", "fills", "splits", "leaves"):
            assert st[k] == rst[k], k


def test_zero_slice_equals_the_2d_julia_image(lib3):
    ask, torch = lib3
    v = Volume(-1.6, 1.5, -1.3, 1.4, -1.2, 1.2, 161, 147, 9, 300, c=(-0.2, 0.6))
    vol = host(gpu_exhaustive(lib3, v), v)
    w = Window(v.x0, v.x1, v.y0, v.y1, v.W, v.H, v.D, julia=v.c)
    ctx = ask.ask_create(0)
    try:
        img = torch.zeros(w.W * w.H, dtype=torch.int32, device="cuda")
        ask.ask_dwell_exhaustive(ctx, ask.window(w), img.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        ask.ask_destroy(ctx)
    assert np.array_equal(vol[4], img.cpu().numpy().view(np.uint32).reshape(w.H, w.W))


def test_repeated_renders_reuse_the_workspace(lib3, ref3):
    """Two renders in a row on one workspace, the second smaller: the control
    block is cleared on the stream, so nothing of the first leaks."""
    ask, torch = lib3
    s = torch.cuda.current_stream().cuda_stream
    big, small = VOLUMES[5], VOLUMES[1]
    vb, pb = ask.volume(big[0]), ask.params3(*big[1:])
    nbytes = ask.ask3_workspace_bytes(vb, pb)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for v, g, r, B in (big, small, big):
        out = torch.zeros(v.voxels, dtype=torch.int32, device="cuda")
        prm = ask.params3(g, r, B)
        assert ask.ask3_workspace_bytes(ask.volume(v), prm) <= nbytes
        st = ask.ask3_dwell_subdiv(ask.volume(v), prm, out.data_ptr(), work.data_ptr(), nbytes, s,
                                   want_stats=True)
        want, rst = ref3.subdiv(v, g, r, B)
        assert np.array_equal(host(out, v), want)
        assert st["regions"] == rst["regions"]


def test_rejects_small_workspace(lib3):
    ask, torch = lib3
    v, g, r, B = VOLUMES[0]
    vol, prm = ask.volume(v), ask.params3(g, r, B)
    nbytes = ask.ask3_workspace_bytes(vol, prm)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(v.voxels, dtype=torch.int32, device="cuda")
    with pytest.raises(ask.AskError):
        ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(), nbytes - 8)


def test_benchmarked_volume(lib3, ref3):
    """The 512^3 volume in the benchmarked parameters: the subdivision volume
    and its counts equal the oracle's in full, and the exhaustive volume on
    sampled voxels."""
    v, p = VOLUME, VOLUME_PARAMS
    print("subdiv3 512^3", flush=True)
    out, st = gpu_subdiv(lib3, v, p.g, p.r, p.B, "morton")
    want, rst = ref3.subdiv(v, p.g, p.r, p.B, "morton")
    assert np.array_equal(host(out, v), want)
    for k in ("levels", "regions", "fills", "splits", "leaves"):
        assert st[k] == rst[k], k
    del out
    print("exhaustive3 512^3", flush=True)
    ex = host(gpu_exhaustive(lib3, v), v)
    rng = np.random.default_rng(3)
    for x, y, z in zip(rng.integers(0, v.W, 2000), rng.integers(0, v.H, 2000),
                       rng.integers(0, v.L, 2000)):
        assert ex[z, y, x] == ref3.voxel_dwell(v, x, y, z)


@pytest.mark.parametrize("curve", CURVES)
def test_graph_replays_equal_the_oracle(lib3, ref3, curve):
    """The render allocates nothing, waits for nothing and clears its control
    block with a kernel, so it captures into a HIP graph: every replay, with
    an eager render on another workspace in between, gives the oracle's
    volume."""
    ask, torch = lib3
    v, g, r, B = VOLUMES[4]
    o, og, orr, oB = VOLUMES[1]
    vol, prm = ask.volume(v), ask.params3(g, r, B, curve)
    nb = ask.ask3_workspace_bytes(vol, prm)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out = torch.zeros(v.voxels, dtype=torch.int32, device="cuda")
    want = ref3.subdiv(v, g, r, B, curve)[0]
    want2 = ref3.subdiv(o, og, orr, oB, curve)[0]
    s = torch.cuda.current_stream()
    ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(), nb, s.cuda_stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(), nb,
                              torch.cuda.current_stream().cuda_stream)
    for rep in range(4):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out, v), want), rep
        out2, _ = gpu_subdiv(lib3, o, og, orr, oB, curve, stats=False)
        assert np.array_equal(host(out2, o), want2), rep
    del graph
