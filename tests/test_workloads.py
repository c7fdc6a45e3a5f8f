"""The seeded workloads: the boundary pool holds what its generator states,
and the deep-zoom, batched and serving workloads have the stated shapes."""
import math

import numpy as np

import workloads as W


def test_boundary_pool_points_have_the_stated_dwell(ref):
    pool = W.boundary_pool()
    assert len(pool) == 1024 and len(set(pool)) == 1024
    for x, y in pool[::8]:
        assert -2.0 <= x <= 0.5 and -1.25 <= y <= 1.25
        assert 4096 <= ref.dwell(x, y, 8192) <= 8110


def test_pool_regenerates_to_the_stored_file():
    from oracle import make_boundary_pool as mk
    assert mk.make(count=16, workers=2) == W.boundary_pool()[:16]


def test_deep_window():
    w = W.deep_window()
    assert (w.W, w.H, w.D) == (32768, 32768, 8192)
    assert math.isclose(w.x1 - w.x0, 1e-6, rel_tol=1e-9)
    assert math.isclose(w.y1 - w.y0, 1e-6, rel_tol=1e-9)
    c = (0.5 * (w.x0 + w.x1), 0.5 * (w.y0 + w.y1))
    assert min(math.hypot(c[0] - x, c[1] - y) for x, y in W.boundary_pool()) < 1e-12
    assert W.deep_window() == w


def test_batch_images_shape():
    ims = W.batch_images()
    assert len(ims) == 256 and ims == W.batch_images()
    sides = np.array([w.W for w in ims])
    assert all(w.W == w.H for w in ims)
    assert sides.min() >= 512 and sides.max() < 8192
    assert {w.D for w in ims} == set(W.BATCH_DWELLS)
    widths = np.array([w.x1 - w.x0 for w in ims])
    assert widths.min() >= 1e-10 * (1 - 1e-9) and widths.max() <= 2.0
    # log-uniform sides: the median near the geometric mean of the range
    assert 1500 < np.median(sides) < 3000
    assert 2.0e9 < sides.astype(np.float64).__pow__(2).sum() < 4.0e9


def test_serving_requests_shape():
    reqs = W.serving_requests()
    times = np.array([t for t, _ in reqs])
    assert np.all(np.diff(times) > 0) and times[-1] < 60.0
    assert 11000 < len(reqs) < 13000  # 200 per second for 60 s
    gaps = np.diff(times)
    assert abs(gaps.mean() - 1 / 200) < 0.1 / 200
    assert W.serving_requests(seconds=1.0) == reqs[:len(W.serving_requests(seconds=1.0))]


def test_batch_params():
    assert W.batch_params(512) == W.Params(2, 2, 128)
    assert W.batch_params(8191) == W.Params(31, 2, 128)
    assert W.batch_params(300) == W.Params(1, 2, 128)


def test_batch_params_levels():
    assert W.batch_params_levels(512) == W.Params(2, 2, 32)
    assert W.batch_params_levels(8191) == W.Params(31, 2, 32)
    assert W.batch_params_levels(300).B == 32
