"""Host logic of the autotuner (CPU), and one small sweep on the GPU."""
import numpy as np
import pytest

from paper_2206_02255_amd import autotune, costmodel
from workloads import paper_window


def synthetic_rows(lam, kappa, P, n=4096, A=1024.0, q=256):
    rows = []
    for g, r, B in autotune.default_grid(n):
        ms = kappa * float(costmodel.time_sbr(n, g, r, B, A, P, lam, q, 64))
        rows.append({"g": g, "r": r, "B": B, "ms": ms, "P": P})
    return rows


@pytest.mark.parametrize("lam", [1.0, 100.0, 10000.0])
def test_fit_recovers_the_model_parameters(lam):
    rows = synthetic_rows(lam, 3e-7, 0.6)
    fl, kappa, P, err = autotune.fit_model(rows, 4096, 1024.0, 256, lambdas=[0.1, 1.0, 100.0, 10000.0])
    assert fl == lam and P == 0.6 and err < 1e-9
    assert kappa == pytest.approx(3e-7, rel=1e-9)


def test_model_optimum_is_the_argmin():
    grid = autotune.default_grid(16384)
    (g, r, B), t = autotune.model_optimum(grid, 16384, 2048.0, 0.5, 10.0, 256)
    ts = [float(costmodel.time_sbr(16384, *p, 2048.0, 0.5, 10.0, 256, 64)) for p in grid]
    assert t == min(ts) and (g, r, B) in grid


def test_default_grid_keeps_a_split_level():
    for g, r, B in autotune.default_grid(1024):
        assert 1024 // g > B


def test_workload_key_classes():
    from paper_2206_02255_amd import ask
    k = autotune.workload_key(ask.window(paper_window(1024, 512)), "persistent")
    assert k == "1024x1024-D512-w1e0-persistent"


@pytest.mark.gpu
def test_small_sweep_on_gpu(tmp_path, monkeypatch):
    from paper_2206_02255_amd import ask
    monkeypatch.setenv("ASK_TUNE_CACHE", str(tmp_path / "tune.json"))
    ctx = ask.ask_create(0)
    try:
        grid = [(4, 2, 32), (16, 2, 16), (32, 4, 16), (64, 2, 16)]
        res = autotune.tune(ctx, ask.window(paper_window(1024, 512)), grid, reps=2)
        assert (res["measured_optimum"]["g"], res["measured_optimum"]["r"],
                res["measured_optimum"]["B"]) in grid
        assert len(res["rows"]) == 4 and all(row["ms"] > 0 for row in res["rows"])
        again = autotune.tune(ctx, ask.window(paper_window(1024, 512)), grid)
        assert again["measured_optimum"] == res["measured_optimum"]  # from the cache
    finally:
        ask.ask_destroy(ctx)
