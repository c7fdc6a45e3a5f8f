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


def test_guided_search_finds_the_optimum_with_few_renders():
    # Synthetic measurements from the model with overheads (known lambda,
    # sigma, kappa and a split probability that grows with the region side):
    # the prior, fitted on 8 pilot renders, must lead to the grid's optimum
    # with at most 16 renders of the 60 and recover lambda and sigma.
    n, A, q = 16384, 2048.0, 256
    curve = lambda s: min(0.95, 0.1 + 0.15 * np.log2(s / 8.0))  # noqa: E731
    lam, sig, kappa = 10.0, 1000.0, 2e-7
    grid = [(g, r, B) for g in (2, 4, 8, 16, 32) for r in (2, 4, 8) for B in (16, 32, 64, 128)]

    def measure(ps):
        rows = []
        for g, r, B in ps:
            L = costmodel.rendered_levels(n, g, r, B)
            sides = costmodel.level_sides(n, g, r, B, L)
            Pl = [curve(s) for s in sides[:-1]] or [0.0]
            ms = kappa * costmodel.time_sbr_levels(n, g, r, B, A, Pl, lam, q, 64, sig, L)
            rows.append({"g": g, "r": r, "B": B, "ms": ms, "P_levels": Pl})
        return rows

    truth = min(measure(grid), key=lambda row: row["ms"])
    res = autotune.guided_search(measure, grid, n, A, q, pilot=8, top=8)
    assert res["measured"] <= 16
    assert (res["best"]["g"], res["best"]["r"], res["best"]["B"]) == (truth["g"], truth["r"], truth["B"])
    assert res["fit"]["lambda"] == pytest.approx(lam, rel=0.5)
    assert res["fit"]["sigma"] == pytest.approx(sig, rel=0.7)
    assert res["fit"]["log_rms"] < 0.05
