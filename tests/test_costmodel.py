"""The cost model (Sec. 4): its oracle pinned by facts that hold independently
of either implementation, and the product evaluator against the oracle."""
import math

import numpy as np
import pytest

from oracle import costmodel_ref as ref
from paper_2206_02255_amd import costmodel as cm

GRID = [(n, g, r, B) for n in (1024, 4096, 16384) for g in (2, 4, 16, 64)
        for r in (2, 4, 8) for B in (8, 16, 32, 128) if n / (g * B) >= r]


@pytest.mark.parametrize("n,g,r,B", GRID[::7])
def test_no_split_costs_one_query_per_region_and_the_fills(n, g, r, B):
    # P = 0: only level 0 is paid, its G queries of 4nA/g and the fill of
    # every pixel: W = 4 g n A + n^2 (and nothing at the last level once
    # tau >= 2).
    A = 512.0
    if ref.tau(n, g, r, B) >= 2:
        assert ref.work_subdivision(n, g, r, B, A, 0.0, 7.0) == pytest.approx(4 * g * n * A + n * n)


@pytest.mark.parametrize("n,g,r,B", GRID[::5])
@pytest.mark.parametrize("P", [0.0, 0.3, 0.7, 1.0])
def test_reduction_factor_never_exceeds_the_work_per_element(n, g, r, B, P):
    # Fills write every pixel of a level that stops and the last level works
    # on every pixel that reaches it, so W >= n^2 and Omega <= A (Sec. 4.2.2).
    for A in (1.0, 64.0, 2048.0):
        assert ref.reduction_factor(n, g, r, B, A, P, 10.0) <= A * (1 + 1e-12)


@pytest.mark.parametrize("n,g,r,B", GRID[::5])
def test_always_splitting_costs_more_than_exhaustive(n, g, r, B):
    # P = 1: every level is paid in full and the last level still works on
    # every pixel, so Omega < 1 as soon as there is a level to pay (tau >= 2;
    # with tau = 1 the model is the exhaustive work and Omega = 1).
    om = ref.reduction_factor(n, g, r, B, 512.0, 1.0, 1.0)
    if ref.tau(n, g, r, B) >= 2:
        assert om < 1.0
    else:
        assert om == 1.0


@pytest.mark.parametrize("n,g,r,B", GRID[::6])
@pytest.mark.parametrize("P", [0.0, 0.25, 0.5, 1.0])
def test_one_core_times_equal_the_work(n, g, r, B, P):
    # With q = c = 1 every ceiling is of an integer (for these dyadic
    # parameters) and both schemes reduce to the total work W_SSD^M.
    A, lam = 128.0, 3.0
    w = ref.work_subdivision(n, g, r, B, A, P, lam)
    assert ref.time_sbr(n, g, r, B, A, P, lam, 1, 1) == pytest.approx(w, rel=1e-12)
    assert ref.time_mbr(n, g, r, B, A, P, lam, 1, 1) == pytest.approx(w, rel=1e-12)
    assert ref.time_exhaustive(n, A, 1, 1) == ref.work_exhaustive(n, A)


def test_depth_is_log_r_of_n_over_gB():
    assert ref.tau(16384, 64, 2, 32) == 3
    assert ref.tau(1024, 4, 2, 32) == 3
    assert ref.tau(4096, 2, 4, 16) == 4
    assert ref.tau(64, 32, 2, 16) == 1   # never below one level


def test_per_level_probabilities_reduce_to_one_probability():
    n, g, r, B, A = 4096, 4, 2, 16, 512.0
    t = ref.tau(n, g, r, B)
    assert ref.work_subdivision(n, g, r, B, A, [0.4] * t, 2.0) == \
        ref.work_subdivision(n, g, r, B, A, 0.4, 2.0)


@pytest.mark.parametrize("P", [0.0, 0.2, 0.5, 0.9, 1.0])
@pytest.mark.parametrize("lam", [0.0, 1.0, 100.0])
def test_product_model_equals_oracle(P, lam):
    A, q, c = 2048.0, 256, 64
    for n, g, r, B in GRID:
        w = ref.work_subdivision(n, g, r, B, A, P, lam)
        assert cm.work_subdivision(n, g, r, B, A, P, lam) == pytest.approx(w, rel=1e-12)
        assert cm.time_sbr(n, g, r, B, A, P, lam, q, c) == pytest.approx(
            ref.time_sbr(n, g, r, B, A, P, lam, q, c), rel=1e-12)
        assert cm.time_mbr(n, g, r, B, A, P, lam, q, c) == pytest.approx(
            ref.time_mbr(n, g, r, B, A, P, lam, q, c), rel=1e-12)
        assert int(cm.tau(n, g, r, B)) == ref.tau(n, g, r, B)


def test_product_model_broadcasts_over_grids():
    gs = np.array([2, 4, 8, 16, 32])[:, None, None]
    rs = np.array([2, 4, 8])[None, :, None]
    Bs = np.array([16, 32, 64, 128])[None, None, :]
    t = cm.time_sbr(16384, gs, rs, Bs, 2048.0, 0.5, 10.0, 256, 64)
    assert t.shape == (5, 3, 4)
    for i, g in enumerate((2, 4, 8, 16, 32)):
        for j, r in enumerate((2, 4, 8)):
            for k, B in enumerate((16, 32, 64, 128)):
                assert t[i, j, k] == pytest.approx(
                    ref.time_sbr(16384, g, r, B, 2048.0, 0.5, 10.0, 256, 64), rel=1e-12)


def test_measured_split_probability():
    st = {"regions": [16, 56, 200, 680], "splits": [14, 50, 170, 0]}
    assert cm.split_probability(st) == pytest.approx((14 / 16 + 50 / 56 + 170 / 200) / 3)


# --- the model with measured overheads: per-level P_i and a per-region cost sigma ---

@pytest.mark.parametrize("n,g,r,B", GRID[::6])
@pytest.mark.parametrize("P", [0.0, 0.4, 1.0])
def test_levels_model_reduces_to_the_paper_model(n, g, r, B, P):
    # One P for every level and sigma = 0 is the time of Sec. 4.3.1.
    t1 = ref.time_sbr(n, g, r, B, 2048.0, P, 3.0, 256, 64)
    assert ref.time_sbr_levels(n, g, r, B, 2048.0, P, 3.0, 256, 64) == pytest.approx(t1, rel=1e-12)
    t = ref.tau(n, g, r, B)
    assert ref.time_sbr_levels(n, g, r, B, 2048.0, [P] * t, 3.0, 256, 64) == pytest.approx(t1, rel=1e-12)


@pytest.mark.parametrize("n,g,r,B", GRID[::6])
def test_sigma_is_paid_once_per_region_round(n, g, r, B):
    # With P = 1 every level is reached, so sigma adds sigma times the number
    # of block rounds, sum_i ceil(G R^i / q) over the tau levels.
    q = 256
    rounds = sum(math.ceil(g * g * (r * r) ** i / q) for i in range(ref.tau(n, g, r, B)))
    t0 = ref.time_sbr_levels(n, g, r, B, 512.0, 1.0, 2.0, q, 64, sigma=0.0)
    t1 = ref.time_sbr_levels(n, g, r, B, 512.0, 1.0, 2.0, q, 64, sigma=7.0)
    assert t1 - t0 == pytest.approx(7.0 * rounds, rel=1e-9)


def test_no_split_at_level_zero_ignores_deeper_levels():
    # P_0 = 0: no region reaches level 1, whatever the deeper P_i.
    n, g, r, B = 16384, 16, 4, 16
    a = ref.time_sbr_levels(n, g, r, B, 2048.0, [0.0, 0.1, 0.2, 0.3], 5.0, 256, 64, sigma=9.0)
    b = ref.time_sbr_levels(n, g, r, B, 2048.0, [0.0, 0.9, 0.8, 0.7], 5.0, 256, 64, sigma=9.0)
    assert a == b
    level0 = (math.ceil(4.0 * n / (g * 64)) * 2048.0 + math.ceil(float(n) * n / (g * g * 64)) + 9.0)
    assert a == pytest.approx(level0 * math.ceil(g * g / 256), rel=1e-12)


def test_levels_model_product_matches_the_oracle():
    rng = np.random.default_rng(7)
    for n, g, r, B in GRID:
        t = ref.tau(n, g, r, B)
        Ps = list(rng.uniform(0, 1, t))
        sig = float(rng.uniform(0, 1e4))
        want = ref.time_sbr_levels(n, g, r, B, 1024.0, Ps, 4.0, 256, 64, sigma=sig)
        got = cm.time_sbr_levels(n, g, r, B, 1024.0, Ps, 4.0, 256, 64, sigma=sig)
        assert got == pytest.approx(want, rel=1e-12)


def test_split_curve_interpolates_in_log_side_and_clamps():
    P = cm.split_curve([(256, 0.2), (1024, 0.6), (256, 0.4)])
    assert P(256) == pytest.approx(0.3) and P(1024) == pytest.approx(0.6)
    assert P(512) == pytest.approx(0.45)  # halfway in log2
    assert P(64) == pytest.approx(0.3) and P(1 << 20) == pytest.approx(0.6)


def test_level_sides_and_probabilities():
    # tau as printed (log_4(16384 / (64 * 16)) = 2 model levels; the render
    # itself has a third, 16-pixel level -- the reading of the stop rule)
    assert cm.level_sides(16384, 64, 4, 16) == [256.0, 64.0]
    assert cm.level_sides(16384, 16, 2, 32) == [1024.0, 512.0, 256.0, 128.0, 64.0]
    st = {"splits": [10, 30, 0], "regions": [20, 160, 480]}
    assert cm.split_probabilities(st) == [0.5, 30 / 160]


def test_rendered_levels_match_the_library():
    # The level count the model uses for measured renders is the one the
    # library computes for the same parameters (a host call, no GPU).
    from paper_2206_02255_amd import ask
    from workloads import Window
    for n, g, r, B in GRID + [(16384, 64, 4, 16), (16384, 16, 2, 32), (1000, 3, 3, 7)]:
        w = ask.window(Window(-1.5, 0.5, -1.0, 1.0, n, n, 256))
        assert cm.rendered_levels(n, g, r, B) == ask.ask_level_count(w, ask.params(g, r, B)), (n, g, r, B)


def test_rendered_levels_product_matches_the_oracle():
    rng = np.random.default_rng(8)
    for n, g, r, B in GRID[::3]:
        L = cm.rendered_levels(n, g, r, B)
        Ps = list(rng.uniform(0, 1, L))
        want = ref.time_sbr_levels(n, g, r, B, 1024.0, Ps, 4.0, 256, 64, sigma=50.0, levels=L)
        got = cm.time_sbr_levels(n, g, r, B, 1024.0, Ps, 4.0, 256, 64, sigma=50.0, levels=L)
        assert got == pytest.approx(want, rel=1e-12)
