"""Pins of the oracle's filled-Julia-set images: the escape-time workload of
the same self-similar class whose point is z0 = the pixel and whose c is
fixed (z_k = z_{k-1}^2 + c, dwell = first k >= 1 with |z_k|^2 > 4, else D).

The pins come from the mathematics, not from the oracle's own formula:

* c = 0: z_k = z0^(2^k), so |z_k| = |z0|^(2^k) and the dwell is the least
  k >= 1 with |z0|^(2^k) > 2 -- 1 when |z0| > 2 and D when |z0| < 1;
* c = -2 maps the real segment [-2, 2] onto itself (x^2 - 2), also after
  rounding, so every real z0 in it has dwell D;
* z -> -z leaves z^2 unchanged, so z0 and -z0 have the same orbit from
  k = 1: a window centred on 0 gives an image with 180-degree symmetry;
  for real c, z -> conj(z) commutes with the map: mirror symmetry in y;
* at z0 = 0 the orbit is the Mandelbrot orbit of c;
* the subdivision image follows the rule of Sec. 4.2.1 (the checks of the
  Mandelbrot subdivision pins, applied to Julia windows).
"""
import math

import numpy as np
import pytest

from test_oracle_subdiv import check_subdivision
from workloads import Window

JULIA_C = [(-0.8, 0.156), (-0.4, 0.6), (0.285, 0.01), (-0.7269, 0.1889), (-1.0, 0.0)]


def closed_form_c0(rho, D):
    """Dwell of |z0| = rho for c = 0, or None when rho is too close to a
    threshold for rounding to be ruled out."""
    if rho > 2.0:
        return 1
    if rho < 1.0:
        return D
    if rho == 1.0:
        return None
    t = math.log2(math.log(2.0) / math.log(rho))  # need 2^k > 2^t
    k = max(1, math.floor(t) + 1)
    if abs(t - round(t)) < 1e-6 and round(t) >= 1:
        return None
    return min(k, D)


def test_c_zero_closed_form(ref):
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(3000):
        rho = float(np.exp(rng.uniform(np.log(0.5), np.log(2.5))))
        th = float(rng.uniform(0, 2 * np.pi))
        want = closed_form_c0(rho, 64)
        if want is None:
            continue
        zr, zi = rho * math.cos(th), rho * math.sin(th)
        assert ref.dwell_julia(zr, zi, 0.0, 0.0, 64) == want, (rho, th)
        checked += 1
    assert checked > 2900


@pytest.mark.parametrize("x,k", [(1.1, 3), (1.5, 1), (1.05, 4), (1.01, 7), (2.0001, 1),
                                 (1.4, 2)])
def test_c_zero_real_axis_values(ref, x, k):
    # 1.1^8 = 2.14 > 2 > 1.1^4; 1.5^2 = 2.25; 1.05^16 = 2.18 > 2 > 1.05^8;
    # 1.01^128 = 3.57 > 2 > 1.01^64 = 1.89; 1.4^4 = 3.84 > 2 > 1.4^2 = 1.96
    assert ref.dwell_julia(x, 0.0, 0.0, 0.0, 500) == k
    assert ref.dwell_julia(-x, 0.0, 0.0, 0.0, 500) == k
    assert ref.dwell_julia(0.0, x, 0.0, 0.0, 500) == k


def test_c_minus_two_real_segment_never_escapes(ref):
    for x in np.linspace(-2.0, 2.0, 1001):
        assert ref.dwell_julia(float(x), 0.0, -2.0, 0.0, 300) == 300


def test_z0_zero_is_the_mandelbrot_orbit(ref):
    rng = np.random.default_rng(12)
    for _ in range(500):
        cr, ci = float(rng.uniform(-2, 0.6)), float(rng.uniform(-1.2, 1.2))
        assert ref.dwell_julia(0.0, 0.0, cr, ci, 700) == ref.dwell(cr, ci, 700)


@pytest.mark.parametrize("c", JULIA_C)
def test_point_symmetry_of_centred_window(ref, c):
    w = Window(-1.6, 1.6, -1.1, 1.1, 97, 64, 300, julia=c)
    E, _ = ref.exhaustive(w)
    assert np.array_equal(E, E[::-1, ::-1])


def test_mirror_symmetry_for_real_c(ref):
    w = Window(-1.9, 1.7, -1.2, 1.2, 90, 71, 400, julia=(-1.0, 0.0))
    E, _ = ref.exhaustive(w)
    assert np.array_equal(E, E[::-1, :])
    # the same window for a non-real c is not mirror-symmetric
    E2, _ = ref.exhaustive(Window(-1.9, 1.7, -1.2, 1.2, 90, 71, 400, julia=(-0.8, 0.156)))
    assert not np.array_equal(E2, E2[::-1, :])


def test_julia_differs_from_mandelbrot_window(ref):
    w = Window(-1.5, 0.5, -1.0, 1.0, 40, 40, 200)
    Em, _ = ref.exhaustive(w)
    Ej, _ = ref.exhaustive(Window(w.x0, w.x1, w.y0, w.y1, w.W, w.H, w.D, julia=(-0.8, 0.156)))
    assert not np.array_equal(Em, Ej)


def test_sampled_pixels_equal_full_images(ref):
    w = Window(-1.6, 1.6, -1.0, 1.0, 83, 59, 250, julia=(-0.8, 0.156))
    E, _ = ref.exhaustive(w)
    S, _ = ref.subdiv(w, 4, 2, 8)
    rng = np.random.default_rng(13)
    px = rng.integers(0, w.W, 300)
    py = rng.integers(0, w.H, 300)
    assert np.array_equal(ref.dwell_pixels(w, px, py), E[py, px])
    assert np.array_equal(ref.subdiv_pixels(w, 4, 2, 8, px, py), S[py, px])


JULIA_CASES = [
    (Window(-1.6, 1.6, -1.0, 1.0, 128, 96, 256, julia=(-0.8, 0.156)), 4, 2, 16),
    (Window(-1.6, 1.6, -1.0, 1.0, 100, 77, 300, julia=(-0.4, 0.6)), 3, 3, 5),
    (Window(-0.3, 0.2, -0.1, 0.4, 96, 80, 500, julia=(0.285, 0.01)), 5, 2, 7),
    (Window(-2.0, 2.0, -1.5, 1.5, 64, 64, 128, julia=(-1.0, 0.0)), 8, 8, 1),
]


@pytest.mark.parametrize("w,g,r,B", JULIA_CASES)
def test_julia_subdivision_follows_the_rule(ref, w, g, r, B):
    E, _ = ref.exhaustive(w)
    S, st, recs = ref.subdiv(w, g, r, B, records=True)
    check_subdivision(E, S, recs, st, g, r, B)


def test_julia_depth_first_equals_level_order(ref):
    w, g, r, B = JULIA_CASES[0]
    S0, st0 = ref.subdiv(w, g, r, B, order="bfs")
    S1, st1 = ref.subdiv(w, g, r, B, order="dfs")
    assert np.array_equal(S0, S1) and st0 == st1
