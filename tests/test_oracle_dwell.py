"""Pins of the oracle's dwell and pixel mapping to what the mathematics fixes.

None of these re-type the oracle's own loop in binary64: they use closed-form
orbits, textbook interior regions, published asymptotics, an exact-arithmetic
(decimal, 80 digits) evaluation of the definition, and exact symmetry.
"""
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

from workloads import Window

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_closed_form():
    rows = []
    with open(os.path.join(GOLDEN, "dwell_closed_form.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            cr, ci, D, want = line.split()[:4]
            rows.append((float(cr), float(ci), int(D), int(want)))
    return rows


@pytest.mark.parametrize("cr,ci,D,want", load_closed_form())
def test_closed_form_orbits(ref, cr, ci, D, want):
    assert ref.dwell(cr, ci, D) == want


def test_outside_radius_two_escapes_at_once(ref):
    # |c| > 2: |z_1|^2 = |c|^2 > 4, so the dwell is 1 (Sec. 6, escape radius 2).
    rng = np.random.default_rng(11)
    rho = rng.uniform(2.0001, 50.0, 2000)
    th = rng.uniform(0, 2 * math.pi, 2000)
    for a, t in zip(rho, th):
        assert ref.dwell(a * math.cos(t), a * math.sin(t), 5000) == 1


def test_main_cardioid_and_period2_bulb_never_escape(ref):
    # Textbook closed forms: c = mu/2 - mu^2/4 (|mu| < 1) has an attracting
    # fixed point; c = -1 + mu/4 (|mu| < 1) an attracting 2-cycle. Kept to
    # |mu| <= 0.9 so the orbit contracts quickly: the dwell is D.
    rng = np.random.default_rng(12)
    for _ in range(1500):
        mu = rng.uniform(0, 0.9) * np.exp(1j * rng.uniform(0, 2 * math.pi))
        c1 = mu / 2 - mu * mu / 4
        c2 = -1 + mu / 4
        assert ref.dwell(c1.real, c1.imag, 3000) == 3000
        assert ref.dwell(c2.real, c2.imag, 3000) == 3000


@pytest.mark.parametrize("eps", [1e-4, 1e-5, 1e-6, 1e-8])
def test_parabolic_gate_at_quarter(ref, eps):
    # Published asymptotic for c = 1/4 + eps: the orbit needs about
    # pi / sqrt(eps) iterations to pass the gate near z = 1/2.
    d = ref.dwell(0.25 + eps, 0.0, 10**7)
    assert abs(d - math.pi / math.sqrt(eps)) <= 3.5


@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-4, 1e-5])
def test_parabolic_gate_at_three_quarters(ref, eps):
    # Published asymptotic for c = -3/4 + i eps: about pi / eps iterations.
    d = ref.dwell(-0.75, eps, 10**8)
    assert abs(d - math.pi / eps) <= 2.5


def exact_dwell(cr, ci, D, prec=80):
    """Dwell of the exact c in 80-digit decimal arithmetic, and the smallest
    distance of |z_k|^2 from 4 over the checked iterations."""
    getcontext().prec = prec
    cr, ci = Decimal(cr), Decimal(ci)
    zr = zi = Decimal(0)
    margin = Decimal(10)
    four = Decimal(4)
    for k in range(1, D + 1):
        zr, zi = zr * zr - zi * zi + cr, 2 * zr * zi + ci
        mag = zr * zr + zi * zi
        margin = min(margin, abs(mag - four))
        if mag > four:
            return k, margin
    return D, margin


def test_dwell_matches_exact_arithmetic(ref):
    # For short orbits, binary64 rounding (and the rounding of c) moves |z_k|^2
    # by far less than 1e-6; wherever the exact orbit stays that far from the
    # escape circle at every check, the dwell must be the exact one.
    rng = np.random.default_rng(13)
    D = 12
    checked = 0
    for _ in range(4000):
        cr, ci = rng.uniform(-2.2, 0.8), rng.uniform(-1.3, 1.3)
        want, margin = exact_dwell(cr, ci, D)
        if margin < Decimal("1e-6"):
            continue
        assert ref.dwell(cr, ci, D) == want, (cr, ci)
        checked += 1
    assert checked > 3500


def test_pixel_centres_exact(ref):
    # Pixel centres of [-2, 2] x [-1, 1] at 4 x 2 pixels are exact binary64
    # values: x in {-1.5, -0.5, 0.5, 1.5}, y in {-0.5, 0.5}; row 0 is y0.
    w = Window(-2.0, 2.0, -1.0, 1.0, 4, 2, 10)
    for py in range(2):
        for px in range(4):
            assert ref.pixel_c(w, px, py) == (-1.5 + px, -0.5 + py)


def test_mapping_constants(ref):
    w = Window(-1.5, 0.5, -1.0, 1.0, 1024, 768, 10)
    cxm, cym, hx, hy = ref.mapping(w)
    assert cxm == -0.5 and cym == 0.0
    assert hx == 2.0 / 2048 and hy == 2.0 / 1536


def exact_image(w, D):
    """Exhaustive image in exact decimal arithmetic with the exact pixel
    centre x0 + (px + 1/2)(x1 - x0)/W; entries whose orbit passes within 1e-6
    of the escape circle are marked -1."""
    getcontext().prec = 80
    x0, x1, y0, y1 = (Decimal(v) for v in (w.x0, w.x1, w.y0, w.y1))
    out = np.empty((w.H, w.W), dtype=np.int64)
    for py in range(w.H):
        ci = y0 + (Decimal(py) + Decimal("0.5")) * (y1 - y0) / w.H
        for px in range(w.W):
            cr = x0 + (Decimal(px) + Decimal("0.5")) * (x1 - x0) / w.W
            k, margin = exact_dwell(cr, ci, D)
            out[py, px] = k if margin > Decimal("1e-6") else -1
    return out


@pytest.mark.parametrize("w", [
    Window(-2.1, 0.7, -1.2, 0.9, 17, 11, 12),    # non-square, odd sizes
    Window(-0.9, -0.3, 0.2, 1.1, 9, 14, 12),      # taller than wide
    Window(-2.5, 1.5, -2.0, 2.0, 13, 13, 12),     # reaches |c| > 2
])
def test_exhaustive_image_matches_exact_arithmetic(ref, w):
    # Pins the pixel mapping, orientation (row 0 on y0) and row-major layout
    # of the exhaustive image together with the dwell.
    img, iters = ref.exhaustive(w, threads=2)
    want = exact_image(w, w.D)
    ok = want >= 0
    assert ok.mean() > 0.9
    assert np.array_equal(img[ok], want[ok].astype(np.uint32))
    assert iters == int(img.astype(np.uint64).sum())


@pytest.mark.parametrize("W,H", [(64, 48), (33, 31), (1, 7)])
def test_exhaustive_mirror_symmetry(ref, W, H):
    # y0 = -y1: the window centre is 0 and ky negates exactly, and every
    # operation is sign-symmetric under round-to-nearest-even, so row py and
    # row H-1-py are identical bit for bit (the set is symmetric under
    # conjugation).
    w = Window(-1.9, 0.6, -1.1, 1.1, W, H, 400)
    img, _ = ref.exhaustive(w, threads=3)
    assert np.array_equal(img, img[::-1])


def test_exhaustive_threads_agree(ref):
    w = Window(-1.5, 0.5, -1.0, 1.0, 97, 61, 200)
    a, ia = ref.exhaustive(w, threads=1)
    b, ib = ref.exhaustive(w, threads=5)
    assert np.array_equal(a, b) and ia == ib


def test_dwell_pixels_agree_with_image(ref):
    w = Window(-1.5, 0.5, -1.0, 1.0, 80, 70, 300)
    img, _ = ref.exhaustive(w)
    rng = np.random.default_rng(3)
    px = rng.integers(0, w.W, 500)
    py = rng.integers(0, w.H, 500)
    assert np.array_equal(ref.dwell_pixels(w, px, py), img[py, px])


def test_bad_windows_rejected(ref):
    for w in [Window(0.5, -1.5, -1, 1, 8, 8, 10), Window(-1, 1, -1, 1, 0, 8, 10),
              Window(-1, 1, -1, 1, 8, 8, 0), Window(-1, float("nan"), -1, 1, 8, 8, 10),
              Window(-1, 1, -1, 1, 65537, 8, 10)]:
        with pytest.raises(ValueError):
            ref.exhaustive(w)
