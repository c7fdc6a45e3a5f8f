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


# --------------------------------------------------------------------------
# The binary64 operation order (the paper fixes no order; the reading taken:
# per iteration zr2 = zr*zr, zi2 = zi*zi, zri = zr*zi, zr = (zr2 - zi2) + cr,
# zi = (zri + zri) + ci, escape when zr*zr + zi*zi > 4, every operation
# rounded on its own, no fused multiply-add). The exact-arithmetic pins above
# cannot see the rounding order: they skip every orbit that passes near the
# escape circle. These pins evaluate the same reading independently, with
# numpy binary64 arrays (each ufunc call is one correctly rounded operation;
# numpy never fuses two calls) and, on a subset, with Python floats, over
# windows chosen so that a reassociated or contracted evaluation changes
# dwells: orbits near c = -2 and |c| = 2, where |z|^2 sits on 4 for many
# iterations, and long orbits near the boundary, where a one-ulp difference
# grows until it moves the escape.
# --------------------------------------------------------------------------

def binary64_points(w):
    """Pixel points of a window in binary64, in the order of the mapping
    reading: centre, half pitch, then centre + (2p + 1 - N) * half pitch."""
    cxm = 0.5 * (w.x0 + w.x1)
    cym = 0.5 * (w.y0 + w.y1)
    hx = (w.x1 - w.x0) / (2.0 * w.W)
    hy = (w.y1 - w.y0) / (2.0 * w.H)
    kx = (2 * np.arange(w.W, dtype=np.int64) + 1 - w.W).astype(np.float64)
    ky = (2 * np.arange(w.H, dtype=np.int64) + 1 - w.H).astype(np.float64)
    pr = cxm + np.multiply(kx, hx)
    pi = cym + np.multiply(ky, hy)
    return np.broadcast_to(pr[None, :], (w.H, w.W)), np.broadcast_to(pi[:, None], (w.H, w.W))


def binary64_dwells(zr, zi, cr, ci, D):
    """Dwells of orbits started at z0 = (zr, zi) with constants (cr, ci)
    (arrays of one shape, or scalars broadcast to it), evaluated with one
    numpy operation per binary64 operation of the reading; lanes leave the
    arrays as they escape."""
    zr, zi, cr, ci = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64)
                                           for a in (zr, zi, cr, ci)))
    shape = zr.shape
    zr, zi = zr.ravel().copy(), zi.ravel().copy()
    cr, ci = cr.ravel().copy(), ci.ravel().copy()
    out = np.full(zr.size, D, dtype=np.int64)
    np.seterr(over="ignore", invalid="ignore")  # escaped orbits may overflow; they leave
    idx = np.arange(zr.size)
    for k in range(1, D + 1):
        zr2 = np.multiply(zr, zr)
        zi2 = np.multiply(zi, zi)
        zri = np.multiply(zr, zi)
        zr = np.add(np.subtract(zr2, zi2), cr)
        zi = np.add(np.add(zri, zri), ci)
        mag = np.add(np.multiply(zr, zr), np.multiply(zi, zi))
        esc = mag > 4.0
        if esc.any():
            out[idx[esc]] = k
            keep = ~esc
            idx, zr, zi, cr, ci = idx[keep], zr[keep], zi[keep], cr[keep], ci[keep]
            if idx.size == 0:
                break
    return out.reshape(shape)


def python_float_dwell(zr, zi, cr, ci, D):
    """The same reading with Python floats (IEEE binary64, never fused)."""
    zr, zi, cr, ci = float(zr), float(zi), float(cr), float(ci)
    for k in range(1, D + 1):
        zr2 = zr * zr
        zi2 = zi * zi
        zri = zr * zi
        zr = (zr2 - zi2) + cr
        zi = (zri + zri) + ci
        if zr * zr + zi * zi > 4.0:
            return k
    return D


def _deep_window(n, D):
    from workloads import deep_window
    return deep_window(n=n, D=D)


# Windows of the op-order pins: 9 windows, 1.3e5 pixels in all.
OP_ORDER_WINDOWS = [
    # c = -2 and its neighbourhood: the orbit 0, -2, 2, 2, ... has |z|^2 = 4.
    Window(-2.0 - 3e-6, -2.0 + 3e-6, -3e-6, 3e-6, 96, 96, 3000),
    # across the circle |c| = 2 at two angles (|z_1|^2 = |c|^2 on 4)
    Window(-1.4142135623730951 - 2e-3, -1.4142135623730951 + 2e-3,
           1.4142135623730951 - 2e-3, 1.4142135623730951 + 2e-3, 96, 96, 2000),
    Window(1.9999, 2.0001, -1e-4, 1e-4, 64, 64, 500),
    # the boundary of the paper's window, seahorse valley and a deep spiral
    Window(-0.7465, -0.7445, 0.1025, 0.1045, 128, 128, 4000),
    Window(-1.5, 0.5, -1.0, 1.0, 128, 128, 2048),
    # the deep-zoom window (width 1e-6 around a stored boundary point, D = 8192)
    "deep",
    # filled Julia sets: basilica, rabbit, Cantor dust
    Window(-1.7, 1.7, -1.7, 1.7, 128, 128, 2048, julia=(-1.0, 0.0)),
    Window(-0.4, -0.2, 0.45, 0.65, 96, 96, 3000, julia=(-0.123, 0.745)),
    Window(-1.6, 1.6, -1.0, 1.0, 128, 96, 1000, julia=(-0.8, 0.156)),
]


def _op_window(w):
    return _deep_window(160, 8192) if w == "deep" else w


@pytest.mark.parametrize("w", OP_ORDER_WINDOWS, ids=lambda w: w if isinstance(w, str) else
                         "%g_%g_%dx%d" % (w.x0, w.y0, w.W, w.H))
def test_operation_order_binary64(ref, w):
    w = _op_window(w)
    img, iters = ref.exhaustive(w)
    pr, pi = binary64_points(w)
    if w.julia is None:
        want = binary64_dwells(0.0, 0.0, pr, pi, w.D)
    else:
        want = binary64_dwells(pr, pi, w.julia[0], w.julia[1], w.D)
    diff = np.argwhere(img != want)
    assert diff.size == 0, "oracle differs from the binary64 reading at %d pixels, first %s" % (
        len(diff), diff[:5].tolist())
    assert iters == int(want.sum())


def test_op_order_windows_cover_enough_pixels():
    n = sum(_op_window(w).pixels for w in OP_ORDER_WINDOWS)
    assert n >= 100000, n


def test_op_order_windows_are_rounding_sensitive():
    # The windows above must tell the reading apart from its nearest
    # alternatives; otherwise matching them would pin nothing. Evaluated
    # here with numpy, with the alternative written out: the real part
    # reassociated as zr2 - (zi2 - cr).
    changed = 0
    np.seterr(over="ignore", invalid="ignore")
    for w in OP_ORDER_WINDOWS[:5]:
        w = _op_window(w)
        pr, pi = binary64_points(w)
        a = binary64_dwells(0.0, 0.0, pr, pi, w.D)
        zr = np.zeros(pr.shape)
        zi = np.zeros(pr.shape)
        out = np.full(pr.shape, w.D, dtype=np.int64)
        live = np.ones(pr.shape, dtype=bool)
        for k in range(1, w.D + 1):
            zr2, zi2, zri = zr * zr, zi * zi, zr * zi
            zr = zr2 - (zi2 - pr)
            zi = (zri + zri) + pi
            esc = live & (zr * zr + zi * zi > 4.0)
            out[esc] = k
            live &= ~esc
            if not live.any():
                break
        changed += int((out != a).sum())
    assert changed > 0


def test_operation_order_python_floats(ref):
    # Python floats on random points of three sensitive windows, through the
    # oracle's single-point entry points.
    rng = np.random.default_rng(41)
    for w in (OP_ORDER_WINDOWS[0], OP_ORDER_WINDOWS[3], OP_ORDER_WINDOWS[7]):
        for _ in range(300):
            x = float(rng.uniform(w.x0, w.x1))
            y = float(rng.uniform(w.y0, w.y1))
            if w.julia is None:
                assert ref.dwell(x, y, w.D) == python_float_dwell(0.0, 0.0, x, y, w.D), (x, y)
            else:
                assert ref.dwell_julia(x, y, *w.julia, w.D) == python_float_dwell(
                    x, y, w.julia[0], w.julia[1], w.D), (x, y)
