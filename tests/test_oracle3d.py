"""Pins of the 3-D oracle (the subdivision at higher dimensions, k = 3): the
quaternion Julia dwell volume, the level grids and their space-filling
curves, and the subdivision over boxes.

What pins it, from outside its own formulas:

* the j = 0 slice of a volume is the filled Julia image of the same complex
  c, bit for bit, as the 2-D oracle (a separate source) computes it;
* c = 0: the quaternion norm is multiplicative, so |q_k| = |q0|^(2^k) and the
  dwell has the closed form of the complex case;
* z -> -z commutes with the map (mirror symmetry in z); for real c so does
  the exchange y <-> z (the volume is symmetric under it);
* the canonical curve and the Morton curve are bijections with known values;
  the floor grids of consecutive levels nest;
* the subdivision volume and its per-level counts equal a brute-force
  re-derivation of the rule from the exhaustive volume, and the level-0
  count is the number of non-empty cells, min(g, n) per axis;
* planted mistakes in a copy of the source fail at least one of these.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import askref3 as R
from oracle import build as oracle_build
from workloads import Volume, Window

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ref3():
    R.lib()
    return R


# --------------------------------------------------------------------------
# The dwell


@pytest.mark.parametrize("c", [(-0.2, 0.6), (-1.0, 0.0), (0.285, 0.01)])
def test_zero_slice_is_the_julia_image(ref3, ref, c):
    v = Volume(-1.6, 1.5, -1.3, 1.4, -1.2, 1.2, 61, 47, 9, 300, c=c)
    E = ref3.exhaustive(v)
    J, _ = ref.exhaustive(Window(v.x0, v.x1, v.y0, v.y1, v.W, v.H, v.D, julia=c))
    assert np.array_equal(E[4], J)
    assert not np.array_equal(E[3], J)


def test_c_zero_closed_form(ref3):
    rng = np.random.default_rng(31)
    checked = 0
    for _ in range(2000):
        rho = float(np.exp(rng.uniform(np.log(0.5), np.log(2.5))))
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        if rho > 2.0:
            want = 1
        elif rho < 1.0:
            want = 64
        else:
            t = math.log2(math.log(2.0) / math.log(rho))
            if abs(t - round(t)) < 1e-6:
                continue
            want = min(max(1, math.floor(t) + 1), 64)
        a, b, e = (rho * u).tolist()
        assert ref3.dwell(a, b, e, 0.0, 0.0, 64) == want, (rho, u)
        checked += 1
    assert checked > 1900


@pytest.mark.parametrize("x,k", [(1.1, 3), (1.5, 1), (1.05, 4), (1.4, 2)])
def test_c_zero_axis_values(ref3, x, k):
    # 1.1^8 > 2 > 1.1^4; 1.5^2 > 2; 1.05^16 > 2 > 1.05^8; 1.4^4 > 2 > 1.4^2
    for q in ((x, 0, 0), (0, x, 0), (0, 0, x), (0, 0, -x)):
        assert ref3.dwell(*q, 0.0, 0.0, 500) == k


def test_volume_c_zero_closed_form(ref3):
    """c = 0 on a whole volume: each voxel's dwell follows from |q0| alone, with
    q0 mapped from the voxel here (centre + (2p + 1 - n) * half pitch, per axis)."""
    v = Volume(-1.9, 1.3, -1.5, 0.7, -0.5, 2.0, 23, 19, 17, 40, c=(0.0, 0.0))
    E = ref3.exhaustive(v)
    axes = []
    for lo, hi, n in ((v.x0, v.x1, v.W), (v.y0, v.y1, v.H), (v.z0, v.z1, v.L)):
        half = (hi - lo) / (2.0 * n)
        axes.append(0.5 * (lo + hi) + (2 * np.arange(n) + 1 - n) * half)
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    rho = np.sqrt(x * x + y * y + z * z)
    checked = 0
    for idx in np.ndindex(E.shape):
        p = float(rho[idx])
        if abs(p - 1.0) < 1e-9:
            continue
        if p > 2.0:
            want = 1
        elif p < 1.0:
            want = v.D
        else:
            t = math.log2(math.log(2.0) / math.log(p))
            if abs(t - round(t)) < 1e-6:
                continue
            want = min(max(1, math.floor(t) + 1), v.D)
        assert E[idx] == want, (idx, p)
        checked += 1
    assert checked > 0.99 * E.size


def test_mirror_in_z(ref3):
    v = Volume(-1.5, 1.3, -1.2, 1.1, -1.0, 1.0, 33, 29, 24, 200, c=(-0.2, 0.6))
    E = ref3.exhaustive(v)
    assert np.array_equal(E, E[::-1])


def test_y_z_exchange_for_real_c(ref3):
    v = Volume(-1.7, 1.5, -1.1, 1.1, -1.1, 1.1, 31, 26, 26, 200, c=(-1.0, 0.0))
    E = ref3.exhaustive(v)
    assert np.array_equal(E, E.transpose(1, 0, 2))
    v2 = Volume(-1.7, 1.5, -1.1, 1.1, -1.1, 1.1, 31, 26, 26, 200, c=(-0.2, 0.6))
    E2 = ref3.exhaustive(v2)
    assert not np.array_equal(E2, E2.transpose(1, 0, 2))


# The binary64 operation order of the quaternion step (the reading taken:
# a2 = a*a, b2 = b*b, e2 = e*e, ab = a*b, ae = a*e; a = (a2 - (b2 + e2)) + cr;
# b = (ab + ab) + ci; e = (ae + ae) + 0; escape when a*a + (b*b + e*e) > 4;
# each operation rounded on its own), evaluated independently with numpy
# binary64 arrays, one ufunc call per operation, over volumes where long
# escaping orbits make a reassociated or contracted step change dwells.
def binary64_volume(v):
    axes = []
    for lo, hi, n in ((v.x0, v.x1, v.W), (v.y0, v.y1, v.H), (v.z0, v.z1, v.L)):
        centre = 0.5 * (lo + hi)
        half = (hi - lo) / (2.0 * n)
        k = (2 * np.arange(n, dtype=np.int64) + 1 - n).astype(np.float64)
        axes.append(centre + np.multiply(k, half))
    shape = (v.L, v.H, v.W)
    a = np.broadcast_to(axes[0][None, None, :], shape).ravel().copy()
    b = np.broadcast_to(axes[1][None, :, None], shape).ravel().copy()
    e = np.broadcast_to(axes[2][:, None, None], shape).ravel().copy()
    cr, ci = float(v.c[0]), float(v.c[1])
    out = np.full(a.size, v.D, dtype=np.int64)
    idx = np.arange(a.size)
    with np.errstate(over="ignore", invalid="ignore"):
        for k in range(1, v.D + 1):
            a2 = np.multiply(a, a)
            b2 = np.multiply(b, b)
            e2 = np.multiply(e, e)
            ab = np.multiply(a, b)
            ae = np.multiply(a, e)
            a = np.add(np.subtract(a2, np.add(b2, e2)), cr)
            b = np.add(np.add(ab, ab), ci)
            e = np.add(np.add(ae, ae), 0.0)
            mag = np.add(np.multiply(a, a), np.add(np.multiply(b, b), np.multiply(e, e)))
            esc = mag > 4.0
            if esc.any():
                out[idx[esc]] = k
                keep = ~esc
                idx, a, b, e = idx[keep], a[keep], b[keep], e[keep]
                if idx.size == 0:
                    break
    return out.reshape(shape)


OP_ORDER_VOLUMES = [
    # a Cantor dust: every orbit escapes, the whole volume is near the set
    Volume(-1.6, 1.6, -1.0, 1.0, -1.0, 1.0, 64, 48, 48, 2000, c=(-0.8, 0.156)),
    Volume(-1.6, 1.6, -1.0, 1.0, -0.5, 0.5, 64, 40, 32, 1000, c=(-0.8, 0.156)),
    # the benchmark's c, and a c near the parabolic point -3/4
    Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 48, 48, 48, 256, c=(-0.2, 0.6)),
    Volume(-1.2, 1.2, -0.8, 0.8, 0.0, 0.8, 64, 48, 24, 2000, c=(-0.75, 0.1)),
]


@pytest.mark.parametrize("v", OP_ORDER_VOLUMES,
                         ids=lambda v: "c%g_%g_%dx%dx%d" % (v.c[0], v.c[1], v.W, v.H, v.L))
def test_operation_order_binary64(ref3, v):
    got = ref3.exhaustive(v)
    want = binary64_volume(v)
    diff = np.argwhere(got != want)
    assert diff.size == 0, "3-D oracle differs from the binary64 reading at %d voxels, first %s" % (
        len(diff), diff[:5].tolist())


def test_op_order_volumes_cover_enough_voxels():
    assert sum(v.voxels for v in OP_ORDER_VOLUMES) >= 300000


def test_voxel_dwell_equals_volume(ref3):
    v = Volume(-1.6, 1.6, -1.6, 1.6, -1.0, 1.4, 20, 17, 13, 150, c=(-0.2, 0.6))
    E = ref3.exhaustive(v)
    rng = np.random.default_rng(32)
    for _ in range(200):
        x, y, z = int(rng.integers(v.W)), int(rng.integers(v.H)), int(rng.integers(v.L))
        assert ref3.voxel_dwell(v, x, y, z) == E[z, y, x]


# --------------------------------------------------------------------------
# Level grids and space-filling curves


def test_canonical_curve(ref3):
    G = 5
    seen = set()
    for z in range(G):
        for y in range(G):
            for x in range(G):
                s = ref3.canonical(G, (x, y, z))
                assert s == x + G * y + G * G * z
                assert ref3.canonical_inv(G, s) == (x, y, z)
                seen.add(s)
    assert seen == set(range(G ** 3))


def test_morton_curve(ref3):
    known = {(1, 0, 0): 1, (0, 1, 0): 2, (0, 0, 1): 4, (2, 0, 0): 8, (0, 2, 0): 16,
             (3, 3, 3): 63, (5, 0, 0): 65, (0, 0, 2): 32, (7, 7, 7): 511}
    for p, s in known.items():
        assert ref3.morton(p) == s and ref3.morton_inv(s) == p
    codes = [ref3.morton((x, y, z)) for z in range(8) for y in range(8) for x in range(8)]
    assert sorted(codes) == list(range(512))
    # every aligned 2^k cube is one contiguous run of codes
    for k in (1, 2):
        s = 1 << k
        for z0 in range(0, 8, s):
            run = sorted(ref3.morton((x, y, z)) for z in range(z0, z0 + s)
                         for y in range(s) for x in range(s))
            assert run == list(range(run[0], run[0] + s ** 3))
    big = (2 ** 21 - 1, 12345, 2 ** 20)
    assert ref3.morton_inv(ref3.morton(big)) == big


def test_level_grids_nest(ref3):
    rng = np.random.default_rng(33)
    for _ in range(300):
        n = int(rng.integers(1, 3000))
        g = int(rng.integers(1, 40))
        r = int(rng.integers(2, 6))
        i = int(rng.integers(0, 4))
        G = g * r ** i
        j = int(rng.integers(0, G))
        assert ref3.cell_lo(j, G, n) == (j * n) // G
        assert ref3.cell_lo(j * r, G * r, n) == ref3.cell_lo(j, G, n)
        assert ref3.cell_lo(j * r + r, G * r, n) == ref3.cell_lo(j + 1, G, n)
    assert ref3.cell_lo(7, 7, 100) == 100


# --------------------------------------------------------------------------
# The subdivision


def brute_subdiv(E, g, r, B):
    """The rule of the subdivision applied to the exhaustive volume: level
    grids G_i = g r^i, floor partitions per axis, boxes decided by their
    surface, children of split boxes on the next grid (empty ones dropped)."""
    L_, H_, W_ = E.shape
    n = (W_, H_, L_)
    S = np.zeros_like(E)
    stats = {"regions": [], "fills": [], "splits": [], "leaves": [],
             "iters_surface": 0, "iters_leaf": 0}

    def span(j, G, m):
        return (j * m) // G, ((j + 1) * m) // G

    def nonempty(p, G):
        return all(span(p[d], G, n[d])[1] > span(p[d], G, n[d])[0] for d in range(3))

    level = [(x, y, z) for z in range(g) for y in range(g) for x in range(g)
             if nonempty((x, y, z), g)]
    G = g
    while level:
        nxt = []
        f = s = lf = 0
        for p in level:
            (x0, x1), (y0, y1), (z0, z1) = (span(p[d], G, n[d]) for d in range(3))
            blk = E[z0:z1, y0:y1, x0:x1]
            surf = np.ones(blk.shape, bool)
            surf[1:-1, 1:-1, 1:-1] = False
            vals = blk[surf]
            # the work counters: every decided box's whole surface, and the
            # inside of every leaf box
            stats["iters_surface"] += int(vals.sum(dtype=np.int64))
            if (vals == vals[0]).all():
                S[z0:z1, y0:y1, x0:x1] = vals[0]
                f += 1
            elif max(x1 - x0, y1 - y0, z1 - z0) <= B:
                S[z0:z1, y0:y1, x0:x1] = blk
                stats["iters_leaf"] += int(blk[~surf].sum(dtype=np.int64))
                lf += 1
            else:
                s += 1
                for kz in range(r):
                    for ky in range(r):
                        for kx in range(r):
                            c = (p[0] * r + kx, p[1] * r + ky, p[2] * r + kz)
                            if nonempty(c, G * r):
                                nxt.append(c)
        for k, val in zip(("regions", "fills", "splits", "leaves"), (len(level), f, s, lf)):
            stats[k].append(val)
        level, G = nxt, G * r
    stats["levels"] = len(stats["regions"])
    return S, stats


CASES = [
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 40, 40, 40, 256, c=(-0.2, 0.6)), 4, 2, 4),
    (Volume(-1.5, 1.4, -1.3, 1.2, -0.9, 1.1, 37, 29, 23, 300, c=(-1.0, 0.0)), 3, 3, 2),
    (Volume(-0.8, 0.4, -0.2, 0.9, -0.5, 0.5, 26, 31, 19, 400, c=(-0.125, 0.65)), 5, 2, 3),
    (Volume(-1.6, 1.6, -1.6, 1.6, -1.6, 1.6, 24, 24, 24, 128, c=(-0.2, 0.6)), 2, 4, 1),
    (Volume(-1.3, 1.1, -1.2, 1.2, -1.1, 1.3, 64, 56, 48, 256, c=(-0.2, 0.6)), 8, 2, 2),
]


@pytest.mark.parametrize("order", ["canonical", "morton"])
@pytest.mark.parametrize("v,g,r,B", CASES)
def test_subdivision_follows_the_rule(ref3, v, g, r, B, order):
    E = ref3.exhaustive(v)
    S, st = ref3.subdiv(v, g, r, B, order)
    S2, st2 = brute_subdiv(E, g, r, B)
    assert np.array_equal(S, S2)
    assert st == st2
    assert st["regions"][0] == min(g, v.W) * min(g, v.H) * min(g, v.L)
    assert st["levels"] >= 2 and sum(st["splits"]) > 0 and sum(st["fills"]) > 0


def test_orders_agree(ref3):
    v, g, r, B = CASES[1]
    a = ref3.subdiv(v, g, r, B, "canonical")
    b = ref3.subdiv(v, g, r, B, "morton")
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_degenerate_volumes(ref3):
    one = Volume(-0.1, 0.1, -0.1, 0.1, -0.1, 0.1, 1, 1, 1, 50, c=(-0.2, 0.6))
    S, st = ref3.subdiv(one, 4, 2, 1)
    assert S[0, 0, 0] == ref3.voxel_dwell(one, 0, 0, 0)
    assert st["regions"] == [1] and st["fills"] == [1]
    line = Volume(-1.6, 1.6, -0.01, 0.01, -0.01, 0.01, 57, 1, 1, 100, c=(-1.0, 0.0))
    S, st = ref3.subdiv(line, 3, 2, 2)
    assert np.array_equal(S, ref3.exhaustive(line))
    assert st["regions"][0] == 3
    # g larger than every side: one cell per voxel on level 0
    small = Volume(-1.0, 1.0, -1.0, 1.0, -1.0, 1.0, 3, 5, 2, 60, c=(-0.2, 0.6))
    S, st = ref3.subdiv(small, 8, 2, 1)
    assert np.array_equal(S, ref3.exhaustive(small))
    assert st["regions"] == [30] and st["fills"] == [30]


def test_uniform_volume_fills_at_level_zero(ref3):
    # every point of this box has |q0| > 2, so every dwell is 1
    v = Volume(3.0, 4.0, 3.0, 4.0, 3.0, 4.0, 30, 20, 10, 100, c=(-0.2, 0.6))
    S, st = ref3.subdiv(v, 4, 2, 2)
    assert (S == 1).all()
    # Every box's whole surface is scanned, at one iteration a voxel. The
    # boxes are 7, 8, 7, 8 wide, 5 high and 2, 3, 2, 3 deep: only the 3-deep
    # ones have an inside, (w - 2) * 3 * 1 voxels each.
    inside = 2 * 4 * (5 + 6 + 5 + 6) * 3
    assert st == {"levels": 1, "regions": [64], "fills": [64], "splits": [0], "leaves": [0],
                  "iters_surface": 30 * 20 * 10 - inside, "iters_leaf": 0}


def test_bad_arguments(ref3):
    v = CASES[0][0]
    for g, r, B in ((0, 2, 4), (4, 1, 4), (4, 2, 0)):
        with pytest.raises(ValueError):
            ref3.subdiv(v, g, r, B)


# --------------------------------------------------------------------------
# Planted mistakes

SRC = os.path.join(ROOT, "oracle", "askref3.c")
PINS = ["test_zero_slice_is_the_julia_image", "test_c_zero_closed_form",
        "test_operation_order_binary64",
        "test_volume_c_zero_closed_form",
        "test_mirror_in_z", "test_y_z_exchange_for_real_c", "test_canonical_curve",
        "test_morton_curve", "test_level_grids_nest", "test_subdivision_follows_the_rule",
        "test_degenerate_volumes"]

MUTANTS = {
    "dropped_z_square": ("a = (a2 - (b2 + e2)) + cr;", "a = (a2 - b2) + cr;"),
    "z_part_not_doubled": ("e = (ae + ae) + 0.0;", "e = ae + 0.0;"),
    "z_missing_in_modulus": ("double mag = a * a + (b * b + e * e);", "double mag = a * a + b * b;"),
    "z_pitch_from_y": ("m[5] = (box[5] - box[4]) / (2.0 * (double)L);",
                       "m[5] = (box[3] - box[2]) / (2.0 * (double)L);"),
    "morton_axes_swapped": ("s |= (uint64_t)((p[d] >> t) & 1u) << (3 * t + d);",
                            "s |= (uint64_t)((p[d] >> t) & 1u) << (3 * t + 2 - d);"),
    "canonical_transposed": ("return ((uint64_t)p[2] * G + p[1]) * G + p[0];",
                             "return ((uint64_t)p[0] * G + p[1]) * G + p[2];"),
    "surface_misses_top": ("y == b->lo[1] || y == b->hi[1] - 1 ||", "y == b->lo[1] ||"),
    "leaf_rule_any_side": ("if (b->hi[0] - b->lo[0] <= B && b->hi[1] - b->lo[1] <= B &&",
                           "if (b->hi[0] - b->lo[0] <= B || b->hi[1] - b->lo[1] <= B &&"),
    "child_grid_not_refined": ("uint64_t G1 = G * r, n1 = 0, cap1 = 0;",
                               "uint64_t G1 = G * r + 1, n1 = 0, cap1 = 0;"),
    "ceil_partition": ("return (uint32_t)(j * (uint64_t)n / G);",
                       "return (uint32_t)((j * (uint64_t)n + G - 1) / G);"),
    # binary64 operation order of the quaternion step
    "reassoc_a_part": ("a = (a2 - (b2 + e2)) + cr;", "a = ((a2 - b2) - e2) + cr;"),
    "reassoc_b_part": ("b = (ab + ab) + ci;", "b = ab + (ab + ci);"),
}

# The unchanged source built with contraction into fused multiply-adds.
FLAG_MUTANTS = {"contracted_build": ("-ffp-contract=fast", "-mfma")}


@pytest.mark.slow
def test_every_planted_mistake_is_caught(tmp_path):
    src = open(SRC).read()
    escaped = []
    for name in list(MUTANTS) + list(FLAG_MUTANTS):
        text, extra = src, ("-Wno-error",)
        if name in FLAG_MUTANTS:
            extra += FLAG_MUTANTS[name]
        else:
            a, b = MUTANTS[name]
            assert src.count(a) == 1, name
            text = src.replace(a, b)
        path = tmp_path / ("m_%s.c" % name)
        path.write_text(text)
        lib = oracle_build.build(extra=extra, src=str(path),
                                 out=str(tmp_path / ("lib_%s.so" % name)))
        env = dict(os.environ, ASKREF3_LIB=lib)
        p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle3d.py"),
                            "-k", " or ".join(PINS)],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
        if p.returncode == 0:
            escaped.append(name)
    assert not escaped, "planted mistakes not caught: %s" % escaped
