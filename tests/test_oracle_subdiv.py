"""Pins of the oracle's Mariani-Silver subdivision image.

The region records the oracle reports are checked against the rule itself,
evaluated here with numpy on the (separately pinned) exhaustive image E:

* level 0 is the g x g floor partition of the image (Sec. 4.2, G = g^2);
* a region whose ring dwells in E are all equal is filled with that value
  (Sec. 4.2.1: uniform perimeter -> terminal work T);
* otherwise a region no larger than B x B is computed pixel by pixel (the
  last-level work L), and a larger one is split into the r x r floor
  partition (S), whose non-empty pieces are exactly the next-level regions;
* the terminal regions partition the image, so each pixel is written once.

Together these fix the subdivision image completely, for every (g, r, B).
"""
import numpy as np
import pytest

from workloads import Window, random_params, random_windows

FILL, LEAF, SPLIT = 1, 2, 3


def floor_parts(a, length, parts):
    return [(a + (j * length) // parts, a + ((j + 1) * length) // parts) for j in range(parts)]


def ring_values(E, x, y, w, h):
    blk = E[y:y + h, x:x + w]
    if w <= 2 or h <= 2:
        return blk.ravel()
    return np.concatenate([blk[0], blk[-1], blk[1:-1, 0], blk[1:-1, -1]])


def check_subdivision(E, S, recs, st, g, r, B):
    H, W = E.shape
    by_level = {}
    for rec in recs:
        by_level.setdefault(int(rec["level"]), set()).add(
            (int(rec["x"]), int(rec["y"]), int(rec["w"]), int(rec["h"])))
    # level 0 is the g x g floor partition
    want0 = {(xa, ya, xb - xa, yb - ya) for (ya, yb) in floor_parts(0, H, g)
             for (xa, xb) in floor_parts(0, W, g)}
    assert by_level[0] == want0
    cover = np.zeros_like(E, dtype=np.int32)
    iters_ring = iters_leaf = ring_new = leaf_inner = ring_filled = 0
    kids_expected = {}
    for rec in recs:
        x, y, w, h, lv, kind, v = (int(rec[k]) for k in ("x", "y", "w", "h", "level", "kind", "value"))
        ring = ring_values(E, x, y, w, h)
        iters_ring += int(ring.astype(np.int64).sum())
        uniform = bool((ring == ring[0]).all())
        if kind == FILL:
            ring_filled += int(ring.astype(np.int64).sum())
            assert uniform and v == ring[0]
            assert (S[y:y + h, x:x + w] == v).all()
            cover[y:y + h, x:x + w] += 1
        elif kind == LEAF:
            assert not uniform and w <= B and h <= B
            assert np.array_equal(S[y:y + h, x:x + w], E[y:y + h, x:x + w])
            cover[y:y + h, x:x + w] += 1
            iters_leaf += int(E[y:y + h, x:x + w].astype(np.int64).sum())
            inner = E[y + 1:y + h - 1, x + 1:x + w - 1]
            leaf_inner += int(inner.astype(np.int64).sum())
        else:
            assert kind == SPLIT
            assert not uniform and (w > B or h > B)
            kids = {(xa, ya, xb - xa, yb - ya) for (ya, yb) in floor_parts(y, h, r)
                    for (xa, xb) in floor_parts(x, w, r) if xb > xa and yb > ya}
            for k in kids:
                kids_expected.setdefault(lv + 1, set()).add(k)
                kx, ky, kw, kh = k
                # ring pixels of the child that are not on this region's ring
                blk = np.zeros((kh, kw), dtype=bool)
                blk[0, :] = blk[-1, :] = True
                blk[:, 0] = blk[:, -1] = True
                yy, xx = np.nonzero(blk)
                yy, xx = yy + ky, xx + kx
                on_parent = (xx == x) | (xx == x + w - 1) | (yy == y) | (yy == y + h - 1)
                ring_new += int(E[yy[~on_parent], xx[~on_parent]].astype(np.int64).sum())
    for lv, kids in kids_expected.items():
        assert by_level.get(lv, set()) == kids
    assert set(by_level) == {0} | set(kids_expected)
    for x, y, w, h in by_level[0]:
        ring_new += int(ring_values(E, x, y, w, h).astype(np.int64).sum())
    assert (cover == 1).all()
    # the subdivision image differs from E only strictly inside filled regions
    for rec in recs:
        if int(rec["kind"]) == FILL:
            x, y, w, h = (int(rec[k]) for k in ("x", "y", "w", "h"))
            cover[y + 1:y + h - 1, x + 1:x + w - 1] = 0
    assert ((S != E) <= (cover == 0)).all()
    # statistics agree with the records
    assert st["iters_ring"] == iters_ring and st["iters_leaf"] == iters_leaf
    assert st["iters_ring_new"] == ring_new and st["iters_leaf_inner"] == leaf_inner
    assert st["iters_ring_filled"] == ring_filled
    for lv in range(st["levels"]):
        assert st["regions"][lv] == len(by_level[lv])
        recs_lv = recs[recs["level"] == lv]
        assert st["fills"][lv] == int((recs_lv["kind"] == FILL).sum())
        assert st["leaves"][lv] == int((recs_lv["kind"] == LEAF).sum())
        assert st["splits"][lv] == int((recs_lv["kind"] == SPLIT).sum())


CASES = [
    (Window(-1.5, 0.5, -1.0, 1.0, 128, 128, 256), 4, 2, 16),
    (Window(-1.5, 0.5, -1.0, 1.0, 128, 128, 256), 2, 4, 8),
    (Window(-1.5, 0.5, -1.0, 1.0, 100, 77, 300), 3, 3, 5),
    (Window(-0.8, -0.7, 0.05, 0.15, 96, 80, 500), 5, 2, 7),
    (Window(-2.1, 0.7, -1.3, 1.3, 61, 127, 64), 1, 5, 3),
    (Window(-1.5, 0.5, -1.0, 1.0, 64, 64, 128), 8, 8, 1),
]


@pytest.mark.parametrize("w,g,r,B", CASES)
def test_subdivision_follows_the_rule(ref, w, g, r, B):
    E, _ = ref.exhaustive(w)
    S, st, recs = ref.subdiv(w, g, r, B, records=True)
    check_subdivision(E, S, recs, st, g, r, B)


def test_subdivision_brute_force_all_parameters(ref):
    # Every (g, r, B) on tiny ragged images.
    for w in [Window(-1.5, 0.5, -1.0, 1.0, 13, 11, 60),
              Window(-0.2, 0.45, 0.3, 0.9, 12, 12, 100)]:
        E, _ = ref.exhaustive(w)
        for g in range(1, min(w.W, w.H) + 1):
            for r in range(2, 14):
                for B in range(1, 14):
                    S, st, recs = ref.subdiv(w, g, r, B, records=True, threads=1)
                    check_subdivision(E, S, recs, st, g, r, B)


def test_random_windows_follow_the_rule(ref):
    for i, w in enumerate(random_windows(21, 25, max_side=70, max_dwell=200)):
        E, _ = ref.exhaustive(w)
        for p in random_params(100 + i, w, 3):
            S, st, recs = ref.subdiv(w, p.g, p.r, p.B, records=True)
            check_subdivision(E, S, recs, st, p.g, p.r, p.B)


@pytest.mark.parametrize("w,g,r,B", CASES)
def test_depth_first_equals_level_order(ref, w, g, r, B):
    a, sa = ref.subdiv(w, g, r, B, order="bfs")
    b, sb = ref.subdiv(w, g, r, B, order="dfs", threads=1)
    assert np.array_equal(a, b)
    assert sa == sb


def test_threads_agree(ref):
    w = Window(-1.5, 0.5, -1.0, 1.0, 300, 260, 400)
    a, sa = ref.subdiv(w, 4, 2, 16, threads=1)
    b, sb = ref.subdiv(w, 4, 2, 16, threads=7)
    assert np.array_equal(a, b) and sa == sb


def test_window_outside_radius_two_fills_at_level_zero(ref):
    w = Window(2.5, 3.5, 2.5, 3.5, 200, 150, 1000)
    S, st = ref.subdiv(w, 4, 2, 16)
    assert (S == 1).all()
    assert st["levels"] == 1 and st["fills"][0] == 16 and st["iters_leaf"] == 0


def test_window_inside_cardioid_fills_at_level_zero(ref):
    w = Window(-0.3, -0.1, -0.1, 0.1, 120, 120, 700)
    S, st = ref.subdiv(w, 3, 2, 16)
    assert (S == 700).all()
    assert st["levels"] == 1 and st["fills"][0] == 9


def test_all_ring_regions_give_the_exhaustive_image(ref):
    # g >= max(W, H) / 2: every level-0 region is at most 2 x 2, all ring,
    # so S = E whatever B is; with B >= 2 nothing splits.
    w = Window(-1.5, 0.5, -1.0, 1.0, 40, 40, 300)
    E, _ = ref.exhaustive(w)
    for B in (1, 2, 5):
        S, st = ref.subdiv(w, 20, 2, B)
        assert np.array_equal(S, E)
        assert st["levels"] == (2 if B == 1 else 1)


def test_stop_size_above_level_zero_side_never_splits(ref):
    w = Window(-1.5, 0.5, -1.0, 1.0, 90, 90, 300)
    E, _ = ref.exhaustive(w)
    S, st = ref.subdiv(w, 3, 2, 30)
    assert st["levels"] == 1 and st["splits"][0] == 0
    assert st["fills"][0] + st["leaves"][0] == 9


def test_sampled_pixels_equal_full_image(ref):
    for w, g, r, B in CASES:
        S, _ = ref.subdiv(w, g, r, B)
        rng = np.random.default_rng(5)
        px = rng.integers(0, w.W, 300)
        py = rng.integers(0, w.H, 300)
        assert np.array_equal(ref.subdiv_pixels(w, g, r, B, px, py), S[py, px])


def test_mirror_symmetry_of_subdivision(ref):
    # With H divisible by g * r^levels the partition is mirror-symmetric, so
    # the subdivision image inherits the exhaustive image's exact symmetry.
    w = Window(-1.9, 0.6, -1.1, 1.1, 128, 128, 300)
    S, _ = ref.subdiv(w, 4, 2, 8)
    assert np.array_equal(S, S[::-1])


def test_bad_parameters_rejected(ref):
    w = Window(-1.5, 0.5, -1.0, 1.0, 32, 32, 50)
    for g, r, B in [(0, 2, 4), (33, 2, 4), (4, 1, 4), (4, 2, 0)]:
        with pytest.raises(ValueError):
            ref.subdiv(w, g, r, B)
