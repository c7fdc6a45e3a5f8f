"""Host logic of the serving loop (CPU): the output arena's allocator."""
import numpy as np

from paper_2206_02255_amd.serve import FirstFit


def test_first_fit_reuses_and_merges():
    a = FirstFit(100)
    x, y, z = a.alloc(30), a.alloc(30), a.alloc(30)
    assert (x, y, z) == (0, 30, 60) and a.alloc(20) is None
    a.release(y, 30)
    assert a.alloc(40) is None and a.alloc(25) == 30
    a.release(30, 25)
    a.release(x, 30)
    a.release(z, 30)
    assert a.free == [(0, 100)]


def test_first_fit_never_overlaps():
    rng = np.random.default_rng(3)
    a = FirstFit(1000)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off = list(live)[int(rng.integers(len(live)))]
            a.release(off, live.pop(off))
        else:
            n = int(rng.integers(1, 120))
            off = a.alloc(n)
            if off is not None:
                live[off] = n
        used = np.zeros(1000, dtype=int)
        for o, n in live.items():
            used[o:o + n] += 1
        for o, n in a.free:
            used[o:o + n] += 1
        assert used.max() == 1 and used.min() == 1  # live and free ranges tile [0, 1000)
