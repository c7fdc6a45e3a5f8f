"""Write the pool of boundary points that the deep-zoom, batched and serving
workloads centre their windows on (test and workload infrastructure; it
calls only the oracle).

Rejection sampling: c uniform in [-2, 0.5] x [-1.25, 1.25] from numpy's
PCG64 seeded with SEED, drawn in blocks of BLOCK candidates (real parts, then
imaginary parts); candidates strictly inside the main cardioid or the
period-2 bulb are skipped (their dwell is the maximum); a candidate is kept
when 4096 <= dwell(c, 8192) <= 8110, i.e. between half and 99 % of the
maximum dwell, which puts it within a few pixel widths of the set's
boundary at any zoom the workloads use. The first COUNT kept points, in
draw order, are written one per line as two hex floats.

    python -m oracle.make_boundary_pool [--out inputs/boundary_pool.txt]
"""
import argparse
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

SEED = 2206
COUNT = 1024
BLOCK = 1 << 16
D = 8192
LO, HI = 4096, 8110
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(os.path.dirname(HERE), "inputs", "boundary_pool.txt")


def inside_cardioid_or_bulb(x, y):
    """Main cardioid q (q + (x - 1/4)) < y^2 / 4 with q = (x - 1/4)^2 + y^2,
    or the disc (x + 1)^2 + y^2 < 1/16."""
    q = (x - 0.25) ** 2 + y * y
    return (q * (q + (x - 0.25)) < 0.25 * y * y) | ((x + 1.0) ** 2 + y * y < 1.0 / 16.0)


def accepted(xy):
    from oracle import askref
    xs, ys = xy
    return [i for i, (x, y) in enumerate(zip(xs, ys)) if LO <= askref.dwell(x, y, D) <= HI]


def make(count=COUNT, workers=8):
    rng = np.random.default_rng(SEED)
    pool = []
    with ProcessPoolExecutor(workers) as ex:
        while len(pool) < count:
            blocks = []
            for _ in range(workers):
                x = rng.uniform(-2.0, 0.5, BLOCK)
                y = rng.uniform(-1.25, 1.25, BLOCK)
                keep = ~inside_cardioid_or_bulb(x, y)
                blocks.append((x[keep].tolist(), y[keep].tolist()))
            for (xs, ys), idx in zip(blocks, ex.map(accepted, blocks)):
                pool.extend((xs[i], ys[i]) for i in idx)
    return pool[:count]


def write(pool, path):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("# boundary points c = x + iy, %d <= dwell(c, %d) <= %d; written by "
                "oracle/make_boundary_pool.py (seed %d)\n" % (LO, D, HI, SEED))
        for x, y in pool:
            f.write("%s %s\n" % (float(x).hex(), float(y).hex()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--count", type=int, default=COUNT)
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    write(make(args.count, args.workers), args.out)


if __name__ == "__main__":
    main()
