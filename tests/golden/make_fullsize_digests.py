"""Write fullsize_mandelbrot16384_D2048.txt: SHA-256 digests of the oracle's
full 16384 x 16384 images of the paper's window (Sec. 6.1 window, D = 2048),
for every point of the (g, r, B) sweep of Sec. 6.2 and the benchmark's
(64, 4, 16), and of the exhaustive image, with each subdivision image's
algorithmic iteration count (ring dwells of every scanned region plus leaf
dwells) and its mismatch count against the exhaustive image.

Only the CPU oracle runs here; the GPU tests compare digests of their own
images with these. Run: python tests/golden/make_fullsize_digests.py [threads]
"""
import hashlib
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import askref  # noqa: E402
from workloads import LARGE, LARGE_DEFAULT, LARGE_SWEEP  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_mandelbrot16384_D2048.txt")


def digest(img):
    return hashlib.sha256(np.ascontiguousarray(img, dtype="<u4").tobytes()).hexdigest()


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    w = LARGE
    t = time.time()
    E, iters_e = askref.exhaustive(w, threads=threads)
    lines = ["# Oracle digests of the 16384 x 16384 paper window [-1.5, 0.5] x [-1, 1], D = 2048.",
             "# Written by tests/golden/make_fullsize_digests.py (oracle only).",
             "# exhaustive <sha256 of the uint32 little-endian image> <sum of dwells>",
             "# g r B <sha256> <algorithmic iterations> <pixels differing from the exhaustive image>",
             "exhaustive %s %d" % (digest(E), iters_e)]
    print("exhaustive %.1f s" % (time.time() - t), flush=True)
    configs = list(LARGE_SWEEP) + [LARGE_DEFAULT]
    for p in configs:
        t = time.time()
        S, st = askref.subdiv(w, p.g, p.r, p.B, threads=threads)
        lines.append("%d %d %d %s %d %d" % (p.g, p.r, p.B, digest(S), st["iters_alg"],
                                            int(np.count_nonzero(S != E))))
        print(lines[-1], "%.1f s" % (time.time() - t), flush=True)
        del S
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
