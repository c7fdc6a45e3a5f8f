"""The 3-D subdivision's algorithmic work, from the oracle (test
infrastructure: documentation figures, not the product path).

For each (g, r, B): the dwell iterations of every decided box's whole
surface and of the voxels inside its leaf boxes (the oracle's counters), and
the exhaustive volume's sum of dwells, on the benchmark's quaternion Julia
volume. Their ratio bounds what the subdivision can gain at equal kernel
efficiency.

    python -m oracle.work3 32,2,8 64,2,8
"""
import sys

from . import askref3


def main(argv):
    sys.path.insert(0, ".")
    import workloads
    v = workloads.VOLUME
    ex = int(askref3.exhaustive(v).sum(dtype="int64"))
    print("exhaustive: %d iterations" % ex)
    for spec in argv or ["32,2,8"]:
        g, r, B = (int(x) for x in spec.split(","))
        _, st = askref3.subdiv(v, g, r, B)
        w = st["iters_surface"] + st["iters_leaf"]
        print("(%d, %d, %d): surfaces %d + leaf insides %d = %d iterations; exhaustive / "
              "subdivision = %.3f; boxes per level %s"
              % (g, r, B, st["iters_surface"], st["iters_leaf"], w, ex / w, st["regions"]))


if __name__ == "__main__":
    main(sys.argv[1:])
