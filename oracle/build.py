"""Build the CPU oracle library (test infrastructure).

Compiles ``askref.c`` (2-D images) and ``askref3.c`` (3-D volumes) with gcc at
-O2, with floating-point contraction off and no fast-math, so that every
binary64 operation is rounded on its own.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libaskref.so")
LIB3 = os.path.join(HERE, "libaskref3.so")
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
         "-shared", "-pthread", "-Wall", "-Wextra", "-Werror"]


def build(extra=(), src=None, out=None):
    """Compile the oracle (``askref.c``, or another source such as a copy
    with a planted mistake) and return the library path."""
    src = src or os.path.join(HERE, "askref.c")
    out = out or LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *FLAGS, "-I", HERE, *extra, src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build3():
    """Compile the 3-D oracle (``askref3.c``) and return the library path."""
    return build(src=os.path.join(HERE, "askref3.c"), out=LIB3)


if __name__ == "__main__":
    print(build())
    print(build3())
