"""Seeded synthetic inputs shared by the tests and the benchmark.

This module only describes inputs: windows of the complex plane, image sizes,
maximum dwells and subdivision parameters. It holds none of the dwell or
subdivision arithmetic, so the GPU path and the CPU oracle can both use it
without sharing any of the method.

Workloads follow the paper's experiment (Sec. 6.1): the Mandelbrot set over
the window with corners (-1.5, -1) and (0.5, 1), square images, dwell limit
512, and the subdivision parameter grid {g, r, B} (Sec. 6.2).
"""
from dataclasses import dataclass
import math

import numpy as np


@dataclass(frozen=True)
class Window:
    """Complex rectangle [x0, x1] x [y0, y1] rendered at W x H pixels with
    maximum dwell D. Row 0 of an image lies on the y0 side."""
    x0: float
    x1: float
    y0: float
    y1: float
    W: int
    H: int
    D: int

    @property
    def pixels(self):
        return self.W * self.H


@dataclass(frozen=True)
class Params:
    """Subdivision parameters: initial g x g grid, r x r split, stop size B."""
    g: int
    r: int
    B: int


# Sec. 6.1: window corners (-1.5, -1) and (0.5, 1), i.e. [-1.5, 0.5] x [-1, 1].
PAPER_WINDOW = (-1.5, 0.5, -1.0, 1.0)


def paper_window(n, D):
    """The paper's window at n x n pixels and dwell limit D."""
    return Window(*PAPER_WINDOW, n, n, D)


# 1024 x 1024, D = 512, subdivision {4, 2, 32}: the small single-image case.
SMALL = paper_window(1024, 512)
SMALL_PARAMS = Params(4, 2, 32)

# 16384 x 16384, D = 2048: the large single-image case and its {g, r, B} sweep.
LARGE = paper_window(16384, 2048)
LARGE_SWEEP = [Params(g, r, B) for g in (2, 4, 8, 16, 32)
               for r in (2, 4, 8) for B in (16, 32, 64, 128)]
# The benchmark's launch configuration for the large image.
LARGE_DEFAULT = Params(64, 2, 32)
LARGE_DEFAULT_FORM = "persistent"


def random_windows(seed, count, max_side=96, max_dwell=300):
    """Small random windows over the region of interest [-2.2, 0.8] x [-1.3, 1.3]
    with ragged, non-square pixel sizes, for parity tests."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        cx = rng.uniform(-2.0, 0.6)
        cy = rng.uniform(-1.2, 1.2)
        span = math.exp(rng.uniform(math.log(1e-3), math.log(3.0)))
        aspect = rng.uniform(0.5, 2.0)
        W = int(rng.integers(1, max_side + 1))
        H = int(rng.integers(1, max_side + 1))
        D = int(rng.integers(1, max_dwell + 1))
        hw, hh = span / 2, span * aspect / 2
        out.append(Window(cx - hw, cx + hw, cy - hh, cy + hh, W, H, D))
    return out


def random_params(seed, window, count):
    """Random valid (g, r, B) for a window."""
    rng = np.random.default_rng(seed)
    lim = min(window.W, window.H)
    out = []
    for _ in range(count):
        g = int(rng.integers(1, min(lim, 16) + 1))
        r = int(rng.integers(2, 9))
        B = int(rng.integers(1, 64))
        out.append(Params(g, r, B))
    return out
