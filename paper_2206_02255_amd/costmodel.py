"""The paper's subdivision cost model (Sec. 4), evaluated for parameter grids.

Host-side tool for the autotuner: it predicts which (g, r, B) a subdivision
should use, from the self-similar-density form of the model (Sec. 4.2.1,
P_i = P for every level, square images, g = g_x = g_y, r = r_x = r_y) with
the Mandelbrot terms Q_i = 4 n A / (g r^i), T_i = n^2 / (G R^i), S = lambda A.
Notation: n image side, A application work per element (the dwell limit),
G = g^2, R = r^2, tau = log_r(n / (g B)) levels, q multiprocessors of c cores.

The work uses the closed form of the level sums (geometric series); the times
keep the ceilings of Sec. 4.3.1 and 4.3.2 and are summed level by level.
Every function accepts numpy arrays for g, r, B, P and lam (broadcast).
"""
import numpy as np


def tau(n, g, r, B):
    """Number of levels tau = log_r(n / (g B)), rounded, at least 1."""
    g, r, B = (np.asarray(v, dtype=np.float64) for v in (g, r, B))
    return np.maximum(1, np.rint(np.log(n / (g * B)) / np.log(r))).astype(np.int64)


def _geometric(x, m):
    """sum_{i=0}^{m-1} x^i."""
    x = np.asarray(x, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    near_one = np.abs(1.0 - x) < 1e-12
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (1.0 - x ** m) / (1.0 - x)
    return np.where(near_one, m, s)


def work_exhaustive(n, A):
    """W_E = n^2 A (Sec. 4.1)."""
    return float(n) * n * A


def work_subdivision(n, g, r, B, A, P, lam):
    """W_SSD^M (Sec. 4.2.1):
    sum_{i<tau-1} [Q_i + P S + (1-P) T_i] G R^i P^i + n^2 A P^{tau-1}
    = 4 n A g sum (rP)^i + lam A G P sum (RP)^i + n^2 (1 - P^{tau-1})
      + n^2 A P^{tau-1}."""
    g, r, B, P, lam = (np.asarray(v, dtype=np.float64) for v in (g, r, B, P, lam))
    m = tau(n, g, r, B) - 1
    n2 = float(n) * n
    return (4.0 * n * A * g * _geometric(r * P, m)
            + lam * A * g * g * P * _geometric(r * r * P, m)
            + n2 * (1.0 - P ** m) + n2 * A * P ** m)


def reduction_factor(n, g, r, B, A, P, lam):
    """Omega = W_E / W_SSD^M (Sec. 4.2.2); never above A."""
    return work_exhaustive(n, A) / work_subdivision(n, g, r, B, A, P, lam)


def time_exhaustive(n, A, q, c):
    """T_Ex = ceil(n^2 / (q c)) A (Sec. 4.3)."""
    return np.ceil(float(n) * n / (q * c)) * A


def _levels(n, g, r, B, P, lam):
    g, r, B, P, lam = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64)
                                           for v in (g, r, B, P, lam)))
    t = tau(n, g, r, B)
    return g, r, B, P, lam, t


def time_sbr(n, g, r, B, A, P, lam, q, c):
    """T_SBR (Sec. 4.3.1): one block of c cores per region, the G R^i regions
    of level i in ceil(G R^i / q) rounds."""
    g, r, B, P, lam, t = _levels(n, g, r, B, P, lam)
    n = float(n)
    total = np.zeros(g.shape)
    for i in range(int(t.max()) - 1):
        live = i < t - 1
        GRi = g * g * (r * r) ** i
        per_region = (np.ceil(4.0 * n / (g * r ** i * c)) * A + P * lam * A
                      + (1.0 - P) * np.ceil(n * n / (GRi * c)))
        total += np.where(live, per_region * np.ceil(GRi / q) * P ** i, 0.0)
    last = t - 1
    GRl = g * g * (r * r) ** last
    total += A * np.ceil(n * n / (GRl * c)) * np.ceil(GRl / q) * P ** last
    return total


def time_mbr(n, g, r, B, A, P, lam, q, c):
    """T_MBR (Sec. 4.3.2): queries and splits one block per region; fills and
    the last level on all q c cores."""
    g, r, B, P, lam, t = _levels(n, g, r, B, P, lam)
    n = float(n)
    total = np.zeros(g.shape)
    for i in range(int(t.max()) - 1):
        live = i < t - 1
        GRi = g * g * (r * r) ** i
        term = (np.ceil(4.0 * n / (g * r ** i * c)) * np.ceil(GRi / q) * A * P ** i
                + np.ceil(GRi / q) * lam * A * P ** (i + 1)
                + np.ceil(n * n * P ** i * (1.0 - P) / (q * c)))
        total += np.where(live, term, 0.0)
    total += A * np.ceil(n * n / (q * c)) * P ** (t - 1)
    return total


def speedup_sbr(n, g, r, B, A, P, lam, q, c):
    return time_exhaustive(n, A, q, c) / time_sbr(n, g, r, B, A, P, lam, q, c)


def speedup_mbr(n, g, r, B, A, P, lam, q, c):
    return time_exhaustive(n, A, q, c) / time_mbr(n, g, r, B, A, P, lam, q, c)


def split_probability(stats):
    """Measured P: the mean over the levels that can split of the fraction
    of scanned regions that split (SSD assumption i)."""
    ps = [s / max(1, n) for s, n in zip(stats["splits"], stats["regions"]) if n]
    ps = ps[:-1] if len(ps) > 1 else ps
    return float(np.mean(ps)) if ps else 0.0


# ---------------------------------------------------------------------------
# Model with measured GPU overheads: a split probability per level, read from
# the render's counters or, for parameters not yet rendered, from the split
# probability as a function of the region side; and a per-region scheduling
# cost sigma. Evaluated one (g, r, B) at a time.
# ---------------------------------------------------------------------------

def rendered_levels(n, g, r, B):
    """The levels a render has: 1 + the number of r-fold splits that take
    the level-0 side ceil(n / g) down to B or below (the paper's tau as
    printed counts one fewer; see the stop rule's reading)."""
    s, levels = -(-int(n) // int(g)), 1
    while s > B:
        s = -(-s // int(r))
        levels += 1
    return levels


def level_sides(n, g, r, B, levels=None):
    """Region side n / (g r^i) of each model level i (tau as printed, or
    the given level count)."""
    t = int(tau(n, g, r, B)) if levels is None else int(levels)
    return [float(n) / (g * r ** i) for i in range(t)]


def split_probabilities(stats):
    """Measured P_i of every level that can split: splits / regions."""
    ps = [s / max(1, n) for s, n in zip(stats["splits"], stats["regions"]) if n]
    return ps[:-1] if len(ps) > 1 else ps


def time_sbr_levels(n, g, r, B, A, P, lam, q, c, sigma=0.0, levels=None):
    """T_SBR (Sec. 4.3.1) with a split probability per level (a sequence;
    its last value serves deeper levels), a per-region cost sigma in the
    units of the other terms, and tau as printed or the given level count.
    One P for every level, sigma = 0 and tau as printed give time_sbr."""
    t = int(tau(n, g, r, B)) if levels is None else int(levels)
    Ps = list(np.atleast_1d(np.asarray(P, dtype=np.float64)))
    Ps = (Ps + [Ps[-1]] * t)[:t]
    G, R, n = float(g) * g, float(r) * r, float(n)
    levels = np.arange(t - 1)
    GRi = G * R ** levels
    reach = np.concatenate(([1.0], np.cumprod(Ps[:t - 1])))  # prod_{j<i} P_j, i = 0..t-1
    P_arr = np.asarray(Ps[:t - 1])
    per_region = (np.ceil(4.0 * n / (g * r ** levels * c)) * A + P_arr * lam * A
                  + (1.0 - P_arr) * np.ceil(n * n / (GRi * c)) + sigma)
    total = float(np.sum(per_region * np.ceil(GRi / q) * reach[:t - 1]))
    GRl = G * R ** (t - 1)
    total += (A * np.ceil(n * n / (GRl * c)) + sigma) * np.ceil(GRl / q) * reach[t - 1]
    return float(total)


def split_curve(points):
    """P as a function of the region side, from measured (side, P) pairs:
    the mean P of each distinct side, linear in log2(side) between them and
    constant beyond the ends."""
    by_side = {}
    for s, p in points:
        by_side.setdefault(float(s), []).append(float(p))
    xs = np.log2(np.array(sorted(by_side)))
    ys = np.array([np.mean(by_side[s]) for s in sorted(by_side)])

    def P(side):
        return float(np.interp(np.log2(float(side)), xs, ys))
    return P


def predict_sbr(n, g, r, B, A, curve, lam, q, c, sigma=0.0):
    """time_sbr_levels over the rendered levels, each level's P read from
    curve(side)."""
    L = rendered_levels(n, g, r, B)
    sides = level_sides(n, g, r, B, L)
    Ps = [curve(s) for s in sides[:-1]] or [0.0]
    return time_sbr_levels(n, g, r, B, A, Ps, lam, q, c, sigma, L)
